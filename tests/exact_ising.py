"""Exact references that pin the oracle (test infrastructure; independent of the oracle).

* Exhaustive spin enumeration of the L x L periodic Ising model (Z = sum over all 2^(L^2)
  configurations of exp(beta * sum_<ij> s_i s_j), J = 1, h = 0), evaluated from the exact
  histogram of bond sums in mpmath at 30 digits.
* Brute-force bond sums for a 2 x 2 periodic network of one arbitrary rank-4 tensor: every one
  of the D^8 bond configurations is visited and its product of four tensor entries added.  The
  gradient of Z with respect to the tensor is the sum of the four one-hole environments, also
  by brute force.
* Onsager's closed form for the infinite square lattice: free energy by quadrature (mpmath) and
  internal energy through the complete elliptic integral K (both written from the textbook
  solution, not from the paper).  At the exact critical coupling the free energy reduces to
  ln(2)/2 + 2 G / pi (G = Catalan's constant), which checks the quadrature.
"""

from __future__ import annotations

import functools
import itertools

import mpmath
import numpy as np

mpmath.mp.dps = 30


@functools.lru_cache(maxsize=None)
def torus_bond_sum_histogram(L: int) -> dict:
    """Histogram {E: count} of E = sum over the 2 L^2 nearest-neighbour bonds of s_i s_j."""
    n = L * L
    if n > 20:
        raise ValueError("enumeration limited to 20 spins")
    idx = np.arange(1 << n, dtype=np.int64)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(n)[None, :]) & 1)       # (2^n, n) of +-1
    s = spins.reshape(-1, L, L)
    E = (s * np.roll(s, 1, axis=1)).sum(axis=(1, 2)) + (s * np.roll(s, 1, axis=2)).sum(axis=(1, 2))
    vals, counts = np.unique(E, return_counts=True)
    return {int(v): int(c) for v, c in zip(vals, counts)}


def torus_lnZ_per_site(L: int, beta: float):
    """(lnZ/N, (1/N) d lnZ/d beta) of the periodic L x L Ising model, exact (mpmath)."""
    hist = torus_bond_sum_histogram(L)
    b = mpmath.mpf(beta)
    Z = mpmath.fsum(c * mpmath.exp(b * E) for E, c in hist.items())
    dZ = mpmath.fsum(c * E * mpmath.exp(b * E) for E, c in hist.items())
    N = L * L
    return float(mpmath.log(Z) / N), float(dZ / Z / N)


def bruteforce_2x2(T_lurd: np.ndarray):
    """Z and dZ/dT of the 2 x 2 periodic network of T[l][u][r][d], by visiting all D^8 bond states.

    Sites (x, y), x, y in {0, 1}.  Bond h[x][y] joins the right leg of (x, y) to the left leg of
    (x+1 mod 2, y); bond v[x][y] joins the down leg of (x, y) to the up leg of (x, y+1 mod 2).
    Site (x, y) therefore sees legs (l, u, r, d) = (h[x-1][y], v[x][y-1], h[x][y], v[x][y]).
    """
    D = T_lurd.shape[0]
    T = np.asarray(T_lurd, dtype=np.float64)
    grid = np.array(list(itertools.product(range(D), repeat=8)), dtype=np.int64)   # (D^8, 8)
    h = grid[:, 0:4].reshape(-1, 2, 2)   # h[:, x, y]
    v = grid[:, 4:8].reshape(-1, 2, 2)   # v[:, x, y]
    legs = []
    for x in range(2):
        for y in range(2):
            legs.append((h[:, (x - 1) % 2, y], v[:, x, (y - 1) % 2], h[:, x, y], v[:, x, y]))
    vals = [T[l, u, r, d] for (l, u, r, d) in legs]
    prod = vals[0] * vals[1] * vals[2] * vals[3]
    Z = float(np.sum(prod))
    dZ = np.zeros_like(T)
    for s, (l, u, r, d) in enumerate(legs):
        others = np.ones_like(prod)
        for t in range(4):
            if t != s:
                others = others * vals[t]
        np.add.at(dZ, (l, u, r, d), others)
    return Z, dZ


def onsager_lnZ_per_site(beta: float) -> float:
    """ln Z / N = ln(2 cosh 2b) + (1/pi) int_0^{pi/2} ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt,
    k = 2 sinh 2b / cosh^2 2b."""
    b = mpmath.mpf(beta)
    k = 2 * mpmath.sinh(2 * b) / mpmath.cosh(2 * b) ** 2
    f = lambda t: mpmath.log((1 + mpmath.sqrt(1 - k * k * mpmath.sin(t) ** 2)) / 2)
    integral = mpmath.quad(f, [0, mpmath.pi / 4, mpmath.pi / 2])
    return float(mpmath.log(2 * mpmath.cosh(2 * b)) + integral / mpmath.pi)


def onsager_dlnZ_dbeta(beta: float) -> float:
    """-u per site, u = -coth 2b [1 + (2/pi)(2 tanh^2 2b - 1) K(k)], K the complete elliptic integral
    of the first kind with modulus k = 2 sinh 2b / cosh^2 2b (evaluated through the complementary
    modulus k' = |1 - sinh^2 2b| / cosh^2 2b for accuracy near criticality)."""
    b = mpmath.mpf(beta)
    s2, c2 = mpmath.sinh(2 * b), mpmath.cosh(2 * b)
    kp = abs(1 - s2 * s2) / (c2 * c2)
    # K(k) = pi / (2 AGM(1, k'))
    K = mpmath.pi / (2 * mpmath.agm(1, kp))
    u = -(c2 / s2) * (1 + (2 / mpmath.pi) * (2 * mpmath.tanh(2 * b) ** 2 - 1) * K)
    return float(-u)


def _onsager_energy_mp(b):
    s2, c2 = mpmath.sinh(2 * b), mpmath.cosh(2 * b)
    kp = abs(1 - s2 * s2) / (c2 * c2)
    K = mpmath.pi / (2 * mpmath.agm(1, kp))
    return -(c2 / s2) * (1 + (2 / mpmath.pi) * (2 * mpmath.tanh(2 * b) ** 2 - 1) * K)


def onsager_specific_heat(beta: float) -> float:
    """Specific heat per site c = beta^2 d^2(lnZ/N)/dbeta^2 = -beta^2 du/dbeta, the derivative of the
    closed-form energy above taken by mpmath at 30 digits (off the critical point, where c is finite)."""
    b = mpmath.mpf(beta)
    return float(-b * b * mpmath.diff(_onsager_energy_mp, b))


def onsager_critical_lnZ_per_site() -> float:
    """ln Z / N at the exact critical coupling: ln(2)/2 + 2 G / pi."""
    return float(mpmath.log(2) / 2 + 2 * mpmath.catalan / mpmath.pi)


BETA_C_EXACT = float(mpmath.log(1 + mpmath.sqrt(2)) / 2)
