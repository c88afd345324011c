"""Exact references for the spin-1/2 XY chain H = sum_i S^x_i S^x_{i+1} + S^y_i S^y_{i+1} (J = 1)
(test infrastructure; independent of the oracle and of the HIP path).

* Dense exact diagonalisation of the periodic N-spin chain (N <= 12).
* The Jordan-Wigner solution (paper, Supplemental Material G): spinless fermions with dispersion
  e_q = cos q, the partition function split into the even and odd fermion-parity sectors with
  their momentum sets; it is checked here against the dense diagonalisation, not taken on trust.
* The infinite chain: ln Z / N = (1/2 pi) int_0^{2 pi} ln(1 + exp(-beta cos q)) dq, by the
  trapezoid rule on a periodic grid (spectrally accurate; the grid is doubled until two successive
  values agree to 1e-15 relative).
* Dense products of the second-order Trotter gates on a ring of two-spin cells, the operator the
  MPO of paper_1912_02780_amd.inputs.xy_trotter_mpo represents.
"""

from __future__ import annotations

import math

import numpy as np

SX = np.array([[0.0, 0.5], [0.5, 0.0]])
SY_IM = np.array([[0.0, -0.5], [0.5, 0.0]])   # S^y = i * SY_IM; S^y S^y = -(SY_IM x SY_IM)


def _site_op(op, i, N):
    out = np.array([[1.0]])
    for j in range(N):
        out = np.kron(out, op if j == i else np.eye(2))
    return out


def bond_h(N, i, j):
    """S^x_i S^x_j + S^y_i S^y_j on N spins (spin 0 is the most significant bit; up = 0)."""
    return _site_op(SX, i, N) @ _site_op(SX, j, N) - _site_op(SY_IM, i, N) @ _site_op(SY_IM, j, N)


def dense_hamiltonian(N):
    """Periodic N-spin XY chain."""
    H = np.zeros((2 ** N, 2 ** N))
    for i in range(N):
        H += bond_h(N, i, (i + 1) % N)
    return H


def ed_lnZ(beta, N):
    """ln Tr exp(-beta H) of the periodic N-spin chain by full diagonalisation."""
    ev = np.linalg.eigvalsh(dense_hamiltonian(N))
    m = np.min(-beta * ev)
    return float(m + np.log(np.sum(np.exp(-beta * ev - m))))


def jw_lnZ(beta, N):
    """ln(Z_+ + Z_-) of the periodic N-spin chain from the Jordan-Wigner fermions: even-parity states
    of the modes q = 2 pi (n + 1/2) / N and odd-parity states of the modes q = 2 pi n / N (the sector
    momenta that reproduce the dense diagonalisation for even N, see the pins)."""
    n = np.arange(N)

    def logs(q):
        # ln prod(1 + x) and (ln |prod(1 - x)|, sign of prod(1 - x)), x = exp(-beta cos q)
        x = np.exp(-beta * np.cos(q))
        with np.errstate(divide="ignore"):
            lm = np.log(np.abs(1.0 - x))
        sgn = float(np.prod(np.sign(1.0 - x)))
        return float(np.sum(np.log1p(x))), float(np.sum(lm)), sgn

    ap, am, sa = logs(2.0 * np.pi * (n + 0.5) / N)
    pp, pm, sp = logs(2.0 * np.pi * n / N)
    terms = [(ap, 1.0), (am, sa), (pp, 1.0), (pm, -sp)]
    m = max(a for a, s_ in terms if s_ != 0.0)
    return m + math.log(0.5 * sum(s_ * math.exp(a - m) for a, s_ in terms if s_ != 0.0))


def lnZ_per_spin_infinite(beta, tol=1e-15):
    """(1/2 pi) int_0^{2 pi} ln(1 + exp(-beta cos q)) dq by the periodic trapezoid rule."""
    M = 256
    prev = None
    while True:
        q = 2.0 * np.pi * np.arange(M) / M
        v = float(np.mean(np.logaddexp(0.0, -beta * np.cos(q))))
        if prev is not None and abs(v - prev) <= tol * abs(v):
            return v
        prev = v
        M *= 2
        if M > 1 << 24:
            raise RuntimeError("quadrature did not converge")


def dense_trotter_rho(tau, n_cells):
    """exp(-tau/2 H_o) exp(-tau H_e) exp(-tau/2 H_o) on a ring of n_cells two-spin cells (2 n_cells
    spins): H_o the bonds (2c, 2c+1) inside the cells, H_e the bonds (2c+1, 2c+2) between them."""
    from scipy.linalg import expm
    N = 2 * n_cells
    Ho = sum(bond_h(N, 2 * c, 2 * c + 1) for c in range(n_cells))
    He = sum(bond_h(N, 2 * c + 1, (2 * c + 2) % N) for c in range(n_cells))
    eo = expm(-0.5 * tau * Ho)
    return eo @ expm(-tau * He) @ eo
