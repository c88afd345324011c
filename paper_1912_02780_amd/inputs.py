"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module builds the initial site tensor T0 of the square-lattice network and nothing
else: it holds none of the coarse-graining arithmetic. Both the product path and the CPU
oracle take their inputs from here, so the two sides see bit-identical T0.

Layout of every tensor returned here: ``T0[l][u][r][d]`` (left, up, right, down), float64,
C-contiguous.

* Ising model (paper, Supplemental Material A, first equation): the partition function of
  the ferromagnet H = -J sum_<ij> s_i s_j (J = 1, h = 0) is the trace of a network of rank-4
  tensors T0_{lurd} = sum_s W_{sl} W_{su} W_{sr} W_{sd}, where W is the symmetric square
  root of the bond Boltzmann matrix [[e^b, e^-b], [e^-b, e^b]].  The site weight carries the
  four half-bonds around a spin, so one tensor per spin reproduces Z exactly.
* Random rank-4 tensor: i.i.d. uniform [0, 1) entries from ``numpy.random.default_rng(seed)``,
  averaged over the eight leg permutations of the square's point group (four rotations, each
  with and without the left/right mirror), so that it is invariant under the lattice
  symmetries.
* Chiral random tensor: the same entries averaged over the four rotations only, so that the
  tensor has no mirror symmetry and the Grams of the left and right unfoldings of a pair differ.
* Quantum XY chain H = sum_i S^x_i S^x_{i+1} + S^y_i S^y_{i+1} (spin 1/2, J = 1; paper, main text
  "Infinite quantum XY chain" and Supplemental Material F): the matrix-product operator of the
  second-order Trotter-Suzuki density operator rho(tau) = exp(-tau/2 H_o) exp(-tau H_e)
  exp(-tau/2 H_o), H_o (H_e) the bonds inside (between) two-spin cells.  One MPO tensor per cell
  M[l][u][r][d]: l, r the bonds to the neighbouring cells, u the cell's two-spin output index,
  d its input index (4 values each: 2 s1 + s2, spin up = 0).
* Random matrix-product operator tensor M[l][u][r][d]: i.i.d. uniform [0, 1) entries plus 0.1 from
  ``numpy.random.default_rng(seed)``, no symmetry (its transfer matrix is not symmetric).
"""

from __future__ import annotations

import math

import numpy as np

BETA_CRITICAL_CONFIG = 0.4406868  # the critical-temperature value used by the workloads


def ising_bond_root(beta: float) -> tuple[np.ndarray, np.ndarray]:
    """Return (W, dW/dbeta) with W the principal symmetric square root of the Boltzmann matrix.

    W = [[p, q], [q, p]], p = (sqrt(2 cosh b) + sqrt(2 sinh b)) / 2,
    q = (sqrt(2 cosh b) - sqrt(2 sinh b)) / 2, so that W @ W = [[e^b, e^-b], [e^-b, e^b]].
    Valid for beta > 0.
    """
    if not beta > 0.0:
        raise ValueError("beta must be positive")
    ch, sh = math.cosh(beta), math.sinh(beta)
    rc, rs = math.sqrt(2.0 * ch), math.sqrt(2.0 * sh)
    p, q = 0.5 * (rc + rs), 0.5 * (rc - rs)
    # d sqrt(2 cosh b)/db = sinh b / sqrt(2 cosh b);  d sqrt(2 sinh b)/db = cosh b / sqrt(2 sinh b)
    drc, drs = sh / rc, ch / rs
    dp, dq = 0.5 * (drc + drs), 0.5 * (drc - drs)
    W = np.array([[p, q], [q, p]], dtype=np.float64)
    dW = np.array([[dp, dq], [dq, dp]], dtype=np.float64)
    return W, dW


def ising_T0(beta: float) -> np.ndarray:
    """Ising site tensor T0[l][u][r][d] = sum_s W[s,l] W[s,u] W[s,r] W[s,d] (D = 2)."""
    W, _ = ising_bond_root(beta)
    return np.ascontiguousarray(np.einsum("sl,su,sr,sd->lurd", W, W, W, W))


def ising_T0_torch(beta):
    """``ising_T0`` from a 0-d float64 torch tensor beta with torch operations, so that autograd
    carries d/dbeta through T0 (elementwise products and a sum over s; no batched matmul)."""
    import torch
    ch, sh = torch.cosh(beta), torch.sinh(beta)
    rc, rs = torch.sqrt(2.0 * ch), torch.sqrt(2.0 * sh)
    p, q = 0.5 * (rc + rs), 0.5 * (rc - rs)
    W = torch.stack([torch.stack([p, q]), torch.stack([q, p])])   # W[s][leg]
    return (W[:, :, None, None, None] * W[:, None, :, None, None] * W[:, None, None, :, None]
            * W[:, None, None, None, :]).sum(0)


def ising_dT0_dbeta(beta: float) -> np.ndarray:
    """Derivative of ``ising_T0`` with respect to beta (product rule over the four W factors)."""
    W, dW = ising_bond_root(beta)
    e = "sl,su,sr,sd->lurd"
    d = (np.einsum(e, dW, W, W, W) + np.einsum(e, W, dW, W, W)
         + np.einsum(e, W, W, dW, W) + np.einsum(e, W, W, W, dW))
    return np.ascontiguousarray(d)


def square_group_images(T: np.ndarray) -> list[np.ndarray]:
    """The eight images of a [l][u][r][d] tensor under the square's point group.

    Rotation by a quarter turn relabels the legs cyclically (l -> u -> r -> d -> l); the mirror
    exchanges left and right.  Rotations r^k and r^k composed with the mirror give all eight.
    """
    rot = (1, 2, 3, 0)
    mirror = (2, 1, 0, 3)
    out = []
    cur = T
    for _ in range(4):
        out.append(cur)
        out.append(np.transpose(cur, mirror))
        cur = np.transpose(cur, rot)
    return out


def random_d4_T0(seed: int = 0, D: int = 4) -> np.ndarray:
    """Random non-negative [l][u][r][d] tensor, uniform [0,1) entries, symmetrised over the
    square's point group (average of its eight images)."""
    rng = np.random.default_rng(seed)
    T = rng.random((D, D, D, D))
    acc = np.zeros_like(T)
    for img in square_group_images(T):
        acc += img
    return np.ascontiguousarray(acc / 8.0)


def random_c4_T0(seed: int = 0, D: int = 4) -> np.ndarray:
    """Random non-negative [l][u][r][d] tensor, uniform [0,1) entries, averaged over the four
    rotations only: invariant under quarter turns but not under the mirror (a chiral tensor)."""
    rng = np.random.default_rng(seed)
    T = rng.random((D, D, D, D))
    acc = np.zeros_like(T)
    cur = T
    for _ in range(4):
        acc += cur
        cur = np.transpose(cur, (1, 2, 3, 0))
    return np.ascontiguousarray(acc / 4.0)


def mirror_T0(T0: np.ndarray) -> np.ndarray:
    """The left/right mirror image of a [l][u][r][d] tensor (the lattice reflected about a vertical
    line has the same partition function)."""
    return np.ascontiguousarray(np.transpose(T0, (2, 1, 0, 3)))


def batch_betas(n: int = 256, lo: float = 0.30, hi: float = 0.60) -> np.ndarray:
    """Deterministic temperature grid beta_i = lo + (hi - lo) * i / (n - 1), i = 0..n-1."""
    if n == 1:
        return np.array([lo])
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / (n - 1)


def batch_chis(n: int = 256, mix: tuple[int, ...] = (32, 16, 24)) -> np.ndarray:
    """Bond dimensions of the mixed batch: chi_i = mix[i mod len(mix)]."""
    return np.array([mix[i % len(mix)] for i in range(n)], dtype=np.int64)


def xy_bond_gate(t: float) -> np.ndarray:
    """exp(-t h) for one XY bond h = S^x S^x + S^y S^y on two spins, as G[a_out][b_out][a_in][b_in].

    h couples only |01> and |10> (matrix element 1/2 each way), so exp(-t h) is the identity on |00>,
    |11> and cosh(t/2) 1 - sinh(t/2) sigma_x on the {|01>, |10>} pair."""
    g = np.eye(4)
    ch, sh = math.cosh(0.5 * t), math.sinh(0.5 * t)
    g[1, 1] = g[2, 2] = ch
    g[1, 2] = g[2, 1] = -sh
    return g.reshape(2, 2, 2, 2)


def xy_bond_split(tau: float):
    """The gate exp(-tau h) of one XY bond as sum_k L[a_out][a_in][k] R[b_out][b_in][k] (k < 4).

    h = (X X + Y Y) / 4 = (X X - J J) / 4 with X = sigma_x and J = i sigma_y = [[0, 1], [-1, 0]]
    (real); the two terms commute and square to the identity, so with c = cosh(tau/4),
    s = sinh(tau/4):  exp(-tau h) = (c - s X X)(c + s J J) = c^2 I I - c s X X + c s J J - s^2 Z Z.
    I, X, J, Z are orthogonal with norm sqrt 2 under the Frobenius inner product of the
    (a_out a_in) x (b_out b_in) unfolding, so this is its singular value decomposition with the
    singular values 2 (c^2, c s, c s, s^2) shared as square roots, written in one fixed basis: a
    numerical SVD may rotate the degenerate pair (c s, c s) arbitrarily from one tau to the next,
    while this factorisation is smooth in tau."""
    c, s = math.cosh(0.25 * tau), math.sinh(0.25 * tau)
    ops = [np.eye(2), np.array([[0.0, 1.0], [1.0, 0.0]]), np.array([[0.0, 1.0], [-1.0, 0.0]]),
           np.array([[1.0, 0.0], [0.0, -1.0]])]
    coef = [c * c, -c * s, c * s, -s * s]
    Lg = np.empty((2, 2, 4))
    Rg = np.empty((2, 2, 4))
    for k, (o, a) in enumerate(zip(ops, coef)):
        r = math.sqrt(abs(a))
        Lg[:, :, k] = r * o
        Rg[:, :, k] = math.copysign(r, a) * o
    return Lg, Rg


def xy_trotter_mpo(tau: float) -> np.ndarray:
    """MPO tensor M[l][u][r][d] of rho(tau) for the infinite XY chain in two-spin cells.

    The gate exp(-tau h) on the bond between cells (spin 2 of one cell, spin 1 of the next) is split
    as sum_k L[a_out, a_in, k] R[b_out, b_in, k] (xy_bond_split, all four terms kept); the cell's
    tensor applies exp(-tau/2 h) on its inner bond, then R on spin 1 (bond l) and L on spin 2
    (bond r), then exp(-tau/2 h) again."""
    if not tau > 0.0:
        raise ValueError("tau must be positive")
    Lg, Rg = xy_bond_split(tau)
    gh = xy_bond_gate(0.5 * tau).reshape(4, 4)           # inner bond, [(s1 s2)_out][(s1 s2)_in]
    # E[(s1 s2)_out, (s1 s2)_in, l, r] = R[s1_out, s1_in, l] L[s2_out, s2_in, r]
    E = np.einsum("acl,bdr->abcdlr", Rg, Lg).reshape(4, 4, 4, 4)
    M = np.einsum("uA,ABlr,Bd->lurd", gh, E, gh)
    return np.ascontiguousarray(M)


def random_mpo(seed: int = 0, D: int = 3, d: int = 2) -> np.ndarray:
    """Random positive MPO tensor [l][u][r][d] (bond D, physical d) without symmetries."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((D, d, D, d)) + 0.1)
