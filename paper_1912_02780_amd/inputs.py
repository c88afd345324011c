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


def batch_betas(n: int = 256, lo: float = 0.30, hi: float = 0.60) -> np.ndarray:
    """Deterministic temperature grid beta_i = lo + (hi - lo) * i / (n - 1), i = 0..n-1."""
    if n == 1:
        return np.array([lo])
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / (n - 1)


def batch_chis(n: int = 256, mix: tuple[int, ...] = (32, 16, 24)) -> np.ndarray:
    """Bond dimensions of the mixed batch: chi_i = mix[i mod len(mix)]."""
    return np.array([mix[i % len(mix)] for i in range(n)], dtype=np.int64)
