"""FP64 CPU oracle of the paper's scheme (b): vertical-only renormalisation of a matrix-product
operator, contracted exactly as a one-dimensional chain, and its reverse-mode adjoint; with the
differentiable-TRG isometry optimisation on it.

TEST INFRASTRUCTURE ONLY, like oracle/hotrg.py (whose step it reuses): nothing in the product path
imports it.  Plain NumPy.

What is computed (paper, main text Fig. 1(b) and the "Infinite quantum XY chain" paragraphs;
Supplemental Material F, exponential cooling):
* The input is one MPO tensor M[l][u][r][d] of the density operator rho(tau) of an infinite chain
  (l, r: bonds to the neighbouring cells; u, d: the cell's output and input states).  A step
  squares the operator, rho(2 t) = rho(t) rho(t): two copies are joined along the physical leg (the
  upper copy's input with the lower copy's output) and the doubled bonds on each side are
  compressed by one isometry w, which is the HOTRG step of oracle/hotrg.py with the merge always
  vertical (no alternation of directions; the physical legs keep their dimension).  w comes from
  the same local higher-order SVD (leading eigenvectors of the Gram of the (x1, x2) unfolding).
* After n steps the cell tensor represents rho(2^n tau).  The chain of infinitely many cells is
  contracted exactly through its transfer matrix E[l, r] = sum_u M_n[l, r, u, u] (the trace over
  the physical legs is Tr rho): Z per cell -> the dominant eigenvalue lambda of E.
* Normalisation as in HOTRG: each step's output is divided by its Frobenius norm c_k and the logs
  are accumulated with weight 2^-k, so the returned
      L = ln c_0 + sum_k 2^-k ln c_k + 2^-n ln lambda
  is ln Z per cell per Trotter slice: ln Z(beta = 2^n tau) per cell = 2^n L.
* Backward: d ln lambda / dE = l r^T / (lambda l^T r) with the left and right dominant eigenvectors
  (first-order perturbation of a simple eigenvalue), spread over the diagonal of the physical legs,
  then the HOTRG step adjoints in reverse order (oracle/hotrg.py; no transposes between steps).
* Differentiable TRG on scheme (b): the isometries of the last `depth` truncating steps are
  optimised for ln Z at the final temperature (paper: optimisation depth n_d, "optimizing the
  current layer" for n_d = 1) by MERA updates w <- U V^T of the environment E_w = w_bar / N_i
  (Eq. EGrad; SVD E_w = U S V^T), n_i inner iterations per layer, layers visited from the lowest
  to the highest, n_s sweeps.

Readings where the paper is not explicit (each also listed in the design notes):
* two-spin cells (one MPO tensor per bond pair, so that the second-order Trotter product is
  translation invariant with a one-tensor unit cell);
* the dominant eigenvalue of E is simple, real and positive (checked; the run stops otherwise);
* the optimisation window is the last `depth` truncating steps of the run to the target
  temperature; the isometries below it keep their local HOSVD values;
* the environment of the last step's isometry has rank <= 2 (the derivative of the closing
  eigenvalue is l r^T), so Tr(E^T w) does not determine the rest of w: the update is
  w <- polar(E + mu |E|_F w) with mu = 1e-6, which keeps the current isometry where the environment
  is silent (and changes the well-determined directions by O(mu)).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import hotrg as H
from .dtrg import polar

POLAR_TIE_BREAK = 1e-6


@dataclass
class ChainResult:
    lnZ_per_tensor: float     # L above: ln Z per cell per Trotter slice
    steps: list               # H.StepRecord per step (T in [l][r][u][d])
    c0: float
    final_T: np.ndarray       # normalised M_n, [l][r][u][d]
    lam: float                # dominant eigenvalue of the final transfer matrix
    l_vec: np.ndarray         # its left eigenvector
    r_vec: np.ndarray         # its right eigenvector
    lnZ_at_step: list         # ln Z per cell per slice at beta = 2^k tau, k = 1..n


def transfer_matrix(T: np.ndarray) -> np.ndarray:
    """E[l, r] = sum_u T[l, r, u, u] (T in [l][r][u][d])."""
    return np.einsum("lruu->lr", T)


def dominant(E: np.ndarray):
    """Largest-magnitude eigenvalue of E with its right and left eigenvectors; it must be simple,
    real and positive."""
    ev, R = np.linalg.eig(E)
    i = int(np.argmax(np.abs(ev)))
    lam = ev[i]
    rest = np.delete(np.abs(ev), i)
    if rest.size and not np.max(rest) < np.abs(lam) * (1.0 - 1e-12):
        raise FloatingPointError("dominant eigenvalue of the transfer matrix is not simple")
    if abs(lam.imag) > 1e-12 * abs(lam) or not lam.real > 0.0:
        raise FloatingPointError("dominant eigenvalue of the transfer matrix is not real and positive")
    evl, Lv = np.linalg.eig(E.T)
    j = int(np.argmin(np.abs(evl - lam)))
    r = np.real(R[:, i])
    l = np.real(Lv[:, j])
    return float(lam.real), l, r


def chain_forward(M0_lurd: np.ndarray, chi: int, n_steps: int, w_fixed=None) -> ChainResult:
    """L = ln Z per cell per Trotter slice of the infinite chain of rho(2^n tau), with chi-truncated
    vertical steps.  w_fixed as in oracle/hotrg.hotrg_forward."""
    M0 = np.asarray(M0_lurd, dtype=np.float64)
    if M0.ndim != 4 or M0.shape[0] != M0.shape[2] or M0.shape[1] != M0.shape[3]:
        raise ValueError("M0 must be a D x d x D x d tensor [l][u][r][d]")
    if chi < 1 or n_steps < 1:
        raise ValueError("chi and n_steps must be positive")
    T = H.to_internal(M0)
    c0 = float(np.linalg.norm(T))
    if not c0 > 0.0:
        raise FloatingPointError("M0 is zero")
    T = T / c0
    L = math.log(c0)
    steps, at = [], []
    for k in range(1, n_steps + 1):
        X = T.shape[0]
        if w_fixed is not None and k in w_fixed:
            w = np.asarray(w_fixed[k], dtype=np.float64)
            chi_kept = min(chi, X * X)
            if w.shape != (X, X, chi_kept):
                raise ValueError(f"step {k}: isometry must have shape {(X, X, chi_kept)}")
            rec = H.StepRecord(T=T, c=0.0, U=None, lam=None, trace_G=math.nan, G_hat=None, A=None, B=None,
                               chi_kept=chi_kept, w_fixed=w)
        else:
            A, B = H.half_environments(T)
            G_hat, t, lam, U, chi_kept = H.isometry(H.gram(A, B), chi)
            w = U[:, :chi_kept].reshape(X, X, chi_kept)
            rec = H.StepRecord(T=T, c=0.0, U=U, lam=lam, trace_G=t, G_hat=G_hat, A=A, B=B, chi_kept=chi_kept)
        _, _, Tn = H.project(T, w)
        c = float(np.linalg.norm(Tn))
        if not (c > 0.0 and math.isfinite(c)):
            raise FloatingPointError(f"step {k}: output norm is not positive and finite")
        rec.c = c
        steps.append(rec)
        T = Tn / c
        L += math.ldexp(math.log(c), -k)
        lam_k, _, _ = dominant(transfer_matrix(T))
        at.append(L + math.ldexp(math.log(lam_k), -k))
    lam, l, r = dominant(transfer_matrix(T))
    L += math.ldexp(math.log(lam), -n_steps)
    return ChainResult(lnZ_per_tensor=L, steps=steps, c0=c0, final_T=T, lam=lam, l_vec=l, r_vec=r,
                       lnZ_at_step=at)


def chain_backward(fwd: ChainResult, gbar: float = 1.0, eps: float = H.DEFAULT_BROADENING,
                   w_bar_out=None) -> np.ndarray:
    """d(gbar * L)/dM0 in the input layout [l][u][r][d]; isometry gradients of steps with a given
    isometry go to w_bar_out[k] when it is given (as in oracle/hotrg.hotrg_backward)."""
    n = len(fwd.steps)
    T = fwd.final_T
    X, Y = T.shape[0], T.shape[2]
    # L += 2^-n ln lambda(E),  E[l, r] = sum_u T[l, r, u, u]
    E_bar = math.ldexp(gbar, -n) * np.outer(fwd.l_vec, fwd.r_vec) / (fwd.lam * float(fwd.l_vec @ fwd.r_vec))
    T_bar = np.zeros((X, X, Y, Y))
    for u in range(Y):
        T_bar[:, :, u, u] = E_bar
    for k in range(n, 0, -1):
        rec = fwd.steps[k - 1]
        if rec.w_fixed is not None:
            T_bar, w_bar = H.projection_adjoint(rec, T_bar / rec.c)
            if w_bar_out is not None:
                w_bar_out[k] = w_bar
        else:
            T_bar = H.step_adjoint(rec, T_bar / rec.c, eps)
    T_bar = T_bar / fwd.c0
    return np.ascontiguousarray(np.transpose(T_bar, (0, 2, 1, 3)))


def ring_lnZ(fwd: ChainResult, n_cells: int) -> float:
    """ln Z of a ring of n_cells cells of the final operator: ln Tr E_true^n_cells, with
    E_true = exp(2^n (L - 2^-n ln lambda)) E.  Exact (to rounding) when no step truncated."""
    n = len(fwd.steps)
    log_scale = math.ldexp(fwd.lnZ_per_tensor - math.ldexp(math.log(fwd.lam), -n), n)
    E = transfer_matrix(fwd.final_T)
    ev = np.linalg.eigvals(E)
    tr = float(np.real(np.sum(ev ** n_cells)))
    return n_cells * log_scale + math.log(tr)


def truncating_steps(fwd: ChainResult) -> list:
    return [k for k, rec in enumerate(fwd.steps, start=1) if rec.chi_kept < rec.T.shape[0] ** 2]


def isometry_of(rec) -> np.ndarray:
    if rec.w_fixed is not None:
        return rec.w_fixed
    X = rec.T.shape[0]
    return np.ascontiguousarray(rec.U[:, :rec.chi_kept].reshape(X, X, rec.chi_kept))


def lnZ_and_wbar(M0, chi, n_steps, w_fixed, eps=H.DEFAULT_BROADENING):
    fwd = chain_forward(M0, chi, n_steps, w_fixed=w_fixed)
    wbar = {}
    chain_backward(fwd, 1.0, eps, w_bar_out=wbar)
    return fwd.lnZ_per_tensor, wbar, fwd


def optimize(M0, chi, n_steps, depth=1, n_inner=5, n_sweeps=3, eps=H.DEFAULT_BROADENING):
    """Isometry optimisation of the last `depth` truncating steps for ln Z at the final temperature.

    Returns (L of plain scheme (b), L after the optimisation, history after every MERA update, the
    optimised isometries)."""
    fwd0 = chain_forward(M0, chi, n_steps)
    steps = truncating_steps(fwd0)[-depth:] if depth > 0 else []
    w = {k: isometry_of(fwd0.steps[k - 1]) for k in steps}
    history = []
    for _ in range(n_sweeps):
        for k in steps:
            for _ in range(n_inner):
                _, wbar, _ = lnZ_and_wbar(M0, chi, n_steps, w, eps)
                X, K = w[k].shape[0], w[k].shape[2]
                E = wbar[k].reshape(X * X, K)
                E = E + POLAR_TIE_BREAK * np.linalg.norm(E) * w[k].reshape(X * X, K)
                w[k] = polar(E).reshape(X, X, K)
                history.append(chain_forward(M0, chi, n_steps, w_fixed=w).lnZ_per_tensor)
    L = history[-1] if history else fwd0.lnZ_per_tensor
    return fwd0.lnZ_per_tensor, L, history, w
