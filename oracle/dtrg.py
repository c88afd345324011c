"""FP64 CPU oracle of the differentiable-TRG isometry optimisation on HOTRG (the paper's scheme (a)).

TEST INFRASTRUCTURE ONLY, like oracle/hotrg.py (which it builds on): nothing in the product path
imports it.  Plain NumPy, in the paper's order and notation.

What is computed (paper, main text, "Differentiable tensor renormalization group" and the Fig. 2
discussion; Eq. EGrad):
* The partition function of the truncated network is a function of the isometries w^(i) of the RG
  steps.  Its gradient with respect to w^(i) is the isometry's environment up to the number of times
  w^(i) appears (Eq. EGrad, E_w = w_bar / N_i); the backward pass (SRG recursion = chain rule) gives
  it for free.
* MERA update: the SVD E_w = U S V^T and the replacement w <- U V^T, the isometry that maximises
  Tr(E_w^T w); the environment depends on w itself, so the update is iterated n_i times ("inner
  iterations").
* Sweeps: the optimised layers are visited from the first (finest) scale up, n_s times.

Readings where the paper is not explicit (also listed in the design notes):
* Which layers: the first `layers` steps whose isometry truncates (chi' < X^2); the paper's Fig. 2
  runs update the first scale by the MERA step and keep HOTRG's local isometries above it.  Steps
  that do not truncate have square orthogonal isometries, which cannot change Z.
* The isometries above the optimised layers stay HOTRG's (leading eigenvectors of each step's
  local Gram), recomputed in every forward pass from the updated lower layers, and the environment
  of an optimised w includes their dependence on it (the derivative through their eigensolves).
* The positive factor between the gradient of ln Z / N and E_w (Z times the site count over N_i)
  does not change the polar factor U V^T, so the gradient of ln Z / N is used as it is.
"""

from __future__ import annotations

import numpy as np

from . import hotrg as H


def polar(E: np.ndarray) -> np.ndarray:
    """U V^T from the thin SVD E = U S V^T (n x K, n >= K): the isometry maximising Tr(E^T w)."""
    U, _, Vt = np.linalg.svd(E, full_matrices=False)
    return U @ Vt


def truncating_steps(fwd: H.ForwardResult) -> list:
    """Step numbers k whose isometry truncates (chi' < X^2), in order."""
    return [k for k, rec in enumerate(fwd.steps, start=1) if rec.chi_kept < rec.T.shape[0] ** 2]


def isometry_of(rec: H.StepRecord) -> np.ndarray:
    """The isometry w[x1][x2][a] a forward step used."""
    if rec.w_fixed is not None:
        return rec.w_fixed
    X = rec.T.shape[0]
    return np.ascontiguousarray(rec.U[:, :rec.chi_kept].reshape(X, X, rec.chi_kept))


def lnZ_and_wbar(T0, chi, n_steps, w_fixed, eps=H.DEFAULT_BROADENING):
    """ln Z / N with the given isometries, and d(ln Z / N)/dw for each of them."""
    fwd = H.hotrg_forward(T0, chi, n_steps, w_fixed=w_fixed)
    wbar = {}
    H.hotrg_backward(fwd, 1.0, eps, w_bar_out=wbar)
    return fwd.lnZ_per_site, wbar, fwd


def optimize(T0, chi, n_steps, layers=1, n_inner=5, n_sweeps=4, eps=H.DEFAULT_BROADENING):
    """Isometry optimisation of the first `layers` truncating steps.

    Returns (ln Z / N of plain HOTRG, ln Z / N after the optimisation, history, isometries): the
    history holds ln Z / N after every MERA update (n_sweeps x layers x n_inner entries)."""
    fwd0 = H.hotrg_forward(T0, chi, n_steps)
    steps = truncating_steps(fwd0)[:layers]
    w = {k: isometry_of(fwd0.steps[k - 1]) for k in steps}
    history = []
    for _ in range(n_sweeps):
        for k in steps:
            for _ in range(n_inner):
                _, wbar, _ = lnZ_and_wbar(T0, chi, n_steps, w, eps)
                X = w[k].shape[0]
                K = w[k].shape[2]
                w[k] = polar(wbar[k].reshape(X * X, K)).reshape(X, X, K)
                fwd = H.hotrg_forward(T0, chi, n_steps, w_fixed=w)
                history.append(fwd.lnZ_per_site)
    L = history[-1] if history else fwd0.lnZ_per_site
    return fwd0.lnZ_per_site, L, history, w
