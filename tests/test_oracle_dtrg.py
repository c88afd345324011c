"""CPU pins of the oracle's differentiable-TRG isometry optimisation (oracle/dtrg.py): what the paper
and the mathematics fix, independently of the oracle's own code.

* A forward pass with HOTRG's own isometries given as fixed parameters is the plain HOTRG pass.
* The isometry gradient (Eq. EGrad: the environment up to a positive factor) against central finite
  differences of ln Z / N in random directions of isometry space, with the higher layers' local
  isometries recomputed in every perturbed pass (the reading the oracle takes).
* The MERA update w = U V^T maximises Tr(E^T w) over isometries; its maximum is the nuclear norm of E,
  computed here from the eigenvalues of E^T E, not from an SVD.
* Untruncated steps: a square orthogonal isometry cannot change Z.
* The paper's Fig. 2 claim, checked as a property: near the critical temperature, the optimised
  network's free energy is closer to Onsager's than plain HOTRG's, and ln Z grows over the sweeps.
* Mutations planted in the oracle (one isometry occurrence dropped from the gradient, the transpose
  of the polar factor) are caught.
"""

import math

import numpy as np
import pytest

import exact_ising as E
from oracle import dtrg as DT
from oracle import hotrg as O
from paper_1912_02780_amd import inputs as I


def _fd_direction(T0, chi, n, w, k, V, h=1e-6):
    wp = dict(w); wp[k] = w[k] + h * V
    wm = dict(w); wm[k] = w[k] - h * V
    Lp = O.hotrg_forward(T0, chi, n, w_fixed=wp).lnZ_per_site
    Lm = O.hotrg_forward(T0, chi, n, w_fixed=wm).lnZ_per_site
    return (Lp - Lm) / (2 * h)


def test_fixed_isometries_reproduce_hotrg():
    T0 = I.ising_T0(0.43)
    fwd = O.hotrg_forward(T0, 8, 14)
    steps = DT.truncating_steps(fwd)
    assert steps and steps[0] == 3          # D = 2: the first two steps keep everything
    w = {k: DT.isometry_of(fwd.steps[k - 1]) for k in steps[:3]}
    fix = O.hotrg_forward(T0, 8, 14, w_fixed=w)
    assert fix.lnZ_per_site == fwd.lnZ_per_site
    assert [r.c for r in fix.steps] == [r.c for r in fwd.steps]


@pytest.mark.parametrize("case", ["ising_bc", "random_d3"])
def test_isometry_gradient_matches_finite_differences(case):
    if case == "ising_bc":
        T0, chi, n = I.ising_T0(0.4406868), 8, 12
    else:
        T0, chi, n = np.random.default_rng(11).random((3, 3, 3, 3)) + 0.2, 7, 8
    fwd = O.hotrg_forward(T0, chi, n)
    steps = DT.truncating_steps(fwd)[:2]
    w = {k: DT.isometry_of(fwd.steps[k - 1]) for k in steps}
    L, wbar, _ = DT.lnZ_and_wbar(T0, chi, n, w)
    assert L == fwd.lnZ_per_site and sorted(wbar) == steps
    rng = np.random.default_rng(3)
    for k in steps:
        for _ in range(3):
            V = rng.normal(size=w[k].shape)
            fd = _fd_direction(T0, chi, n, w, k, V)
            ad = float(np.sum(wbar[k] * V))
            assert abs(ad - fd) < 1e-7 * max(abs(fd), 1e-3), (k, ad, fd)


def test_polar_factor_maximises_the_overlap():
    rng = np.random.default_rng(7)
    E_ = rng.normal(size=(12, 5))
    w = DT.polar(E_)
    assert np.max(np.abs(w.T @ w - np.eye(5))) < 1e-13
    best = float(np.sum(E_ * w))
    nuclear = float(np.sum(np.sqrt(np.linalg.eigvalsh(E_.T @ E_))))
    assert abs(best - nuclear) < 1e-12 * nuclear
    for _ in range(200):
        q, _ = np.linalg.qr(rng.normal(size=(12, 5)))
        assert float(np.sum(E_ * q)) <= best + 1e-12


def test_square_isometry_does_not_change_Z():
    # a non-truncating step with any orthogonal w in place of HOTRG's gives the same Z
    T0 = np.random.default_rng(5).random((3, 3, 3, 3))
    fwd = O.hotrg_forward(T0, 9, 3)
    assert fwd.steps[0].chi_kept == 9
    q, _ = np.linalg.qr(np.random.default_rng(6).normal(size=(9, 9)))
    fix = O.hotrg_forward(T0, 9, 3, w_fixed={1: q.reshape(3, 3, 9)})
    assert abs(fix.lnZ_per_site - fwd.lnZ_per_site) < 1e-14 * abs(fwd.lnZ_per_site)


@pytest.mark.parametrize("beta", [0.42, 0.4406868, 0.46])
def test_optimisation_beats_hotrg_near_Tc(beta):
    """Fig. 2 of the paper: the optimised (dTRG) free energy is closer to Onsager's than HOTRG's."""
    T0 = I.ising_T0(beta)
    L0, L, hist, _ = DT.optimize(T0, 6, 20, layers=3, n_inner=5, n_sweeps=2)
    Lx = float(E.onsager_lnZ_per_site(beta))
    e0, e1 = abs(L0 / Lx - 1), abs(L / Lx - 1)
    assert L > L0                        # the truncated network's Z grows toward the exact one
    assert e1 < 0.9 * e0, (e0, e1)
    assert hist[0] > L0 and hist[-1] >= hist[0]


def test_converged_isometry_is_a_fixed_point_of_the_update():
    T0 = I.ising_T0(0.44)
    _, _, hist, w = DT.optimize(T0, 6, 16, layers=1, n_inner=25, n_sweeps=1)
    (k,) = list(w)
    _, wbar, _ = DT.lnZ_and_wbar(T0, 6, 16, w)
    X, K = w[k].shape[0], w[k].shape[2]
    upd = DT.polar(wbar[k].reshape(X * X, K))
    assert np.max(np.abs(upd - w[k].reshape(X * X, K))) < 1e-6
    assert abs(hist[-1] - hist[-2]) < 1e-13


def test_mutations_are_caught():
    """A gradient that drops the right-hand occurrence of w, and a transposed polar factor, each fail
    a pin above."""
    T0, chi, n = I.ising_T0(0.4406868), 8, 12
    fwd = O.hotrg_forward(T0, chi, n)
    k = DT.truncating_steps(fwd)[0]
    w = {k: DT.isometry_of(fwd.steps[k - 1])}
    orig = O.projection_adjoint

    def dropped(rec, Tn_bar):
        T_bar, w_bar = orig(rec, Tn_bar)
        if rec.w_fixed is None:
            return T_bar, w_bar
        wR = np.einsum("acyz,iyamz->imc", Tn_bar, O.project(rec.T, rec.w_fixed)[1], optimize=True)
        return T_bar, w_bar - wR

    O.projection_adjoint = dropped
    try:
        _, wbar, _ = DT.lnZ_and_wbar(T0, chi, n, w)
    finally:
        O.projection_adjoint = orig
    V = np.random.default_rng(1).normal(size=w[k].shape)
    fd = _fd_direction(T0, chi, n, w, k, V)
    assert abs(float(np.sum(wbar[k] * V)) - fd) > 1e-3 * abs(fd)
    E_ = np.random.default_rng(2).normal(size=(9, 9))
    U, _, Vt = np.linalg.svd(E_)
    assert float(np.sum(E_ * (U @ Vt).T)) < float(np.sum(E_ * DT.polar(E_))) - 1e-6
