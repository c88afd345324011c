"""CPU pins of the scheme-(b) oracle (oracle/xtrg.py) and of the XY-chain references it is judged by:
what the paper and the mathematics fix, independently of the oracle's own code.

* The Jordan-Wigner partition function of the periodic chain against dense exact diagonalisation,
  and the infinite-chain integral against the finite formula at large N.
* The Trotter MPO: a ring of cells traced through the MPO equals the trace of the dense
  second-order Trotter product operator; that operator's error against exp(-tau H) is third order
  in tau.
* Squaring without truncation is exact: ln Tr rho(2^n tau)^... of a ring from the chain oracle equals
  the dense matrix power.
* The infinite chain against Jordan-Wigner: the error of the Trotter density operator is second
  order in tau (halving tau divides it by four) when nothing is truncated that matters.
* The adjoint (transfer-matrix eigenvalue, vertical steps, isometry gradients) against central
  finite differences, also along dM/dtau (the energy's direction; the MPO's bond split is smooth in
  tau); planted mistakes in the eigenvalue adjoint are caught.
* The paper's Fig. 3(a) claim as a property: optimising the isometries of the last layers (depth
  n_d) raises ln Z monotonically over the MERA updates and brings the free energy closer to the
  exact one than the plain local truncation, more so with larger depth.
"""

import math

import numpy as np
import pytest

import exact_xy as X
from oracle import hotrg as O
from oracle import xtrg as C
from paper_1912_02780_amd import inputs as I


@pytest.mark.parametrize("N", [4, 6, 8, 10])
def test_jordan_wigner_matches_dense_diagonalisation(N):
    for beta in (0.3, 1.7, 5.0):
        assert abs(X.jw_lnZ(beta, N) - X.ed_lnZ(beta, N)) < 1e-12 * max(1.0, abs(X.ed_lnZ(beta, N)))


def test_infinite_chain_integral_matches_large_ring():
    for beta in (0.5, 1.0, 2.0):
        assert abs(X.jw_lnZ(beta, 4000) / 4000 / X.lnZ_per_spin_infinite(beta) - 1) < 1e-12
    # high temperature: ln 2 - beta^2 <cos^2>/2 / 4 ... to second order ln 2 + beta^2 / 16
    b = 1e-3
    assert abs(X.lnZ_per_spin_infinite(b) - (math.log(2.0) + b * b / 16.0)) < 1e-12


def test_trotter_mpo_ring_equals_dense_trotter_operator():
    for tau in (0.1, 0.37):
        M = I.xy_trotter_mpo(tau)
        E = np.einsum("luru->lr", M)
        for n_cells in (2, 3):
            rho = X.dense_trotter_rho(tau, n_cells)
            assert abs(np.trace(np.linalg.matrix_power(E, n_cells)) / np.trace(rho) - 1) < 1e-13


def test_trotter_operator_error_is_third_order():
    from scipy.linalg import expm
    errs = []
    for tau in (0.2, 0.1, 0.05):
        rho = X.dense_trotter_rho(tau, 3)
        ex = expm(-tau * X.dense_hamiltonian(6))
        errs.append(np.linalg.norm(rho - ex))
    assert 6.5 < errs[0] / errs[1] < 9.5 and 6.5 < errs[1] / errs[2] < 9.5


@pytest.mark.parametrize("n", [1, 2])
def test_untruncated_squaring_is_exact(n):
    tau = 0.21
    M = I.xy_trotter_mpo(tau)
    fwd = C.chain_forward(M, 10 ** 6, n)
    assert all(rec.chi_kept == rec.T.shape[0] ** 2 for rec in fwd.steps)
    for n_cells in (2, 3):
        rho = X.dense_trotter_rho(tau, n_cells)
        ex = math.log(np.trace(np.linalg.matrix_power(rho, 2 ** n)))
        assert abs(C.ring_lnZ(fwd, n_cells) - ex) < 1e-12 * abs(ex)


def test_infinite_chain_trotter_error_is_second_order():
    # beta = 0.8 with tau and tau / 2; chi = 64 keeps what matters at this temperature
    errs = []
    for tau, n in ((0.1, 3), (0.05, 4), (0.025, 5)):
        fwd = C.chain_forward(I.xy_trotter_mpo(tau), 64, n)
        per_spin = math.ldexp(fwd.lnZ_per_tensor, n) / 2.0
        errs.append(per_spin - X.lnZ_per_spin_infinite(0.8))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4
    assert abs(errs[2]) < 1e-5


def test_lnZ_at_steps_and_dominant_eigenvalue():
    fwd = C.chain_forward(I.xy_trotter_mpo(0.05), 10, 7)
    assert fwd.lnZ_at_step[-1] == fwd.lnZ_per_tensor
    E = C.transfer_matrix(fwd.final_T)
    ev = np.linalg.eigvals(E)
    assert abs(fwd.lam - np.max(np.abs(ev))) < 1e-13 * fwd.lam
    assert np.allclose(E @ fwd.r_vec, fwd.lam * fwd.r_vec, rtol=0, atol=1e-12 * np.abs(fwd.r_vec).max() * fwd.lam)
    assert np.allclose(fwd.l_vec @ E, fwd.lam * fwd.l_vec, rtol=0, atol=1e-12 * np.abs(fwd.l_vec).max() * fwd.lam)


def _fd_input(M, chi, n, V, h=1e-6):
    Lp = C.chain_forward(M + h * V, chi, n).lnZ_per_tensor
    Lm = C.chain_forward(M - h * V, chi, n).lnZ_per_tensor
    return (Lp - Lm) / (2 * h)


@pytest.mark.parametrize("case,chi,n", [("xy", 6, 4), ("xy", 10, 6), ("random", 5, 5)])
def test_input_gradient_matches_finite_differences(case, chi, n):
    M = I.xy_trotter_mpo(0.1) if case == "xy" else I.random_mpo(4, 3, 2)
    fwd = C.chain_forward(M, chi, n)
    if case == "random":      # a transfer matrix that is not symmetric: l and r differ
        assert np.linalg.norm(fwd.l_vec / np.linalg.norm(fwd.l_vec) - fwd.r_vec / np.linalg.norm(fwd.r_vec)) > 1e-2
    g = C.chain_backward(fwd)
    rng = np.random.default_rng(chi)
    for _ in range(3):
        V = rng.standard_normal(M.shape)
        fd = _fd_input(M, chi, n, V)
        assert abs(float(np.sum(g * V)) / fd - 1) < 2e-6


def test_mpo_is_smooth_in_tau_and_its_split_is_exact():
    """The bond split of the MPO is the gate's SVD written in one fixed operator basis: it
    reproduces the gate, and the MPO is smooth in tau (a numerical SVD may rotate the degenerate pair
    of singular values from one tau to the next, which makes finite differences of M meaningless)."""
    for tau in (1e-4, 0.05, 0.3):
        L, R = I.xy_bond_split(tau)
        G = np.transpose(I.xy_bond_gate(tau), (0, 2, 1, 3)).reshape(4, 4)
        assert np.max(np.abs(np.einsum("abk,cdk->abcd", L, R).reshape(4, 4) - G)) < 1e-15
    tau = 0.05
    d5 = (I.xy_trotter_mpo(tau * (1 + 1e-5)) - I.xy_trotter_mpo(tau * (1 - 1e-5))) / (2e-5 * tau)
    d6 = (I.xy_trotter_mpo(tau * (1 + 1e-6)) - I.xy_trotter_mpo(tau * (1 - 1e-6))) / (2e-6 * tau)
    assert np.max(np.abs(d5 - d6)) < 1e-8 * np.max(np.abs(d5))


@pytest.mark.parametrize("chi,n", [(10, 6), (12, 8)])
def test_tau_derivative_of_lnZ(chi, n):
    """The gradient contracted with dM/dtau (the internal energy's direction: ln Z per cell at
    beta = 2^n tau is 2^n L) against central differences of L in tau, through the truncations."""
    tau = 0.05
    M = I.xy_trotter_mpo(tau)
    g = C.chain_backward(C.chain_forward(M, chi, n))
    h = 1e-6
    dM = (I.xy_trotter_mpo(tau * (1 + h)) - I.xy_trotter_mpo(tau * (1 - h))) / (2 * h * tau)
    ht = 1e-5 * tau
    fd = (C.chain_forward(I.xy_trotter_mpo(tau + ht), chi, n).lnZ_per_tensor
          - C.chain_forward(I.xy_trotter_mpo(tau - ht), chi, n).lnZ_per_tensor) / (2 * ht)
    assert abs(float(np.sum(g * dM)) / fd - 1) < 1e-6


def test_isometry_gradient_matches_finite_differences():
    M, chi, n = I.xy_trotter_mpo(0.1), 8, 6
    fwd = C.chain_forward(M, chi, n)
    steps = C.truncating_steps(fwd)[-2:]
    w = {k: C.isometry_of(fwd.steps[k - 1]) for k in steps}
    L, wbar, _ = C.lnZ_and_wbar(M, chi, n, w)
    assert L == fwd.lnZ_per_tensor and sorted(wbar) == steps
    rng = np.random.default_rng(5)
    h = 1e-6
    for k in steps:
        V = rng.standard_normal(w[k].shape)
        wp = dict(w); wp[k] = w[k] + h * V
        wm = dict(w); wm[k] = w[k] - h * V
        fd = (C.chain_forward(M, chi, n, w_fixed=wp).lnZ_per_tensor -
              C.chain_forward(M, chi, n, w_fixed=wm).lnZ_per_tensor) / (2 * h)
        assert abs(float(np.sum(wbar[k] * V)) / fd - 1) < 2e-6


@pytest.mark.parametrize("mutation", ["unnormalised", "right_only"])
def test_planted_eigenvalue_adjoint_mistakes_are_caught(mutation):
    # a random MPO: its transfer matrix is not symmetric, so that l r^T and r r^T differ
    M, chi, n = I.random_mpo(4, 3, 2), 5, 5
    fwd = C.chain_forward(M, chi, n)
    if mutation == "unnormalised":
        fwd.l_vec = fwd.l_vec * 3.0           # the adjoint must divide by l^T r
        fwd.l_vec = fwd.l_vec / float(np.linalg.norm(fwd.l_vec))
        fwd.r_vec = fwd.r_vec / float(np.linalg.norm(fwd.r_vec)) * 2.0
        # a version that forgets the normalisation: multiply E_bar by l^T r
        orig = C.chain_backward

        def bad(f, gbar=1.0, eps=O.DEFAULT_BROADENING, w_bar_out=None):
            return orig(f, gbar * float(f.l_vec @ f.r_vec), eps, w_bar_out)
        g = bad(fwd)
    else:
        fwd.l_vec = fwd.r_vec.copy()          # r r^T in place of l r^T
        g = C.chain_backward(fwd)
    V = np.random.default_rng(9).standard_normal(M.shape)
    fd = _fd_input(M, chi, n, V)
    assert abs(float(np.sum(g * V)) / fd - 1) > 1e-3


def test_isometry_optimisation_beats_local_truncation():
    """Fig. 3(a) as a property: at beta = 12.8 (tau = 0.05, 8 squarings) and D = 12 the optimised
    isometries raise ln Z at every MERA update and bring the free energy closer to Jordan-Wigner than
    the local truncation, by more with depth 2 than with depth 1."""
    M, D, n = I.xy_trotter_mpo(0.05), 12, 8
    ex = X.lnZ_per_spin_infinite(2 ** n * 0.05)
    errs = []
    for depth in (1, 2):
        L0, L1, hist, _ = C.optimize(M, D, n, depth=depth, n_inner=5, n_sweeps=3)
        assert all(b >= a - 1e-13 for a, b in zip(hist, hist[1:]))
        assert hist[0] > L0
        e0 = abs(math.ldexp(L0, n) / 2 / ex - 1)
        e1 = abs(math.ldexp(L1, n) / 2 / ex - 1)
        errs.append(e1)
        assert e1 < 0.5 * e0
    assert errs[1] < 0.5 * errs[0]
