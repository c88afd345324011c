"""Pins of the oracle's side rule (oracle/hotrg.py, side_rule="min"): the isometry of each step taken
from the unfolding of the pair, left (x1, x2) or right (x1', x2'), whose discarded eigenvalues weigh
less.  It matters for tensors without the left/right mirror symmetry: chiral tensors (invariant
under quarter turns only) and generic ones.

* The exact partition function does not change when the lattice is mirrored.  The rule is mirror
  covariant (the mirror exchanges the two unfoldings of every step that merges along the mirrored
  legs), so the truncated ln Z / N of a tensor and of its mirror image agree to rounding, and the
  gradient of the mirror image is the mirror image of the gradient.  Taking the left unfolding
  always (the planted mistake) breaks both by far more than rounding.
* The gradient with the rule against central finite differences in random directions, on generic
  tensors whose steps pick both sides with clear margins.
* Inputs with the mirror symmetry (the D4 random tensor, Ising) have equal spectra on both sides:
  every step keeps the left unfolding and the result is bit for bit the plain rule's.
* Untruncated, either rule is exact (2 x 2 brute force).
"""

import math

import numpy as np
import pytest

import exact_ising as E
from oracle import hotrg as O
from paper_1912_02780_amd import inputs as I


def _generic(seed, D=3):
    rng = np.random.default_rng(seed)
    return rng.random((D, D, D, D)) + 0.2


@pytest.mark.parametrize("seed,D,chi,n", [(1, 4, 8, 8), (0, 3, 6, 8), (2, 4, 12, 10)])
def test_mirror_invariance_chiral(seed, D, chi, n):
    T = I.random_c4_T0(seed, D)
    Tm = I.mirror_T0(T)
    a = O.hotrg_forward(T, chi, n, side_rule="min")
    b = O.hotrg_forward(Tm, chi, n, side_rule="min")
    assert any(r.side == "R" for r in a.steps) and any(r.side == "R" for r in b.steps)
    assert abs(a.lnZ_per_site / b.lnZ_per_site - 1) < 1e-14
    # the planted mistake: the left unfolding on every step
    la = O.hotrg_forward(T, chi, n).lnZ_per_site
    lb = O.hotrg_forward(Tm, chi, n).lnZ_per_site
    assert abs(la / lb - 1) > 1e-12


@pytest.mark.parametrize("seed,chi,n", [(0, 6, 6), (2, 5, 6)])
def test_mirror_covariance_generic(seed, chi, n):
    T = _generic(seed)
    Tm = I.mirror_T0(T)
    La, ga, fa = O.lnZ_and_grad(T, chi, n, side_rule="min")
    Lb, gb, fb = O.lnZ_and_grad(Tm, chi, n, side_rule="min")
    # the mirror flips the side on every step that merges along the mirrored legs (odd steps)
    for k, (ra, rb) in enumerate(zip(fa.steps, fb.steps), start=1):
        assert (ra.side != rb.side) == (k % 2 == 1)
    assert abs(La / Lb - 1) < 1e-14
    gm = I.mirror_T0(ga)
    assert np.max(np.abs(gm - gb)) < 1e-12 * np.max(np.abs(gb))
    la, gla, _ = O.lnZ_and_grad(T, chi, n)
    lb, glb, _ = O.lnZ_and_grad(Tm, chi, n)
    assert abs(la / lb - 1) > 1e-9
    assert np.max(np.abs(I.mirror_T0(gla) - glb)) > 1e-7 * np.max(np.abs(glb))


@pytest.mark.parametrize("seed,chi,n", [(0, 6, 6), (2, 5, 6), (3, 8, 8)])
def test_fd_random_directions_side_rule(seed, chi, n):
    T0 = _generic(seed)
    # unbroadened adjoint: the exact derivative of a spectrum without degeneracies
    L, g, fwd = O.lnZ_and_grad(T0, chi, n, eps=0.0, side_rule="min")
    sides = "".join(r.side for r in fwd.steps)
    assert "R" in sides and "L" in sides
    # every step's choice has a clear margin, so that the perturbed passes choose alike
    for r in fwd.steps:
        a, b = r.trunc_LR
        assert abs(a - b) > 1e-3 * max(a, b)
    rng = np.random.default_rng(100 + seed)
    h = 1e-5
    for _ in range(3):
        V = rng.normal(size=T0.shape)
        fp = O.hotrg_forward(T0 + h * V, chi, n, side_rule="min")
        fm = O.hotrg_forward(T0 - h * V, chi, n, side_rule="min")
        assert [r.side for r in fp.steps] == [r.side for r in fm.steps] == list(sides)
        fd = (fp.lnZ_per_site - fm.lnZ_per_site) / (2 * h)
        ad = float(np.sum(g * V))
        assert abs(fd - ad) < 1e-7 * max(abs(ad), 1e-3)


def test_planted_adjoint_mistake_is_caught(monkeypatch):
    """The right side's Gram adjoint taken on T instead of its mirror (and not mirrored back)."""
    T0, chi, n = _generic(0), 6, 6
    L, g_ok, _ = O.lnZ_and_grad(T0, chi, n, eps=0.0, side_rule="min")
    fwd = O.hotrg_forward(T0, chi, n, side_rule="min")
    monkeypatch.setattr(O, "mirror_lr", lambda T: T)
    g_bad = O.hotrg_backward(fwd, 1.0, 0.0)
    rng = np.random.default_rng(7)
    V = rng.normal(size=T0.shape)
    h = 1e-5
    monkeypatch.undo()
    fd = (O.hotrg_forward(T0 + h * V, chi, n, side_rule="min").lnZ_per_site
          - O.hotrg_forward(T0 - h * V, chi, n, side_rule="min").lnZ_per_site) / (2 * h)
    assert abs(fd - float(np.sum(g_ok * V))) < 1e-7 * abs(fd)
    assert abs(fd - float(np.sum(g_bad * V))) > 1e-4 * abs(fd)


@pytest.mark.parametrize("case", ["d4", "ising"])
def test_mirror_symmetric_inputs_keep_the_left_side(case):
    T0 = I.random_d4_T0(0, 4) if case == "d4" else I.ising_T0(I.BETA_CRITICAL_CONFIG)
    chi, n = (8, 8) if case == "d4" else (8, 10)
    La, ga, fa = O.lnZ_and_grad(T0, chi, n, side_rule="min")
    Lb, gb, _ = O.lnZ_and_grad(T0, chi, n)
    assert all(r.side == "L" for r in fa.steps)
    assert La == Lb and np.array_equal(ga, gb)


def test_chosen_side_truncates_less():
    T0, chi, n = _generic(3), 8, 8
    fwd = O.hotrg_forward(T0, chi, n, side_rule="min")
    for r in fwd.steps:
        a, b = r.trunc_LR
        assert O.truncated_weight(r.lam, r.chi_kept) == (b if r.side == "R" else a)
        assert (b if r.side == "R" else a) <= min(a, b) + O.SIDE_MARGIN


def test_untruncated_either_side_is_exact():
    """2 x 2 periodic network (two steps, nothing truncated) of a generic tensor against brute-force
    bond sums, Z and the full gradient."""
    T0 = _generic(5, D=4)
    Z, dZ = E.bruteforce_2x2(T0)
    L, g, fwd = O.lnZ_and_grad(T0, 16, 2, side_rule="min")
    assert abs(L - math.log(Z) / 4) <= 1e-14
    ref = dZ / Z / 4.0
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))
