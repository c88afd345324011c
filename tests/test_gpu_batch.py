"""GPU tests of the batched path (dtrg_batch_create / dtrg_batch_run through the C ABI): many Ising
temperatures with mixed chi in one call, adaptive runs and HIP-graph replays.

  * every instance of a small mixed-chi batch against the FP64 oracle (same bars as the
    single-instance parity tests: ln Z / N 1e-12, d(lnZ/N)/dbeta 1e-10, T0bar 1e-10 relative);
  * the batch against the single-instance path on the same inputs;
  * graph replays reproduce the adaptive run that recorded their schedule bit for bit, replay after
    replay with other device work in between;
  * a replay on changed inputs either reports that the recorded schedule does not fit them or
    agrees with a fresh adaptive run on them;
  * split-bf16 and FP32 batches against the FP64 batch (ln Z / N 1e-6, dbeta per the precision's
    gradient bound);
  * full-size batch (n = 30, chi in {16, 24, 32}, the shapes of the 256-temperature workload) with
    instances whose FP64 oracle results are stored (beta = 0.30, 0.4406868, 0.50 at chi = 32):
    those against the stored values, every instance's energy and free energy against Onsager.
"""

import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02780_amd import binding
    return binding


def _ising_inputs(betas):
    from paper_1912_02780_amd import inputs as I
    T0s = np.stack([I.ising_T0(b) for b in betas])
    dT0s = np.stack([I.ising_dT0_dbeta(b) for b in betas])
    dev = torch.device("cuda:0")
    return torch.from_numpy(T0s).to(dev), torch.from_numpy(dT0s).to(dev)


def _run(B, batch, T0s, dT0s, replay=False):
    L, g, d = B.dtrg_batch_run(batch, T0s, dT0s, 1.0, backward=True, replay=replay)
    return np.array(L), g.cpu().numpy(), np.array(d)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


SMALL_BETAS = [0.30, 0.40, 0.4406868, 0.50, 0.35, 0.45, 0.60]
SMALL_CHIS = [8, 12, 16, 8, 12, 16, 12]
SMALL_N = 12


def test_batch_small_vs_oracle(B):
    from oracle import hotrg as O
    from paper_1912_02780_amd import inputs as I
    _say(f"[gpu] batch of {len(SMALL_BETAS)} Ising instances, chi {sorted(set(SMALL_CHIS))}, n={SMALL_N}, fp64")
    T0s, dT0s = _ising_inputs(SMALL_BETAS)
    batch = B.dtrg_batch_create(2, SMALL_CHIS, SMALL_N)
    L, g, d = _run(B, batch, T0s, dT0s)
    for i, (beta, chi) in enumerate(zip(SMALL_BETAS, SMALL_CHIS)):
        T0 = I.ising_T0(beta)
        Lo, go, fwd = O.lnZ_and_grad(T0, chi, SMALL_N)
        do = float(np.sum(go * I.ising_dT0_dbeta(beta)))
        _say(f"    beta={beta} chi={chi}: lnZ rel {abs(L[i] / Lo - 1):.1e} dbeta rel {abs(d[i] / do - 1):.1e} "
             f"T0bar rel {_rel(g[i], go):.1e}")
        assert abs(L[i] / Lo - 1) < 1e-12
        assert abs(d[i] / do - 1) < 1e-10
        assert _rel(g[i], go) < 1e-10
        for k, rec in enumerate(fwd.steps, start=1):
            info = batch.step_info(i, k)
            assert info["chi_kept"] == rec.chi_kept
            assert abs(info["c"] / rec.c - 1) < 1e-11 + rec.lam[rec.chi_kept - 1]


def test_batch_matches_single_instance(B):
    _say("[gpu] batch vs single-instance path")
    betas, chis = [0.38, 0.4406868, 0.52, 0.41], [16, 16, 24, 24]
    n = 14
    T0s, dT0s = _ising_inputs(betas)
    batch = B.dtrg_batch_create(2, chis, n)
    L, g, d = _run(B, batch, T0s, dT0s)
    for i in range(len(betas)):
        plan, Ls = B.dtrg_hotrg_forward(T0s[i].contiguous(), chis[i], n)
        gs, ds = B.dtrg_hotrg_backward(plan, 1.0, dT0s[i].contiguous())
        gs = gs.cpu().numpy()
        _say(f"    {i}: lnZ {abs(L[i] - Ls):.1e} dbeta rel {abs(d[i] / ds - 1):.1e} T0bar rel {_rel(g[i], gs):.1e}")
        assert abs(L[i] / Ls - 1) < 1e-13
        assert abs(d[i] / ds - 1) < 1e-11
        assert _rel(g[i], gs) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
def test_batch_replay_reproduces_adaptive(B, prec):
    _say(f"[gpu] batch graph replay ({prec})")
    betas = [0.33, 0.4406868, 0.47, 0.55, 0.39]
    chis = [16, 24, 16, 24, 12]
    n = 16
    T0s, dT0s = _ising_inputs(betas)
    batch = B.dtrg_batch_create(2, chis, n, B.default_options(contract=prec))
    L0, g0, d0 = _run(B, batch, T0s, dT0s, replay=False)
    dev = torch.device("cuda:0")
    for r in range(3):
        # unrelated eager work (and a synchronisation) between the replays
        x = torch.randn(1 << 16, device=dev, dtype=torch.float64)
        _ = float((x * x).sum())
        L1, g1, d1 = _run(B, batch, T0s, dT0s, replay=True)
        _say(f"    replay {r}: max |dlnZ| {np.max(np.abs(L1 - L0)):.1e}  max |dT0bar| {np.max(np.abs(g1 - g0)):.1e}")
        assert np.array_equal(L1, L0)
        assert np.array_equal(d1, d0)
        assert np.array_equal(g1, g0)


def test_batch_replay_on_changed_inputs(B):
    _say("[gpu] batch replay on changed inputs")
    betas = [0.36, 0.4406868, 0.51]
    chis = [16, 16, 24]
    n = 16
    T0s, dT0s = _ising_inputs(betas)
    batch = B.dtrg_batch_create(2, chis, n)
    _run(B, batch, T0s, dT0s, replay=False)
    _run(B, batch, T0s, dT0s, replay=True)   # capture
    new_betas = [b + 2e-3 for b in betas]
    T1, dT1 = _ising_inputs(new_betas)
    T0s.copy_(T1)
    dT0s.copy_(dT1)
    ref = B.dtrg_batch_create(2, chis, n)
    Lr, gr, dr = _run(B, ref, T1, dT1, replay=False)
    try:
        L, g, d = _run(B, batch, T0s, dT0s, replay=True)
    except B.DtrgError as e:
        _say(f"    replay refused the new inputs: {e}")
        assert e.status in (B.DTRG_ENOCONV, B.DTRG_ENONPOS)
        assert "replay = 0" in str(e)
    else:
        _say(f"    replay accepted: lnZ rel {np.max(np.abs(L / Lr - 1)):.1e} dbeta rel {np.max(np.abs(d / dr - 1)):.1e}")
        assert np.max(np.abs(L / Lr - 1)) < 1e-12
        assert np.max(np.abs(d / dr - 1)) < 1e-9
    # a new adaptive run records a schedule for them, which replays exactly
    L2, g2, d2 = _run(B, batch, T0s, dT0s, replay=False)
    L3, g3, d3 = _run(B, batch, T0s, dT0s, replay=True)
    assert np.array_equal(L2, L3) and np.array_equal(g2, g3)


def test_batch_replay_needs_schedule(B):
    T0s, dT0s = _ising_inputs([0.4])
    batch = B.dtrg_batch_create(2, [8], 6)
    with pytest.raises(B.DtrgError) as e:
        B.dtrg_batch_run(batch, T0s, dT0s, 1.0, backward=True, replay=True)
    assert e.value.status == B.DTRG_ESTATE
    # a forward-only schedule does not cover a backward replay
    B.dtrg_batch_run(batch, T0s, None, 1.0, backward=False, replay=False)
    with pytest.raises(B.DtrgError) as e:
        B.dtrg_batch_run(batch, T0s, dT0s, 1.0, backward=True, replay=True)
    assert e.value.status == B.DTRG_ESTATE
    L, _, _ = B.dtrg_batch_run(batch, T0s, None, 1.0, backward=False, replay=True)
    assert np.isfinite(L[0])


# Gradient tolerance per contraction format.  FP32 and three-plane split-bf16 (six products) meet the
# 1e-5 target.  Two-plane split-bf16 (three products) carries ~2^-17 relative error per product (the
# two-plane representation and the dropped x1*y1 term); the broadened eigen-adjoint amplifies it:
# over the 256-temperature Ising sweep (chi <= 32, 30 steps) its d(lnZ/N)/dbeta differs from the
# FP64 path by 3e-5 at the median and 2.5e-4 at worst, so that format is bounded by 3e-4 and does not
# meet the target.
GRAD_TOL = {"fp32": 1e-5, "bf16x3": 3e-4, "bf16x6": 1e-5}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_batch_mixed_precision_vs_fp64(B, prec):
    _say(f"[gpu] batch {prec} vs fp64")
    betas = [0.32, 0.4406868, 0.48, 0.58]
    chis = [24, 24, 16, 16]
    n = 20
    T0s, dT0s = _ising_inputs(betas)
    ref = B.dtrg_batch_create(2, chis, n)
    Lr, _, dr = _run(B, ref, T0s, dT0s)
    batch = B.dtrg_batch_create(2, chis, n, B.default_options(contract=prec))
    L, _, d = _run(B, batch, T0s, dT0s)
    _say(f"    lnZ rel {np.max(np.abs(L / Lr - 1)):.1e}  dbeta rel {np.max(np.abs(d / dr - 1)):.1e}")
    assert np.max(np.abs(L / Lr - 1)) < 1e-6
    assert np.max(np.abs(d / dr - 1)) < GRAD_TOL[prec]


# Onsager bounds for HOTRG at these chi after 30 steps (relative).  The energy bound is set by the
# truncation error at the critical point, the worst temperature of the range: 4.8e-4 at chi = 16,
# 2.2e-5 at chi = 32 for the FP64 oracle; the free energy is far more accurate (1e-6 is loose).
ONSAGER_U_TOL = {16: 1e-3, 24: 3e-4, 32: 1e-4}
ONSAGER_F_TOL = 1e-6


def test_batch_full_shapes_vs_golden_and_onsager(B):
    """n = 30 and chi in {16, 24, 32}: the shapes of the 256-temperature workload."""
    import exact_ising as E
    goldens = ["ising_b0.30_chi32_n30", "ising_b0.4406868_chi32_n30", "ising_b0.50_chi32_n30"]
    gds = []
    for name in goldens:
        path = os.path.join(GOLDEN, name + ".json")
        if not os.path.exists(path):
            pytest.skip(f"golden {name} not generated")
        with open(path) as f:
            gds.append(json.load(f))
    betas = [gd["param"] for gd in gds] + [0.31, 0.4406868, 0.57, 0.34, 0.4406868, 0.59]
    chis = [32, 32, 32, 24, 24, 24, 16, 16, 16]
    n = 30
    _say(f"[gpu] full-shape batch: {len(betas)} instances, chi {chis}, n={n}")
    T0s, dT0s = _ising_inputs(betas)
    batch = B.dtrg_batch_create(2, chis, n)
    L, g, d = _run(B, batch, T0s, dT0s)
    for i, gd in enumerate(gds):
        go = np.array(gd["T0bar"]).reshape(gd["T0bar_shape"])
        tol = max(1e-10, 10 * gd["rounding_sensitivity_T0bar"])
        _say(f"    golden {gd['name']}: lnZ rel {abs(L[i] / gd['lnZ_per_site'] - 1):.1e} "
             f"dbeta rel {abs(d[i] / gd['dlnZ_dbeta'] - 1):.1e} T0bar rel {_rel(g[i], go):.1e}")
        assert abs(L[i] / gd["lnZ_per_site"] - 1) < 1e-12
        assert abs(d[i] / gd["dlnZ_dbeta"] - 1) < 1e-10
        assert _rel(g[i], go) < tol
    for i, (beta, chi) in enumerate(zip(betas, chis)):
        f_ex = float(E.onsager_lnZ_per_site(beta))
        u_ex = float(E.onsager_dlnZ_dbeta(beta))
        ef, eu = abs(L[i] / f_ex - 1), abs(d[i] / u_ex - 1)
        _say(f"    beta={beta:.7f} chi={chi}: lnZ vs Onsager {ef:.1e}, energy vs Onsager {eu:.1e}")
        assert ef < ONSAGER_F_TOL
        assert eu < ONSAGER_U_TOL[chi]
    # the replay of the recorded schedule gives the same numbers
    L1, g1, d1 = _run(B, batch, T0s, dT0s, replay=True)
    assert np.array_equal(L1, L) and np.array_equal(d1, d) and np.array_equal(g1, g)


def test_batch_256_temperatures_replay_vs_onsager(B):
    """The whole 256-temperature workload (beta_i = 0.30 + 0.30 i / 255, chi_i = (32, 16, 24)[i mod 3],
    30 steps) in the benchmark's configuration (three-plane split-bf16, tile autotuner): the adaptive
    run, then two replays of its HIP graph, every instance's free energy and energy against Onsager at
    the bounds above, and the replays bit for bit equal to the adaptive run."""
    import exact_ising as E
    from paper_1912_02780_amd import inputs as I
    betas = I.batch_betas(256)
    chis = [int(c) for c in I.batch_chis(256)]
    T0s, dT0s = _ising_inputs(betas)
    _say("[gpu] 256-temperature batch: adaptive run")
    batch = B.dtrg_batch_create(2, chis, 30, B.default_options(contract="bf16x6", autotune=1))
    L, g, d = _run(B, batch, T0s, dT0s)
    for rep in range(2):
        _say(f"[gpu] 256-temperature batch: replay {rep}")
        L1, g1, d1 = _run(B, batch, T0s, dT0s, replay=True)
        assert np.array_equal(L1, L) and np.array_equal(d1, d) and np.array_equal(g1, g)
    worst = {}
    for i, (beta, chi) in enumerate(zip(betas, chis)):
        ef = abs(L[i] / float(E.onsager_lnZ_per_site(beta)) - 1)
        eu = abs(d[i] / float(E.onsager_dlnZ_dbeta(beta)) - 1)
        worst[chi] = max(worst.get(chi, (0, 0)), (eu, ef))
        assert ef < ONSAGER_F_TOL, (beta, chi, ef)
        assert eu < ONSAGER_U_TOL[chi], (beta, chi, eu)
    _say("    worst (energy, free energy) vs Onsager per chi: "
         + ", ".join(f"chi={c}: {u:.1e}, {f:.1e}" for c, (u, f) in sorted(worst.items())))
