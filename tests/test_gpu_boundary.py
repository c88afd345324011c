"""GPU tests of the boundary (through the C ABI): the torch.autograd wrapper with beta entering through
a torch-built Ising tensor, the single-call batch, the caller's allocator, the persisted tuning table,
forced eigensolver non-convergence and the per-step diagnostics, against the FP64 oracle."""

import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02780_amd import binding
    return binding


def test_gpu_autograd_dbeta_through_torch_tensor(B):
    """beta is a leaf tensor; T0(beta) is built with torch ops; lnZ/N = HOTRGFunction.apply(T0);
    torch.autograd.grad(lnZ, beta) chains the library's T0bar into dT0/dbeta."""
    from oracle import hotrg as O
    from paper_1912_02780_amd import inputs as I
    from paper_1912_02780_amd.autograd import HOTRGFunction
    for beta0, chi, n in ((0.40, 16, 20), (0.4406868, 24, 16)):
        _say(f"[gpu] autograd beta={beta0} chi={chi} n={n}")
        beta = torch.tensor(beta0, dtype=torch.float64, device="cuda:0", requires_grad=True)
        T0 = I.ising_T0_torch(beta)
        assert np.allclose(T0.detach().cpu().numpy(), I.ising_T0(beta0), rtol=1e-15, atol=0)
        lnZ = HOTRGFunction.apply(T0, chi, n, None)
        (dbeta,) = torch.autograd.grad(lnZ, beta)
        Lo, go, _ = O.lnZ_and_grad(I.ising_T0(beta0), chi, n)
        do = float(np.sum(go * I.ising_dT0_dbeta(beta0)))
        _say(f"    lnZ rel {abs(lnZ.item() / Lo - 1):.1e}  dbeta rel {abs(dbeta.item() / do - 1):.1e}")
        assert lnZ.dtype == torch.float64 and lnZ.dim() == 0
        assert abs(lnZ.item() / Lo - 1) < 1e-10
        assert abs(dbeta.item() / do - 1) < 1e-10


def test_gpu_autograd_second_backward_and_scaling(B):
    """The backward is seeded with the incoming gradient (here 7 d lnZ) and may run twice on one forward
    (retain_graph).  The two backward passes round differently (the seed scales every intermediate):
    entry by entry they agree to 9e-15 to 1.1e-14 here (the eigen-adjoint's broadened inverse gaps
    d / (d^2 + 1e-12) reach up to 5e5), held to 5e-14."""
    from paper_1912_02780_amd import inputs as I
    from paper_1912_02780_amd.autograd import HOTRGFunction
    T0 = torch.from_numpy(I.random_d4_T0(2)).to("cuda:0").requires_grad_(True)
    lnZ = HOTRGFunction.apply(T0, 12, 8, None)
    (g1,) = torch.autograd.grad(lnZ, T0, retain_graph=True)
    (g2,) = torch.autograd.grad(7.0 * lnZ, T0)
    d = (g2 - 7.0 * g1).abs()
    _say(f"[gpu] second backward: max |g2 - 7 g1| / |7 g1| = {float((d / (7.0 * g1).abs()).max()):.2e}, "
         f"normwise {float(d.norm() / (7.0 * g1).norm()):.2e}")
    assert torch.allclose(g2, 7.0 * g1, rtol=5e-14, atol=0)
    assert abs(float((g1 * T0.detach()).sum()) - 1.0) < 1e-12      # Euler identity


def test_gpu_forced_nonconvergence_is_enoconv(B):
    """One subspace iteration with tolerance 0 cannot resolve the kept vectors from a random start."""
    from paper_1912_02780_amd import inputs as I
    _say("[gpu] forced ENOCONV")
    T0 = torch.from_numpy(I.ising_T0(0.4406868)).to("cuda:0")
    with pytest.raises(B.DtrgError) as e:
        B.dtrg_hotrg_forward(T0, 16, 8, B.default_options(max_subspace_iters=1, subspace_tol=0.0))
    assert e.value.status == B.DTRG_ENOCONV
    assert "eigensolve" in str(e.value)


def test_gpu_hotrg_batched_single_call(B):
    """dtrg_hotrg_batched equals create + one adaptive run of a batch, bit for bit, and the oracle."""
    from oracle import hotrg as O
    from paper_1912_02780_amd import inputs as I
    betas, chis, n = [0.35, 0.4406868, 0.55, 0.42], [8, 12, 8, 16], 10
    dev = torch.device("cuda:0")
    T0s = torch.from_numpy(np.stack([I.ising_T0(b) for b in betas])).to(dev)
    dT0s = torch.from_numpy(np.stack([I.ising_dT0_dbeta(b) for b in betas])).to(dev)
    _say("[gpu] dtrg_hotrg_batched")
    L1, g1, d1 = B.dtrg_hotrg_batched(T0s, chis, n, 1.0, dT0s)
    bt = B.dtrg_batch_create(2, chis, n)
    L2, g2, d2 = B.dtrg_batch_run(bt, T0s, dT0s, 1.0, backward=True)
    assert L1 == L2 and d1 == d2 and torch.equal(g1, g2)
    for i, (beta, chi) in enumerate(zip(betas, chis)):
        Lo, go, _ = O.lnZ_and_grad(I.ising_T0(beta), chi, n)
        assert abs(L1[i] / Lo - 1) < 1e-12
        assert abs(d1[i] / float(np.sum(go * I.ising_dT0_dbeta(beta))) - 1) < 1e-10
    Lf, gf, df = B.dtrg_hotrg_batched(T0s, chis, n, None)
    assert Lf == L1 and gf is None and df is None


def test_gpu_plan_memory_comes_from_torch_allocator(B):
    """With the default binding options the plan's device memory is allocated by PyTorch's caching
    allocator (and returned to it); with hipMalloc the results are bit-identical."""
    from paper_1912_02780_amd import inputs as I
    T0 = torch.from_numpy(I.random_d4_T0(1)).to("cuda:0")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    plan, L = B.dtrg_hotrg_forward(T0, 16, 8)
    g, _ = B.dtrg_hotrg_backward(plan)
    held = torch.cuda.memory_allocated() - before
    _say(f"[gpu] plan {plan.device_bytes() / 2**20:.1f} MiB, torch allocator holds {held / 2**20:.1f} MiB more")
    assert held >= plan.device_bytes() > 0
    plan.close()
    assert torch.cuda.memory_allocated() - before < held
    plan2, L2 = B.dtrg_hotrg_forward(T0, 16, 8, B.default_options(torch_allocator=False))
    g2, _ = B.dtrg_hotrg_backward(plan2)
    assert L2 == L and torch.equal(g2, g)


_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r})
from paper_1912_02780_amd import binding as B, inputs as I
T0 = torch.from_numpy(I.random_d4_T0(5)).to("cuda:0")
o = B.default_options(contract="bf16x6", autotune=1, tile_table={path!r})
plan, L = B.dtrg_hotrg_forward(T0, 24, 8, o)
g, _ = B.dtrg_hotrg_backward(plan)
np.save({out!r}, np.concatenate([[L], g.cpu().numpy().ravel()]))
print("child tuned shapes", B.tuned_shapes(), flush=True)
"""


def test_gpu_tile_table_persists_across_processes(B, tmp_path):
    """A process that tunes with a tile_table file writes it; a second process that loads the file
    takes every configuration from it (it times nothing) and reproduces the first's results bit for bit."""
    path = str(tmp_path / "tune.txt")
    outs = [str(tmp_path / f"r{i}.npy") for i in range(2)]
    for i in range(2):
        _say(f"[gpu] tile table: process {i}")
        src = _CHILD.format(root=ROOT, path=path, out=outs[i])
        r = subprocess.run([sys.executable, "-c", src], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        _say("    " + r.stdout.strip().splitlines()[-1])
        if i == 0:
            lines = open(path).read().splitlines()
            assert lines[0] == "dtrg-tune 1" and len(lines) > 1
            mtime = os.path.getmtime(path)
    assert os.path.getmtime(path) == mtime          # nothing new was tuned the second time
    a, b = np.load(outs[0]), np.load(outs[1])
    assert np.array_equal(a, b)


_CHILD48 = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r})
from paper_1912_02780_amd import binding as B, inputs as I
T0 = torch.from_numpy(I.random_d4_T0(0)).to("cuda:0")
o = B.default_options(contract="bf16x6", autotune=1, tile_table={path!r})
plan, L = B.dtrg_hotrg_forward(T0, 48, 24, o)
g, _ = B.dtrg_hotrg_backward(plan)
np.save({out!r}, np.concatenate([[L], g.cpu().numpy().ravel()]))
"""


def test_gpu_forced_deep_tile_chi48_vs_golden(B, tmp_path):
    """Every contraction the three-stage 256 x 256 tile can take (K-contiguous operands, K a multiple
    of 16, at least 256 rows and columns) forced onto it through a tile_table: the full chi = 48 pass,
    with its bf16-plane outputs written by the tile's 16-byte epilogue, against the FP64 golden at the
    three-plane tolerance."""
    tile = 6
    import json
    path = str(tmp_path / "tune.txt")
    outs = [str(tmp_path / f"r{i}.npy") for i in range(2)]
    src = _CHILD48.format(root=ROOT, path=path, out=outs[0])
    _say(f"[gpu] forced tile {tile}: tuning child")
    r = subprocess.run([sys.executable, "-c", src], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = open(path).read().splitlines()
    forced = 0
    out_lines = [lines[0]]
    for ln in lines[1:]:
        v = [int(x) for x in ln.split()]
        prec, M, N, K, akm, bkm = v[0], v[2], v[3], v[4], v[7], v[8]
        # prec 2 / 3: the bf16-plane formats (FP64 symmetric outputs carry prec + 16 sym)
        if prec in (2, 3) and not akm and not bkm and M >= 256 and N >= 256 and K % 16 == 0:
            v[10] = tile
            forced += 1
        out_lines.append(" ".join(str(x) for x in v))
    assert forced >= 3, forced
    open(path, "w").write("\n".join(out_lines) + "\n")
    _say(f"    {forced} of {len(lines) - 1} shapes forced onto tile {tile}")
    src = _CHILD48.format(root=ROOT, path=path, out=outs[1])
    r = subprocess.run([sys.executable, "-c", src], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    res = np.load(outs[1])
    gd = json.load(open(os.path.join(ROOT, "tests", "golden", "random_d4_seed0_chi48_n24.json")))
    go = np.array(gd["T0bar"]).ravel()
    lnZ, g = float(res[0]), res[1:]
    rel_l = abs(lnZ / gd["lnZ_per_site"] - 1)
    rel_g = float(np.linalg.norm(g - go) / np.linalg.norm(go))
    _say(f"    lnZ rel {rel_l:.2e}  T0bar rel {rel_g:.2e}")
    assert rel_l < 1e-6
    assert rel_g < 1e-5


def test_gpu_step_info_diagnostics_vs_oracle(B):
    """trunc_weight, cut_gap and min_kept_gap of every step against the oracle's full spectrum
    (absolute 1e-12 on the trace-normalised spectrum)."""
    from oracle import hotrg as O
    from paper_1912_02780_amd import inputs as I
    T0 = I.ising_T0(0.4406868)
    chi, n = 16, 12
    plan, _ = B.dtrg_hotrg_forward(torch.from_numpy(T0).to("cuda:0"), chi, n)
    fwd = O.hotrg_forward(T0, chi, n)
    inv = O.step_invariants(fwd)
    for k, (rec, iv) in enumerate(zip(fwd.steps, inv), start=1):
        info = plan.step_info(k)
        lam = rec.lam
        K = rec.chi_kept
        assert info["mixed"] == 0
        assert abs(info["trunc_weight"] - iv["trunc_weight"]) < 1e-12, k
        gap = iv["cut_gap"] if K < lam.size else 0.0
        assert abs(info["cut_gap"] - gap) < 1e-12, k
        mkg = float(np.min(lam[:K - 1] - lam[1:K])) if K > 1 else 0.0
        assert abs(info["min_kept_gap"] - mkg) < 1e-12, k


@pytest.mark.parametrize("beta,tol_onsager", [(0.30, 1e-5), (0.50, 1e-4)])
def test_gpu_specific_heat(B, beta, tol_onsager):
    """The specific heat from the autograd energy (Richardson central difference of the reverse-mode
    energy, h = 1e-4): against the same difference of the oracle's energy at chi = 12 (the same
    function of beta, so to rounding / h), and against Onsager at chi = 24."""
    import exact_ising as E
    from oracle import hotrg as O
    from paper_1912_02780_amd import inputs as I
    from paper_1912_02780_amd.autograd import ising_specific_heat

    def u(b):
        _, g, _ = O.lnZ_and_grad(I.ising_T0(b), 12, 16)
        return -float(np.sum(g * I.ising_dT0_dbeta(b)))
    h = 1e-4
    d1 = (u(beta + h) - u(beta - h)) / (2 * h)
    d2 = (u(beta + h / 2) - u(beta - h / 2)) / h
    c_oracle = -beta * beta * (4 * d2 - d1) / 3
    c12 = ising_specific_heat(beta, 12, 16, h)
    c24 = ising_specific_heat(beta, 24, 24, h)
    c_ex = E.onsager_specific_heat(beta)
    _say(f"[gpu] specific heat beta={beta}: chi=12 {c12:.12f} (oracle {c_oracle:.12f}); chi=24 {c24:.10f} "
         f"(Onsager {c_ex:.10f}, rel {abs(c24 / c_ex - 1):.1e})")
    assert abs(c12 / c_oracle - 1) < 1e-8
    assert abs(c24 / c_ex - 1) < tol_onsager
