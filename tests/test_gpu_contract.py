"""The MFMA contraction kernel (diagnostic entry point of the C ABI) against float64 matmul.

Covers every precision, the four operand layouts, ragged edges, both tile shapes and split-K.
FP64 must agree to rounding; FP32 to single precision; split-bf16 (three products) to the
~2^-16 relative error of the dropped lo*lo term and the bf16 rounding of lo.
"""

import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SHAPES = [(70, 45, 37), (300, 260, 129), (40, 30, 5000), (16, 16, 4), (1, 1, 1), (129, 257, 65)]
TOL = {"fp64": 1e-13, "fp32": 2e-6, "bf16x3": 3e-5}


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02780_amd import binding
    return binding


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("akm", [False, True])
@pytest.mark.parametrize("bkm", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_contract(B, prec, akm, bkm, shape):
    M, N, K = shape
    print(f"[gpu] contract {prec} akm={akm} bkm={bkm} {shape}", flush=True)
    g = torch.Generator().manual_seed(M * 1000003 + N * 1009 + K)
    A64 = torch.randn((K, M) if akm else (M, K), generator=g, dtype=torch.float64)
    B64 = torch.randn((K, N) if bkm else (N, K), generator=g, dtype=torch.float64)
    C64 = torch.randn((M, N), generator=g, dtype=torch.float64)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A_in, B_in = A64.to(dt), B64.to(dt)
    Am = A_in.double().T if akm else A_in.double()
    Bm = B_in.double() if bkm else B_in.double().T
    ref = 0.75 * (Am @ Bm) - 0.5 * C64
    dev = torch.device("cuda:0")
    for out_dt in ([torch.float64] if prec == "fp64" else [torch.float64, torch.float32]):
        C = C64.to(out_dt).to(dev)
        B.dtrg_contract(prec, A_in.to(dev), B_in.to(dev), C, a_kmajor=akm, b_kmajor=bkm, alpha=0.75, beta=-0.5)
        torch.cuda.synchronize()
        out = C.cpu().double()
        err = (out - ref).norm() / ref.norm()
        tol = TOL[prec] if out_dt == torch.float64 else max(TOL[prec], 1e-6)
        assert err < tol, (prec, akm, bkm, shape, out_dt, float(err))
