"""GPU test of dtrg_contract_noalloc (through the C ABI): the contraction with its scratch in the
library's static device array gives dtrg_contract's result on two calls in a row (the second
smaller, so it runs over what the first left in the array), and a contraction too large for the
array is rejected before any work."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02780_amd import binding
    return binding


def _case(prec, M, N, K, a_kmajor, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = torch.rand((K, M) if a_kmajor else (M, K), generator=g, dtype=torch.float64).to(dt).to("cuda:0")
    Bm = torch.rand((N, K), generator=g, dtype=torch.float64).to(dt).to("cuda:0")
    return A, Bm


# (precision, M, N, K, A K-major): K beyond 4096 splits the split-bf16 contraction into K chunks
# (FP32 chains), and the small FP64 output is split over K to fill the chip: both use partials
CASES = [("bf16x6", 1000, 700, 5000, False), ("fp64", 300, 200, 1500, True)]


@pytest.mark.parametrize("order", [0, 1])
def test_gpu_contract_noalloc_matches_contract(B, order):
    cases = CASES if order == 0 else [("bf16x3", 900, 650, 4500, True), ("fp32", 257, 129, 777, False)]
    for i, (prec, M, N, K, akm) in enumerate(cases):
        A, Bm = _case(prec, M, N, K, akm, 17 + i + 10 * order)
        print(f"[gpu] noalloc {prec} M={M} N={N} K={K} a_kmajor={akm}", flush=True)
        C0 = torch.full((M, N), 0.5, dtype=torch.float64, device="cuda:0")
        C1 = C0.clone()
        B.dtrg_contract(prec, A, Bm, C0, a_kmajor=akm, alpha=1.25, beta=0.5)
        B.dtrg_contract(prec, A, Bm, C1, a_kmajor=akm, alpha=1.25, beta=0.5, noalloc=True)
        torch.cuda.synchronize()
        ref = (1.25 * ((A.double().T if akm else A.double()) @ Bm.double().T) + 0.25).cpu().numpy()
        c0, c1 = C0.cpu().numpy(), C1.cpu().numpy()
        tol = 1e-12 if prec == "fp64" else (1e-4 if prec == "bf16x3" else 1e-6)
        assert np.max(np.abs(c1 - ref) / np.abs(ref)) < tol
        assert np.array_equal(c1, c0), float(np.max(np.abs(c1 - c0)))


def test_gpu_contract_noalloc_rejects_oversize_before_work(B):
    M = N = K = 6144                                  # three bf16 planes of each operand: 453 MiB
    A = torch.zeros((M, K), dtype=torch.float32, device="cuda:0")
    C = torch.full((M, N), 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(B.DtrgError) as e:
        B.dtrg_contract("bf16x6", A, A, C, noalloc=True)
    assert e.value.status == B.DTRG_EINVAL and "static" in str(e.value)
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())                     # nothing was written
