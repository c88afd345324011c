"""The MFMA contraction kernel (diagnostic entry point of the C ABI) against float64 matmul.

Covers every precision, the four operand layouts, ragged edges (K not a multiple of 8: the bf16
planes' masked last chunk), every tile shape (with the tile for outputs of at most 64 columns and
the short, wide case computed as its transpose) and split-K.  FP64 must agree to rounding; FP32 to
single precision; split-bf16 with two planes (three products) to the ~2^-17 relative error of the
two-plane representation and the dropped x1*y1 term; with three planes (six products) to single
precision.
"""

import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SHAPES = [(70, 45, 37), (300, 260, 129), (40, 30, 5000), (16, 16, 4), (1, 1, 1), (129, 257, 65)]
TOL = {"fp64": 1e-13, "fp32": 2e-6, "bf16x3": 3e-5, "bf16x6": 2e-6}
PRECS = ["fp64", "fp32", "bf16x3", "bf16x6"]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02780_amd import binding
    return binding


@pytest.mark.parametrize("prec", PRECS)
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


# enough 256 x 128 tiles to select the largest tile of the bf16-plane kernel (ragged in M, N, K)
@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("layout", [(False, False), (True, True)])
def test_contract_large_tile(B, prec, layout):
    test_contract(B, prec, layout[0], layout[1], (8200, 4100, 70))


# at most 64 output columns and many rows: the full-width-wave tile (ragged in M, N, K); and the
# transposed case, at most 64 rows and many columns, which is computed as its transpose on that tile
# (with split-K for the long K)
@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("layout", [(False, False), (True, True)])
@pytest.mark.parametrize("shape", [(3001, 45, 333), (50, 2100, 5003)])
def test_contract_tall_and_wide(B, prec, layout, shape):
    test_contract(B, prec, layout[0], layout[1], shape)


# every tile code of each precision forced through the configuration entry point, with one and with
# three K-chunks (ragged in M, N and K; both operand layouts)
CONFIG_SHAPES = [(300, 260, 129), (70, 45, 37), (129, 257, 1000)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("layout", [(False, False), (True, True), (True, False)])
@pytest.mark.parametrize("shape", CONFIG_SHAPES)
def test_contract_every_tile(B, prec, layout, shape):
    akm, bkm = layout
    M, N, K = shape
    g = torch.Generator().manual_seed(M * 7919 + N * 31 + K)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A_in = torch.randn((K, M) if akm else (M, K), generator=g, dtype=torch.float64).to(dt)
    B_in = torch.randn((K, N) if bkm else (N, K), generator=g, dtype=torch.float64).to(dt)
    C0 = torch.randn((M, N), generator=g, dtype=torch.float64)
    Am = A_in.double().T if akm else A_in.double()
    Bm = B_in.double() if bkm else B_in.double().T
    ref = 1.25 * (Am @ Bm) + 0.5 * C0
    dev = torch.device("cuda:0")
    tiles = [1, 2] if prec in ("fp64", "fp32") else [1, 2, 3, 4, 5]
    for tile in tiles:
        for splits in (1, 3):
            print(f"[gpu] contract config {prec} {layout} {shape} tile {tile} splits {splits}", flush=True)
            C = C0.to(dev)
            B.dtrg_contract(prec, A_in.to(dev), B_in.to(dev), C, a_kmajor=akm, b_kmajor=bkm, alpha=1.25, beta=0.5,
                            tile=tile, splits=splits)
            torch.cuda.synchronize()
            err = float((C.cpu() - ref).norm() / ref.norm())
            assert err < TOL[prec], (prec, layout, shape, tile, splits, err)


# the three-stage 256 x 256 tile on 32 x 32 MFMA tiles: K-contiguous operands and K a multiple of 16;
# ragged M and N, tile counts per chunk that are and are not multiples of the stage count (steps past
# the last tile), a single K tile, fewer rows than a tile, and split-K with chunk counts that leave a
# short last chunk
DEEP_SHAPES = [(300, 260, 144), (1000, 530, 1008), (257, 300, 16), (100, 700, 4096), (520, 270, 2320)]


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("shape", DEEP_SHAPES)
def test_contract_deep_tiles(B, prec, shape):
    M, N, K = shape
    g = torch.Generator().manual_seed(M * 7919 + N * 31 + K + 5)
    A_in = torch.randn((M, K), generator=g, dtype=torch.float64).float()
    B_in = torch.randn((N, K), generator=g, dtype=torch.float64).float()
    C0 = torch.randn((M, N), generator=g, dtype=torch.float64)
    ref = 1.25 * (A_in.double() @ B_in.double().T) + 0.5 * C0
    dev = torch.device("cuda:0")
    for tile in (6,):
        for splits in (1, 3, 5):
            print(f"[gpu] contract deep {prec} {shape} tile {tile} splits {splits}", flush=True)
            C = C0.to(dev)
            B.dtrg_contract(prec, A_in.to(dev), B_in.to(dev), C, alpha=1.25, beta=0.5, tile=tile, splits=splits)
            torch.cuda.synchronize()
            err = float((C.cpu() - ref).norm() / ref.norm())
            assert err < TOL[prec], (prec, shape, tile, splits, err)
    # K-major operands and K not a multiple of 16 are refused for these tiles
    A = A_in.to(dev)
    for kw in (dict(a_kmajor=True), dict(b_kmajor=True)):
        Ak = A.T.contiguous() if kw.get("a_kmajor") else A
        Bk = B_in.to(dev).T.contiguous() if kw.get("b_kmajor") else B_in.to(dev)
        with pytest.raises(B.DtrgError) as e:
            B.dtrg_contract(prec, Ak, Bk, C0.to(dev), tile=6, splits=1, **kw)
        assert e.value.status == B.DTRG_EINVAL
    with pytest.raises(B.DtrgError) as e:
        B.dtrg_contract(prec, A[:, :K - 8].contiguous(), B_in.to(dev)[:, :K - 8].contiguous(), C0.to(dev), tile=6,
                        splits=1)
    assert e.value.status == B.DTRG_EINVAL


def test_contract_config_rejects_bad_codes(B):
    dev = torch.device("cuda:0")
    A = torch.randn(8, 8, dtype=torch.float64, device=dev)
    C = torch.zeros(8, 8, dtype=torch.float64, device=dev)
    for tile, splits in ((3, 0), (6, 0), (-1, 0), (1, 65), (1, -2)):
        with pytest.raises(B.DtrgError) as e:
            B.dtrg_contract("fp64", A, A, C, tile=tile, splits=splits)
        assert e.value.status == B.DTRG_EINVAL
