// Host dispatch of the MFMA contraction kernel (tile choice, split-K, bounds checks) and the
// deterministic split-K reduction.  The kernels themselves are in gemm_kernels.hpp.
#include "gemm_kernels.hpp"

#include <algorithm>

namespace dtrg {

// Sum of split-K partials in a fixed order, then the scatter epilogue.
template <class TA, class TO>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(KArgs p) {
    const i64 MN = (i64)p.M * p.N;
    const i64 total = MN * p.batch;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const i64 zb = idx / MN, rc = idx % MN;
        const int r = (int)(rc / p.N), c = (int)(rc % p.N);
        const TA* W = (const TA*)p.W + zb * p.splits * MN + rc;
        double s = 0.0;
        for (int q = 0; q < p.splits; ++q) s += (double)W[(i64)q * MN];
        TO* C = (TO*)p.C + zb * p.c_bs;
        const i64 off = idx_off(p.rmap, r) + idx_off(p.cmap, c);
        double v = p.alpha * s;
        if (p.beta != 0.0) v += p.beta * (double)C[off];
        C[off] = (TO)v;
    }
}

namespace {

i64 map_max(const IdxMap& m, i64 count) {
    if (count <= 0) return 0;
    const i64 last = count - 1;
    if (last < m.div) return last * m.s0;
    return (last / m.div) * m.s1 + (m.div - 1) * m.s0;
}

}  // namespace

void gemm(Prec prec, bool out_f64, const GemmOp& op, hipStream_t s, Scratch& ws) {
    DTRG_REQUIRE(op.M >= 0 && op.N >= 0 && op.K >= 0 && op.batch >= 1, DTRG_EINVAL, "gemm: bad sizes");
    if (op.M == 0 || op.N == 0) return;
    if (op.K > 0 && op.a_cap >= 0) {
        const i64 mx = (op.a_kmajor ? (i64)(op.K - 1) * op.lda + (op.M - 1) : (i64)(op.M - 1) * op.lda + (op.K - 1)) +
                       (i64)(op.batch - 1) * op.a_bs;
        DTRG_REQUIRE(mx < op.a_cap, DTRG_EINVAL, "gemm: operand A out of bounds");
    }
    if (op.K > 0 && op.b_cap >= 0) {
        const i64 mx = (op.b_kmajor ? (i64)(op.K - 1) * op.ldb + (op.N - 1) : (i64)(op.N - 1) * op.ldb + (op.K - 1)) +
                       (i64)(op.batch - 1) * op.b_bs;
        DTRG_REQUIRE(mx < op.b_cap, DTRG_EINVAL, "gemm: operand B out of bounds");
    }
    if (op.c_cap >= 0) {
        const i64 mx = map_max(op.rmap, op.M) + map_max(op.cmap, op.N) + (i64)(op.batch - 1) * op.c_bs;
        DTRG_REQUIRE(mx < op.c_cap, DTRG_EINVAL, "gemm: output C out of bounds");
    }
    KArgs a;
    a.M = op.M; a.N = op.N; a.K = op.K;
    a.A = op.A; a.lda = op.lda; a.a_bs = op.a_bs;
    a.B = op.B; a.ldb = op.ldb; a.b_bs = op.b_bs;
    a.C = op.C; a.c_bs = op.c_bs;
    a.rmap = op.rmap; a.cmap = op.cmap;
    a.alpha = op.alpha; a.beta = op.beta;
    a.batch = op.batch;
    a.W = nullptr;

    // tile shape: 128x128 for large outputs, 64x64 otherwise
    const bool big = (op.M >= 256 && op.N >= 128) || (op.N >= 256 && op.M >= 128);
    const int BM = big ? 128 : 64, BN = big ? 128 : 64;
    const int BK = (prec == Prec::BF16X3) ? 32 : 16;
    const i64 tiles = (i64)((op.M + BM - 1) / BM) * ((op.N + BN - 1) / BN) * op.batch;
    int splits = op.splits;
    if (splits <= 0) {
        splits = 1;
        // fill the 256 CUs (several blocks each) when the output is small and K is long
        if (tiles < 512) {
            const i64 want = (1024 + tiles - 1) / tiles;
            const i64 maxs = std::max<i64>(1, op.K / (BK * 8));
            splits = (int)std::min<i64>({want, maxs, 64});
        }
    }
    const int k_chunk_raw = (op.K + splits - 1) / std::max(splits, 1);
    a.k_chunk = std::max(BK, ((k_chunk_raw + BK - 1) / BK) * BK);
    splits = std::max(1, (op.K + a.k_chunk - 1) / a.k_chunk);
    if (op.K == 0) splits = 1;
    a.splits = splits;
    DTRG_REQUIRE((i64)op.batch * splits < 65536, DTRG_EINVAL, "gemm: batch x splits too large");

    const bool acc_f64 = (prec == Prec::F64);
    if (splits > 1) {
        const i64 need_elems = (i64)op.batch * splits * op.M * op.N;
        const i64 need_d = acc_f64 ? need_elems : (need_elems + 1) / 2;
        ws.splitk.ensure((size_t)need_d);
        a.W = ws.splitk.p;
    }
    a.tiles_m = (op.M + BM - 1) / BM;
    a.tiles_n = (op.N + BN - 1) / BN;
    const i64 total = (i64)a.tiles_m * a.tiles_n;
    const i64 chunk = (total + kXcds - 1) / kXcds;
    DTRG_REQUIRE(total < (1LL << 30), DTRG_EINVAL, "gemm: grid too large");
    dim3 grid((unsigned)(chunk * kXcds), 1, op.batch * splits);

    switch (prec) {
        case Prec::F64:
            DTRG_REQUIRE(out_f64, DTRG_EINVAL, "gemm: FP64 contraction must write FP64");
            launch_gemm_f64(a, grid, op.a_kmajor, op.b_kmajor, op.tag, big, s);
            break;
        case Prec::F32:
            launch_gemm_f32(a, grid, op.a_kmajor, op.b_kmajor, op.tag, big, out_f64, s);
            break;
        case Prec::BF16X3:
            launch_gemm_bf16x3(a, grid, op.a_kmajor, op.b_kmajor, op.tag, big, out_f64, s);
            break;
    }
    DTRG_HIP(hipGetLastError());
    if (splits > 1) {
        const i64 total = (i64)op.M * op.N * op.batch;
        const int nb = (int)std::min<i64>((total + 255) / 256, 4096);
        if (acc_f64) hipLaunchKernelGGL((splitk_reduce_kernel<double, double>), dim3(nb), dim3(256), 0, s, a);
        else if (out_f64) hipLaunchKernelGGL((splitk_reduce_kernel<float, double>), dim3(nb), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((splitk_reduce_kernel<float, float>), dim3(nb), dim3(256), 0, s, a);
        DTRG_HIP(hipGetLastError());
    }
}

}  // namespace dtrg
