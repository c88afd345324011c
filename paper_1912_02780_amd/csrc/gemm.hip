// Host dispatch of the MFMA contraction kernels (tile choice, split-K, bounds checks) and the
// deterministic split-K reduction.  The kernels are in gemm_kernels.hpp (FP64, FP32) and
// gemm_split.hpp (bf16 planes).
#include "gemm_kernels.hpp"

#include <algorithm>
#include <cstdint>

namespace dtrg {

// Sum of split-K partials in a fixed order (q = 0, 1, ...), then the shared epilogue.  The
// partials are loaded sixteen at a time before they are added (the last group padded with zeros,
// which leave the sum unchanged), so that a thread waits for one memory round trip per sixteen
// splits rather than per split.
template <class TA, int OUT>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(KArgs p) {
    constexpr int U = 16;
    const i64 MN = (i64)p.M * p.N;
    const i64 total = MN * p.batch * p.batch2;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const i64 zb = idx / MN, rc = idx % MN;
        const int r = (int)(rc / p.N), c = (int)(rc % p.N);
        // a symmetric output's tiles above the diagonal have no partials: they are written as the
        // mirror images of the tiles below it
        if (p.sym == 1 && r / p.sym_tile < c / p.sym_tile) continue;
        const TA* W = (const TA*)p.W + zb * p.splits * MN + rc;
        double s = 0.0;
        for (int q = 0; q < p.splits; q += U) {
            TA v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = q + u < p.splits ? W[(i64)(q + u) * MN] : TA(0);
#pragma unroll
            for (int u = 0; u < U; ++u) s += (double)v[u];
        }
        write_out<OUT>(p, (int)zb, r, c, p.alpha * s);
    }
}

namespace {

i64 map_max(const IdxMap& m, i64 count) {
    if (count <= 0) return 0;
    const i64 last = count - 1;
    if (last < m.div) return last * m.s0;
    return (last / m.div) * m.s1 + (m.div - 1) * m.s0;
}

// K tile of the kernel that runs a configuration (split-K chunks are multiples of it)
int bk_of(Prec prec, int tile) { return prec_planes(prec) == 1 || tile == 6 ? 16 : 32; }

int out_code(Prec prec, Out out) {
    if (out == Out::F64) return 0;
    if (out == Out::F32) return 1;
    return prec_planes(prec);
}

i64 round8(i64 x) { return (x + 7) / 8 * 8; }

// K chunk and number of K chunks a resolved configuration runs with (chunks are whole K tiles)
void resolve_chunks(Prec prec, const GemmOp& op, const GemmCfg& cfg, int& k_chunk, int& splits) {
    const int BK = bk_of(prec, cfg.tile);
    splits = std::max(1, cfg.splits);
    const int k_chunk_raw = (op.K + splits - 1) / splits;
    k_chunk = std::max(BK, ((k_chunk_raw + BK - 1) / BK) * BK);
    splits = std::max(1, (op.K + k_chunk - 1) / k_chunk);
    if (op.K == 0) splits = 1;
}

// a short, wide split-bf16 output is computed as its transpose (see gemm)
bool run_transposed(Prec prec, const GemmOp& op) {
    return prec_planes(prec) > 1 && op.cfg.tile == 0 && op.M <= 64 && op.N >= 1024;
}

// the largest split-K workspace (elements) and count spent on keeping FP32 accumulation chains short
constexpr i64 kMaxChainPartials = 1LL << 32;
constexpr i64 kMaxChainSplits = 256;

}  // namespace

int prec_planes(Prec p) { return p == Prec::BF16X3 ? 2 : (p == Prec::BF16X6 ? 3 : 1); }

namespace {
// rows of the full output (a symmetric output with packed rows has rdig^2)
i64 full_rows(const GemmOp& op) { return op.sym == 2 ? (i64)op.rdig * op.rdig : op.M; }

// output tiles a configuration computes per batch element (a sym = 1 output: the lower triangle)
i64 tile_count(const GemmOp& op, int BM, int BN) {
    const i64 tm = (op.M + BM - 1) / BM, tn = (op.N + BN - 1) / BN;
    return op.sym == 1 ? tm * (tm + 1) / 2 : tm * tn;
}
}  // namespace

i64 gemm_c_extent(const GemmOp& op) {
    if (op.M == 0 || op.N == 0) return 0;
    return map_max(op.rmap, full_rows(op)) + map_max(op.cmap, op.N) + (i64)(op.batch - 1) * op.c_bs +
           (i64)(op.batch2 - 1) * op.c_bs2 + 1;
}

GemmCfg gemm_resolve(Prec prec, const GemmOp& op) {
    GemmCfg c = op.cfg;
    const bool split = prec_planes(prec) > 1;
    if (c.tile == 0) {
        // 128 x 128 for large outputs (256 x 128 for the split kernel when there are enough of
        // them to fill the chip), 64 x 64 otherwise; for the split kernel, 64 x 64 on waves of 16
        // full-width rows when the output has at most 64 columns and many rows (a tall operand
        // streamed past a narrow one: 10% faster than 2 x 2 waves; 128 x 64 and 256 x 64 tiles,
        // which re-read the narrow operand less often, were not faster)
        const bool big = (op.M >= 256 && op.N >= 128) || (op.N >= 256 && op.M >= 128);
        c.tile = big ? 2 : 1;
        if (split && big && op.M >= 256) {
            // the largest tile when it alone fills the chip, or when K is long enough for split-K to
            const i64 t3 = (i64)((op.M + 255) / 256) * ((op.N + 127) / 128) * op.batch * op.batch2;
            if (t3 >= 512 || (op.N >= 128 && op.K >= 4096)) c.tile = 3;
        }
        if (split && op.N <= 64 && op.M >= 1024) c.tile = 4;
    }
    const int BM = tile_rows(c.tile), BN = tile_cols(c.tile);
    const int BK = bk_of(prec, c.tile);
    if (c.splits <= 0) {
        const i64 nz = (i64)op.batch * op.batch2;
        const i64 tiles = tile_count(op, BM, BN) * nz;
        c.splits = 1;
        // fill the 256 CUs (several blocks each) when the output is small and K is long
        if (tiles < 512) {
            const i64 want = (1024 + tiles - 1) / tiles;
            const i64 maxs = std::max<i64>(1, op.K / (BK * 8));
            c.splits = (int)std::min<i64>({want, maxs, 64});
        }
        c.splits = std::max(c.splits, gemm_chain_splits(prec, op));
    }
    return c;
}

i64 gemm_workspace(Prec prec, const GemmOp& op) {
    if (op.M == 0 || op.N == 0) return 0;
    if (run_transposed(prec, op)) {
        GemmOp t = op;
        std::swap(t.M, t.N);
        return gemm_workspace(prec, t);
    }
    int k_chunk = 0, splits = 1;
    resolve_chunks(prec, op, gemm_resolve(prec, op), k_chunk, splits);
    if (splits <= 1) return 0;
    const i64 elems = (i64)op.batch * op.batch2 * splits * op.M * op.N;
    return prec == Prec::F64 ? elems : (elems + 1) / 2;
}

int gemm_chain_splits(Prec prec, const GemmOp& op) {
    // FP32 accumulation: no chain longer than op.max_chain products per output (the partials are
    // summed in FP64), where the partials fit in kMaxChainPartials elements; otherwise as many
    // splits as fit
    const i64 cap = std::max(op.max_chain, 32);
    if (prec == Prec::F64 || op.K <= cap) return 1;
    const i64 nz = (i64)op.batch * op.batch2;
    i64 need = std::min<i64>(kMaxChainSplits, (op.K + cap - 1) / cap);
    const i64 fit = kMaxChainPartials / std::max<i64>(1, nz * (i64)op.M * op.N);
    need = std::min(need, fit);
    while (need > 1 && nz * need >= 65536) --need;
    return (int)std::max<i64>(1, need);
}

void gemm(Prec prec, Out out, const GemmOp& op, hipStream_t s, Scratch& ws) {
    DTRG_REQUIRE(op.M >= 0 && op.N >= 0 && op.K >= 0 && op.batch >= 1 && op.batch2 >= 1, DTRG_EINVAL,
                 "gemm: bad sizes");
    if (op.M == 0 || op.N == 0) return;
    const int np = prec_planes(prec);
    const bool split = np > 1;
    if (run_transposed(prec, op)) {
        // a short, wide output is computed as its transpose, C(r, c) = sum_k B(c, k) A(r, k) with
        // the roles of the operands and of the index maps exchanged, so that the tall-operand tile
        // streams the long operand once
        GemmOp t = op;
        std::swap(t.M, t.N);
        std::swap(t.A, t.B); std::swap(t.lda, t.ldb); std::swap(t.a_bs, t.b_bs); std::swap(t.a_bs2, t.b_bs2);
        std::swap(t.a_ps, t.b_ps); std::swap(t.a_kmajor, t.b_kmajor); std::swap(t.a_cap, t.b_cap);
        std::swap(t.rmap, t.cmap);
        gemm(prec, out, t, s, ws);
        return;
    }
    DTRG_REQUIRE(prec != Prec::F64 || out == Out::F64, DTRG_EINVAL, "gemm: FP64 contraction must write FP64");
    if (op.sym != 0) {
        DTRG_REQUIRE(prec == Prec::F64 && op.beta == 0.0 && (op.sym == 1 || op.sym == 2), DTRG_EINVAL,
                     "gemm: symmetric outputs are FP64 contractions with beta = 0");
        DTRG_REQUIRE(op.sym != 1 || op.M == op.N, DTRG_EINVAL, "gemm: sym = 1 needs a square output");
        DTRG_REQUIRE(op.sym != 2 || (op.rdig >= 1 && op.cdig >= 1 && (i64)op.M == (i64)op.rdig * (op.rdig + 1) / 2 &&
                                     (i64)op.N == (i64)op.cdig * op.cdig),
                     DTRG_EINVAL, "gemm: sym = 2 needs M = rdig (rdig + 1) / 2 packed rows and N = cdig^2");
    }
    DTRG_REQUIRE(out != Out::Split || (split && op.beta == 0.0), DTRG_EINVAL,
                 "gemm: split output needs a split contraction and beta = 0");
    if (split) {
        // planes with 16-byte aligned rows padded to a multiple of 8 elements: K-contiguous rows of
        // at least round8(K) elements, or K-major rows of at least round8(M) (round8(N)) elements,
        // the latter only into FP64 or FP32 outputs
        DTRG_REQUIRE(op.lda % 8 == 0 && op.ldb % 8 == 0, DTRG_EINVAL,
                     "gemm: split operand rows must be padded to a multiple of 8 elements");
        DTRG_REQUIRE(op.lda >= round8(op.a_kmajor ? op.M : op.K) && op.ldb >= round8(op.b_kmajor ? op.N : op.K),
                     DTRG_EINVAL, "gemm: split operand rows shorter than their padded extent");
        DTRG_REQUIRE(!(op.a_kmajor || op.b_kmajor) || out != Out::Split, DTRG_EINVAL,
                     "gemm: K-major split operands need an FP64 or FP32 output");
        DTRG_REQUIRE((op.a_ps | op.b_ps | op.a_bs | op.b_bs | op.a_bs2 | op.b_bs2) % 8 == 0, DTRG_EINVAL,
                     "gemm: split operand strides must be multiples of 8 elements");
        DTRG_REQUIRE(((uintptr_t)op.A | (uintptr_t)op.B) % 16 == 0, DTRG_EINVAL,
                     "gemm: split operands must be 16-byte aligned");
    }
    // the kernels read whole 16-byte chunks of split rows: the row extent is padded to 8 elements
    auto ext = [&](i64 x) { return split ? round8(x) : x; };
    if (op.K > 0 && op.a_cap >= 0) {
        const i64 rows = full_rows(op);   // rows read from A (packed rows stand for rows below rdig^2)
        const i64 mx = (op.a_kmajor ? (i64)(op.K - 1) * op.lda + (ext(rows) - 1) : (i64)(rows - 1) * op.lda + (ext(op.K) - 1)) +
                       (i64)(op.batch - 1) * op.a_bs + (i64)(op.batch2 - 1) * op.a_bs2 + (i64)(np - 1) * op.a_ps;
        DTRG_REQUIRE(mx < op.a_cap, DTRG_EINVAL, "gemm: operand A out of bounds");
    }
    if (op.K > 0 && op.b_cap >= 0) {
        const i64 mx = (op.b_kmajor ? (i64)(op.K - 1) * op.ldb + (ext(op.N) - 1) : (i64)(op.N - 1) * op.ldb + (ext(op.K) - 1)) +
                       (i64)(op.batch - 1) * op.b_bs + (i64)(op.batch2 - 1) * op.b_bs2 + (i64)(np - 1) * op.b_ps;
        DTRG_REQUIRE(mx < op.b_cap, DTRG_EINVAL, "gemm: operand B out of bounds");
    }
    const int onp = out == Out::Split ? np : 1;
    if (op.c_cap >= 0)
        DTRG_REQUIRE(gemm_c_extent(op) + (i64)(onp - 1) * op.c_ps <= op.c_cap, DTRG_EINVAL,
                     "gemm: output C out of bounds");
    KArgs a;
    a.M = op.M; a.N = op.N; a.K = op.K;
    a.A = op.A; a.lda = op.lda; a.a_bs = op.a_bs; a.a_bs2 = op.a_bs2; a.a_ps = op.a_ps;
    a.B = op.B; a.ldb = op.ldb; a.b_bs = op.b_bs; a.b_bs2 = op.b_bs2; a.b_ps = op.b_ps;
    a.C = op.C; a.c_bs = op.c_bs; a.c_bs2 = op.c_bs2; a.c_ps = op.c_ps;
    a.rmap = op.rmap; a.cmap = op.cmap;
    a.alpha = op.alpha; a.beta = op.beta;
    a.batch = op.batch; a.batch2 = op.batch2;
    a.W = nullptr;
    a.sym = op.sym; a.rdig = op.rdig; a.cdig = op.cdig; a.sym_tile = 1;
    {
        // 16-byte epilogue stores of bf16 planes: every aligned group of 8 output columns must be
        // contiguous and start on a multiple of 8 elements in every plane and batch element
        auto al8 = [](i64 x) { return x % 8 == 0; };
        const bool cols = op.cmap.s0 == 1 && (op.cmap.div >= (1LL << 62) || al8(op.cmap.div)) && al8(op.cmap.s1);
        const bool rows = al8(op.rmap.s0) && al8(op.rmap.s1);
        a.vec_out = out == Out::Split && cols && rows && al8(op.c_bs) && al8(op.c_bs2) && al8(op.c_ps) &&
                    (uintptr_t)op.C % 16 == 0;
    }

    const GemmCfg cfg = gemm_resolve(prec, op);
    DTRG_REQUIRE(cfg.tile == 1 || cfg.tile == 2 || ((cfg.tile >= 3 && cfg.tile <= 6) && split), DTRG_EINVAL,
                 "gemm: bad tile configuration");
    DTRG_REQUIRE(cfg.tile != 6 || (!op.a_kmajor && !op.b_kmajor && op.K % 16 == 0), DTRG_EINVAL,
                 "gemm: tile 6 takes K-contiguous operands and K a multiple of 16 only");
    const int BM = tile_rows(cfg.tile), BN = tile_cols(cfg.tile);
    DTRG_REQUIRE(op.sym != 1 || BM == BN, DTRG_EINVAL, "gemm: sym = 1 needs square tiles");
    a.sym_tile = BM;
    int splits = 1;
    resolve_chunks(prec, op, cfg, a.k_chunk, splits);
    a.splits = splits;
    const i64 nz = (i64)op.batch * op.batch2;
    DTRG_REQUIRE(nz * splits < 65536, DTRG_EINVAL, "gemm: batch x splits too large");

    const bool acc_f64 = (prec == Prec::F64);
    if (splits > 1) {
        ws.splitk.ensure((size_t)gemm_workspace(prec, op));
        a.W = ws.splitk.p;
    }
    a.tiles_m = (op.M + BM - 1) / BM;
    a.tiles_n = (op.N + BN - 1) / BN;
    const i64 total = tile_count(op, BM, BN);
    const i64 chunk = (total + kXcds - 1) / kXcds;
    DTRG_REQUIRE(total < (1LL << 30), DTRG_EINVAL, "gemm: grid too large");
    dim3 grid((unsigned)(chunk * kXcds), 1, (unsigned)(nz * splits));

    const int oc = out_code(prec, out);
    switch (prec) {
        case Prec::F64:
            launch_gemm_f64(a, grid, op.a_kmajor, op.b_kmajor, op.tag, cfg.tile == 2, s);
            break;
        case Prec::F32:
            launch_gemm_f32(a, grid, op.a_kmajor, op.b_kmajor, op.tag, cfg.tile == 2, out == Out::F64, s);
            break;
        case Prec::BF16X3:
        case Prec::BF16X6:
            launch_gemm_split(a, grid, np, oc, cfg.tile, op.tag, op.a_kmajor, op.b_kmajor, s);
            break;
    }
    DTRG_HIP(hipGetLastError());
    if (splits > 1) {
        const i64 tot = (i64)op.M * op.N * nz;
        const dim3 g((unsigned)std::min<i64>((tot + 255) / 256, 4096));
        if (acc_f64) hipLaunchKernelGGL((splitk_reduce_kernel<double, 0>), g, dim3(256), 0, s, a);
        else if (oc == 0) hipLaunchKernelGGL((splitk_reduce_kernel<float, 0>), g, dim3(256), 0, s, a);
        else if (oc == 1) hipLaunchKernelGGL((splitk_reduce_kernel<float, 1>), g, dim3(256), 0, s, a);
        else if (oc == 2) hipLaunchKernelGGL((splitk_reduce_kernel<float, 2>), g, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((splitk_reduce_kernel<float, 3>), g, dim3(256), 0, s, a);
        DTRG_HIP(hipGetLastError());
    }
}

}  // namespace dtrg
