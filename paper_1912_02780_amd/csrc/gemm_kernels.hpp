// MFMA contraction kernel for gfx950: C = alpha * A B^T + beta * C with strided operands,
// batching, split-K and a two-level scatter epilogue.
//
// Every tensor contraction of the HOTRG step and its adjoint is one call of this kernel: the
// operands are read either K-contiguous or M/N-contiguous straight from the layout their
// producer wrote, and the epilogue writes each output element at
//     C + batch * c_bs + (r / rdiv) * rs1 + (r % rdiv) * rs0 + (c / cdiv) * cs1 + (c % cdiv) * cs0,
// which is enough to emit every intermediate directly in the layout its consumer reads.
//
// Tiling: WGM x WGN waves (2 x 2 by default; FP64 runs 128 x 128 tiles on 4 x 2 waves so that two
// waves share each SIMD); block tile BM x BN x BK staged through LDS with one register-prefetched
// stage (one barrier per K tile); each wave owns (BM/WGM) x (BN/WGN) outputs as 16 x 16 MFMA tiles.
// FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32.  The kernel for operands split into
// bf16 planes is in gemm_split.hpp.
#pragma once

#include "common.hpp"

namespace dtrg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

// Tile of a block.  The grid is one-dimensional in x (z = batch x split-K).  Blocks are handed
// to the 8 XCDs round-robin (block b runs on XCD b % 8), so block b = 8 q + x is given the q-th
// tile of XCD x's contiguous share of the tile sequence; the sequence walks bands of kGroupM
// row tiles across all column tiles, so the blocks of one XCD reuse the same A and B tiles from
// that XCD's L2.
constexpr int kXcds = 8;
constexpr int kGroupM = 4;

// Packed index p of the pairs (r1, r0) with r1 >= r0, in the order (0,0), (1,0), (1,1), (2,0), ...:
// p = r1 (r1 + 1) / 2 + r0.
// (The root is off by at most one for the index range used here; one correction each way.)
__host__ __device__ inline void tri_pair(int p, int& r1, int& r0) {
    int a = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    a -= (a * (a + 1) / 2 > p) ? 1 : 0;
    a += ((a + 1) * (a + 2) / 2 <= p) ? 1 : 0;
    r1 = a;
    r0 = p - a * (a + 1) / 2;
}

// With `lower`, only the tiles on or below the diagonal of a square tile grid (tiles_m x tiles_m),
// taken row by row (the same XCD split of the sequence; no bands).
__device__ inline bool tile_of(int pid, int tiles_m, int tiles_n, int& tm, int& tn, bool lower = false) {
    if (lower) {
        const int total = tiles_m * (tiles_m + 1) / 2;
        const int chunk = (total + kXcds - 1) / kXcds;
        const int t = (pid % kXcds) * chunk + pid / kXcds;
        if (t >= total) return false;
        tri_pair(t, tm, tn);
        return true;
    }
    const int total = tiles_m * tiles_n;
    const int chunk = (total + kXcds - 1) / kXcds;
    const int t = (pid % kXcds) * chunk + pid / kXcds;
    if (t >= total) return false;
    const int band = t / (kGroupM * tiles_n);
    const int rows = min(kGroupM, tiles_m - band * kGroupM);
    const int r = t - band * kGroupM * tiles_n;
    tm = band * kGroupM + r % rows;
    tn = r / rows;
    return true;
}

struct KArgs {
    int M, N, K;
    const void* A; i64 lda, a_bs, a_bs2, a_ps;
    const void* B; i64 ldb, b_bs, b_bs2, b_ps;
    void* C; i64 c_bs, c_bs2, c_ps;
    IdxMap rmap, cmap;
    double alpha, beta;
    int splits, k_chunk, batch, batch2;
    int tiles_m, tiles_n;
    void* W;  // split-K partials [batch2 * batch * splits][M][N], accumulator type
    int vec_out;  // bf16-plane output whose aligned groups of 8 columns are 16-byte aligned and
                  // contiguous in every plane (the epilogue then stores 16 bytes per lane)
    int sym, sym_tile, rdig, cdig;  // symmetric output (GemmOp::sym; FP64 kernel only), its tile size
};

// offset of batch element zb = z2 * batch + z1 in an operand with strides (bs, bs2)
__host__ __device__ inline i64 batch_off(const KArgs& p, int zb, i64 bs, i64 bs2) {
    return (i64)(zb % p.batch) * bs + (i64)(zb / p.batch) * bs2;
}

// Output element writers.  OUT = 0: double, 1: float, 2 / 3: the value rounded to FP32 and split
// into that many bf16 planes (plane q = bf16 of what the planes before it leave; planes ps apart).
template <int OUT>
__device__ inline void put_out(void* base, i64 off, i64 ps, double v, double beta) {
    if constexpr (OUT == 0) {
        double* C = (double*)base;
        if (beta != 0.0) v += beta * C[off];
        C[off] = v;
    } else if constexpr (OUT == 1) {
        float* C = (float*)base;
        if (beta != 0.0) v += beta * (double)C[off];
        C[off] = (float)v;
    } else {
        __bf16* C = (__bf16*)base;
        float r = (float)v;
#pragma unroll
        for (int q = 0; q < OUT; ++q) {
            const __bf16 h = (__bf16)r;
            C[q * ps + off] = h;
            r -= (float)h;
        }
    }
}

// write output element (zb, r, c) = v
template <int OUT>
__device__ inline void write_elem(const KArgs& p, int zb, int r, int c, double v) {
    put_out<OUT>(p.C, batch_off(p, zb, p.c_bs, p.c_bs2) + idx_off(p.rmap, r) + idx_off(p.cmap, c), p.c_ps, v, p.beta);
}

// write the output element of kernel row r (a packed row for sym = 2) and column c, and its mirror
// image where the symmetric output has one that is not computed itself
template <int OUT>
__device__ inline void write_out(const KArgs& p, int zb, int r, int c, double v) {
    if (p.sym == 2) {
        int r1, r0;
        tri_pair(r, r1, r0);
        write_elem<OUT>(p, zb, r1 * p.rdig + r0, c, v);
        if (r1 != r0) {
            const int c1 = c / p.cdig, c0 = c - c1 * p.cdig;
            write_elem<OUT>(p, zb, r0 * p.rdig + r1, c0 * p.cdig + c1, v);
        }
        return;
    }
    write_elem<OUT>(p, zb, r, c, v);
    if (p.sym == 1 && r / p.sym_tile > c / p.sym_tile) write_elem<OUT>(p, zb, c, r, v);
}



// ------------------------------------------------------------------------------------------
// FP64 / FP32: 16x16x4 MFMA.  Fragment layout (A 16x4, B 4x16, D 16x16) for lane l:
//   A[i = l % 16][k = l / 16], B[k = l / 16][j = l % 16];
//   accumulator register r of lane l holds D[row(l / 16, r)][j = l % 16] with
//   row = 4 * (l / 16) + r for the f32 instruction and row = l / 16 + 4 * r for the f64 one
//   (measured on gfx950 with an in-bounds 16x16x4 product).
// ------------------------------------------------------------------------------------------
template <class T> struct Mfma4;
template <> struct Mfma4<double> {
    typedef v4d acc_t;
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma4<float> {
    typedef v4f acc_t;
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

// TAG only distinguishes kernel symbols in profiles (7, 8, 9: the three chi^7 contractions).
// WGM x WGN waves per block, each owning (BM / WGM) x (BN / WGN) outputs.
template <class T, class TO, int BM, int BN, int BK, bool AKM, bool BKM, int TAG, int WGM = 2, int WGN = 2>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_mfma4_kernel(KArgs p) {
    typedef typename Mfma4<T>::acc_t acc_t;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
    constexpr int PAD = 1;   // odd row stride: the transposing LDS stores of K-contiguous tiles spread over banks
    constexpr bool SYM = sizeof(T) == 8;   // symmetric outputs: FP64 contractions only
    static_assert(AE >= 1 && BE >= 1, "tile too small");
    __shared__ T As[2][BK][BM + PAD];
    __shared__ T Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;
    int tmi, tni;
    if (!tile_of(blockIdx.x, p.tiles_m, p.tiles_n, tmi, tni, p.sym == 1)) return;
    const int m0 = tmi * BM, n0 = tni * BN;
    const int zb = blockIdx.z / p.splits, zs = blockIdx.z % p.splits;
    const int kbeg = zs * p.k_chunk;
    const int kend = min(p.K, kbeg + p.k_chunk);
    const T* A = (const T*)p.A + batch_off(p, zb, p.a_bs, p.a_bs2);
    const T* B = (const T*)p.B + batch_off(p, zb, p.b_bs, p.b_bs2);
    // the operand row each thread's A elements come from (-1 past the last row): the kernel row,
    // or for sym = 2 the row its packed index stands for
    int arow[AE];
#pragma unroll
    for (int e = 0; e < AE; ++e) {
        const int idx = tid + e * NT;
        const int gm = m0 + (AKM ? idx % BM : idx / BK);
        int r = gm < p.M ? gm : -1;
        if (SYM && p.sym == 2 && r >= 0) {
            int r1, r0;
            tri_pair(gm, r1, r0);
            r = r1 * p.rdig + r0;
        }
        arow[e] = r;
    }

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0};

    T ra[AE], rb[BE];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = tid + e * NT;
            const int k = AKM ? idx / BM : idx % BK;
            const int gr = arow[e], gk = k0 + k;
            ra[e] = (gr >= 0 && gk < kend) ? (AKM ? A[(i64)gk * p.lda + gr] : A[(i64)gr * p.lda + gk]) : T(0);
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            int n, k;
            if (BKM) { int idx = tid + e * NT; k = idx / BN; n = idx % BN; }
            else { int idx = tid + e * NT; n = idx / BK; k = idx % BK; }
            int gn = n0 + n, gk = k0 + k;
            rb[e] = (gn < p.N && gk < kend) ? (BKM ? B[(i64)gk * p.ldb + gn] : B[(i64)gn * p.ldb + gk]) : T(0);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            int m, k;
            if (AKM) { int idx = tid + e * NT; k = idx / BM; m = idx % BM; }
            else { int idx = tid + e * NT; m = idx / BK; k = idx % BK; }
            As[buf][k][m] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            int n, k;
            if (BKM) { int idx = tid + e * NT; k = idx / BN; n = idx % BN; }
            else { int idx = tid + e * NT; n = idx / BK; k = idx % BK; }
            Bs[buf][k][n] = rb[e];
        }
    };

    const int ntiles = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    if (ntiles > 0) {
        load(kbeg);
        store(0);
    }
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles) load(kbeg + (t + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = As[buf][kk + lk][wm0 + i * 16 + li];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[buf][kk + lk][wn0 + j * 16 + li];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Mfma4<T>::mma(af[i], bf[j], acc[i][j]);
        }
        if (t + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    // epilogue
    if (p.splits > 1) {
        T* W = (T*)p.W + (i64)blockIdx.z * p.M * p.N;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int gm = m0 + wm0 + i * 16 + Mfma4<T>::row(lk, r), gn = n0 + wn0 + j * 16 + li;
                    if (gm < p.M && gn < p.N) W[(i64)gm * p.N + gn] = acc[i][j][r];
                }
        return;
    }
    constexpr int OUT = sizeof(TO) == 8 ? 0 : 1;
    // a symmetric output: tiles below the diagonal (sym = 1) and packed rows with r1 > r0 (sym = 2)
    // also write their mirror images
    const bool mirror_tile = SYM && p.sym == 1 && tmi > tni;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gm = m0 + wm0 + i * 16 + Mfma4<T>::row(lk, r);
            if (gm >= p.M) continue;
            int orow = gm, mrow = -1;   // output row and mirrored row (sym = 2)
            if (SYM && p.sym == 2) {
                int r1, r0;
                tri_pair(gm, r1, r0);
                orow = r1 * p.rdig + r0;
                if (r1 != r0) mrow = r0 * p.rdig + r1;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int gn = n0 + wn0 + j * 16 + li;
                if (gn >= p.N) continue;
                const double v = p.alpha * (double)acc[i][j][r];
                write_elem<OUT>(p, zb, orow, gn, v);
                if (mirror_tile) write_elem<OUT>(p, zb, gn, gm, v);
                if (SYM && mrow >= 0) {
                    const int c1 = gn / p.cdig, c0 = gn - c1 * p.cdig;
                    write_elem<OUT>(p, zb, mrow, c0 * p.cdig + c1, v);
                }
            }
        }
}

template <class T, class TO, int BM, int BN, int BK, int TAG, int WGM, int WGN>
void launch_mfma4_t(const KArgs& a, dim3 grid, bool akm, bool bkm, hipStream_t s) {
    const dim3 blk(64 * WGM * WGN);
    if (akm && bkm) hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, true, true, TAG, WGM, WGN>), grid, blk, 0, s, a);
    else if (akm) hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, true, false, TAG, WGM, WGN>), grid, blk, 0, s, a);
    else if (bkm) hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, false, true, TAG, WGM, WGN>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, false, false, TAG, WGM, WGN>), grid, blk, 0, s, a);
}

// tags 7, 8, 9 (the three chi^7 contractions) get their own symbols on the large tiles only
template <class T, class TO, int BM, int BN, int BK, int WGM = 2, int WGN = 2>
void launch_mfma4(const KArgs& a, dim3 grid, bool akm, bool bkm, int tag, hipStream_t s) {
    if constexpr (BM == 128) {
        if (tag == 7) { launch_mfma4_t<T, TO, BM, BN, BK, 7, WGM, WGN>(a, grid, akm, bkm, s); return; }
        if (tag == 8) { launch_mfma4_t<T, TO, BM, BN, BK, 8, WGM, WGN>(a, grid, akm, bkm, s); return; }
        if (tag == 9) { launch_mfma4_t<T, TO, BM, BN, BK, 9, WGM, WGN>(a, grid, akm, bkm, s); return; }
    }
    launch_mfma4_t<T, TO, BM, BN, BK, 0, WGM, WGN>(a, grid, akm, bkm, s);
}

// per-precision launchers (one translation unit each, compiled in parallel)
void launch_gemm_f64(const KArgs& a, dim3 grid, bool akm, bool bkm, int tag, bool big, hipStream_t s);
void launch_gemm_f32(const KArgs& a, dim3 grid, bool akm, bool bkm, int tag, bool big, bool out_f64, hipStream_t s);
// split-bf16 planes (gemm_split*.hip): np = 2 or 3 planes per operand, out = 0 double, 1 float,
// 2 / 3 bf16 planes; tile as in GemmCfg; akm / bkm: K-major operand (FP64 or FP32 output only)
void launch_gemm_split(const KArgs& a, dim3 grid, int np, int out, int tile, int tag, bool akm, bool bkm,
                       hipStream_t s);

}  // namespace dtrg
