// MFMA contraction kernel for gfx950: C = alpha * A B^T + beta * C with strided operands,
// batching, split-K and a two-level scatter epilogue.
//
// Every tensor contraction of the HOTRG step and its adjoint is one call of this kernel: the
// operands are read either K-contiguous or M/N-contiguous straight from the layout their
// producer wrote, and the epilogue writes each output element at
//     C + batch * c_bs + (r / rdiv) * rs1 + (r % rdiv) * rs0 + (c / cdiv) * cs1 + (c % cdiv) * cs0,
// which is enough to emit every intermediate directly in the layout its consumer reads.
//
// Tiling: 256 threads = 4 waves (2 x 2); block tile BM x BN x BK staged through LDS with one
// register-prefetched stage (one barrier per K tile); each wave owns (BM/2) x (BN/2) outputs as
// 16 x 16 MFMA tiles.  FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32; the split-
// bf16 path uses v_mfma_f32_16x16x32_bf16 three times per K step (hi*hi + hi*lo + lo*hi).
#include "common.hpp"

#include <algorithm>

namespace dtrg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct KArgs {
    int M, N, K;
    const void* A; i64 lda, a_bs;
    const void* B; i64 ldb, b_bs;
    void* C; i64 c_bs;
    IdxMap rmap, cmap;
    double alpha, beta;
    int splits, k_chunk, batch;
    void* W;  // split-K partials [batch * splits][M][N], accumulator type
};

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

template <class T, class TO, int BM, int BN, int BK, bool AKM, bool BKM>
__global__ __launch_bounds__(256) void gemm_mfma4_kernel(KArgs p) {
    typedef typename Mfma4<T>::acc_t acc_t;
    constexpr int NT = 256;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
    constexpr int PAD = 0;
    static_assert(AE >= 1 && BE >= 1, "tile too small");
    __shared__ T As[2][BK][BM + PAD];
    __shared__ T Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int zb = blockIdx.z / p.splits, zs = blockIdx.z % p.splits;
    const int kbeg = zs * p.k_chunk;
    const int kend = min(p.K, kbeg + p.k_chunk);
    const T* A = (const T*)p.A + (i64)zb * p.a_bs;
    const T* B = (const T*)p.B + (i64)zb * p.b_bs;

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0};

    T ra[AE], rb[BE];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            int m, k;
            if (AKM) { int idx = tid + e * NT; k = idx / BM; m = idx % BM; }
            else { int idx = tid * AE + e; m = idx / BK; k = idx % BK; }
            int gm = m0 + m, gk = k0 + k;
            ra[e] = (gm < p.M && gk < kend) ? (AKM ? A[(i64)gk * p.lda + gm] : A[(i64)gm * p.lda + gk]) : T(0);
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            int n, k;
            if (BKM) { int idx = tid + e * NT; k = idx / BN; n = idx % BN; }
            else { int idx = tid * BE + e; n = idx / BK; k = idx % BK; }
            int gn = n0 + n, gk = k0 + k;
            rb[e] = (gn < p.N && gk < kend) ? (BKM ? B[(i64)gk * p.ldb + gn] : B[(i64)gn * p.ldb + gk]) : T(0);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            int m, k;
            if (AKM) { int idx = tid + e * NT; k = idx / BM; m = idx % BM; }
            else { int idx = tid * AE + e; m = idx / BK; k = idx % BK; }
            As[buf][k][m] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            int n, k;
            if (BKM) { int idx = tid + e * NT; k = idx / BN; n = idx % BN; }
            else { int idx = tid * BE + e; n = idx / BK; k = idx % BK; }
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
    TO* C = (TO*)p.C + (i64)zb * p.c_bs;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm0 + i * 16 + Mfma4<T>::row(lk, r), gn = n0 + wn0 + j * 16 + li;
                if (gm < p.M && gn < p.N) {
                    i64 off = idx_off(p.rmap, gm) + idx_off(p.cmap, gn);
                    double v = p.alpha * (double)acc[i][j][r];
                    if (p.beta != 0.0) v += p.beta * (double)C[off];
                    C[off] = (TO)v;
                }
            }
}

// ------------------------------------------------------------------------------------------
// split-bf16 x3 on v_mfma_f32_16x16x32_bf16.  Fragment layout (A 16x32, B 32x16) for lane l:
//   A[i = l % 16][k = 8 * (l / 16) + e], B[k = 8 * (l / 16) + e][j = l % 16], e = 0..7;
//   D as for the 16x16x4 instructions.
// Operands arrive as FP32; each element is split into hi = bf16(x) and lo = bf16(x - hi) while
// it is staged into LDS.
// ------------------------------------------------------------------------------------------
__device__ inline __bf16 f2bf(float x) { return (__bf16)x; }

template <class TO, int BM, int BN, bool AKM, bool BKM>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(KArgs p) {
    constexpr int BK = 32;
    constexpr int NT = 256;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
    constexpr int KP = BK + 8;  // k-contiguous rows of bf16, padded
    __shared__ __bf16 Ah[2][BM][KP], Al[2][BM][KP];
    __shared__ __bf16 Bh[2][BN][KP], Bl[2][BN][KP];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int zb = blockIdx.z / p.splits, zs = blockIdx.z % p.splits;
    const int kbeg = zs * p.k_chunk;
    const int kend = min(p.K, kbeg + p.k_chunk);
    const float* A = (const float*)p.A + (i64)zb * p.a_bs;
    const float* B = (const float*)p.B + (i64)zb * p.b_bs;

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    float ra[AE], rb[BE];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            int m, k;
            if (AKM) { int idx = tid + e * NT; k = idx / BM; m = idx % BM; }
            else { int idx = tid * AE + e; m = idx / BK; k = idx % BK; }
            int gm = m0 + m, gk = k0 + k;
            ra[e] = (gm < p.M && gk < kend) ? (AKM ? A[(i64)gk * p.lda + gm] : A[(i64)gm * p.lda + gk]) : 0.f;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            int n, k;
            if (BKM) { int idx = tid + e * NT; k = idx / BN; n = idx % BN; }
            else { int idx = tid * BE + e; n = idx / BK; k = idx % BK; }
            int gn = n0 + n, gk = k0 + k;
            rb[e] = (gn < p.N && gk < kend) ? (BKM ? B[(i64)gk * p.ldb + gn] : B[(i64)gn * p.ldb + gk]) : 0.f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            int m, k;
            if (AKM) { int idx = tid + e * NT; k = idx / BM; m = idx % BM; }
            else { int idx = tid * AE + e; m = idx / BK; k = idx % BK; }
            __bf16 h = f2bf(ra[e]);
            Ah[buf][m][k] = h;
            Al[buf][m][k] = f2bf(ra[e] - (float)h);
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            int n, k;
            if (BKM) { int idx = tid + e * NT; k = idx / BN; n = idx % BN; }
            else { int idx = tid * BE + e; n = idx / BK; k = idx % BK; }
            __bf16 h = f2bf(rb[e]);
            Bh[buf][n][k] = h;
            Bl[buf][n][k] = f2bf(rb[e] - (float)h);
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
        v8bf ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            ah[i] = *(const v8bf*)&Ah[buf][wm0 + i * 16 + li][8 * lk];
            al[i] = *(const v8bf*)&Al[buf][wm0 + i * 16 + li][8 * lk];
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            bh[j] = *(const v8bf*)&Bh[buf][wn0 + j * 16 + li][8 * lk];
            bl[j] = *(const v8bf*)&Bl[buf][wn0 + j * 16 + li][8 * lk];
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        if (t + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    if (p.splits > 1) {
        float* W = (float*)p.W + (i64)blockIdx.z * p.M * p.N;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int gm = m0 + wm0 + i * 16 + 4 * lk + r, gn = n0 + wn0 + j * 16 + li;
                    if (gm < p.M && gn < p.N) W[(i64)gm * p.N + gn] = acc[i][j][r];
                }
        return;
    }
    TO* C = (TO*)p.C + (i64)zb * p.c_bs;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm0 + i * 16 + 4 * lk + r, gn = n0 + wn0 + j * 16 + li;
                if (gm < p.M && gn < p.N) {
                    i64 off = idx_off(p.rmap, gm) + idx_off(p.cmap, gn);
                    double v = p.alpha * (double)acc[i][j][r];
                    if (p.beta != 0.0) v += p.beta * (double)C[off];
                    C[off] = (TO)v;
                }
            }
}

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

// ------------------------------------------------------------------------------------------
// host dispatch
// ------------------------------------------------------------------------------------------
namespace {

template <class T, class TO, int BM, int BN, int BK>
void launch_mfma4(const KArgs& a, dim3 grid, bool akm, bool bkm, hipStream_t s) {
    if (akm && bkm) hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, true, true>), grid, dim3(256), 0, s, a);
    else if (akm) hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, true, false>), grid, dim3(256), 0, s, a);
    else if (bkm) hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, false, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((gemm_mfma4_kernel<T, TO, BM, BN, BK, false, false>), grid, dim3(256), 0, s, a);
}

template <class TO, int BM, int BN>
void launch_bf16x3(const KArgs& a, dim3 grid, bool akm, bool bkm, hipStream_t s) {
    if (akm && bkm) hipLaunchKernelGGL((gemm_bf16x3_kernel<TO, BM, BN, true, true>), grid, dim3(256), 0, s, a);
    else if (akm) hipLaunchKernelGGL((gemm_bf16x3_kernel<TO, BM, BN, true, false>), grid, dim3(256), 0, s, a);
    else if (bkm) hipLaunchKernelGGL((gemm_bf16x3_kernel<TO, BM, BN, false, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((gemm_bf16x3_kernel<TO, BM, BN, false, false>), grid, dim3(256), 0, s, a);
}

}  // namespace

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
    dim3 grid((op.M + BM - 1) / BM, (op.N + BN - 1) / BN, op.batch * splits);
    DTRG_REQUIRE(grid.y < 65536 && grid.x < (1u << 31), DTRG_EINVAL, "gemm: grid too large");

    switch (prec) {
        case Prec::F64:
            DTRG_REQUIRE(out_f64, DTRG_EINVAL, "gemm: FP64 contraction must write FP64");
            if (big) launch_mfma4<double, double, 128, 128, 16>(a, grid, op.a_kmajor, op.b_kmajor, s);
            else launch_mfma4<double, double, 64, 64, 16>(a, grid, op.a_kmajor, op.b_kmajor, s);
            break;
        case Prec::F32:
            if (out_f64) {
                if (big) launch_mfma4<float, double, 128, 128, 16>(a, grid, op.a_kmajor, op.b_kmajor, s);
                else launch_mfma4<float, double, 64, 64, 16>(a, grid, op.a_kmajor, op.b_kmajor, s);
            } else {
                if (big) launch_mfma4<float, float, 128, 128, 16>(a, grid, op.a_kmajor, op.b_kmajor, s);
                else launch_mfma4<float, float, 64, 64, 16>(a, grid, op.a_kmajor, op.b_kmajor, s);
            }
            break;
        case Prec::BF16X3:
            if (out_f64) {
                if (big) launch_bf16x3<double, 128, 128>(a, grid, op.a_kmajor, op.b_kmajor, s);
                else launch_bf16x3<double, 64, 64>(a, grid, op.a_kmajor, op.b_kmajor, s);
            } else {
                if (big) launch_bf16x3<float, 128, 128>(a, grid, op.a_kmajor, op.b_kmajor, s);
                else launch_bf16x3<float, 64, 64>(a, grid, op.a_kmajor, op.b_kmajor, s);
            }
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
