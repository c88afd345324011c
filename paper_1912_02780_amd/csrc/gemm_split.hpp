// MFMA contraction kernel for operands split into bf16 planes (gfx950).
//
// An FP32 value x is carried as NP bf16 planes, x ~ x_0 + x_1 (+ x_2), plane q being the bf16
// rounding of what the planes before it leave.  The product of two such operands is accumulated
// in FP32 on v_mfma_f32_16x16x32_bf16 from the partial products that matter at this precision,
// smallest first:
//   NP = 2 (3 products):  a1 b0 + a0 b1 + a0 b0              (relative error ~2^-17 per product)
//   NP = 3 (6 products):  a2 b0 + a1 b1 + a0 b2 + a1 b0 + a0 b1 + a0 b0   (below FP32 rounding)
//
// Both operands are stored K-contiguous (row r of plane q at base + q * ps + r * ld, ld a multiple
// of 8 elements, 16-byte aligned), so every global load and every LDS store moves 16 bytes
// (8 bf16 along K) and the MFMA fragments (8 consecutive K values per lane) are single 16-byte LDS
// reads; there is no conversion work in the K loop.  K beyond the operand's extent is masked to
// zero in the last tile, so row padding is never read as data.
//
// Tiles: BM x BN per block, WGM x WGN waves of (BM / WGM) x (BN / WGN) outputs each, BK per K tile,
// one or two LDS stages (with one stage the next tile waits in registers).  The epilogue is the
// shared one: alpha scaling, optional beta, two-level scatter, and output as
// FP64, FP32 or NP bf16 planes.
#pragma once

#include "gemm_kernels.hpp"

namespace dtrg {

template <int NP, int OUT, int BM, int BN, int WGM, int WGN, int BK, int STAGES, int TAG>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_split_kernel(KArgs p) {
    constexpr int NT = 64 * WGM * WGN;
    constexpr int KP = BK + 8;   // row stride in LDS (bf16), padded
    constexpr int WM = BM / WGM, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
    constexpr int CPR = BK / 8;                      // 16-byte chunks per tile row
    constexpr int ACH = (BM * CPR + NT - 1) / NT;    // chunks per thread per plane
    constexpr int BCH = (BN * CPR + NT - 1) / NT;
    static_assert(TM >= 1 && TN >= 1 && BK % 32 == 0, "bad tile");
    __shared__ __bf16 As[STAGES][NP][BM][KP];
    __shared__ __bf16 Bs[STAGES][NP][BN][KP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;
    int tmi, tni;
    if (!tile_of(blockIdx.x, p.tiles_m, p.tiles_n, tmi, tni)) return;
    const int m0 = tmi * BM, n0 = tni * BN;
    const int zb = blockIdx.z / p.splits, zs = blockIdx.z % p.splits;
    const int kbeg = zs * p.k_chunk;
    const int kend = min(p.K, kbeg + p.k_chunk);
    const __bf16* A = (const __bf16*)p.A + batch_off(p, zb, p.a_bs, p.a_bs2);
    const __bf16* B = (const __bf16*)p.B + batch_off(p, zb, p.b_bs, p.b_bs2);

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    v8bf ra[NP][ACH], rb[NP][BCH];
    auto chunk = [&](const __bf16* X, i64 ld, i64 ps, int q, int row, int nrows, int gk) -> v8bf {
        v8bf v = {};
        if (row < nrows && gk < kend) {
            v = *(const v8bf*)(X + q * ps + (i64)row * ld + gk);
            if (gk + 8 > kend) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (gk + t >= kend) v[t] = (__bf16)0.f;
            }
        }
        return v;
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
#pragma unroll
            for (int e = 0; e < ACH; ++e) {
                const int c = tid + e * NT, m = c / CPR, kc = (c % CPR) * 8;
                ra[q][e] = m < BM ? chunk(A, p.lda, p.a_ps, q, m0 + m, p.M, k0 + kc) : v8bf{};
            }
#pragma unroll
            for (int e = 0; e < BCH; ++e) {
                const int c = tid + e * NT, n = c / CPR, kc = (c % CPR) * 8;
                rb[q][e] = n < BN ? chunk(B, p.ldb, p.b_ps, q, n0 + n, p.N, k0 + kc) : v8bf{};
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
#pragma unroll
            for (int e = 0; e < ACH; ++e) {
                const int c = tid + e * NT, m = c / CPR, kc = (c % CPR) * 8;
                if (m < BM) *(v8bf*)&As[buf][q][m][kc] = ra[q][e];
            }
#pragma unroll
            for (int e = 0; e < BCH; ++e) {
                const int c = tid + e * NT, n = c / CPR, kc = (c % CPR) * 8;
                if (n < BN) *(v8bf*)&Bs[buf][q][n][kc] = rb[q][e];
            }
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
        const int buf = STAGES == 2 ? (t & 1) : 0;
        if (t + 1 < ntiles) load(kbeg + (t + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            v8bf a[NP][TM], b[NP][TN];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
#pragma unroll
                for (int i = 0; i < TM; ++i) a[q][i] = *(const v8bf*)&As[buf][q][wm0 + i * 16 + li][kk + 8 * lk];
#pragma unroll
                for (int j = 0; j < TN; ++j) b[q][j] = *(const v8bf*)&Bs[buf][q][wn0 + j * 16 + li][kk + 8 * lk];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if constexpr (NP == 2) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
                    } else {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
                    }
                }
        }
        if (t + 1 < ntiles) {
            if (STAGES == 1) __syncthreads();   // every wave is done reading the stage
            store(STAGES == 2 ? (buf ^ 1) : 0);
        }
        __syncthreads();
    }

    // epilogue: D row of accumulator register r of lane l is 4 (l / 16) + r, column l % 16
    if (p.splits > 1) {
        float* W = (float*)p.W + (i64)blockIdx.z * p.M * p.N;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = m0 + wm0 + i * 16 + 4 * lk + r, gn = n0 + wn0 + j * 16 + li;
                    if (gm < p.M && gn < p.N) W[(i64)gm * p.N + gn] = acc[i][j][r];
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm0 + i * 16 + 4 * lk + r, gn = n0 + wn0 + j * 16 + li;
                if (gm < p.M && gn < p.N) write_elem<OUT>(p, zb, gm, gn, p.alpha * (double)acc[i][j][r]);
            }
}

// Tile shapes: 1 = 64 x 64 (4 waves of 32 x 32), 2 = 128 x 128 (4 waves of 64 x 64),
// 3 = 256 x 128 (8 waves of 64 x 64).  LDS: at most 120 KiB.
template <int NP, int OUT, int TAG>
void launch_split_tile(const KArgs& a, dim3 grid, int tile, hipStream_t s) {
    if (tile == 3) {
        if constexpr (NP == 2)
            hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 256, 128, 4, 2, 64, 1, TAG>), grid, dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 256, 128, 4, 2, 32, 1, TAG>), grid, dim3(512), 0, s, a);
    } else if (tile == 2) {
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 128, 128, 2, 2, 32, 2, TAG>), grid, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 64, 64, 2, 2, 32, 2, 0>), grid, dim3(256), 0, s, a);
    }
}

// tags 7, 8, 9 (the three chi^7 contractions) get their own symbols on the large tiles only
template <int NP, int OUT>
void launch_split_tag(const KArgs& a, dim3 grid, int tile, int tag, hipStream_t s) {
    if (tile >= 2 && tag == 7) { launch_split_tile<NP, OUT, 7>(a, grid, tile, s); return; }
    if (tile >= 2 && tag == 8) { launch_split_tile<NP, OUT, 8>(a, grid, tile, s); return; }
    if (tile >= 2 && tag == 9) { launch_split_tile<NP, OUT, 9>(a, grid, tile, s); return; }
    launch_split_tile<NP, OUT, 0>(a, grid, tile, s);
}

}  // namespace dtrg
