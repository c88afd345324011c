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
// of 8 elements, 16-byte aligned), so the K tiles (32 bf16 = 64 bytes per row and plane) go from
// global memory straight into LDS with 16-byte direct-to-LDS loads (no registers, no LDS store
// instructions), double-buffered so that the next tile is in flight while the current one is
// multiplied, and the MFMA fragments (8 consecutive K values per lane) are single 16-byte LDS
// reads; there is no conversion work in the K loop.  Elements at or beyond the end of K in the
// last tile are zeroed in LDS, so row padding is never read as data.
//
// Tiles: BM x BN per block, WGM x WGN waves of (BM / WGM) x (BN / WGN) outputs each.  The epilogue
// applies alpha (and beta), scatters through the two-level index maps and writes FP64, FP32 or NP
// bf16 planes; bf16 planes whose aligned groups of 8 columns are contiguous go out as 16-byte
// stores through a per-wave LDS slab.
#pragma once

#include "gemm_kernels.hpp"

namespace dtrg {

// Epilogue of a bf16-plane output with 16-byte stores.  A wave passes its WM x WN accumulator
// tile through its own LDS slab of 16 rows (stride WN + 4 floats) one row of MFMA tiles at a time;
// each lane then reads 8 consecutive columns of a row, splits them into the OUT planes and stores
// 16 bytes per plane (element by element at the ragged right edge).  Only the wave's own lanes
// touch its slab, and LDS instructions of a wave complete in order, so no barrier is needed.
template <int OUT, int TM, int TN>
__device__ inline void store_planes_vec(const KArgs& p, int zb, const v4f (&acc)[TM][TN], int r0, int c0, float* slab) {
    constexpr int WN = TN * 16, SLD = WN + 4, GPR = WN / 8;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const i64 cbase = batch_off(p, zb, p.c_bs, p.c_bs2);
    __bf16* C = (__bf16*)p.C;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) slab[(4 * lk + r) * SLD + j * 16 + li] = acc[i][j][r];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int g = lane; g < 16 * GPR; g += 64) {
            const int row = g / GPR, cg = (g % GPR) * 8;
            const int gm = r0 + i * 16 + row, gn = c0 + cg;
            if (gm < p.M && gn < p.N) {
                float v[8];
                if (p.alpha == 1.0) {   // exact: (float)(1.0 * (double)x) == x
#pragma unroll
                    for (int t = 0; t < 8; ++t) v[t] = slab[row * SLD + cg + t];
                } else {
#pragma unroll
                    for (int t = 0; t < 8; ++t) v[t] = (float)(p.alpha * (double)slab[row * SLD + cg + t]);
                }
                const i64 off = cbase + idx_off(p.rmap, gm) + idx_off(p.cmap, gn);
                if (gn + 8 <= p.N) {
#pragma unroll
                    for (int q = 0; q < OUT; ++q) {
                        v8bf h;
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            h[t] = (__bf16)v[t];
                            v[t] -= (float)h[t];
                        }
                        __builtin_nontemporal_store(h, (v8bf*)(C + q * p.c_ps + off));
                    }
                } else {
                    for (int t = 0; t < 8 && gn + t < p.N; ++t) put_out<OUT>(p.C, off + t, p.c_ps, (double)v[t], 0.0);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_cvoid_t;

// Position (in bf16 elements) of element k of row r in a 64-byte LDS row: the four 16-byte chunks
// of row r are permuted by r / 2 mod 4, which spreads the 16 rows x 4 chunks read by one
// ds_read_b128 of the MFMA fragment loads over all banks (measured on gfx950; a row stride of 80
// or 72 bytes, or the permutation by r mod 4, leaves two-way conflicts).
__device__ inline int lds_pos(int r, int k) { return ((((k >> 3) ^ (r >> 1)) & 3) << 3) | (k & 7); }

template <int NP, int OUT, int BM, int BN, int WGM, int WGN, int TAG>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_split_kernel(KArgs p) {
    constexpr int BK = 32, NW = WGM * WGN;
    constexpr int WM = BM / WGM, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
    constexpr int AI = NP * BM / 16, BI = NP * BN / 16;   // 1 KiB direct-to-LDS loads per stage
    static_assert(TM >= 1 && TN >= 1, "bad tile");
    // two stages in distinct arrays, so that the compiler can tell the stage being filled from the
    // one being read and does not wait for the loads in flight before reading
    __shared__ __attribute__((aligned(16))) __bf16 As0[NP][BM][BK], As1[NP][BM][BK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs0[NP][BN][BK], Bs1[NP][BN][BK];
    // the 16-byte plane epilogue needs a slab of 16 x (WN + 4) floats per wave in As0 and As1
    constexpr bool kVecEpilogue = 16 * (WN + 4) * 4 * ((NW + 1) / 2) <= (int)sizeof(As0);

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

    // Direct-to-LDS loads: one instruction of a wave fills 16 rows x 64 bytes of one plane, lane
    // l writing the 16 bytes at l * 16, i.e. row l / 4, chunk position l % 4, which holds the
    // chunk of logical index (l % 4) ^ (row / 2 mod 4).  Rows beyond M (N) are clamped to the last
    // row (they only feed outputs that are never stored); chunks at or beyond kend load any valid
    // chunk and are zeroed in LDS afterwards (zero_tail).
    const int lr = lane >> 2, lp = lane & 3;
    auto issue = [&](auto& As, auto& Bs, int k0) {
#pragma unroll
        for (int e = 0; e < (AI + NW - 1) / NW; ++e) {
            const int g = wave + NW * e, q = g / (BM / 16), rb = g % (BM / 16);
            if (AI % NW != 0 && g >= AI) break;   // wave-uniform
            const int row = rb * 16 + lr;
            const int gk = k0 + 8 * ((lp ^ (row >> 1)) & 3);
            const __bf16* src = A + q * p.a_ps + (i64)min(m0 + row, p.M - 1) * p.lda + (gk < kend ? gk : kbeg);
            __builtin_amdgcn_global_load_lds((gbl_cvoid_t*)src, (lds_void_t*)&As[q][rb * 16][0], 16, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < (BI + NW - 1) / NW; ++e) {
            const int g = wave + NW * e, q = g / (BN / 16), rb = g % (BN / 16);
            if (BI % NW != 0 && g >= BI) break;   // wave-uniform
            const int row = rb * 16 + lr;
            const int gk = k0 + 8 * ((lp ^ (row >> 1)) & 3);
            const __bf16* src = B + q * p.b_ps + (i64)min(n0 + row, p.N - 1) * p.ldb + (gk < kend ? gk : kbeg);
            __builtin_amdgcn_global_load_lds((gbl_cvoid_t*)src, (lds_void_t*)&Bs[q][rb * 16][0], 16, 0, 0);
        }
    };
    // zero the elements k >= kend of a stage holding the last, partial K tile (after its loads landed)
    auto zero_tail = [&](auto& As, auto& Bs, int k0) {
        const int kv = kend - k0;
        for (int idx = tid; idx < NP * (BM + BN) * BK; idx += 64 * NW) {
            const int k = idx % BK, rr = idx / BK, q = rr / (BM + BN), row = rr % (BM + BN);
            if (k < kv) continue;
            if (row < BM) As[q][row][lds_pos(row, k)] = (__bf16)0.f;
            else Bs[q][row - BM][lds_pos(row - BM, k)] = (__bf16)0.f;
        }
    };
    const int li = lane & 15, lk = lane >> 4;
    auto compute = [&](auto& As, auto& Bs) {
        v8bf a[NP][TM], b[NP][TN];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int r = wm0 + i * 16 + li;
                a[q][i] = *(const v8bf*)&As[q][r][lds_pos(r, 8 * lk)];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int r = wn0 + j * 16 + li;
                b[q][j] = *(const v8bf*)&Bs[q][r][lds_pos(r, 8 * lk)];
            }
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
    };
    // every wave's loads have landed and are visible to the block
    auto landed = [&]() {
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    // K tiles t = 0 .. nt-1; tile t in stage t % 2; the loads of tile t + 1 are in flight while
    // tile t is multiplied
    const int nt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    const bool ragged = (kend - kbeg) % BK != 0;
    if (nt > 0) {
        issue(As0, Bs0, kbeg);
        landed();
        if (nt == 1 && ragged) {
            zero_tail(As0, Bs0, kbeg);
            __syncthreads();
        }
    }
    for (int t = 0; t < nt; t += 2) {
        if (t + 1 < nt) issue(As1, Bs1, kbeg + (t + 1) * BK);
        compute(As0, Bs0);
        landed();
        if (t + 1 >= nt) break;
        if (t + 2 == nt && ragged) {
            zero_tail(As1, Bs1, kbeg + (t + 1) * BK);
            __syncthreads();
        }
        if (t + 2 < nt) issue(As0, Bs0, kbeg + (t + 2) * BK);
        compute(As1, Bs1);
        landed();
        if (t + 3 == nt && ragged) {
            zero_tail(As0, Bs0, kbeg + (t + 2) * BK);
            __syncthreads();
        }
    }

    // epilogue: D row of accumulator register r of lane l is 4 (l / 16) + r, column l % 16
    if constexpr (OUT >= 2 && kVecEpilogue) {
        if (p.vec_out && p.splits == 1) {
            float* slab = (wave < (NW + 1) / 2 ? (float*)&As0[0][0][0] : (float*)&As1[0][0][0]) +
                          (wave % ((NW + 1) / 2)) * 16 * (WN + 4);
            store_planes_vec<OUT>(p, zb, acc, m0 + wm0, n0 + wn0, slab);
            return;
        }
    }
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
// 3 = 256 x 128 (8 waves of 64 x 64), 4 = 64 x 64 as 4 waves of 16 rows x 64 columns (outputs of at
// most 64 columns: every wave covers all of them).  LDS: two stages of NP x (BM + BN) x 64 bytes (at
// most 144 KiB).
template <int NP, int OUT, int TAG>
void launch_split_tile(const KArgs& a, dim3 grid, int tile, hipStream_t s) {
    if (tile == 4)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 64, 64, 4, 1, 0>), grid, dim3(256), 0, s, a);
    else if (tile == 3)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 256, 128, 4, 2, TAG>), grid, dim3(512), 0, s, a);
    else if (tile == 2)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 128, 128, 2, 2, TAG>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 64, 64, 2, 2, 0>), grid, dim3(256), 0, s, a);
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
