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

// K-major operands (stored X[k][m], m contiguous) keep that layout in LDS: K-tile row k holds the R
// values m of the tile, its 16-byte chunks permuted by kswz(k) so that the four rows (at one
// column range) that a transposing fragment read touches, and the four lane groups of a wave, fall
// on different banks.
template <int R>
__device__ inline int kswz_pos(int k, int m) {
    const int sw = (2 * (k & 3) + 8 * ((k >> 3) & 3)) & (R / 8 - 1);
    return k * R + ((((m >> 3) ^ sw) & (R / 8 - 1)) << 3) + (m & 7);
}

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) v4s lds_v4s_t;

// One operand of the contraction (R rows of the block tile, NP planes, KM: K-major storage) in LDS
// as 32-wide K tiles: loads, tail zeroing and MFMA fragment reads.
template <int NP, int R, bool KM>
struct SplitOperand {
    // Direct-to-LDS loads of K tile k0: instruction g of the block fills 1 KiB of one plane, lane l
    // the 16 bytes at l * 16.  K-contiguous: 16 rows x 64 bytes; position l % 4 of row l / 4 holds
    // the chunk of logical index (l % 4) ^ (row / 2 mod 4).  K-major: 1024 / (2 R) K rows of R
    // values; the position holds the chunk kswz_pos puts there.  Rows beyond the operand are
    // clamped to its last row (they only feed outputs that are never stored); chunks beyond kend,
    // and K-major chunks past the row's padded end, load any valid chunk, and kend's tail is zeroed
    // in LDS afterwards.
    // (NW waves; a trip count known at compile time keeps the loads in one unrolled block, free to
    // be scheduled among the MFMAs)
    template <int NW>
    __device__ static void issue(const __bf16* X, i64 ld, i64 ps, int rows, int base, __bf16 (&L)[NP][R * 32],
                                 int k0, int kbeg, int kend, int wave, int lane) {
        constexpr int NI = NP * R / 16;
#pragma unroll
        for (int e = 0; e < (NI + NW - 1) / NW; ++e) {
            const int g = wave + NW * e;
            if (NI % NW != 0 && g >= NI) break;   // wave-uniform
            const int q = g / (R / 16), rb = g % (R / 16);
            const __bf16* src;
            if constexpr (!KM) {
                const int row = rb * 16 + (lane >> 2);
                const int gk = k0 + 8 * (((lane & 3) ^ (row >> 1)) & 3);
                src = X + q * ps + (i64)min(base + row, rows - 1) * ld + (gk < kend ? gk : kbeg);
            } else {
                const int e = rb * 512 + lane * 8, k = e / R;
                const int sw = (2 * (k & 3) + 8 * ((k >> 3) & 3)) & (R / 8 - 1);
                const int m = ((((e % R) >> 3) ^ sw) & (R / 8 - 1)) << 3;
                const int gk = k0 + k;
                const int gm = base + m < ((rows + 7) & ~7) ? base + m : 0;
                src = X + q * ps + (i64)(gk < kend ? gk : kbeg) * ld + gm;
            }
            __builtin_amdgcn_global_load_lds((gbl_cvoid_t*)src, (lds_void_t*)&L[q][rb * 512], 16, 0, 0);
        }
    }
    // zero the K values at or beyond kv of a stage holding a partial K tile
    __device__ static void zero_tail(__bf16 (&L)[NP][R * 32], int kv, int tid, int nthr) {
        for (int idx = tid; idx < NP * R * 32; idx += nthr) {
            const int q = idx / (R * 32), e = idx % (R * 32);
            int k;
            if constexpr (!KM) {
                const int row = e / 32, pk = e % 32;
                k = (((pk >> 3) ^ (row >> 1)) & 3) * 8 + (pk & 7);   // lds_pos is an involution per row
            } else {
                k = e / R;
            }
            if (k >= kv) L[q][e] = (__bf16)0.f;
        }
    }
    // MFMA fragment of plane q for rows rbase .. rbase + 15: lane l holds row rbase + l % 16,
    // K values 8 (l / 16) .. 8 (l / 16) + 7.  K-major: two ds_read_b64_tr_b16, each of which hands
    // lane j of a 16-lane group element j of four consecutive K rows (measured on gfx950: of the
    // 16 lanes' 8-byte chunks, lane j receives element j % 4 of chunks j / 4, j / 4 + 4, ...).
    __device__ static v8bf frag(const __bf16 (&L)[NP][R * 32], int q, int rbase, int lane) {
        const int li = lane & 15, lk = lane >> 4;
        if constexpr (!KM) {
            const int r = rbase + li;
            return *(const v8bf*)&L[q][r * 32 + lds_pos(r, 8 * lk)];
        } else {
            const int m = rbase + 4 * (li & 3);
            const int k0 = 8 * lk + (li >> 2);
            const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s_t*)&L[q][kswz_pos<R>(k0, m)]);
            const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s_t*)&L[q][kswz_pos<R>(k0 + 4, m)]);
            const v8s w = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            return __builtin_bit_cast(v8bf, w);
        }
    }
};

template <int NP, int OUT, int BM, int BN, int WGM, int WGN, int TAG, bool AKM = false, bool BKM = false, int ST = 2>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_split_kernel(KArgs p) {
    constexpr int BK = 32, NW = WGM * WGN;
    constexpr int WM = BM / WGM, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
    static_assert(TM >= 1 && TN >= 1, "bad tile");
    typedef SplitOperand<NP, BM, AKM> OpA;
    typedef SplitOperand<NP, BN, BKM> OpB;
    // ST = 2: two stages in distinct arrays, so that the compiler can tell the stage being filled
    // from the one being read and does not wait for the loads in flight before reading.  ST = 1: one
    // stage (half the LDS, so that two blocks share a compute unit and one block's output stores
    // overlap the other's loads; for short K, where there is little to pipeline)
    static_assert(ST == 1 || ST == 2, "one or two stages");
    __shared__ __attribute__((aligned(16))) __bf16 As0[NP][BM * BK], As1[ST == 2 ? NP : 1][ST == 2 ? BM * BK : 8];
    __shared__ __attribute__((aligned(16))) __bf16 Bs0[NP][BN * BK], Bs1[ST == 2 ? NP : 1][ST == 2 ? BN * BK : 8];
    // the 16-byte plane epilogue needs a slab of 16 x (WN + 4) floats per wave: in As0 and As1 with
    // two stages, in As0 with one
    constexpr bool kVecEpilogue = 16 * (WN + 4) * 4 * (ST == 2 ? (NW + 1) / 2 : NW) <= (int)sizeof(As0);

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

    auto issue = [&](auto& As, auto& Bs, int k0) {
        OpA::template issue<NW>(A, p.lda, p.a_ps, p.M, m0, As, k0, kbeg, kend, wave, lane);
        OpB::template issue<NW>(B, p.ldb, p.b_ps, p.N, n0, Bs, k0, kbeg, kend, wave, lane);
    };
    // zero the elements k >= kend of a stage holding the last, partial K tile (after its loads landed)
    auto zero_tail = [&](auto& As, auto& Bs, int k0) {
        OpA::zero_tail(As, kend - k0, tid, 64 * NW);
        OpB::zero_tail(Bs, kend - k0, tid, 64 * NW);
    };
    const int li = lane & 15, lk = lane >> 4;
    auto compute = [&](auto& As, auto& Bs) {
        v8bf a[NP][TM], b[NP][TN];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
#pragma unroll
            for (int i = 0; i < TM; ++i) a[q][i] = OpA::frag(As, q, wm0 + i * 16, lane);
#pragma unroll
            for (int j = 0; j < TN; ++j) b[q][j] = OpB::frag(Bs, q, wn0 + j * 16, lane);
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

    // K tiles t = 0 .. nt-1; with two stages, tile t is in stage t % 2 and the loads of tile t + 1
    // are in flight while tile t is multiplied
    const int nt = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    const bool ragged = (kend - kbeg) % BK != 0;
    if constexpr (ST == 1) {
        // one stage: load, multiply, and a barrier before the next tile overwrites the stage
        for (int t = 0; t < nt; ++t) {
            issue(As0, Bs0, kbeg + t * BK);
            landed();
            if (t == nt - 1 && ragged) {
                zero_tail(As0, Bs0, kbeg + t * BK);
                __syncthreads();
            }
            compute(As0, Bs0);
            __syncthreads();
        }
    } else {
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
    }

    // epilogue: D row of accumulator register r of lane l is 4 (l / 16) + r, column l % 16
    if constexpr (OUT >= 2 && kVecEpilogue) {
        if (p.vec_out && p.splits == 1) {
            float* slab = ST == 1 ? (float*)&As0[0][0] + wave * 16 * (WN + 4)
                                  : (wave < (NW + 1) / 2 ? (float*)&As0[0][0] : (float*)&As1[0][0]) +
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

// ------------------------------------------------------------------------------------------
// 256 x 256 tiles on v_mfma_f32_32x32x16_bf16 with K tiles of 16 and three LDS stages (tile code 6;
// K-contiguous operands, K a multiple of 16).  Three bf16 planes of a 256 x 256 block tile at BK = 16
// take 48 KiB per stage, so that three stages fit in 144 KiB and a K tile's loads are issued two tiles
// before it is multiplied (the 256 x 128 tile at BK = 32 on the 16 x 16 MFMA has room for two stages
// only), and each operand row loaded feeds twice the outputs of the 256 x 128 tile's B rows.
// Operand layout in LDS: row r of plane q holds the tile's 16 K values (32 bytes) as two 16-byte
// chunks, chunk c at position c ^ ((r >> 3) & 1), so that the 16 rows read by a 16-lane group of a
// fragment load cover all 256 bytes of the banks once.  Fragment of a 32-row block for lane l: row
// l % 32, the 8 K values of chunk l / 32 (A and B use the same K assignment, so the dot products are
// those of the contraction).  Accumulator register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.
// ------------------------------------------------------------------------------------------
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ inline int s32_pos(int r, int c) { return r * 16 + ((c ^ ((r >> 3) & 1)) << 3); }

// s_waitcnt immediate: at most n vector-memory operations of this wave still in flight, no wait on
// the other counters
template <int N>
__device__ inline void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int NP, int R>
struct Split32Operand {
    static constexpr int NI = NP * R / 32;   // 1 KiB direct-to-LDS loads per K tile
    static_assert(NI >= 8, "at least one load per wave");
    // loads of K tile k0: instruction g of the block fills 1 KiB of one plane (32 rows x 32 bytes),
    // lane l the chunk at LDS position l; rows beyond the operand are clamped to its last row (they
    // only feed outputs that are never stored) and chunks at or beyond kend load the chunk at kbeg
    // (every wave issues the same number, PW: where NW does not divide NI, the waves past the end
    // repeat their previous load, the same 16 bytes to the same place, so that the count of loads in
    // flight is the same in every wave)
    template <int NW>
    static constexpr int PW = (NI + NW - 1) / NW;
    template <int NW>
    __device__ static void issue(const __bf16* X, i64 ld, i64 ps, int rows, int base, __bf16 (&L)[NP][R * 16],
                                 int k0, int kbeg, int kend, int wave, int lane) {
#pragma unroll
        for (int e = 0; e < PW<NW>; ++e) {
            const int g = wave + NW * e < NI ? wave + NW * e : wave + NW * (e - 1);
            const int q = g / (R / 32), rb = g % (R / 32);
            const int row = rb * 32 + (lane >> 1);
            const int c = (lane & 1) ^ ((row >> 3) & 1);
            const int gk = k0 + 8 * c;
            const __bf16* src = X + q * ps + (i64)min(base + row, rows - 1) * ld + (gk < kend ? gk : kbeg);
            __builtin_amdgcn_global_load_lds((gbl_cvoid_t*)src, (lds_void_t*)&L[q][rb * 512], 16, 0, 0);
        }
    }
    __device__ static v8bf frag(const __bf16 (&L)[NP][R * 16], int q, int rbase, int lane) {
        const int r = rbase + (lane & 31);
        return *(const v8bf*)&L[q][s32_pos(r, lane >> 5)];
    }
};

template <int NP, int OUT, int TAG>
__global__ __launch_bounds__(512) void gemm_split32_kernel(KArgs p) {
    constexpr int BM = 256, BN = 256, BK = 16, ST = 3, NW = 8, WGM = 2, WGN = 4;
    constexpr int WM = BM / WGM, WN = BN / WGN, TM = WM / 32, TN = WN / 32;
    typedef Split32Operand<NP, BM> OpA;
    typedef Split32Operand<NP, BN> OpB;
    // one LDS variable per stage (both operands), so that the compiler's alias analysis tells the
    // stage being filled from the one being read and inserts no wait for the loads in flight before
    // the fragment reads (it tracks the direct-to-LDS writes of a few distinct variables only)
    struct Stage {
        __bf16 a[NP][BM * BK];
        __bf16 b[NP][BN * BK];
    };
    __shared__ __attribute__((aligned(16))) Stage S0, S1, S2;

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

    // an (empty) use of an accumulation register makes the compiler keep the MFMA accumulators in
    // the AGPR half of the register file, apart from the fragments and addresses
    asm volatile("" ::: "a0");
    v16f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    auto stage = [&](auto I) -> Stage& {
        constexpr int s = decltype(I)::value;
        if constexpr (s == 0) return S0;
        else if constexpr (s == 1) return S1;
        else return S2;
    };
    auto stA = [&](auto I) -> auto& { return stage(I).a; };
    auto stB = [&](auto I) -> auto& { return stage(I).b; };
    auto issue = [&](auto& As, auto& Bs, int k0) {
        OpA::template issue<NW>(A, p.lda, p.a_ps, p.M, m0, As, k0, kbeg, kend, wave, lane);
        OpB::template issue<NW>(B, p.ldb, p.b_ps, p.N, n0, Bs, k0, kbeg, kend, wave, lane);
    };
    // fragments of a stage, and the MFMAs on them
    struct Frags {
        v8bf a[NP][TM], b[NP][TN];
    };
    auto read = [&](auto& As, auto& Bs, Frags& f) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
#pragma unroll
            for (int j = 0; j < TN; ++j) f.b[q][j] = OpB::frag(Bs, q, wn0 + j * 32, lane);
#pragma unroll
            for (int i = 0; i < TM; ++i) f.a[q][i] = OpA::frag(As, q, wm0 + i * 32, lane);
        }
    };
    auto multiply = [&](const Frags& f) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (NP == 2) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[1][i], f.b[0][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0][i], f.b[1][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0][i], f.b[0][j], acc[i][j], 0, 0, 0);
                } else {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[2][i], f.b[0][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[1][i], f.b[1][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0][i], f.b[2][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[1][i], f.b[0][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0][i], f.b[1][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0][i], f.b[0][j], acc[i][j], 0, 0, 0);
                }
            }
    };
    // Tile t is in stage t % 3.  Step t waits until only the loads of tile t + 1 are in flight (and for
    // its LDS reads); the barrier then makes every wave's loads of tile t visible, and every wave has
    // finished tile t - 1, whose stage takes the loads of tile t + 2; then the fragments of tile t are
    // read and multiplied.  s_barrier goes through inline assembly with a memory clobber:
    // __syncthreads would also wait for the loads of tile t + 1.
    // The loop runs whole groups of three steps, and every step issues its loads and reads its stage;
    // steps past the last tile skip only the multiply, and their loads (K at or beyond the chunk end:
    // the chunk's first K values, by issue's rule) go to stages that are not multiplied.  Every path
    // through the loop then issues the same loads in the same order, which is what the compiler's own
    // wait analysis needs to agree that the wait suffices (it cannot follow conditions on the tile
    // count, and would otherwise wait for every load in flight before each fragment read); and the
    // loop has a single exit, which keeps the accumulators in place (with several exits the compiler
    // copies them between register halves on every trip).  Every wave issues LPW loads per tile.
    // Chunks are whole K tiles: the host admits this tile for K a multiple of 16 only.
    constexpr int LPW = OpA::template PW<NW> + OpB::template PW<NW>;
    static_assert(LPW < 16, "vmcnt range");
    const int nt = kend > kbeg ? (kend - kbeg) / BK : 0;
    auto step = [&](auto I, int t) {
        constexpr int s = decltype(I)::value;
        __builtin_amdgcn_sched_barrier(0);
        wait_vm<LPW>();
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        // the next loads go out first (a scheduling barrier keeps them ahead of the MFMAs)
        constexpr int sn = (s + 2) % 3;
        issue(stA(std::integral_constant<int, sn>()), stB(std::integral_constant<int, sn>()), kbeg + (t + 2) * BK);
        __builtin_amdgcn_sched_barrier(0);
        Frags f;
        read(stA(I), stB(I), f);
        if (t < nt) multiply(f);   // block-uniform
    };
    if (nt > 0) {   // block-uniform; an empty K chunk leaves the accumulators at zero
        issue(S0.a, S0.b, kbeg);
        issue(S1.a, S1.b, kbeg + BK);
        for (int t = 0; t < nt; t += 3) {
            step(std::integral_constant<int, 0>(), t);
            step(std::integral_constant<int, 1>(), t + 1);
            step(std::integral_constant<int, 2>(), t + 2);
        }
    }
    __syncthreads();   // all loads have landed and every wave is done with the stages before they hold epilogue slabs

    const int lc = lane & 31, lg = lane >> 5;
    if constexpr (OUT >= 2) {
        if (p.vec_out && p.splits == 1) {
            // per wave an LDS slab of 16 rows x (WN + 4) floats (four waves per stage); the 32 rows of
            // an MFMA tile go through it in two halves, registers 8 h .. 8 h + 7 holding rows 16 h .. 16 h + 15
            constexpr int SLD = WN + 4, GPR = WN / 8;
            static_assert(4 * 16 * SLD * 4 <= (int)sizeof(Stage), "four slabs per stage");
            float* const slab = (wave < 4 ? (float*)&S0 : (float*)&S1) + (wave & 3) * 16 * SLD;
            const i64 cbase = batch_off(p, zb, p.c_bs, p.c_bs2);
            __bf16* C = (__bf16*)p.C;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int r = 8 * h; r < 8 * h + 8; ++r)
                            slab[(8 * ((r >> 2) - 2 * h) + 4 * lg + (r & 3)) * SLD + j * 32 + lc] = acc[i][j][r];
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int gi = lane; gi < 16 * GPR; gi += 64) {
                        const int row = gi / GPR, cg = (gi % GPR) * 8;
                        const int gm = m0 + wm0 + i * 32 + 16 * h + row, gn = n0 + wn0 + cg;
                        if (gm < p.M && gn < p.N) {
                            float v[8];
#pragma unroll
                            for (int t = 0; t < 8; ++t) {
                                const float x = slab[row * SLD + cg + t];
                                v[t] = p.alpha == 1.0 ? x : (float)(p.alpha * (double)x);
                            }
                            const i64 off = cbase + idx_off(p.rmap, gm) + idx_off(p.cmap, gn);
                            if (gn + 8 <= p.N) {
#pragma unroll
                                for (int q = 0; q < OUT; ++q) {
                                    v8bf hv;
#pragma unroll
                                    for (int t = 0; t < 8; ++t) {
                                        hv[t] = (__bf16)v[t];
                                        v[t] -= (float)hv[t];
                                    }
                                    __builtin_nontemporal_store(hv, (v8bf*)(C + q * p.c_ps + off));
                                }
                            } else {
                                for (int t = 0; t < 8 && gn + t < p.N; ++t) put_out<OUT>(p.C, off + t, p.c_ps, (double)v[t], 0.0);
                            }
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
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
                for (int r = 0; r < 16; ++r) {
                    const int gm = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * lg + (r & 3), gn = n0 + wn0 + j * 32 + lc;
                    if (gm < p.M && gn < p.N) W[(i64)gm * p.N + gn] = acc[i][j][r];
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int gm = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * lg + (r & 3), gn = n0 + wn0 + j * 32 + lc;
                if (gm < p.M && gn < p.N) write_elem<OUT>(p, zb, gm, gn, p.alpha * (double)acc[i][j][r]);
            }
}

// Tile shapes: 1 = 64 x 64 (4 waves of 32 x 32), 2 = 128 x 128 (4 waves of 64 x 64),
// 3 = 256 x 128 (8 waves of 64 x 64), 4 = 64 x 64 as 4 waves of 16 rows x 64 columns (outputs of at
// most 64 columns: every wave covers all of them), 5 = tile 2 with a single LDS stage (short K).
// LDS: two stages of NP x (BM + BN) x 64 bytes (at most 144 KiB), one for tile 5.
template <int NP, int OUT, int TAG, bool AKM, bool BKM>
void launch_split_tile(const KArgs& a, dim3 grid, int tile, hipStream_t s) {
    if (tile == 6) {
        DTRG_REQUIRE(!AKM && !BKM, DTRG_EINVAL, "split contraction: tile 6 takes K-contiguous operands only");
        if constexpr (!AKM && !BKM) hipLaunchKernelGGL((gemm_split32_kernel<NP, OUT, TAG>), grid, dim3(512), 0, s, a);
        return;
    }
    if (tile == 5)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 128, 128, 2, 2, 0, AKM, BKM, 1>), grid, dim3(256), 0, s, a);
    else if (tile == 4)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 64, 64, 4, 1, 0, AKM, BKM>), grid, dim3(256), 0, s, a);
    else if (tile == 3)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 256, 128, 4, 2, TAG, AKM, BKM>), grid, dim3(512), 0, s, a);
    else if (tile == 2)
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 128, 128, 2, 2, TAG, AKM, BKM>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((gemm_split_kernel<NP, OUT, 64, 64, 2, 2, 0, AKM, BKM>), grid, dim3(256), 0, s, a);
}

// tags 7, 8, 9 (the three chi^7 contractions) get their own symbols on the large tiles only
template <int NP, int OUT, bool AKM = false, bool BKM = false>
void launch_split_tag(const KArgs& a, dim3 grid, int tile, int tag, hipStream_t s) {
    if ((tile == 2 || tile == 3 || tile == 6) && tag == 7) { launch_split_tile<NP, OUT, 7, AKM, BKM>(a, grid, tile, s); return; }
    if ((tile == 2 || tile == 3 || tile == 6) && tag == 8) { launch_split_tile<NP, OUT, 8, AKM, BKM>(a, grid, tile, s); return; }
    if ((tile == 2 || tile == 3 || tile == 6) && tag == 9) { launch_split_tile<NP, OUT, 9, AKM, BKM>(a, grid, tile, s); return; }
    launch_split_tile<NP, OUT, 0, AKM, BKM>(a, grid, tile, s);
}

// operand layouts: K-major operands only with FP64 or FP32 outputs (the contractions that read a
// chi^5 intermediate in its producer's layout all write FP64)
template <int NP>
void launch_split_np(const KArgs& a, dim3 grid, int out, int tile, int tag, bool akm, bool bkm, hipStream_t s) {
    if (!akm && !bkm) {
        if (out == 0) launch_split_tag<NP, 0>(a, grid, tile, tag, s);
        else if (out == 1) launch_split_tag<NP, 1>(a, grid, tile, tag, s);
        else launch_split_tag<NP, NP>(a, grid, tile, tag, s);
        return;
    }
    DTRG_REQUIRE(out == 0 || out == 1, DTRG_EINVAL, "split contraction: K-major operands need an FP64 or FP32 output");
    if (akm && bkm) {
        if (out == 0) launch_split_tag<NP, 0, true, true>(a, grid, tile, tag, s);
        else launch_split_tag<NP, 1, true, true>(a, grid, tile, tag, s);
    } else if (akm) {
        if (out == 0) launch_split_tag<NP, 0, true, false>(a, grid, tile, tag, s);
        else launch_split_tag<NP, 1, true, false>(a, grid, tile, tag, s);
    } else {
        if (out == 0) launch_split_tag<NP, 0, false, true>(a, grid, tile, tag, s);
        else launch_split_tag<NP, 1, false, true>(a, grid, tile, tag, s);
    }
}

}  // namespace dtrg
