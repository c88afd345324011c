// Shared host/device definitions of the dtrg library (HIP, gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/dtrg.h"

namespace dtrg {

typedef long long i64;

struct Error : std::runtime_error {
    dtrg_status code;
    Error(dtrg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DTRG_HIP(expr)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::dtrg::Error(DTRG_EHIP, std::string(#expr) + " failed: " +            \
                                               hipGetErrorString(e_));                    \
    } while (0)

#define DTRG_REQUIRE(cond, code, msg)                                                     \
    do {                                                                                  \
        if (!(cond)) throw ::dtrg::Error(code, msg);                                      \
    } while (0)

// The device allocator that DevBuf::alloc uses on this thread: a caller's callbacks (set for the
// duration of an entry point by AllocScope), or hipMalloc / hipFree when there is none.
struct Allocator {
    dtrg_alloc_fn alloc_fn = nullptr;
    dtrg_free_fn free_fn = nullptr;
    void* user = nullptr;
    hipStream_t stream = nullptr;   // stream of the call that allocates
};
inline const Allocator*& current_allocator() {
    static thread_local const Allocator* a = nullptr;
    return a;
}
struct AllocScope {
    const Allocator* prev;
    explicit AllocScope(const Allocator* a) : prev(current_allocator()) { current_allocator() = a; }
    ~AllocScope() { current_allocator() = prev; }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
};

// Owning device buffer (the thread's current allocator, else hipMalloc / hipFree).  A buffer
// holding nb instances of a tensor keeps the instance stride bs (elements): instance i starts at
// p + i * bs.  A buffer from a caller's allocator remembers its release function.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    i64 bs = 0;
    dtrg_free_fn ff = nullptr;   // release callback (nullptr: hipFree)
    void* fu = nullptr;
    hipStream_t fs = nullptr;
    bool borrowed = false;       // a view of memory the buffer does not own: never freed or grown
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { take(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); take(o); }
        return *this;
    }
    ~DevBuf() { release(); }
    void take(DevBuf& o) {
        p = o.p; n = o.n; bs = o.bs; ff = o.ff; fu = o.fu; fs = o.fs; borrowed = o.borrowed;
        o.p = nullptr; o.n = 0; o.bs = 0; o.ff = nullptr; o.fu = nullptr; o.fs = nullptr; o.borrowed = false;
    }
    // view `count` elements at ptr (memory owned elsewhere)
    void borrow(T* ptr, size_t count) {
        release();
        p = ptr;
        n = count;
        borrowed = true;
    }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        const size_t bytes = count * sizeof(T);
        const Allocator* A = current_allocator();
        if (A && A->alloc_fn) {
            void* q = A->alloc_fn(bytes, (void*)A->stream, A->user);
            if (!q) throw Error(DTRG_ENOMEM, "alloc_fn returned NULL for " + std::to_string(bytes) + " bytes");
            if ((uintptr_t)q % 256 != 0) {
                A->free_fn(q, bytes, (void*)A->stream, A->user);
                throw Error(DTRG_EINVAL, "alloc_fn returned memory not aligned to 256 bytes");
            }
            p = (T*)q;
            ff = A->free_fn; fu = A->user; fs = A->stream;
        } else {
            hipError_t e = hipMalloc((void**)&p, bytes);
            if (e != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw Error(DTRG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                             hipGetErrorString(e));
            }
        }
        n = count;
    }
    // nb instances of `per` elements each
    void alloc_inst(int nb, i64 per) {
        alloc((size_t)nb * (size_t)per);
        bs = per;
    }
    void ensure(size_t count) {
        if (count <= n) return;
        if (borrowed) throw Error(DTRG_ENOMEM, "borrowed buffer of " + std::to_string(n * sizeof(T)) +
                                                   " bytes is too small (" + std::to_string(count * sizeof(T)) +
                                                   " needed)");
        alloc(count);
    }
    void release() {
        if (p && !borrowed) {
            if (ff) {
                // a caller's allocator may hand the block out again at once: wait for the device
                // (hipFree waits the same way)
                (void)hipDeviceSynchronize();
                ff(p, n * sizeof(T), (void*)fs, fu);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        n = 0;
        bs = 0;
        ff = nullptr;
        fu = nullptr;
        fs = nullptr;
        borrowed = false;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Two-level index map used by the GEMM epilogue: offset(i) = (i / div) * s1 + (i % div) * s0.
struct IdxMap {
    i64 div = 1LL << 62;
    i64 s1 = 0;
    i64 s0 = 1;
    static IdxMap linear(i64 stride) { IdxMap m; m.div = 1LL << 62; m.s1 = 0; m.s0 = stride; return m; }
    static IdxMap split(i64 div, i64 s1, i64 s0) { IdxMap m; m.div = div; m.s1 = s1; m.s0 = s0; return m; }
};

__host__ __device__ inline i64 idx_off(const IdxMap& m, i64 i) {
    if (i < m.div) return i * m.s0;   // every index of a linear map; the first block of a split one
    if (m.div <= 0xffffffffLL && i <= 0xffffffffLL) {
        // 32-bit division (a 64-bit one is a long instruction sequence on the GPU)
        const unsigned q = (unsigned)i / (unsigned)m.div, r = (unsigned)i - q * (unsigned)m.div;
        return (i64)q * m.s1 + (i64)r * m.s0;
    }
    return (i / m.div) * m.s1 + (i % m.div) * m.s0;
}

// Arithmetic of a contraction, which is also the storage format of its operands: FP64, FP32, or
// FP32 values carried as 2 (BF16X3: three bf16 products) or 3 (BF16X6: six products) bf16 planes.
enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2, BF16X6 = 3 };
// Output format of a contraction: FP64, FP32, or the contraction's own bf16 planes.
enum class Out { F64 = 0, F32 = 1, Split = 2 };
int prec_planes(Prec p);   // 1, or the number of bf16 planes

// Tile configuration of one contraction: tile 0 = automatic, 1 = 64 x 64, 2 = 128 x 128,
// 3 = 256 x 128, 4 = 64 x 64 on waves of 16 full-width rows (3 and 4: bf16 planes only);
// splits 0 = automatic split-K.
struct GemmCfg {
    int tile = 0;
    int splits = 0;
};
inline int tile_rows(int tile) { return (tile == 3 || tile == 6) ? 256 : ((tile == 2 || tile == 5) ? 128 : 64); }
inline int tile_cols(int tile) { return tile == 6 ? 256 : ((tile == 2 || tile == 3 || tile == 5) ? 128 : 64); }

// One (batched) contraction C[z](r, c) = alpha * sum_k A[z](r, k) B[z](c, k) + beta * C[z](r, c).
//   A stored as [M][K] (a_kmajor = false: A[m * lda + k]) or [K][M] (a_kmajor = true: A[k * lda + m]).
//   B stored as [N][K] (b_kmajor = false: B[n * ldb + k]) or [K][N] (b_kmajor = true: B[k * ldb + n]).
//   Two batch levels: z = (z2, z1), z1 < batch, z2 < batch2 (the problem instance); operand X of
//   batch element z starts at X + z1 * x_bs + z2 * x_bs2.
//   C element (z, r, c) lives at C + z1 * c_bs + z2 * c_bs2 + idx_off(rmap, r) + idx_off(cmap, c).
//   bf16-plane operands and outputs: plane q at base + q * (a_ps, b_ps, c_ps); such operands are
//   K-contiguous with rows padded to a multiple of 8 elements.
struct GemmOp {
    int M = 0, N = 0, K = 0, batch = 1, batch2 = 1;
    const void* A = nullptr; i64 lda = 0, a_bs = 0, a_bs2 = 0, a_ps = 0; bool a_kmajor = false;
    const void* B = nullptr; i64 ldb = 0, b_bs = 0, b_bs2 = 0, b_ps = 0; bool b_kmajor = false;
    void* C = nullptr; i64 c_bs = 0, c_bs2 = 0, c_ps = 0;
    IdxMap rmap, cmap;
    double alpha = 1.0, beta = 0.0;
    GemmCfg cfg;
    // element capacities of the buffers behind A, B, C (-1: unchecked); checked on the host
    // against the largest offset the kernel can touch before anything is launched
    i64 a_cap = -1, b_cap = -1, c_cap = -1;
    // longest FP32 accumulation chain (products per output and K chunk) of the FP32 and bf16-plane
    // formats; longer K is split and the partials are summed in FP64
    int max_chain = 4096;
    // Symmetric outputs (FP64 contractions only; beta = 0), which are computed on half their rows:
    //   sym = 1: C(r, c) = C(c, r) (M == N).  Only the tiles on or below the diagonal are computed,
    //            and every tile below it also writes its mirror image.
    //   sym = 2: C(r, c) = C(r~, c~), where r = r1 rdig + r0 has r~ = r0 rdig + r1 and
    //            c = c1 cdig + c0 has c~ = c0 cdig + c1 (N == cdig^2).  Only the rows with r1 >= r0
    //            are computed: M = rdig (rdig + 1) / 2, packed row p standing for the row with
    //            p = r1 (r1 + 1) / 2 + r0, read from A and written to C as that row, and every packed
    //            row with r1 > r0 also writes the mirrored row.
    int sym = 0, rdig = 0, cdig = 0;
    int tag = 0;   // own kernel symbol for the chi^7 contractions: 7 the join of the two copies
                   // (forward and its backward recompute; timed when profiling), 8 its adjoint
                   // with respect to the upper copy's product P, 9 with respect to the lower copy;
                   // 10: the products with the step's Gram (timed when profiling scheme (b))
};

// Scratch owned by a plan, grown on demand (not shrunk) and reused by every contraction.
struct Scratch {
    DevBuf<double> splitk;   // split-K partials (FP64 or reinterpreted FP32)
    DevBuf<double> red;      // reduction partials
};

// gemm.hip
// Tile configuration gemm() would pick for op (after the automatic choices are resolved).
GemmCfg gemm_resolve(Prec in_prec, const GemmOp& op);
// smallest split-K count that keeps every FP32 accumulation chain of the contraction short (1 for
// FP64 and short K); gemm_resolve never picks fewer, and the autotuner tries no fewer
int gemm_chain_splits(Prec prec, const GemmOp& op);
// Split-K workspace (doubles) gemm() needs for op (0 when it runs as one K chunk).
i64 gemm_workspace(Prec prec, const GemmOp& op);
// Largest element offset (plus one) the epilogue of op can write, over all batch elements.
i64 gemm_c_extent(const GemmOp& op);
void gemm(Prec prec, Out out, const GemmOp& op, hipStream_t s, Scratch& ws);

// tensor_ops.hip
// Batched helpers: instance i < nb of a buffer p with instance stride bs starts at p + i * bs;
// per-instance device scalars x_dev with stride x_bs are read at x_dev + i * x_bs.
struct PermDesc {
    int rank = 0;
    i64 in_dims[6];
    int perm[6];
    int nb = 1;                      // instances
    i64 in_bs = 0, out_bs = 0;       // instance strides (elements)
    int out_inner = 0;               // output rows = the last out_inner output dims (0: dense output)
    i64 out_ld = 0;                  // output row stride (elements) when out_inner > 0
    i64 out_ps = 0;                  // plane stride of bf16-plane outputs
    i64 in_cap = -1, out_cap = -1;   // element capacities (-1: unchecked)
};
// out = alpha * (scale_dev[i * scale_bs] if scale_dev) * transpose(in, perm) + beta * out
// (numpy transpose semantics, per instance)
void permute(const double* in, double* out, const PermDesc& d, double alpha, double beta,
             const double* scale_dev, i64 scale_bs, hipStream_t s);
// the same (beta = 0) written as out_code 0 double, 1 float, 2 / 3 bf16 planes (the value rounded
// to FP32, plane q the bf16 rounding of what the planes before it leave), rows padded per d
void permute_out(const double* in, void* out, int out_code, const PermDesc& d, double alpha, const double* scale_dev,
                 i64 scale_bs, hipStream_t s);
// planes of an FP32 matrix, K-contiguous: out[q][r][k] from in(r, k) (in[r * ld_in + k], or
// in[k * ld_in + r] if kmajor), rows r < rows, k < cols, row stride ld_out, plane stride ps
void split_matrix(const float* in, i64 ld_in, bool kmajor, int rows, int cols, void* out, i64 ld_out, i64 ps, int np,
                  hipStream_t s);
void convert_f64_to_f32(const double* in, i64 in_bs, float* out, i64 out_bs, i64 n, int nb, hipStream_t s);
void fill(double* p, i64 bs, i64 n, int nb, double v, hipStream_t s);
// y += a * x
void axpy(const double* x, double* y, i64 bs, i64 n, int nb, double a, hipStream_t s, const double* sc = nullptr,
          i64 sc_bs = 0);
// p *= alpha * (scale_dev[i * scale_bs], or its reciprocal)
void scale_inplace(double* p, i64 bs, i64 n, int nb, double alpha, const double* scale_dev, i64 scale_bs,
                   bool reciprocal, hipStream_t s);
// out_dev[i * out_bs] = sqrt(sum x_i^2) (deterministic two-pass reduction)
void norm2(const double* x, i64 bs, i64 n, int nb, double* out_dev, i64 out_bs, hipStream_t s, Scratch& ws);
void dot(const double* x, const double* y, i64 bs, i64 n, int nb, double* out_dev, i64 out_bs, hipStream_t s,
         Scratch& ws);
// out = sum_{x,y} T[x][x][y][y]  for T of shape [X][X][Y][Y]
void trace_xxyy(const double* T, i64 bs, int X, int Y, int nb, double* out_dev, i64 out_bs, hipStream_t s);
// G (n x n, ld n) <- (G + G^T) / (2 t), with t = trace(G) written to t_dev first; flag_dev[i] bit 0
// if t is not positive and finite
void sym_normalise(double* G, i64 bs, int n, int nb, double* t_dev, i64 t_bs, int* flag_dev, hipStream_t s);
// L += weight * log(x); inv = 1 / x (if inv_dev); flag_dev[i] bit 0 if x is not positive, bit 2
// if it is not finite (per instance, scalars at stride sc_bs)
void accum_log(const double* x_dev, double weight, double* L_dev, double* inv_dev, i64 sc_bs, int nb, int* flag_dev,
               hipStream_t s);
void fill_int(int* p, i64 n, int v, hipStream_t s);
// seed of the backward: T[x][x][y][y] = gbar * weight / tr, zero elsewhere
void seed_trace_grad(double* T, i64 bs, int X, int Y, int nb, double gbar_weight, const double* tr_dev, i64 tr_bs,
                     hipStream_t s);
// pseudo-random fill in [-1, 1) from a counter-based hash (stream seed ^ instance)
void hash_fill(double* p, i64 bs, i64 n, int nb, uint64_t seed, hipStream_t s);
// copy a rows x cols block between row-major matrices with leading dimensions
void copy2d(const double* src, i64 lds, i64 src_bs, double* dst, i64 ldd, i64 dst_bs, int rows, int cols, int nb,
            hipStream_t s);
// dst + i * dst_bs <- src + idx[i] * src_bs (len elements; gather) or the reverse (scatter)
void gather_rows(const double* src, i64 src_bs, const int* idx_dev, double* dst, i64 dst_bs, i64 len, int nb,
                 bool scatter, hipStream_t s);
// flag_dev[i] |= bit where max_{j < k} v[i * v_bs + j] > thr (or is not finite); mx_dev[i * mx_bs] = that max
void max_check(const double* v, i64 v_bs, int k, int nb, double thr, double* mx_dev, i64 mx_bs, int* flag_dev,
               int bit, hipStream_t s);

// chain.hip (scheme (b): closing the infinite chain of cells)
// largest transfer matrix the closing kernel takes, its residual bound, and the squarings of E
constexpr int kChainMaxK = 2048;
// largest chi of a scheme (b) plan
constexpr int kChainMaxChi = 512;
constexpr double kChainResidual = 1e-8;
constexpr int kChainSquarings = 24;
// E[l][r] = scale * sum_u T[l][r][u][u] for T [K][K][Y][Y] (scale from scale_dev[i * sc_bs], or 1)
void chain_transfer(const double* T, i64 tbs, int K, int Y, const double* scale_dev, i64 sc_bs, double* E, i64 ebs,
                    int nb, hipStream_t s);
// P /= max |P|; flag_dev[i] |= bit if that maximum is zero or not finite
void chain_normalise(double* P, i64 bs, i64 n, int nb, int* flag_dev, int bit, hipStream_t s);
// lambda (to lam_dev), r (unit norm) and l (l^T r = 1) into lr [r | l] from E and its converged
// normalised power P (both K x K, instance strides ebs, pbs); flag_dev[i] |= bit if lambda is not
// positive or either eigenvector residual exceeds kChainResidual relative
void chain_dominant_finish(const double* E, i64 ebs, const double* P, i64 pbs, int K, int nb, double* lr, i64 lrbs,
                           double* lam_dev, i64 sc_bs, int* flag_dev, int bit, hipStream_t s);
// p[i][j] = (i == j) for a rows x cols row-major block per instance
void eye(double* p, i64 bs, int rows, int cols, int nb, hipStream_t s);
// trace of the Gram G = sum_{j,k} A_jk (x) B_jk of the doubled bond, from the half-environments
// A, B ([X][X][Y][Y], instance strides a_bs, b_bs) into t_dev; flag_dev[i] |= 1 if it is not
// positive or not finite
void kron_trace(const double* A, i64 a_bs, const double* B, i64 b_bs, int X, int Y, int nb, double* t_dev, i64 t_bs,
                int* flag_dev, hipStream_t s);
// backward seed: T[y][z][a][b] = delta(y, z) gw l[a] r[b] / lambda
void chain_seed(double* T, i64 bs, int K, int Y, const double* lr, i64 lrbs, double gw, const double* lam_dev,
                i64 sc_bs, int nb, hipStream_t s);
// out = L + w ln lambda (per instance)
void chain_lnZ_at(const double* L_dev, const double* lam_dev, double w, double* out_dev, i64 sc_bs, int nb,
                  hipStream_t s);

// eig.hip
// Full symmetric eigendecomposition of an n x n matrix (n <= kJacobiMax) by parallel cyclic
// Jacobi, one workgroup per instance: eigenvalues descending into lam_dev[0..n), eigenvectors as
// the columns of V (row-major, leading dimension ldv).  flag_dev (nullable): flag_dev[i] |= flag_bit
// when instance i still rotated in its last allowed sweep.  Off-diagonal entries below
// floor_rel |A|_F are left in place.
constexpr int kJacobiMax = 96;
void jacobi_eig(const double* A, int n, int lda, i64 a_bs, double* lam_dev, i64 lam_bs, double* V, int ldv, i64 v_bs,
                int nb, int max_sweeps, int* sweeps_dev, hipStream_t s, int* flag_dev = nullptr, int flag_bit = 0,
                double floor_rel = 0x1p-60);
// Upper-triangular R^{-1} of the Cholesky factor of (S + shift * I), S b x b (ld b); the
// shift is shift_rel * trace(S).  flag_dev[i] |= 2 on a non-positive pivot.  near_dev (nullable):
// near_dev[i] = 1 if every entry of S_i is within near_tol of the identity's, else 0.  skip_dev
// (nullable): instances with skip_dev[i] != 0 get R^{-1} = I without a factorisation.
void chol_inverse(const double* S, i64 s_bs, int b, double shift_rel, double* Rinv, i64 r_bs, int nb, int* flag_dev,
                  hipStream_t s, const int* skip_dev = nullptr, int* near_dev = nullptr, double near_tol = 0.0);
// norms of the b columns of V (n x b, ld ldv) -> out[0..b)
void col_norms(const double* V, int n, int b, int ldv, i64 v_bs, double* out_dev, i64 out_bs, int nb, hipStream_t s);
// V[:, j] /= nrm[j] where nrm[j] > tiny * max(nrm); other columns replaced by hash noise
void col_normalise(double* V, int n, int b, int ldv, i64 v_bs, const double* nrm_dev, i64 nrm_bs, int nb,
                   uint64_t seed, hipStream_t s);
// res[j] = |Y[:, j] - theta[j] V[:, j]| for j < k
void ritz_residuals(const double* V, const double* Y, int n, int k, int ld, i64 v_bs, const double* theta_dev,
                    i64 th_bs, double* res_dev, i64 res_bs, int nb, hipStream_t s);
// S = [[0, R], [R^T, 0]] (2K x 2K, row-major) from R (K x K): its eigenpairs are +-sigma_j with vectors
// (u_j, +-v_j) / sqrt 2 for the singular triplets of R
void sym_augment(const double* R, i64 r_bs, int K, double* S, i64 s_bs, int nb, hipStream_t s);
// S[i][j] = F(lam_j - lam_i) * (Om[i][j] - Om[j][i]) / 2 on the k x k kept block (F_ii = 0),
// F(d) = d / (d^2 + eps)
void kept_block_adjoint(const double* Om, i64 om_bs, const double* lam_dev, i64 lam_bs, int k, double eps, double* S,
                        i64 s_bs, int nb, hipStream_t s);
// M[i][j] = F(lam_j - theta_i) * Om[i][j] / 2 for i < p, j < k, theta = lam + k
void over_block_adjoint(const double* Om, i64 om_bs, const double* lam_dev, i64 lam_bs, int p, int k, double eps,
                        double* M, i64 m_bs, int nb, hipStream_t s);
// Chebyshev three-term step on n x k blocks (all with instance stride bs), interval [lo, hi] of
// instance i at lohi_dev[i * lohi_bs + {0, 1}]:
//   Vn = a * (2 * Y - (hi + lo) * Vc) - Vp (a = 2 / (hi - lo), or half that for the first step with Vp = 0)
//   X += coef[j] * Vn[:, j]   (first step: X += coef[j] * Vc[:, j] + coef[K + j] * Vn[:, j])
void cheb_step(const double* Y, const double* Vc, const double* Vp, double* Vn, double* X, i64 bs, int n, int k,
               const double* lohi_dev, i64 lohi_bs, bool first, const double* coef_dev, i64 coef_bs, int nb,
               hipStream_t s);
// Interval of the complement expansion of instance i from its Ritz values th (th[0] the largest,
// th[e] the first unresolved one) and res_next (the residual of th[e]), n the matrix order:
//   nu = 64 n 2^-53 max(th[0], 0);  hi = mult * (max(1.1 (max(th[e], 0) + res_next), nu) + 1e-300);
//   lo = -max(nu, 0.05 hi).
void cheb_interval(const double* th, i64 th_bs, int e, const double* res_next, i64 rn_bs, int n, double mult,
                   double* lohi_dev, i64 lohi_bs, int nb, hipStream_t s);
// DCT table of degree m at the N = m + 1 first-kind Chebyshev nodes: ct[q][k] = w_q cos(pi q (k + 1/2) / N),
// w_0 = 1 / N, w_q = 2 / N.
void cheb_table(double* ct, int m, hipStream_t s);
// fv[k][j] = (1/2) d / (d^2 + eps), d = lam[j] - t_k, t_k the k-th node on [lo, hi], k <= m, j < K
void cheb_fvals(const double* lam, i64 lam_bs, int K, double eps, const double* lohi_dev, i64 lohi_bs, int m,
                double* fv, i64 fv_bs, int nb, hipStream_t s);
// ratio[i] = max_{q >= m - 1, j} |c[q][j]| / max_{q, j} |c[q][j]| of instance i's (m + 1) x K coefficients
void cheb_tail(const double* coef, i64 coef_bs, int m, int K, double* ratio_dev, i64 ratio_bs, int nb, hipStream_t s);
// flag_dev[i] |= bit unless |v_m| <= 1.5 |v_0| (both finite): the expansion stayed bounded
void cheb_bound_check(const double* vm_dev, const double* v0_dev, i64 bs, int nb, int* flag_dev, int bit,
                      hipStream_t s);

}  // namespace dtrg
