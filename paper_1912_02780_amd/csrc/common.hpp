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

// Owning device buffer (hipMalloc / hipFree).
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw Error(DTRG_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                         " bytes failed: " + hipGetErrorString(e));
        }
        n = count;
    }
    void ensure(size_t count) { if (count > n) alloc(count); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
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

__host__ __device__ inline i64 idx_off(const IdxMap& m, i64 i) { return (i / m.div) * m.s1 + (i % m.div) * m.s0; }

// Element types of a contraction.
enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2 };

// One (batched) contraction C[b](r, c) = alpha * sum_k A[b](r, k) B[b](c, k) + beta * C[b](r, c).
//   A stored as [M][K] (a_kmajor = false: A[m * lda + k]) or [K][M] (a_kmajor = true: A[k * lda + m]).
//   B stored as [N][K] (b_kmajor = false: B[n * ldb + k]) or [K][N] (b_kmajor = true: B[k * ldb + n]).
//   C element (b, r, c) lives at C + b * c_bs + idx_off(rmap, r) + idx_off(cmap, c).
struct GemmOp {
    int M = 0, N = 0, K = 0, batch = 1;
    const void* A = nullptr; i64 lda = 0, a_bs = 0; bool a_kmajor = false;
    const void* B = nullptr; i64 ldb = 0, b_bs = 0; bool b_kmajor = false;
    void* C = nullptr; i64 c_bs = 0;
    IdxMap rmap, cmap;
    double alpha = 1.0, beta = 0.0;
    int splits = 0;  // 0 = automatic
    // element capacities of the buffers behind A, B, C (-1: unchecked); checked on the host
    // against the largest offset the kernel can touch before anything is launched
    i64 a_cap = -1, b_cap = -1, c_cap = -1;
    int tag = 0;   // own kernel symbol for the chi^7 contractions: 7 the join of the two copies
                   // (forward and its backward recompute; timed when profiling), 8 its adjoint
                   // with respect to the upper copy's product P, 9 with respect to the lower copy
};

// Scratch owned by a plan, grown on demand (not shrunk) and reused by every contraction.
struct Scratch {
    DevBuf<double> splitk;   // split-K partials (FP64 or reinterpreted FP32)
    DevBuf<double> red;      // reduction partials
};

// gemm.hip
void gemm(Prec in_prec, bool out_f64, const GemmOp& op, hipStream_t s, Scratch& ws);

// tensor_ops.hip
struct PermDesc {
    int rank = 0;
    i64 in_dims[6];
    int perm[6];
    i64 in_cap = -1, out_cap = -1;   // element capacities (-1: unchecked)
};
// out = alpha * (*scale_dev if non-null) * transpose(in, perm) + beta * out   (numpy transpose semantics)
void permute(const double* in, double* out, const PermDesc& d, double alpha, double beta,
             const double* scale_dev, hipStream_t s);
void permute_to_f32(const double* in, float* out, const PermDesc& d, hipStream_t s);
void permute_f32(const float* in, float* out, const PermDesc& d, hipStream_t s);
void convert_f64_to_f32(const double* in, float* out, i64 n, hipStream_t s);
void fill(double* p, i64 n, double v, hipStream_t s);
// y += a * x
void axpy(const double* x, double* y, i64 n, double a, hipStream_t s);
void scale_inplace(double* p, i64 n, double alpha, const double* scale_dev, bool reciprocal, hipStream_t s);
// out[0] = sqrt(sum x^2) (deterministic two-pass reduction)
void norm2(const double* x, i64 n, double* out_dev, hipStream_t s, Scratch& ws);
void dot(const double* x, const double* y, i64 n, double* out_dev, hipStream_t s, Scratch& ws);
// out[0] = sum_{x,y} T[x][x][y][y]  for T of shape [X][X][Y][Y]
void trace_xxyy(const double* T, int X, int Y, double* out_dev, hipStream_t s);
// G (n x n, ld n) <- (G + G^T) / (2 * t_dev[0]), with t_dev[0] = trace(G) computed first
void sym_normalise(double* G, int n, double* t_dev, hipStream_t s);
// L_dev[0] += weight * log(x_dev[0]); inv_dev[0] = 1 / x_dev[0] (if inv_dev); flag bit 0 if x is
// not positive and finite
void accum_log(const double* x_dev, double weight, double* L_dev, double* inv_dev, int* flag_dev, hipStream_t s);
void fill_int(int* p, i64 n, int v, hipStream_t s);
// seed of the backward: T[x][x][y][y] = gbar * weight / tr_dev[0], zero elsewhere
void seed_trace_grad(double* T, int X, int Y, double gbar_weight, const double* tr_dev, hipStream_t s);
// pseudo-random fill in [-1, 1) from a counter-based hash
void hash_fill(double* p, i64 n, uint64_t seed, hipStream_t s);
// copy a rows x cols block between row-major matrices with leading dimensions
void copy2d(const double* src, i64 lds, double* dst, i64 ldd, int rows, int cols, hipStream_t s);

// eig.hip
// Full symmetric eigendecomposition of an n x n matrix (n <= kJacobiMax) by parallel cyclic
// Jacobi in one workgroup: eigenvalues descending into lam_dev[0..n), eigenvectors as the
// columns of V (row-major, leading dimension ldv).
constexpr int kJacobiMax = 96;
void jacobi_eig(const double* A, int n, int lda, double* lam_dev, double* V, int ldv, int max_sweeps,
                int* sweeps_dev, hipStream_t s);
// Upper-triangular R^{-1} of the Cholesky factor of (S + shift * I), S b x b (ld b); the
// shift is shift_rel * trace(S).  flag_dev[0] |= 2 on a non-positive pivot.
void chol_inverse(const double* S, int b, double shift_rel, double* Rinv, int* flag_dev, hipStream_t s);
// norms of the b columns of V (n x b, ld ldv) -> out[0..b)
void col_norms(const double* V, int n, int b, int ldv, double* out_dev, hipStream_t s);
// V[:, j] /= nrm[j] where nrm[j] > tiny * max(nrm); other columns replaced by hash noise
void col_normalise(double* V, int n, int b, int ldv, const double* nrm_dev, uint64_t seed, hipStream_t s);
// res[j] = |Y[:, j] - theta[j] V[:, j]| for j < k
void ritz_residuals(const double* V, const double* Y, int n, int k, int ld, const double* theta_dev,
                    double* res_dev, hipStream_t s);
// S[i][j] = F(lam_j - lam_i) * (Om[i][j] - Om[j][i]) / 2 on the k x k kept block (F_ii = 0),
// F(d) = d / (d^2 + eps)
void kept_block_adjoint(const double* Om, const double* lam_dev, int k, double eps, double* S, hipStream_t s);
// M[i][j] = F(lam_j - theta_i) * Om[i][j] / 2 for i < p (oversampled), j < k
void over_block_adjoint(const double* Om, const double* theta_dev, const double* lam_dev, int p, int k,
                        double eps, double* M, hipStream_t s);
// Chebyshev three-term step on n x k blocks:
//   Vn = a * (2 * Y - (hi + lo) * Vc) - Vp (a = 2 / (hi - lo), or half that for the first step with Vp = 0)
//   X += coef[j] * Vn[:, j]   (first step: X += coef[j] * Vc[:, j] + coef[K + j] * Vn[:, j])
void cheb_step(const double* Y, const double* Vc, const double* Vp, double* Vn, double* X, int n, int k,
               double lo, double hi, bool first, const double* coef_dev, hipStream_t s);

}  // namespace dtrg
