// Small dense FP64 eigen kernels of the truncated eigensolve and its adjoint (gfx950).
//
// * jacobi_eig: one workgroup holds an n x n symmetric matrix and its eigenvector accumulator in
//   LDS (n <= 96: 2 x 96 x 97 doubles = 146 KiB of the 160 KiB LDS) and runs cyclic Jacobi in the
//   round-robin (Berger table) order: in every round n/2 disjoint index pairs are rotated at once,
//   rows first, then columns.  A pair is rotated while |a_pq| > 1e-16 sqrt(|a_pp a_qq|) (or above
//   an absolute floor), which keeps small eigenvalues to high relative accuracy.
// * chol_inverse: Cholesky of a (shifted) b x b Gram in LDS and the inverse of its triangular
//   factor, for CholeskyQR of the subspace block.
// * element-wise helpers for Ritz residuals, column normalisation, the broadened inverse gaps of
//   the eigenvector adjoint and the Chebyshev three-term recurrence.
#include "common.hpp"

#include <algorithm>

namespace dtrg {

namespace {

constexpr int JM = kJacobiMax;
constexpr int JLD = JM + 1;
constexpr int JT = 512;    // Jacobi: 8 waves
constexpr int CT = 256;    // Cholesky / inverse: 4 waves

__global__ __launch_bounds__(JT) void jacobi_kernel(const double* __restrict__ Ain, int n, int lda,
                                                     double* __restrict__ lam, double* __restrict__ Vout,
                                                     int ldv, int max_sweeps, int* sweeps_out) {
    __shared__ double A[JM * JLD];
    __shared__ double V[JM * JLD];
    __shared__ int rp[JM / 2], rq[JM / 2];
    __shared__ double rc[JM / 2], rs[JM / 2];
    __shared__ int nrot, nact;
    __shared__ double fro;
    const int tid = threadIdx.x;
    const int m = n + (n & 1);  // players, padded to even with a dummy index n
    for (int i = tid; i < n * n; i += JT) {
        const int r = i / n, c = i % n;
        A[r * JLD + c] = 0.5 * (Ain[(i64)r * lda + c] + Ain[(i64)c * lda + r]);
        V[r * JLD + c] = (r == c) ? 1.0 : 0.0;
    }
    if (tid == 0) fro = 0.0;
    __syncthreads();
    if (tid < 64) {
        double s = 0.0;
        for (int i = tid; i < n * n; i += 64) { const double v = A[(i / n) * JLD + (i % n)]; s += v * v; }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
        if (tid == 0) fro = sqrt(s);
    }
    __syncthreads();
    // entries below the rounding level of the matrix are not rotated away (they are noise; rotating
    // them only costs sweeps on spectra that reach the FP64 floor)
    const double abs_floor = 0x1p-60 * fro + 1e-300;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) nrot = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            // the n/2 pairs of this round are handled by wave 0 (m/2 <= 48 lanes); the pairs that
            // need a rotation are compacted into slots 0..nact-1
            if (tid < 64) {
                int p = 0, q = 0, active = 0;
                double c = 1.0, s = 0.0;
                if (tid < m / 2) {
                    if (tid == 0) { p = m - 1; q = round; }
                    else { p = (round + tid) % (m - 1); q = (round - tid + (m - 1)) % (m - 1); }
                    if (p > q) { const int t = p; p = q; q = t; }
                    if (q < n) {
                        const double apq = A[p * JLD + q];
                        const double app = A[p * JLD + p], aqq = A[q * JLD + q];
                        if (fabs(apq) > fmax(1e-16 * sqrt(fabs(app * aqq)), abs_floor)) {
                            const double theta = (aqq - app) / (2.0 * apq);
                            double t;
                            if (fabs(theta) > 1e150) t = 0.5 / theta;
                            else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                            c = 1.0 / sqrt(1.0 + t * t);
                            s = t * c;
                            active = 1;
                        }
                    }
                }
                const unsigned long long mask = __ballot(active);
                const int slot = __popcll(mask & ((1ull << tid) - 1ull));
                if (active) { rp[slot] = p; rq[slot] = q; rc[slot] = c; rs[slot] = s; }
                if (tid == 0) { nact = __popcll(mask); nrot += nact; }
            }
            __syncthreads();
            const int na = nact;
            if (na > 0) {
                // rows:  row_p <- c row_p - s row_q ; row_q <- s row_p + c row_q
                for (int idx = tid; idx < na * n; idx += JT) {
                    const int i = idx / n, j = idx % n;
                    const int p = rp[i], q = rq[i];
                    const double c = rc[i], s = rs[i];
                    const double ap = A[p * JLD + j], aq = A[q * JLD + j];
                    A[p * JLD + j] = c * ap - s * aq;
                    A[q * JLD + j] = s * ap + c * aq;
                }
                __syncthreads();
                // columns of A and of V
                for (int idx = tid; idx < na * n; idx += JT) {
                    const int i = idx / n, r = idx % n;
                    const int p = rp[i], q = rq[i];
                    const double c = rc[i], s = rs[i];
                    const double ap = A[r * JLD + p], aq = A[r * JLD + q];
                    A[r * JLD + p] = c * ap - s * aq;
                    A[r * JLD + q] = s * ap + c * aq;
                    const double vp = V[r * JLD + p], vq = V[r * JLD + q];
                    V[r * JLD + p] = c * vp - s * vq;
                    V[r * JLD + q] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
        const int done = (nrot == 0);
        __syncthreads();
        if (done) break;
    }
    // sort descending (ties by index) and write out
    for (int i = tid; i < n; i += JT) {
        const double li = A[i * JLD + i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = A[j * JLD + j];
            rank += (lj > li) || (lj == li && j < i);
        }
        lam[rank] = li;
        for (int r = 0; r < n; ++r) Vout[(i64)r * ldv + rank] = V[r * JLD + i];
    }
    if (tid == 0 && sweeps_out) sweeps_out[0] = sweep;
}

// Lower Cholesky factor L of S + shift I in LDS, then Rinv = (L^T)^{-1} (upper) to global.
// Lower Cholesky factor L of (S + shift I) in LDS (right-looking, rank-1 trailing updates in
// parallel), then X = L^{-1} by the same elimination applied to the identity (row k of X is
// final after step k, rows below get a parallel rank-1 update), Rinv = X^T to global.
__global__ __launch_bounds__(CT) void chol_inv_kernel(const double* __restrict__ S, int b, double shift_rel,
                                                       double* __restrict__ Rinv, int* flag) {
    __shared__ double L[JM * JLD];
    __shared__ double Xs[JM * JLD];
    __shared__ double tr;
    const int tid = threadIdx.x;
    for (int i = tid; i < b * b; i += CT) {
        const int r = i / b, c = i % b;
        L[r * JLD + c] = 0.5 * (S[(i64)r * b + c] + S[(i64)c * b + r]);
        Xs[r * JLD + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < b; ++i) s += L[i * JLD + i];
        tr = s;
    }
    __syncthreads();
    const double shift = shift_rel * tr;
    for (int i = tid; i < b; i += CT) L[i * JLD + i] += shift;
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        double d = L[k * JLD + k];
        if (!(d > 0.0) || !isfinite(d)) {
            if (tid == 0 && flag) atomicOr(flag, 2);
            d = 1e-300;
        }
        const double dk = sqrt(d);
        // column k of L below the diagonal; lanes read L[k][k] before it is overwritten
        for (int i = k + 1 + tid; i < b; i += CT) L[i * JLD + k] /= dk;
        __syncthreads();
        if (tid == 0) L[k * JLD + k] = dk;
        const int rem = b - k - 1;
        for (int idx = tid; idx < rem * rem; idx += CT) {
            const int i = k + 1 + idx / rem, j = k + 1 + idx % rem;
            if (j <= i) L[i * JLD + j] -= L[i * JLD + k] * L[j * JLD + k];
        }
        __syncthreads();
    }
    // X = L^{-1}: for k = 0..b-1, scale row k by 1/L[k][k], then remove it from the rows below
    for (int k = 0; k < b; ++k) {
        const double inv = 1.0 / L[k * JLD + k];
        for (int j = tid; j <= k; j += CT) Xs[k * JLD + j] *= inv;
        __syncthreads();
        const int rem = b - k - 1;
        for (int idx = tid; idx < rem * (k + 1); idx += CT) {
            const int i = k + 1 + idx / (k + 1), j = idx % (k + 1);
            Xs[i * JLD + j] -= L[i * JLD + k] * Xs[k * JLD + j];
        }
        __syncthreads();
    }
    // Rinv = (L^{-1})^T
    for (int idx = tid; idx < b * b; idx += CT) {
        const int i = idx / b, j = idx % b;
        Rinv[(i64)i * b + j] = (i <= j) ? Xs[j * JLD + i] : 0.0;
    }
}

__device__ inline double block_sum256(double v) {
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void col_norms_kernel(const double* V, int n, int ldv, double* out) {
    const int j = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) { const double v = V[(i64)r * ldv + j]; s += v * v; }
    s = block_sum256(s);
    if (threadIdx.x == 0) out[j] = sqrt(s);
}

__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void col_normalise_kernel(double* V, int n, int b, int ldv, const double* nrm,
                                                             uint64_t seed) {
    double mx = 0.0;
    for (int j = 0; j < b; ++j) mx = fmax(mx, nrm[j]);
    const double tiny = 1e-200 + 1e-30 * mx;
    const i64 total = (i64)n * b;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int r = (int)(idx / b), j = (int)(idx % b);
        const double d = nrm[j];
        if (d > tiny) V[(i64)r * ldv + j] /= d;
        else {
            const uint64_t h = mix64(seed ^ mix64((uint64_t)idx));
            V[(i64)r * ldv + j] = ((double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0) / sqrt((double)n);
        }
    }
}

__global__ __launch_bounds__(256) void ritz_res_kernel(const double* V, const double* Y, int n, int ld,
                                                        const double* theta, double* res) {
    const int j = blockIdx.x;
    const double th = theta[j];
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) {
        const double v = Y[(i64)r * ld + j] - th * V[(i64)r * ld + j];
        s += v * v;
    }
    s = block_sum256(s);
    if (threadIdx.x == 0) res[j] = sqrt(s);
}

__device__ inline double bgap(double d, double eps) { return d / (d * d + eps); }

__global__ __launch_bounds__(256) void kept_block_kernel(const double* Om, const double* lam, int k, double eps,
                                                          double* S) {
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < k * k; idx += gridDim.x * blockDim.x) {
        const int i = idx / k, j = idx % k;
        S[idx] = (i == j) ? 0.0 : bgap(lam[j] - lam[i], eps) * 0.5 * (Om[i * k + j] - Om[j * k + i]);
    }
}

__global__ __launch_bounds__(256) void over_block_kernel(const double* Om, const double* theta, const double* lam,
                                                          int p, int k, double eps, double* M) {
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < p * k; idx += gridDim.x * blockDim.x) {
        const int i = idx / k, j = idx % k;
        M[idx] = bgap(lam[j] - theta[i], eps) * 0.5 * Om[idx];
    }
}

__global__ __launch_bounds__(256) void cheb_step_kernel(const double* Y, const double* Vc, const double* Vp,
                                                         double* Vn, double* X, int n, int k, double a, double sum,
                                                         int first, const double* coef) {
    const i64 total = (i64)n * k;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int j = (int)(idx % k);
        const double vc = Vc[idx];
        double v = a * (2.0 * Y[idx] - sum * vc);
        if (!first) v -= Vp[idx];
        Vn[idx] = v;
        if (first) X[idx] += coef[j] * vc + coef[k + j] * v;
        else X[idx] += coef[j] * v;
    }
}

int grid_for(i64 n) { return (int)std::max<i64>(1, std::min<i64>((n + 255) / 256, 8192)); }

}  // namespace

void jacobi_eig(const double* A, int n, int lda, double* lam_dev, double* V, int ldv, int max_sweeps,
                int* sweeps_dev, hipStream_t s) {
    DTRG_REQUIRE(n >= 1 && n <= kJacobiMax, DTRG_EINVAL, "jacobi_eig: n out of range");
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(JT), 0, s, A, n, lda, lam_dev, V, ldv, max_sweeps, sweeps_dev);
    DTRG_HIP(hipGetLastError());
}

void chol_inverse(const double* S, int b, double shift_rel, double* Rinv, int* flag_dev, hipStream_t s) {
    DTRG_REQUIRE(b >= 1 && b <= kJacobiMax, DTRG_EINVAL, "chol_inverse: b out of range");
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(CT), 0, s, S, b, shift_rel, Rinv, flag_dev);
    DTRG_HIP(hipGetLastError());
}

void col_norms(const double* V, int n, int b, int ldv, double* out_dev, hipStream_t s) {
    hipLaunchKernelGGL(col_norms_kernel, dim3(b), dim3(256), 0, s, V, n, ldv, out_dev);
    DTRG_HIP(hipGetLastError());
}

void col_normalise(double* V, int n, int b, int ldv, const double* nrm_dev, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(col_normalise_kernel, dim3(grid_for((i64)n * b)), dim3(256), 0, s, V, n, b, ldv, nrm_dev, seed);
    DTRG_HIP(hipGetLastError());
}

void ritz_residuals(const double* V, const double* Y, int n, int k, int ld, const double* theta_dev,
                    double* res_dev, hipStream_t s) {
    hipLaunchKernelGGL(ritz_res_kernel, dim3(k), dim3(256), 0, s, V, Y, n, ld, theta_dev, res_dev);
    DTRG_HIP(hipGetLastError());
}

void kept_block_adjoint(const double* Om, const double* lam_dev, int k, double eps, double* S, hipStream_t s) {
    hipLaunchKernelGGL(kept_block_kernel, dim3(grid_for((i64)k * k)), dim3(256), 0, s, Om, lam_dev, k, eps, S);
    DTRG_HIP(hipGetLastError());
}

void over_block_adjoint(const double* Om, const double* theta_dev, const double* lam_dev, int p, int k, double eps,
                        double* M, hipStream_t s) {
    hipLaunchKernelGGL(over_block_kernel, dim3(grid_for((i64)p * k)), dim3(256), 0, s, Om, theta_dev, lam_dev, p, k,
                       eps, M);
    DTRG_HIP(hipGetLastError());
}

void cheb_step(const double* Y, const double* Vc, const double* Vp, double* Vn, double* X, int n, int k, double lo,
               double hi, bool first, const double* coef_dev, hipStream_t s) {
    const double a = (first ? 1.0 : 2.0) / (hi - lo);
    hipLaunchKernelGGL(cheb_step_kernel, dim3(grid_for((i64)n * k)), dim3(256), 0, s, Y, Vc, Vp, Vn, X, n, k, a,
                       hi + lo, first ? 1 : 0, coef_dev);
    DTRG_HIP(hipGetLastError());
}

}  // namespace dtrg
