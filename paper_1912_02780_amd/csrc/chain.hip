// Closing the infinite chain of the paper's scheme (b): the transfer matrix of the cell tensor, its
// dominant eigenvalue and eigenvectors, and the seed of the backward pass.
//
// The cell tensor T[l][r][u][d] of rho(2^n tau) is traced over its physical legs, E[l][r] =
// sum_u T[l][r][u][u] (K x K), and the chain of infinitely many cells has Z per cell = lambda, the
// dominant eigenvalue of E.  lambda comes from repeated squaring: P_0 = E, P_{j+1} = P_j P_j (each
// rescaled by its largest entry; the products are FP64 MFMA contractions launched by the caller)
// converges to the rank-one projector r l^T / (l^T r) at the rate (lambda_2 / lambda)^(2^j), so that a
// fixed number of squarings resolves any gap above ~2^-20 in a known number of launches.  The column
// and the row of P through its largest entry are r and l; lambda = l^T E r / l^T r, with the
// residuals of both eigenvector equations checked.  The adjoint of ln lambda is l r^T / (lambda l^T r)
// (first-order perturbation of a simple eigenvalue), spread over the diagonal of the physical legs.
#include "common.hpp"

#include <algorithm>

namespace dtrg {

namespace {

__global__ __launch_bounds__(256) void transfer_kernel(const double* T, i64 tbs, int K, int Y, const double* scale,
                                                       i64 sc_bs, double* E, i64 ebs) {
    const int z = blockIdx.y;
    T += z * tbs;
    E += z * ebs;
    const double s = scale ? scale[z * sc_bs] : 1.0;
    const i64 total = (i64)K * K;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
        const double* t = T + i * Y * Y;
        double acc = 0.0;
        for (int u = 0; u < Y; ++u) acc += t[(i64)u * Y + u];
        E[i] = s * acc;
    }
}

template <class T, class Op>
__device__ T block_reduce(T v, T* sh, Op op) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] = op(sh[tid], sh[tid + w]);
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

// tr G for G = sum_{j,k} A_jk (x) B_jk: sum_{j,k} (sum_a A[a][a][j][k]) (sum_c B[c][c][j][k]) (one
// workgroup per instance); a trace that is not positive or not finite sets flag bit 1
__global__ __launch_bounds__(256) void kron_trace_kernel(const double* A, i64 a_bs, const double* B, i64 b_bs, int X,
                                                         int Y, double* out, i64 out_bs, int* flag) {
    __shared__ double sh[256];
    const int z = blockIdx.x;
    A += z * a_bs;
    B += z * b_bs;
    const int YY = Y * Y;
    double s = 0.0;
    for (int jk = threadIdx.x; jk < YY; jk += blockDim.x) {
        double ta = 0.0, tb = 0.0;
        for (int a = 0; a < X; ++a) {
            ta += A[((i64)a * X + a) * YY + jk];
            tb += B[((i64)a * X + a) * YY + jk];
        }
        s += ta * tb;
    }
    s = block_reduce(s, sh, [](double u, double v) { return u + v; });
    if (threadIdx.x == 0) {
        out[z * out_bs] = s;
        if (!(s > 0.0) || !isfinite(s)) flag[z] |= 1;
    }
}

// P /= max |P| (one workgroup per instance); a zero or non-finite P sets flag bit
__global__ __launch_bounds__(1024) void maxabs_normalise_kernel(double* P, i64 bs, i64 n, int* flag, int bit) {
    __shared__ double sh[1024];
    const int z = blockIdx.x;
    P += z * bs;
    double m = 0.0;
    for (i64 i = threadIdx.x; i < n; i += blockDim.x) {
        const double a = fabs(P[i]);
        m = (a > m || a != a) ? a : m;
    }
    m = block_reduce(m, sh, [](double a, double b) { return (a > b || a != a) ? a : b; });
    if (!(m > 0.0) || !isfinite(m)) {
        if (threadIdx.x == 0) flag[z] |= bit;
        return;
    }
    const double inv = 1.0 / m;
    for (i64 i = threadIdx.x; i < n; i += blockDim.x) P[i] *= inv;
}

// lambda, r, l from E and the converged power P (K <= kChainMaxK; one workgroup per instance)
__global__ __launch_bounds__(1024) void dominant_finish_kernel(const double* E, i64 ebs, const double* P, i64 pbs,
                                                               int K, double* lr, i64 lrbs, double* lam, i64 sc_bs,
                                                               int* flag, int bit) {
    __shared__ double sh[1024];
    __shared__ int shi[1024];
    __shared__ double r[kChainMaxK], l[kChainMaxK];
    const int z = blockIdx.x, tid = threadIdx.x;
    E += z * ebs;
    P += z * pbs;
    lr += z * lrbs;
    // the largest entry of P
    double m = -1.0;
    int at = 0;
    for (int i = tid; i < K * K; i += blockDim.x) {
        const double a = fabs(P[i]);
        if (a > m) { m = a; at = i; }
    }
    sh[tid] = m;
    shi[tid] = at;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w && (sh[tid + w] > sh[tid] || (sh[tid + w] == sh[tid] && shi[tid + w] < shi[tid]))) {
            sh[tid] = sh[tid + w];
            shi[tid] = shi[tid + w];
        }
        __syncthreads();
    }
    const int istar = shi[0] / K, jstar = shi[0] % K;
    __syncthreads();
    for (int i = tid; i < K; i += blockDim.x) {
        r[i] = P[(i64)i * K + jstar];
        l[i] = P[(i64)istar * K + i];
    }
    __syncthreads();
    // E r, l^T E, and the scalars of the Rayleigh quotient and the residuals
    double lr_ = 0.0, lEr = 0.0, rr = 0.0, ll = 0.0;
    for (int i = tid; i < K; i += blockDim.x) {
        double er = 0.0;
        for (int j = 0; j < K; ++j) er += E[(i64)i * K + j] * r[j];
        lEr += l[i] * er;
        lr_ += l[i] * r[i];
        rr += r[i] * r[i];
        ll += l[i] * l[i];
    }
    auto add = [](double a, double b) { return a + b; };
    lr_ = block_reduce(lr_, sh, add);
    lEr = block_reduce(lEr, sh, add);
    rr = block_reduce(rr, sh, add);
    ll = block_reduce(ll, sh, add);
    const double lmb = lEr / lr_;
    double res_r = 0.0, res_l = 0.0;
    for (int i = tid; i < K; i += blockDim.x) {
        double er = 0.0, le = 0.0;
        for (int j = 0; j < K; ++j) {
            er += E[(i64)i * K + j] * r[j];
            le += l[j] * E[(i64)j * K + i];
        }
        res_r += (er - lmb * r[i]) * (er - lmb * r[i]);
        res_l += (le - lmb * l[i]) * (le - lmb * l[i]);
    }
    res_r = block_reduce(res_r, sh, add);
    res_l = block_reduce(res_l, sh, add);
    const bool ok = lmb > 0.0 && isfinite(lmb) && lr_ != 0.0 && sqrt(res_r) <= kChainResidual * lmb * sqrt(rr) &&
                    sqrt(res_l) <= kChainResidual * lmb * sqrt(ll);
    if (!ok) {
        if (tid == 0) flag[z] |= bit;
        return;
    }
    // r with unit norm, l with l^T r = 1
    const double nr = 1.0 / sqrt(rr), nl = sqrt(rr) / lr_;
    for (int i = tid; i < K; i += blockDim.x) {
        lr[i] = r[i] * nr;
        lr[K + i] = l[i] * nl;
    }
    if (tid == 0) lam[z * sc_bs] = lmb;
}

// Tbar[y][z][a][b] = delta(y, z) gw l[a] r[b] / lambda  (layout [Y][Y][K][K])
__global__ __launch_bounds__(256) void chain_seed_kernel(double* T, i64 bs, int K, int Y, const double* lr, i64 lrbs,
                                                         double gw, const double* lam, i64 sc_bs) {
    const int z = blockIdx.y;
    T += z * bs;
    lr += z * lrbs;
    const double v = gw / lam[z * sc_bs];
    const i64 KK = (i64)K * K, total = (i64)Y * Y * KK;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
        const i64 yz = i / KK, ab = i % KK;
        const int y = (int)(yz / Y), zz = (int)(yz % Y);
        const int a = (int)(ab / K), b = (int)(ab % K);
        T[i] = y == zz ? v * lr[K + a] * lr[b] : 0.0;
    }
}

// out = L + w ln lambda
__global__ void lnZ_at_kernel(const double* L, const double* lam, double w, double* out, i64 sc_bs, int nb) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nb) return;
    out[z * sc_bs] = L[z * sc_bs] + w * log(lam[z * sc_bs]);
}

dim3 grid_of(i64 n, int nb) {
    const i64 per = std::max<i64>(1, std::min<i64>((n + 255) / 256, std::max<i64>(1, 8192 / nb)));
    return dim3((unsigned)per, (unsigned)nb);
}

}  // namespace

void kron_trace(const double* A, i64 a_bs, const double* B, i64 b_bs, int X, int Y, int nb, double* t_dev, i64 t_bs,
                int* flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(kron_trace_kernel, dim3(nb), dim3(256), 0, s, A, a_bs, B, b_bs, X, Y, t_dev, t_bs, flag_dev);
    DTRG_HIP(hipGetLastError());
}

void chain_transfer(const double* T, i64 tbs, int K, int Y, const double* scale_dev, i64 sc_bs, double* E, i64 ebs,
                    int nb, hipStream_t s) {
    hipLaunchKernelGGL(transfer_kernel, grid_of((i64)K * K, nb), dim3(256), 0, s, T, tbs, K, Y, scale_dev, sc_bs, E,
                       ebs);
    DTRG_HIP(hipGetLastError());
}

void chain_normalise(double* P, i64 bs, i64 n, int nb, int* flag_dev, int bit, hipStream_t s) {
    hipLaunchKernelGGL(maxabs_normalise_kernel, dim3(nb), dim3(1024), 0, s, P, bs, n, flag_dev, bit);
    DTRG_HIP(hipGetLastError());
}

void chain_dominant_finish(const double* E, i64 ebs, const double* P, i64 pbs, int K, int nb, double* lr, i64 lrbs,
                           double* lam_dev, i64 sc_bs, int* flag_dev, int bit, hipStream_t s) {
    DTRG_REQUIRE(K >= 1 && K <= kChainMaxK, DTRG_EINVAL, "chain transfer matrix larger than the closing kernel takes");
    hipLaunchKernelGGL(dominant_finish_kernel, dim3(nb), dim3(1024), 0, s, E, ebs, P, pbs, K, lr, lrbs, lam_dev,
                       sc_bs, flag_dev, bit);
    DTRG_HIP(hipGetLastError());
}

void chain_seed(double* T, i64 bs, int K, int Y, const double* lr, i64 lrbs, double gw, const double* lam_dev,
                i64 sc_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(chain_seed_kernel, grid_of((i64)Y * Y * K * K, nb), dim3(256), 0, s, T, bs, K, Y, lr, lrbs, gw,
                       lam_dev, sc_bs);
    DTRG_HIP(hipGetLastError());
}

void chain_lnZ_at(const double* L_dev, const double* lam_dev, double w, double* out_dev, i64 sc_bs, int nb,
                  hipStream_t s) {
    hipLaunchKernelGGL(lnZ_at_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, L_dev, lam_dev, w, out_dev, sc_bs, nb);
    DTRG_HIP(hipGetLastError());
}

}  // namespace dtrg
