// Memory-bound helpers of the HOTRG path: permutations, conversions, deterministic reductions,
// traces, log-scale accumulation, the backward's seed and pseudo-random fills.
#include "common.hpp"

#include <algorithm>

namespace dtrg {

namespace {

constexpr int kRedBlocks = 1024;   // fixed number of partials: reductions are bit-reproducible

struct PermK {
    int rank;
    i64 odims[6];     // output dims
    i64 istr[6];      // input stride of each output axis
    i64 total;
};

PermK make_perm(const PermDesc& d) {
    DTRG_REQUIRE(d.rank >= 1 && d.rank <= 6, DTRG_EINVAL, "permute: rank out of range");
    PermK k;
    k.rank = d.rank;
    i64 in_str[6];
    in_str[d.rank - 1] = 1;
    for (int i = d.rank - 2; i >= 0; --i) in_str[i] = in_str[i + 1] * d.in_dims[i + 1];
    k.total = 1;
    int seen = 0;
    for (int i = 0; i < d.rank; ++i) {
        DTRG_REQUIRE(d.perm[i] >= 0 && d.perm[i] < d.rank && !(seen & (1 << d.perm[i])), DTRG_EINVAL,
                     "permute: not a permutation");
        seen |= 1 << d.perm[i];
        k.odims[i] = d.in_dims[d.perm[i]];
        k.istr[i] = in_str[d.perm[i]];
        k.total *= k.odims[i];
    }
    for (int i = d.rank; i < 6; ++i) { k.odims[i] = 1; k.istr[i] = 0; }
    DTRG_REQUIRE(d.in_cap < 0 || k.total <= d.in_cap, DTRG_EINVAL, "permute: input out of bounds");
    DTRG_REQUIRE(d.out_cap < 0 || k.total <= d.out_cap, DTRG_EINVAL, "permute: output out of bounds");
    return k;
}

__device__ inline i64 perm_src(const PermK& p, i64 idx) {
    i64 off = 0;
    for (int i = p.rank - 1; i >= 0; --i) {
        const i64 q = idx / p.odims[i];
        off += (idx - q * p.odims[i]) * p.istr[i];
        idx = q;
    }
    return off;
}

template <class TI, class TO>
__global__ __launch_bounds__(256) void permute_kernel(const TI* __restrict__ in, TO* __restrict__ out, PermK p,
                                                      double alpha, double beta, const double* scale) {
    const double a = scale ? alpha * scale[0] : alpha;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < p.total; i += (i64)gridDim.x * blockDim.x) {
        double v = a * (double)in[perm_src(p, i)];
        if (beta != 0.0) v += beta * (double)out[i];
        out[i] = (TO)v;
    }
}

int grid_for(i64 n) { return (int)std::max<i64>(1, std::min<i64>((n + 255) / 256, 8192)); }

__device__ inline double block_sum(double v) {
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void sumsq_partial_kernel(const double* x, const double* y, i64 n, double* part) {
    double s = 0.0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        s += x[i] * (y ? y[i] : x[i]);
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void finish_sum_kernel(const double* part, int np, double* out, int take_sqrt) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(s) : s;
}

__global__ __launch_bounds__(256) void fill_kernel(double* p, i64 n, double v) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void axpy_kernel(const double* x, double* y, i64 n, double a) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) y[i] += a * x[i];
}

__global__ __launch_bounds__(256) void scale_kernel(double* p, i64 n, double alpha, const double* sc, int recip) {
    double a = alpha;
    if (sc) a *= recip ? 1.0 / sc[0] : sc[0];
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] *= a;
}

__global__ __launch_bounds__(256) void convert_kernel(const double* in, float* out, i64 n) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

__global__ __launch_bounds__(256) void trace_xxyy_kernel(const double* T, int X, int Y, double* out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < X * Y; i += blockDim.x) {
        const int x = i / Y, y = i % Y;
        s += T[(((i64)x * X + x) * Y + y) * Y + y];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(256) void diag_sum_kernel(const double* G, int n, double* out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += G[(i64)i * n + i];
    s = block_sum(s);
    if (threadIdx.x == 0) out[0] = s;
}

// G <- (G + G^T) / (2 t), one thread per (i <= j) pair
__global__ __launch_bounds__(256) void sym_norm_kernel(double* G, int n, const double* t) {
    const double inv = 0.5 / t[0];
    const i64 total = (i64)n * n;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int i = (int)(idx / n), j = (int)(idx % n);
        if (j < i) continue;
        const double v = (G[(i64)i * n + j] + G[(i64)j * n + i]) * inv;
        G[(i64)i * n + j] = v;
        G[(i64)j * n + i] = v;
    }
}

__global__ void accum_log_kernel(const double* x, double w, double* L, double* inv, int* flag) {
    const double v = x[0];
    if (!(v > 0.0) || !isfinite(v)) { if (flag) flag[0] |= 1; return; }
    L[0] += w * log(v);
    if (inv) inv[0] = 1.0 / v;
}

__global__ __launch_bounds__(256) void fill_int_kernel(int* p, i64 n, int v) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void seed_kernel(double* T, int X, int Y, double gw, const double* tr) {
    const i64 total = (i64)X * X * Y * Y;
    const double v = gw / tr[0];
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
        i64 r = i;
        const int d = (int)(r % Y); r /= Y;
        const int u = (int)(r % Y); r /= Y;
        const int rr = (int)(r % X); r /= X;
        const int l = (int)r;
        T[i] = (l == rr && u == d) ? v : 0.0;
    }
}

__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void hash_fill_kernel(double* p, i64 n, uint64_t seed) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)i));
        p[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

__global__ __launch_bounds__(256) void copy2d_kernel(const double* src, i64 lds, double* dst, i64 ldd, int rows, int cols) {
    const i64 total = (i64)rows * cols;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
        const i64 r = i / cols, c = i % cols;
        dst[r * ldd + c] = src[r * lds + c];
    }
}

}  // namespace

void permute(const double* in, double* out, const PermDesc& d, double alpha, double beta,
             const double* scale_dev, hipStream_t s) {
    PermK k = make_perm(d);
    hipLaunchKernelGGL((permute_kernel<double, double>), dim3(grid_for(k.total)), dim3(256), 0, s, in, out, k, alpha,
                       beta, scale_dev);
    DTRG_HIP(hipGetLastError());
}

void permute_to_f32(const double* in, float* out, const PermDesc& d, hipStream_t s) {
    PermK k = make_perm(d);
    hipLaunchKernelGGL((permute_kernel<double, float>), dim3(grid_for(k.total)), dim3(256), 0, s, in, out, k, 1.0,
                       0.0, (const double*)nullptr);
    DTRG_HIP(hipGetLastError());
}

void permute_f32(const float* in, float* out, const PermDesc& d, hipStream_t s) {
    PermK k = make_perm(d);
    hipLaunchKernelGGL((permute_kernel<float, float>), dim3(grid_for(k.total)), dim3(256), 0, s, in, out, k, 1.0,
                       0.0, (const double*)nullptr);
    DTRG_HIP(hipGetLastError());
}

void convert_f64_to_f32(const double* in, float* out, i64 n, hipStream_t s) {
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    DTRG_HIP(hipGetLastError());
}

void fill(double* p, i64 n, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    DTRG_HIP(hipGetLastError());
}

void axpy(const double* x, double* y, i64 n, double a, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, y, n, a);
    DTRG_HIP(hipGetLastError());
}

void scale_inplace(double* p, i64 n, double alpha, const double* scale_dev, bool reciprocal, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, alpha, scale_dev, reciprocal ? 1 : 0);
    DTRG_HIP(hipGetLastError());
}

void norm2(const double* x, i64 n, double* out_dev, hipStream_t s, Scratch& ws) {
    ws.red.ensure(kRedBlocks);
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, x, (const double*)nullptr, n, ws.red.p);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)ws.red.p, kRedBlocks, out_dev, 1);
    DTRG_HIP(hipGetLastError());
}

void dot(const double* x, const double* y, i64 n, double* out_dev, hipStream_t s, Scratch& ws) {
    ws.red.ensure(kRedBlocks);
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, x, y, n, ws.red.p);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)ws.red.p, kRedBlocks, out_dev, 0);
    DTRG_HIP(hipGetLastError());
}

void trace_xxyy(const double* T, int X, int Y, double* out_dev, hipStream_t s) {
    hipLaunchKernelGGL(trace_xxyy_kernel, dim3(1), dim3(256), 0, s, T, X, Y, out_dev);
    DTRG_HIP(hipGetLastError());
}

void sym_normalise(double* G, int n, double* t_dev, hipStream_t s) {
    hipLaunchKernelGGL(diag_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)G, n, t_dev);
    hipLaunchKernelGGL(sym_norm_kernel, dim3(grid_for((i64)n * n)), dim3(256), 0, s, G, n, (const double*)t_dev);
    DTRG_HIP(hipGetLastError());
}

void accum_log(const double* x_dev, double weight, double* L_dev, double* inv_dev, int* flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(accum_log_kernel, dim3(1), dim3(1), 0, s, x_dev, weight, L_dev, inv_dev, flag_dev);
    DTRG_HIP(hipGetLastError());
}

void fill_int(int* p, i64 n, int v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    DTRG_HIP(hipGetLastError());
}

void seed_trace_grad(double* T, int X, int Y, double gbar_weight, const double* tr_dev, hipStream_t s) {
    hipLaunchKernelGGL(seed_kernel, dim3(grid_for((i64)X * X * Y * Y)), dim3(256), 0, s, T, X, Y, gbar_weight, tr_dev);
    DTRG_HIP(hipGetLastError());
}

void hash_fill(double* p, i64 n, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(hash_fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, seed);
    DTRG_HIP(hipGetLastError());
}

void copy2d(const double* src, i64 lds, double* dst, i64 ldd, int rows, int cols, hipStream_t s) {
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for((i64)rows * cols)), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
    DTRG_HIP(hipGetLastError());
}

}  // namespace dtrg
