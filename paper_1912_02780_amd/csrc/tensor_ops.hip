// Memory-bound helpers of the HOTRG path: permutations, conversions, deterministic reductions,
// traces, log-scale accumulation, the backward's seed and pseudo-random fills.
//
// Every helper works on nb independent instances at once: blockIdx.y is the instance, the x
// blocks of an instance stride over its elements, so one launch serves a whole batch.
#include "common.hpp"

#include <algorithm>
#include <cstdint>

namespace dtrg {

namespace {

constexpr int kRedBlocks = 1024;   // partials of a single-instance reduction

struct PermK {
    int rank;
    i64 odims[6];     // output dims
    i64 istr[6];      // input stride of each output axis
    i64 total;        // elements per instance
    i64 rowlen;       // output row length (product of the last out_inner output dims), 0: dense
    i64 out_ld;       // output row stride when rowlen > 0
    i64 out_ps;       // plane stride of bf16-plane outputs
};

PermK make_perm(const PermDesc& d, int np = 1) {
    DTRG_REQUIRE(d.rank >= 1 && d.rank <= 6, DTRG_EINVAL, "permute: rank out of range");
    DTRG_REQUIRE(d.nb >= 1 && d.nb < 65536, DTRG_EINVAL, "permute: instance count out of range");
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
    DTRG_REQUIRE(d.out_inner >= 0 && d.out_inner <= d.rank, DTRG_EINVAL, "permute: bad row definition");
    k.rowlen = 0;
    k.out_ld = 0;
    k.out_ps = d.out_ps;
    i64 out_inst = k.total;   // extent of one output instance
    if (d.out_inner > 0) {
        k.rowlen = 1;
        for (int i = d.rank - d.out_inner; i < d.rank; ++i) k.rowlen *= k.odims[i];
        DTRG_REQUIRE(d.out_ld >= k.rowlen, DTRG_EINVAL, "permute: output row stride smaller than a row");
        k.out_ld = d.out_ld;
        out_inst = k.total > 0 ? (k.total / k.rowlen - 1) * k.out_ld + k.rowlen : 0;
    }
    DTRG_REQUIRE(np == 1 || d.out_ps >= (i64)(d.nb - 1) * d.out_bs + out_inst, DTRG_EINVAL,
                 "permute: output planes overlap");
    const i64 in_ext = (i64)(d.nb - 1) * d.in_bs + k.total;
    const i64 out_ext = (i64)(d.nb - 1) * d.out_bs + out_inst + (i64)(np - 1) * d.out_ps;
    DTRG_REQUIRE(d.in_cap < 0 || in_ext <= d.in_cap, DTRG_EINVAL, "permute: input out of bounds");
    DTRG_REQUIRE(d.out_cap < 0 || out_ext <= d.out_cap, DTRG_EINVAL, "permute: output out of bounds");
    DTRG_REQUIRE(d.nb == 1 || (d.in_bs >= k.total && d.out_bs >= out_inst), DTRG_EINVAL,
                 "permute: instance stride smaller than an instance");
    return k;
}

// input offset of output element idx; 32-bit division when the instance has fewer than 2^31
// elements (a 64-bit division is a long instruction sequence on the GPU)
__device__ inline i64 perm_src(const PermK& p, i64 idx) {
    i64 off = 0;
    if (p.total < (1LL << 31)) {
        unsigned u = (unsigned)idx;
        for (int i = p.rank - 1; i >= 0; --i) {
            const unsigned d = (unsigned)p.odims[i], q = u / d;
            off += (i64)(u - q * d) * p.istr[i];
            u = q;
        }
        return off;
    }
    for (int i = p.rank - 1; i >= 0; --i) {
        const i64 q = idx / p.odims[i];
        off += (idx - q * p.odims[i]) * p.istr[i];
        idx = q;
    }
    return off;
}

// output offset of output element i (rows of rowlen elements at stride out_ld, or dense)
__device__ inline i64 perm_dst(const PermK& p, i64 i) {
    if (p.rowlen <= 0) return i;
    if (p.total < (1LL << 31)) {
        const unsigned u = (unsigned)i, r = (unsigned)p.rowlen, q = u / r;
        return (i64)q * p.out_ld + (u - q * r);
    }
    return (i / p.rowlen) * p.out_ld + i % p.rowlen;
}

// x blocks per instance for n elements, keeping the whole grid near 8192 blocks
dim3 grid2(i64 n, int nb) {
    const i64 per = std::max<i64>(1, std::min<i64>((n + 255) / 256, std::max<i64>(1, 8192 / nb)));
    return dim3((unsigned)per, (unsigned)nb);
}

// output writers: OUT = 0 double, 1 float, 2 / 3 the value rounded to FP32 and split into that
// many bf16 planes (plane q = bf16 of what the planes before it leave)
template <int OUT>
__device__ inline void put_elem(void* base, i64 off, i64 ps, double v, double beta) {
    if constexpr (OUT == 0) {
        double* o = (double*)base;
        if (beta != 0.0) v += beta * o[off];
        o[off] = v;
    } else if constexpr (OUT == 1) {
        float* o = (float*)base;
        if (beta != 0.0) v += beta * (double)o[off];
        o[off] = (float)v;
    } else {
        __bf16* o = (__bf16*)base;
        float r = (float)v;
#pragma unroll
        for (int q = 0; q < OUT; ++q) {
            const __bf16 h = (__bf16)r;
            o[q * ps + off] = h;
            r -= (float)h;
        }
    }
}

template <class TI, int OUT>
__global__ __launch_bounds__(256) void permute_kernel(const TI* __restrict__ in, void* __restrict__ out, PermK p,
                                                      i64 in_bs, i64 out_bs, double alpha, double beta,
                                                      const double* scale, i64 scale_bs) {
    const int z = blockIdx.y;
    in += z * in_bs;
    const double a = scale ? alpha * scale[z * scale_bs] : alpha;
    const i64 ob = z * out_bs;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < p.total; i += (i64)gridDim.x * blockDim.x) {
        put_elem<OUT>(out, ob + perm_dst(p, i), p.out_ps, a * (double)in[perm_src(p, i)], beta);
    }
}

// out[q][r][k] (row stride ld_out, plane stride ps) = planes of in(r, k), in(r, k) = in[r * ld_in + k]
// or in[k * ld_in + r] (kmajor)
template <int OUT>
__global__ __launch_bounds__(256) void split_matrix_kernel(const float* in, i64 ld_in, int kmajor, int rows, int cols,
                                                           void* out, i64 ld_out, i64 ps) {
    const i64 total = (i64)rows * cols;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
        const i64 r = i / cols, k = i % cols;
        const float v = kmajor ? in[k * ld_in + r] : in[r * ld_in + k];
        put_elem<OUT>(out, r * ld_out + k, ps, (double)v, 0.0);
    }
}

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

// partial sums of x*y (x*x when y is null): part[z * gridDim.x + blockIdx.x]
__global__ __launch_bounds__(256) void sumsq_partial_kernel(const double* x, const double* y, i64 bs, i64 n,
                                                            double* part) {
    const int z = blockIdx.y;
    x += z * bs;
    if (y) y += z * bs;
    double s = 0.0;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        s += x[i] * (y ? y[i] : x[i]);
    s = block_sum(s);
    if (threadIdx.x == 0) part[(i64)z * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void finish_sum_kernel(const double* part, int np, double* out, i64 out_bs,
                                                         int take_sqrt) {
    const int z = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[(i64)z * np + i];
    s = block_sum(s);
    if (threadIdx.x == 0) out[z * out_bs] = take_sqrt ? sqrt(s) : s;
}

__global__ __launch_bounds__(256) void fill_kernel(double* p, i64 bs, i64 n, double v) {
    p += blockIdx.y * bs;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void axpy_kernel(const double* x, double* y, i64 bs, i64 n, double a,
                                                   const double* sc, i64 sc_bs) {
    x += blockIdx.y * bs;
    y += blockIdx.y * bs;
    if (sc) a *= sc[blockIdx.y * sc_bs];
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) y[i] += a * x[i];
}

__global__ __launch_bounds__(256) void scale_kernel(double* p, i64 bs, i64 n, double alpha, const double* sc,
                                                    i64 sc_bs, int recip) {
    const int z = blockIdx.y;
    p += z * bs;
    double a = alpha;
    if (sc) a *= recip ? 1.0 / sc[z * sc_bs] : sc[z * sc_bs];
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] *= a;
}

__global__ __launch_bounds__(256) void convert_kernel(const double* in, i64 in_bs, float* out, i64 out_bs, i64 n) {
    in += blockIdx.y * in_bs;
    out += blockIdx.y * out_bs;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

__global__ __launch_bounds__(256) void trace_xxyy_kernel(const double* T, i64 bs, int X, int Y, double* out,
                                                         i64 out_bs) {
    const int z = blockIdx.x;
    T += z * bs;
    double s = 0.0;
    for (int i = threadIdx.x; i < X * Y; i += blockDim.x) {
        const int x = i / Y, y = i % Y;
        s += T[(((i64)x * X + x) * Y + y) * Y + y];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) out[z * out_bs] = s;
}

__global__ __launch_bounds__(256) void diag_sum_kernel(const double* G, i64 bs, int n, double* out, i64 out_bs,
                                                       int* flag) {
    const int z = blockIdx.x;
    G += z * bs;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += G[(i64)i * n + i];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        out[z * out_bs] = s;
        if (!(s > 0.0) || !isfinite(s)) flag[z] |= 1;
    }
}

// G <- (G + G^T) / (2 t), one thread per (i <= j) pair
__global__ __launch_bounds__(256) void sym_norm_kernel(double* G, i64 bs, int n, const double* t, i64 t_bs) {
    const int z = blockIdx.y;
    G += z * bs;
    const double inv = 0.5 / t[z * t_bs];
    const i64 total = (i64)n * n;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int i = (int)(idx / n), j = (int)(idx % n);
        if (j < i) continue;
        const double v = (G[(i64)i * n + j] + G[(i64)j * n + i]) * inv;
        G[(i64)i * n + j] = v;
        G[(i64)j * n + i] = v;
    }
}

__global__ void accum_log_kernel(const double* x, double w, double* L, double* inv, i64 sc_bs, int nb, int* flag) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nb) return;
    const double v = x[z * sc_bs];
    if (!isfinite(v)) { flag[z] |= 4; return; }
    if (!(v > 0.0)) { flag[z] |= 1; return; }
    L[z * sc_bs] += w * log(v);
    if (inv) inv[z * sc_bs] = 1.0 / v;
}

__global__ __launch_bounds__(256) void fill_int_kernel(int* p, i64 n, int v) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void seed_kernel(double* T, i64 bs, int X, int Y, double gw, const double* tr,
                                                   i64 tr_bs) {
    const int z = blockIdx.y;
    T += z * bs;
    const i64 total = (i64)X * X * Y * Y;
    const double v = gw / tr[z * tr_bs];
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

__global__ __launch_bounds__(256) void hash_fill_kernel(double* p, i64 bs, i64 n, uint64_t seed) {
    const int z = blockIdx.y;
    p += z * bs;
    const uint64_t sz = z == 0 ? seed : splitmix64(seed ^ (0xa5a5a5a5ULL + (uint64_t)z));
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const uint64_t h = splitmix64(sz ^ splitmix64((uint64_t)i));
        p[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

__global__ __launch_bounds__(256) void copy2d_kernel(const double* src, i64 lds, i64 src_bs, double* dst, i64 ldd,
                                                     i64 dst_bs, int rows, int cols) {
    src += blockIdx.y * src_bs;
    dst += blockIdx.y * dst_bs;
    const i64 total = (i64)rows * cols;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x) {
        const i64 r = i / cols, c = i % cols;
        dst[r * ldd + c] = src[r * lds + c];
    }
}

__global__ __launch_bounds__(256) void gather_kernel(const double* src, i64 src_bs, const int* idx, double* dst,
                                                     i64 dst_bs, i64 len, int scatter) {
    const int z = blockIdx.y;
    const i64 so = scatter ? (i64)z * src_bs : (i64)idx[z] * src_bs;
    const i64 dof = scatter ? (i64)idx[z] * dst_bs : (i64)z * dst_bs;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < len; i += (i64)gridDim.x * blockDim.x)
        dst[dof + i] = src[so + i];
}

__global__ __launch_bounds__(64) void max_check_kernel(const double* v, i64 v_bs, int k, double thr, double* mx,
                                                       i64 mx_bs, int* flag, int bit) {
    const int z = blockIdx.x;
    v += z * v_bs;
    double m = 0.0;
    for (int j = threadIdx.x; j < k; j += 64) m = fmax(m, isfinite(v[j]) ? v[j] : INFINITY);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o));
    if (threadIdx.x == 0) {
        if (mx) mx[z * mx_bs] = m;
        if (!(m <= thr)) flag[z] |= bit;
    }
}

int np_of(int nb) {
    // fixed partial count for a given batch size: reductions are bit-reproducible
    return nb == 1 ? kRedBlocks : std::max(16, std::min(kRedBlocks, 4096 / nb));
}

}  // namespace

void permute(const double* in, double* out, const PermDesc& d, double alpha, double beta,
             const double* scale_dev, i64 scale_bs, hipStream_t s) {
    PermK k = make_perm(d);
    hipLaunchKernelGGL((permute_kernel<double, 0>), grid2(k.total, d.nb), dim3(256), 0, s, in, (void*)out, k, d.in_bs,
                       d.out_bs, alpha, beta, scale_dev, scale_bs);
    DTRG_HIP(hipGetLastError());
}

void permute_out(const double* in, void* out, int out_code, const PermDesc& d, double alpha, const double* scale_dev,
                 i64 scale_bs, hipStream_t s) {
    DTRG_REQUIRE(out_code >= 0 && out_code <= 3, DTRG_EINVAL, "permute: bad output format");
    PermK k = make_perm(d, out_code >= 2 ? out_code : 1);
    const dim3 g = grid2(k.total, d.nb);
    switch (out_code) {
        case 0: hipLaunchKernelGGL((permute_kernel<double, 0>), g, dim3(256), 0, s, in, out, k, d.in_bs, d.out_bs, alpha,
                                   0.0, scale_dev, scale_bs); break;
        case 1: hipLaunchKernelGGL((permute_kernel<double, 1>), g, dim3(256), 0, s, in, out, k, d.in_bs, d.out_bs, alpha,
                                   0.0, scale_dev, scale_bs); break;
        case 2: hipLaunchKernelGGL((permute_kernel<double, 2>), g, dim3(256), 0, s, in, out, k, d.in_bs, d.out_bs, alpha,
                                   0.0, scale_dev, scale_bs); break;
        default: hipLaunchKernelGGL((permute_kernel<double, 3>), g, dim3(256), 0, s, in, out, k, d.in_bs, d.out_bs,
                                    alpha, 0.0, scale_dev, scale_bs); break;
    }
    DTRG_HIP(hipGetLastError());
}

void split_matrix(const float* in, i64 ld_in, bool kmajor, int rows, int cols, void* out, i64 ld_out, i64 ps, int np,
                  hipStream_t s) {
    DTRG_REQUIRE(np == 2 || np == 3, DTRG_EINVAL, "split_matrix: 2 or 3 planes");
    const dim3 g = grid2((i64)rows * cols, 1);
    if (np == 2) hipLaunchKernelGGL((split_matrix_kernel<2>), g, dim3(256), 0, s, in, ld_in, kmajor ? 1 : 0, rows, cols,
                                    out, ld_out, ps);
    else hipLaunchKernelGGL((split_matrix_kernel<3>), g, dim3(256), 0, s, in, ld_in, kmajor ? 1 : 0, rows, cols, out,
                            ld_out, ps);
    DTRG_HIP(hipGetLastError());
}

void convert_f64_to_f32(const double* in, i64 in_bs, float* out, i64 out_bs, i64 n, int nb, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(convert_kernel, grid2(n, nb), dim3(256), 0, s, in, in_bs, out, out_bs, n);
    DTRG_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void eye_kernel(double* p, i64 bs, int rows, int cols) {
    p += blockIdx.y * bs;
    const i64 total = (i64)rows * cols;
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < total; i += (i64)gridDim.x * blockDim.x)
        p[i] = (i / cols == i % cols) ? 1.0 : 0.0;
}

void eye(double* p, i64 bs, int rows, int cols, int nb, hipStream_t s) {
    hipLaunchKernelGGL(eye_kernel, grid2((i64)rows * cols, nb), dim3(256), 0, s, p, bs, rows, cols);
    DTRG_HIP(hipGetLastError());
}

void fill(double* p, i64 bs, i64 n, int nb, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, grid2(n, nb), dim3(256), 0, s, p, bs, n, v);
    DTRG_HIP(hipGetLastError());
}

void axpy(const double* x, double* y, i64 bs, i64 n, int nb, double a, hipStream_t s, const double* sc, i64 sc_bs) {
    if (n <= 0) return;
    hipLaunchKernelGGL(axpy_kernel, grid2(n, nb), dim3(256), 0, s, x, y, bs, n, a, sc, sc_bs);
    DTRG_HIP(hipGetLastError());
}

void scale_inplace(double* p, i64 bs, i64 n, int nb, double alpha, const double* scale_dev, i64 scale_bs,
                   bool reciprocal, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_kernel, grid2(n, nb), dim3(256), 0, s, p, bs, n, alpha, scale_dev, scale_bs,
                       reciprocal ? 1 : 0);
    DTRG_HIP(hipGetLastError());
}

void norm2(const double* x, i64 bs, i64 n, int nb, double* out_dev, i64 out_bs, hipStream_t s, Scratch& ws) {
    const int np = np_of(nb);
    ws.red.ensure((size_t)np * nb);
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(np, nb), dim3(256), 0, s, x, (const double*)nullptr, bs, n, ws.red.p);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(nb), dim3(256), 0, s, (const double*)ws.red.p, np, out_dev, out_bs, 1);
    DTRG_HIP(hipGetLastError());
}

void dot(const double* x, const double* y, i64 bs, i64 n, int nb, double* out_dev, i64 out_bs, hipStream_t s,
         Scratch& ws) {
    const int np = np_of(nb);
    ws.red.ensure((size_t)np * nb);
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(np, nb), dim3(256), 0, s, x, y, bs, n, ws.red.p);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(nb), dim3(256), 0, s, (const double*)ws.red.p, np, out_dev, out_bs, 0);
    DTRG_HIP(hipGetLastError());
}

void trace_xxyy(const double* T, i64 bs, int X, int Y, int nb, double* out_dev, i64 out_bs, hipStream_t s) {
    hipLaunchKernelGGL(trace_xxyy_kernel, dim3(nb), dim3(256), 0, s, T, bs, X, Y, out_dev, out_bs);
    DTRG_HIP(hipGetLastError());
}

void sym_normalise(double* G, i64 bs, int n, int nb, double* t_dev, i64 t_bs, int* flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(diag_sum_kernel, dim3(nb), dim3(256), 0, s, (const double*)G, bs, n, t_dev, t_bs, flag_dev);
    hipLaunchKernelGGL(sym_norm_kernel, grid2((i64)n * n, nb), dim3(256), 0, s, G, bs, n, (const double*)t_dev, t_bs);
    DTRG_HIP(hipGetLastError());
}

void accum_log(const double* x_dev, double weight, double* L_dev, double* inv_dev, i64 sc_bs, int nb, int* flag_dev,
               hipStream_t s) {
    hipLaunchKernelGGL(accum_log_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, x_dev, weight, L_dev, inv_dev, sc_bs,
                       nb, flag_dev);
    DTRG_HIP(hipGetLastError());
}

void fill_int(int* p, i64 n, int v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_int_kernel, grid2(n, 1), dim3(256), 0, s, p, n, v);
    DTRG_HIP(hipGetLastError());
}

void seed_trace_grad(double* T, i64 bs, int X, int Y, int nb, double gbar_weight, const double* tr_dev, i64 tr_bs,
                     hipStream_t s) {
    hipLaunchKernelGGL(seed_kernel, grid2((i64)X * X * Y * Y, nb), dim3(256), 0, s, T, bs, X, Y, gbar_weight, tr_dev,
                       tr_bs);
    DTRG_HIP(hipGetLastError());
}

void hash_fill(double* p, i64 bs, i64 n, int nb, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(hash_fill_kernel, grid2(n, nb), dim3(256), 0, s, p, bs, n, seed);
    DTRG_HIP(hipGetLastError());
}

void copy2d(const double* src, i64 lds, i64 src_bs, double* dst, i64 ldd, i64 dst_bs, int rows, int cols, int nb,
            hipStream_t s) {
    if ((i64)rows * cols <= 0) return;
    hipLaunchKernelGGL(copy2d_kernel, grid2((i64)rows * cols, nb), dim3(256), 0, s, src, lds, src_bs, dst, ldd, dst_bs,
                       rows, cols);
    DTRG_HIP(hipGetLastError());
}

void gather_rows(const double* src, i64 src_bs, const int* idx_dev, double* dst, i64 dst_bs, i64 len, int nb,
                 bool scatter, hipStream_t s) {
    if (len <= 0 || nb <= 0) return;
    hipLaunchKernelGGL(gather_kernel, grid2(len, nb), dim3(256), 0, s, src, src_bs, idx_dev, dst, dst_bs, len,
                       scatter ? 1 : 0);
    DTRG_HIP(hipGetLastError());
}

void max_check(const double* v, i64 v_bs, int k, int nb, double thr, double* mx_dev, i64 mx_bs, int* flag_dev,
               int bit, hipStream_t s) {
    hipLaunchKernelGGL(max_check_kernel, dim3(nb), dim3(64), 0, s, v, v_bs, k, thr, mx_dev, mx_bs, flag_dev, bit);
    DTRG_HIP(hipGetLastError());
}

}  // namespace dtrg
