// Small dense FP64 eigen kernels of the truncated eigensolve and its adjoint (gfx950).
//
// * jacobi_eig: one workgroup holds an n x n symmetric matrix and its eigenvector accumulator in
//   LDS (n <= 96: 2 x 96 x 97 doubles = 146 KiB of the 160 KiB LDS) and runs cyclic Jacobi in the
//   round-robin (Berger table) order: in every round n/2 disjoint index pairs are rotated at once,
//   rows first, then columns, each pass with one thread per row (or column) element of a pair, so
//   that a wave touches consecutive LDS words.  A pair is rotated while |a_pq| > 1e-16
//   sqrt(|a_pp a_qq|) and above an absolute floor (floor_rel |A|_F: 2^-60 for the spectra of the
//   eigensolver, which reach the FP64 floor; the callers may raise it to the rounding level of the
//   matrix, where rotations among large entries keep leaving residues of about u |A| next to small
//   eigenvalues), which keeps small eigenvalues to high relative accuracy.  (One pass over the disjoint 2 x 2 blocks of pair rows and pair columns, with one
//   barrier less per round, measured 40% slower: its LDS accesses scatter over the banks.)
// * chol_inverse: Cholesky of a (shifted) b x b Gram in LDS and the inverse of its triangular
//   factor, for CholeskyQR of the subspace block.  It can report whether the Gram is the identity
//   to a tolerance (the block is nearly orthonormal), and a later call can skip its work on that
//   report and return the identity.
// * element-wise helpers for Ritz residuals, column normalisation, the broadened inverse gaps of
//   the eigenvector adjoint and the Chebyshev expansion of the complement (interval, node values,
//   three-term recurrence, coefficient tail and boundedness checks).
// Every kernel serves nb independent instances (one workgroup or one y-slice of the grid each).
#include "common.hpp"

#include <algorithm>

namespace dtrg {

namespace {

constexpr int JM = kJacobiMax;
constexpr int JLD = JM + 1;
static_assert(JM <= 128, "one row or column element per thread of a group");
constexpr int CG = 32;              // Cholesky / inverse: a CG x CG thread grid for the updates
constexpr int CT = CG * CG;         // (16 waves)

// GW: threads per group, one row (or column) element each, so n <= GW; JT threads in all (a single
// wave is slower: the row and column updates need the width).  12 waves, in groups of GW = 64 for
// n <= 64 and of GW = 96 for n <= 96 (a group may then straddle two waves): every thread of a group
// has an element, and the 12 or 8 groups share the pairs of a round.
template <int GW, int JT>
__global__ __launch_bounds__(JT) void jacobi_kernel(const double* __restrict__ Ain, int n, int lda, i64 a_bs,
                                                     double* __restrict__ lam, i64 lam_bs, double* __restrict__ Vout,
                                                     int ldv, i64 v_bs, int max_sweeps, int* sweeps_out,
                                                     int* flag, int flag_bit, double floor_rel) {
    constexpr int JG = JT / GW;                  // groups
    constexpr int JS = (JM / 2 + JG - 1) / JG;   // pair slots per group
    __shared__ double A[JM * JLD];
    __shared__ double V[JM * JLD];
    __shared__ int rp[JM / 2], rq[JM / 2];
    __shared__ double rc[JM / 2], rs[JM / 2];
    __shared__ int nrot, nact, any_active;
    __shared__ double fro;
    const int tid = threadIdx.x;
    Ain += blockIdx.x * a_bs;
    lam += blockIdx.x * lam_bs;
    Vout += blockIdx.x * v_bs;
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
    const double abs_floor = floor_rel * fro + 1e-300;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // A sweep in which no pair passes the rotation test leaves the matrix as it is, so every round
        // of it sees the matrix the sweep started from: the test over all pairs at once decides that
        // case without running the rounds (the result is the same as running them).
        if (tid == 0) any_active = 0;
        __syncthreads();
        {
            int mine = 0;
            for (int i = tid; i < n * n && !mine; i += JT) {
                const int p = i / n, q = i % n;
                if (q <= p) continue;
                const double apq = A[p * JLD + q];
                const double app = A[p * JLD + p], aqq = A[q * JLD + q];
                mine = fabs(apq) > fmax(1e-16 * sqrt(fabs(app * aqq)), abs_floor);
            }
            if (mine) any_active = 1;
        }
        __syncthreads();
        if (!any_active) break;
        if (tid == 0) nrot = 0;
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            // the n/2 pairs of this round are handled by wave 0 (m/2 <= 48 lanes); the pairs that
            // need a rotation are compacted into slots 0..nact-1
            if (tid < 64) {
                int p = 0, q = 0, active = 0;
                double c = 1.0, sn = 0.0;
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
                            sn = t * c;
                            active = 1;
                        }
                    }
                }
                const unsigned long long mask = __ballot(active);
                const int slot = __popcll(mask & ((1ull << tid) - 1ull));
                if (active) { rp[slot] = p; rq[slot] = q; rc[slot] = c; rs[slot] = sn; }
                if (tid == 0) { nact = __popcll(mask); nrot += nact; }
            }
            __syncthreads();
            const int na = nact;
            if (na > 0) {
                // Slot i = g + JG t of group g (GW threads) is one active pair; thread l of the group
                // takes column l of its two rows, then row l of its two columns (and of V).  A
                // round's pairs are disjoint, so a thread issues every LDS read of a pass before its
                // first store: one round trip per pass instead of one per pair.
                const int g = tid / GW, l = tid % GW;
                const bool lv = l < n;
                const int lc = lv ? l : n - 1;
                const int ns = (na - g + JG - 1) / JG;   // active slots of this group
                int sp[JS], sq[JS];
                double sc[JS], ss[JS];
#pragma unroll
                for (int t = 0; t < JS; ++t) {
                    if (t >= ns) continue;
                    const int i = g + JG * t;
                    sp[t] = rp[i]; sq[t] = rq[i]; sc[t] = rc[i]; ss[t] = rs[i];
                }
                // rows: row_p <- c row_p - s row_q ; row_q <- s row_p + c row_q
                {
                    double ap[JS], aq[JS];
#pragma unroll
                    for (int t = 0; t < JS; ++t) {
                        if (t >= ns) continue;
                        ap[t] = A[sp[t] * JLD + lc];
                        aq[t] = A[sq[t] * JLD + lc];
                    }
#pragma unroll
                    for (int t = 0; t < JS; ++t) {
                        if (t >= ns || !lv) continue;
                        A[sp[t] * JLD + l] = sc[t] * ap[t] - ss[t] * aq[t];
                        A[sq[t] * JLD + l] = ss[t] * ap[t] + sc[t] * aq[t];
                    }
                }
                __syncthreads();
                // columns of A and of V
                {
                    double ap[JS], aq[JS], vp[JS], vq[JS];
#pragma unroll
                    for (int t = 0; t < JS; ++t) {
                        if (t >= ns) continue;
                        ap[t] = A[lc * JLD + sp[t]];
                        aq[t] = A[lc * JLD + sq[t]];
                        vp[t] = V[lc * JLD + sp[t]];
                        vq[t] = V[lc * JLD + sq[t]];
                    }
#pragma unroll
                    for (int t = 0; t < JS; ++t) {
                        if (t >= ns || !lv) continue;
                        A[l * JLD + sp[t]] = sc[t] * ap[t] - ss[t] * aq[t];
                        A[l * JLD + sq[t]] = ss[t] * ap[t] + sc[t] * aq[t];
                        V[l * JLD + sp[t]] = sc[t] * vp[t] - ss[t] * vq[t];
                        V[l * JLD + sq[t]] = ss[t] * vp[t] + sc[t] * vq[t];
                    }
                }
            }
            __syncthreads();
        }
        const int done = (nrot == 0);
        __syncthreads();
        if (done) break;
    }
    // every sweep still rotated something: the matrix is not diagonal to the rotation threshold
    if (tid == 0 && flag && sweep >= max_sweeps) atomicOr(flag + blockIdx.x, flag_bit);
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
    if (tid == 0 && sweeps_out) atomicMax(sweeps_out, sweep);
}

// Lower Cholesky factor L of (S + shift I) in LDS (right-looking, rank-1 trailing updates in
// parallel), then X = L^{-1} by the same elimination applied to the identity (row k of X is
// final after step k, rows below get a parallel rank-1 update), Rinv = X^T to global.  The
// updates run on a CG x CG thread grid, one barrier per column (or row).
//
// An unshifted S = I + E with |E|_F <= kCholSeries (the Gram of a block that one CholeskyQR pass has
// made orthonormal to about that) takes the series instead: with G1 = Phi(E) and
// Phi(M) = (strict lower part of M) + diag(M)/2, the factor is L = I + G1 - Phi(G1 G1^T) + O(|E|^3)
// (from L L^T = I + E order by order), and its inverse
//   X = I - G1 + Phi(G1 G1^T) + G1 G1 + O(|E|^3),
// exact to rounding for |E|_F <= 2^-20 (|E|^3 <= 2^-60).  Two triangular b^3 products with no
// barrier between columns, against 2b barriers of the elimination.
constexpr double kCholSeries = 0x1p-20;

__global__ __launch_bounds__(CT) void chol_inv_kernel(const double* __restrict__ S, i64 s_bs, int b,
                                                       double shift_rel, double* __restrict__ Rinv, i64 r_bs,
                                                       int* flag, const int* __restrict__ skip, int* __restrict__ near,
                                                       double near_tol) {
    __shared__ double L[JM * JLD];
    __shared__ double Xs[JM * JLD];
    __shared__ double tr, efro2;
    __shared__ double wmax[CT / 64], wsum[CT / 64];
    const int tid = threadIdx.x;
    S += blockIdx.x * s_bs;
    Rinv += blockIdx.x * r_bs;
    flag += blockIdx.x;
    if (skip && skip[blockIdx.x]) {
        // the block is orthonormal to working accuracy already: R^{-1} = I
        for (int idx = tid; idx < b * b; idx += CT) Rinv[(i64)(idx / b) * b + idx % b] = (idx / b == idx % b) ? 1.0 : 0.0;
        return;
    }
    double dev = 0.0, e2 = 0.0;
    for (int i = tid; i < b * b; i += CT) {
        const int r = i / b, c = i % b;
        const double v = 0.5 * (S[(i64)r * b + c] + S[(i64)c * b + r]);
        L[r * JLD + c] = v;
        Xs[r * JLD + c] = (r == c) ? 1.0 : 0.0;
        const double e = v - (r == c ? 1.0 : 0.0);
        dev = fmax(dev, fabs(e));   // fmax drops a NaN: checked below
        e2 += e * e;                // a NaN stays: the series test below fails on it
        if (!isfinite(v)) dev = INFINITY;
    }
    for (int o = 32; o > 0; o >>= 1) {
        dev = fmax(dev, __shfl_xor(dev, o));
        e2 += __shfl_xor(e2, o);
    }
    if ((tid & 63) == 0) {
        wmax[tid >> 6] = dev;
        wsum[tid >> 6] = e2;
    }
    __syncthreads();
    if (tid == 0) {
        double s2 = 0.0;
        for (int w = 0; w < CT / 64; ++w) s2 += wsum[w];
        efro2 = s2;
    }
    if (near && tid == 0) {
        double m = 0.0;
        for (int w = 0; w < CT / 64; ++w) m = fmax(m, wmax[w]);
        near[blockIdx.x] = m <= near_tol ? 1 : 0;
    }
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < b; ++i) s += L[i * JLD + i];
        tr = s;
    }
    __syncthreads();
    const int tx = tid % CG, ty = tid / CG;
    if (shift_rel == 0.0 && efro2 <= kCholSeries * kCholSeries) {
        // the series: G1 = Phi(S - I) in L (the strict upper part zeroed)
        for (int i = tid; i < b * b; i += CT) {
            const int r = i / b, c = i % b;
            const double e = L[r * JLD + c] - (r == c ? 1.0 : 0.0);
            L[r * JLD + c] = r > c ? e : (r == c ? 0.5 * e : 0.0);
        }
        __syncthreads();
        // X[i][j] (i >= j) = delta_ij - G1[i][j] + Phi(M)[i][j] + (G1 G1)[i][j], with
        // M[i][j] = sum_{k <= j} G1[i][k] G1[j][k] and (G1 G1)[i][j] = sum_{j <= k <= i} G1[i][k] G1[k][j]
        for (int i = ty; i < b; i += CG)
            for (int j = tx; j <= i; j += CG) {
                double m = 0.0, p = 0.0;
                for (int k = 0; k <= j; ++k) m += L[i * JLD + k] * L[j * JLD + k];
                for (int k = j; k <= i; ++k) p += L[i * JLD + k] * L[k * JLD + j];
                Xs[i * JLD + j] = (i == j ? 1.0 : 0.0) - L[i * JLD + j] + (i > j ? m : 0.5 * m) + p;
            }
        __syncthreads();
        for (int idx = tid; idx < b * b; idx += CT) {
            const int i = idx / b, j = idx % b;
            Rinv[(i64)i * b + j] = (i <= j) ? Xs[j * JLD + i] : 0.0;
        }
        return;
    }
    const double shift = shift_rel * tr;
    for (int i = tid; i < b; i += CT) L[i * JLD + i] += shift;
    __syncthreads();
    // Cholesky, right-looking, one barrier per column: phase k takes the pivot and column k as phase
    // k-1 left them, applies the rank-1 update with the scaled column to the trailing lower
    // triangle, and writes back the scaled column k-1, which phase k no longer reads
    double dprev = 1.0, rprev = 1.0;
    for (int k = 0; k <= b; ++k) {
        if (k > 0) {
            for (int i = k + tid; i < b; i += CT) L[i * JLD + k - 1] *= rprev;
            if (tid == 0) L[(k - 1) * JLD + k - 1] = dprev;
        }
        if (k == b) break;
        double d = L[k * JLD + k];
        if (!(d > 0.0) || !isfinite(d)) {
            if (tid == 0) flag[0] |= 2;
            d = 1e-300;
        }
        const double dk = sqrt(d), rdk = 1.0 / dk;
        for (int i = k + 1 + ty; i < b; i += CG) {
            const double lik = L[i * JLD + k] * rdk;
            for (int j = k + 1 + tx; j <= i; j += CG) L[i * JLD + j] -= lik * (L[j * JLD + k] * rdk);
        }
        dprev = dk;
        rprev = rdk;
        __syncthreads();
    }
    __syncthreads();   // the scaled last column and pivot, written after the last phase's barrier
    // X = L^{-1}, one barrier per row: phase k removes row k, scaled by 1 / L[k][k], from the rows
    // below and writes back the scaled row k-1, which phase k no longer reads
    double inv_prev = 1.0;
    for (int k = 0; k <= b; ++k) {
        if (k > 0)
            for (int j = tid; j < k; j += CT) Xs[(k - 1) * JLD + j] *= inv_prev;
        if (k == b) break;
        const double inv = 1.0 / L[k * JLD + k];
        for (int i = k + 1 + ty; i < b; i += CG) {
            const double lik = L[i * JLD + k];
            for (int j = tx; j <= k; j += CG) Xs[i * JLD + j] -= lik * (Xs[k * JLD + j] * inv);
        }
        inv_prev = inv;
        __syncthreads();
    }
    // the last phase scaled row b-1 of X after its barrier: every thread's scaling must land before
    // any thread reads X below
    __syncthreads();
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

__global__ __launch_bounds__(256) void col_norms_kernel(const double* V, int n, int ldv, i64 v_bs, double* out,
                                                         i64 out_bs) {
    const int j = blockIdx.x;
    V += blockIdx.y * v_bs;
    out += blockIdx.y * out_bs;
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

__global__ __launch_bounds__(256) void col_normalise_kernel(double* V, int n, int b, int ldv, i64 v_bs,
                                                             const double* nrm, i64 nrm_bs, uint64_t seed) {
    V += blockIdx.y * v_bs;
    nrm += blockIdx.y * nrm_bs;
    if (blockIdx.y) seed = mix64(seed ^ (0x5bd1e995ULL + blockIdx.y));
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

__global__ __launch_bounds__(256) void ritz_res_kernel(const double* V, const double* Y, int n, int ld, i64 v_bs,
                                                        const double* theta, i64 th_bs, double* res, i64 res_bs) {
    const int j = blockIdx.x;
    V += blockIdx.y * v_bs;
    Y += blockIdx.y * v_bs;
    theta += blockIdx.y * th_bs;
    res += blockIdx.y * res_bs;
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

// S = [[0, R], [R^T, 0]] (2K x 2K, ld 2K) from R (K x K, ld K)
__global__ __launch_bounds__(256) void sym_augment_kernel(const double* R, i64 r_bs, int K, double* S, i64 s_bs) {
    R += blockIdx.y * r_bs;
    S += blockIdx.y * s_bs;
    const int m = 2 * K;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < m * m; idx += gridDim.x * blockDim.x) {
        const int i = idx / m, j = idx % m;
        double v = 0.0;
        if (i < K && j >= K) v = R[i * K + (j - K)];
        else if (i >= K && j < K) v = R[j * K + (i - K)];
        S[idx] = v;
    }
}

__global__ __launch_bounds__(256) void kept_block_kernel(const double* Om, i64 om_bs, const double* lam,
                                                          i64 lam_bs, int k, double eps, double* S, i64 s_bs) {
    Om += blockIdx.y * om_bs;
    lam += blockIdx.y * lam_bs;
    S += blockIdx.y * s_bs;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < k * k; idx += gridDim.x * blockDim.x) {
        const int i = idx / k, j = idx % k;
        S[idx] = (i == j) ? 0.0 : bgap(lam[j] - lam[i], eps) * 0.5 * (Om[i * k + j] - Om[j * k + i]);
    }
}

__global__ __launch_bounds__(256) void over_block_kernel(const double* Om, i64 om_bs, const double* lam,
                                                          i64 lam_bs, int p, int k, double eps, double* M, i64 m_bs) {
    Om += blockIdx.y * om_bs;
    lam += blockIdx.y * lam_bs;
    M += blockIdx.y * m_bs;
    const double* theta = lam + k;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < p * k; idx += gridDim.x * blockDim.x) {
        const int i = idx / k, j = idx % k;
        M[idx] = bgap(lam[j] - theta[i], eps) * 0.5 * Om[idx];
    }
}

__global__ __launch_bounds__(256) void cheb_step_kernel(const double* Y, const double* Vc, const double* Vp,
                                                         double* Vn, double* X, i64 bs, int n, int k,
                                                         const double* lohi, i64 lohi_bs, int first,
                                                         const double* coef, i64 coef_bs) {
    const int z = blockIdx.y;
    const i64 o = z * bs;
    const double lo = lohi[z * lohi_bs], hi = lohi[z * lohi_bs + 1];
    const double a = (first ? 1.0 : 2.0) / (hi - lo), sum = hi + lo;
    coef += z * coef_bs;
    const i64 total = (i64)n * k;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int j = (int)(idx % k);
        const double vc = Vc[o + idx];
        double v = a * (2.0 * Y[o + idx] - sum * vc);
        if (!first) v -= Vp[o + idx];
        Vn[o + idx] = v;
        if (first) X[o + idx] += coef[j] * vc + coef[k + j] * v;
        else X[o + idx] += coef[j] * v;
    }
}

__global__ void cheb_interval_kernel(const double* th, i64 th_bs, int e, const double* rn, i64 rn_bs, int n,
                                     double mult, double* lohi, i64 lohi_bs, int nb) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nb) return;
    const double* t = th + z * th_bs;
    const double nu = 64.0 * n * 0x1p-53 * fmax(t[0], 0.0);
    const double hi = mult * (fmax(1.1 * (fmax(t[e], 0.0) + rn[z * rn_bs]), nu) + 1e-300);
    lohi[z * lohi_bs] = -fmax(nu, 0.05 * hi);
    lohi[z * lohi_bs + 1] = hi;
}

__global__ __launch_bounds__(256) void cheb_table_kernel(double* ct, int m) {
    const int N = m + 1;
    const i64 total = (i64)N * N;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int q = (int)(idx / N), k = (int)(idx % N);
        // q (k + 1/2) / N reduced modulo 2 keeps the argument of cospi small and exact
        const i64 num = (i64)q * (2 * k + 1) % (4 * (i64)N);
        ct[idx] = (q == 0 ? 1.0 : 2.0) / N * cospi((double)num / (2.0 * N));
    }
}

__global__ __launch_bounds__(256) void cheb_fvals_kernel(const double* lam, i64 lam_bs, int K, double eps,
                                                          const double* lohi, i64 lohi_bs, int m, double* fv,
                                                          i64 fv_bs) {
    const int z = blockIdx.y;
    lam += z * lam_bs;
    fv += z * fv_bs;
    const double lo = lohi[z * lohi_bs], hi = lohi[z * lohi_bs + 1];
    const int N = m + 1;
    const i64 total = (i64)N * K;
    for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
        const int k = (int)(idx / K), j = (int)(idx % K);
        const double x = cospi((2.0 * k + 1.0) / (2.0 * N));
        const double t = 0.5 * (hi - lo) * x + 0.5 * (hi + lo);
        const double d = lam[j] - t;
        fv[idx] = 0.5 * d / (d * d + eps);
    }
}

__global__ __launch_bounds__(256) void cheb_tail_kernel(const double* coef, i64 coef_bs, int m, int K, double* ratio,
                                                         i64 ratio_bs) {
    const int z = blockIdx.x;
    coef += z * coef_bs;
    double mx = 0.0, tail = 0.0;
    const i64 total = (i64)(m + 1) * K;
    for (i64 idx = threadIdx.x; idx < total; idx += 256) {
        const double a = fabs(coef[idx]);
        const double a2 = isfinite(a) ? a : INFINITY;
        mx = fmax(mx, a2);
        if (idx / K >= m - 1) tail = fmax(tail, a2);
    }
    __shared__ double s1[256], s2[256];
    s1[threadIdx.x] = mx;
    s2[threadIdx.x] = tail;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + st]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ratio[z * ratio_bs] = s1[0] > 0.0 ? s2[0] / s1[0] : 0.0;
}

__global__ void cheb_bound_kernel(const double* vm, const double* v0, i64 bs, int nb, int* flag, int bit) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nb) return;
    const double a = vm[z * bs], b = v0[z * bs];
    if (!(isfinite(a) && isfinite(b) && a <= 1.5 * b)) flag[z] |= bit;
}

dim3 grid2(i64 n, int nb) {
    const i64 per = std::max<i64>(1, std::min<i64>((n + 255) / 256, std::max<i64>(1, 8192 / nb)));
    return dim3((unsigned)per, (unsigned)nb);
}

}  // namespace

void jacobi_eig(const double* A, int n, int lda, i64 a_bs, double* lam_dev, i64 lam_bs, double* V, int ldv, i64 v_bs,
                int nb, int max_sweeps, int* sweeps_dev, hipStream_t s, int* flag_dev, int flag_bit, double floor_rel) {
    DTRG_REQUIRE(n >= 1 && n <= kJacobiMax, DTRG_EINVAL, "jacobi_eig: n out of range");
    static_assert(kJacobiMax <= 96, "the widest Jacobi group has 96 threads");
    if (n <= 64)
        hipLaunchKernelGGL((jacobi_kernel<64, 768>), dim3(nb), dim3(768), 0, s, A, n, lda, a_bs, lam_dev, lam_bs, V,
                           ldv, v_bs, max_sweeps, sweeps_dev, flag_dev, flag_bit, floor_rel);
    else
        hipLaunchKernelGGL((jacobi_kernel<96, 768>), dim3(nb), dim3(768), 0, s, A, n, lda, a_bs, lam_dev, lam_bs, V,
                           ldv, v_bs, max_sweeps, sweeps_dev, flag_dev, flag_bit, floor_rel);
    DTRG_HIP(hipGetLastError());
}

void chol_inverse(const double* S, i64 s_bs, int b, double shift_rel, double* Rinv, i64 r_bs, int nb, int* flag_dev,
                  hipStream_t s, const int* skip_dev, int* near_dev, double near_tol) {
    DTRG_REQUIRE(b >= 1 && b <= kJacobiMax, DTRG_EINVAL, "chol_inverse: b out of range");
    DTRG_REQUIRE(flag_dev, DTRG_EINVAL, "chol_inverse: flag array required");
    hipLaunchKernelGGL(chol_inv_kernel, dim3(nb), dim3(CT), 0, s, S, s_bs, b, shift_rel, Rinv, r_bs, flag_dev,
                       skip_dev, near_dev, near_tol);
    DTRG_HIP(hipGetLastError());
}

void col_norms(const double* V, int n, int b, int ldv, i64 v_bs, double* out_dev, i64 out_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(col_norms_kernel, dim3(b, nb), dim3(256), 0, s, V, n, ldv, v_bs, out_dev, out_bs);
    DTRG_HIP(hipGetLastError());
}

void col_normalise(double* V, int n, int b, int ldv, i64 v_bs, const double* nrm_dev, i64 nrm_bs, int nb,
                   uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(col_normalise_kernel, grid2((i64)n * b, nb), dim3(256), 0, s, V, n, b, ldv, v_bs, nrm_dev,
                       nrm_bs, seed);
    DTRG_HIP(hipGetLastError());
}

void ritz_residuals(const double* V, const double* Y, int n, int k, int ld, i64 v_bs, const double* theta_dev,
                    i64 th_bs, double* res_dev, i64 res_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(ritz_res_kernel, dim3(k, nb), dim3(256), 0, s, V, Y, n, ld, v_bs, theta_dev, th_bs, res_dev,
                       res_bs);
    DTRG_HIP(hipGetLastError());
}

void sym_augment(const double* R, i64 r_bs, int K, double* S, i64 s_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(sym_augment_kernel, grid2((i64)4 * K * K, nb), dim3(256), 0, s, R, r_bs, K, S, s_bs);
    DTRG_HIP(hipGetLastError());
}

void kept_block_adjoint(const double* Om, i64 om_bs, const double* lam_dev, i64 lam_bs, int k, double eps, double* S,
                        i64 s_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(kept_block_kernel, grid2((i64)k * k, nb), dim3(256), 0, s, Om, om_bs, lam_dev, lam_bs, k, eps,
                       S, s_bs);
    DTRG_HIP(hipGetLastError());
}

void over_block_adjoint(const double* Om, i64 om_bs, const double* lam_dev, i64 lam_bs, int p, int k, double eps,
                        double* M, i64 m_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(over_block_kernel, grid2((i64)p * k, nb), dim3(256), 0, s, Om, om_bs, lam_dev, lam_bs, p, k,
                       eps, M, m_bs);
    DTRG_HIP(hipGetLastError());
}

void cheb_step(const double* Y, const double* Vc, const double* Vp, double* Vn, double* X, i64 bs, int n, int k,
               const double* lohi_dev, i64 lohi_bs, bool first, const double* coef_dev, i64 coef_bs, int nb,
               hipStream_t s) {
    hipLaunchKernelGGL(cheb_step_kernel, grid2((i64)n * k, nb), dim3(256), 0, s, Y, Vc, Vp, Vn, X, bs, n, k, lohi_dev,
                       lohi_bs, first ? 1 : 0, coef_dev, coef_bs);
    DTRG_HIP(hipGetLastError());
}

void cheb_interval(const double* th, i64 th_bs, int e, const double* res_next, i64 rn_bs, int n, double mult,
                   double* lohi_dev, i64 lohi_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(cheb_interval_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, th, th_bs, e, res_next, rn_bs, n,
                       mult, lohi_dev, lohi_bs, nb);
    DTRG_HIP(hipGetLastError());
}

void cheb_table(double* ct, int m, hipStream_t s) {
    hipLaunchKernelGGL(cheb_table_kernel, grid2((i64)(m + 1) * (m + 1), 1), dim3(256), 0, s, ct, m);
    DTRG_HIP(hipGetLastError());
}

void cheb_fvals(const double* lam, i64 lam_bs, int K, double eps, const double* lohi_dev, i64 lohi_bs, int m,
                double* fv, i64 fv_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(cheb_fvals_kernel, grid2((i64)(m + 1) * K, nb), dim3(256), 0, s, lam, lam_bs, K, eps, lohi_dev,
                       lohi_bs, m, fv, fv_bs);
    DTRG_HIP(hipGetLastError());
}

void cheb_tail(const double* coef, i64 coef_bs, int m, int K, double* ratio_dev, i64 ratio_bs, int nb, hipStream_t s) {
    hipLaunchKernelGGL(cheb_tail_kernel, dim3(nb), dim3(256), 0, s, coef, coef_bs, m, K, ratio_dev, ratio_bs);
    DTRG_HIP(hipGetLastError());
}

void cheb_bound_check(const double* vm_dev, const double* v0_dev, i64 bs, int nb, int* flag_dev, int bit,
                      hipStream_t s) {
    hipLaunchKernelGGL(cheb_bound_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, vm_dev, v0_dev, bs, nb, flag_dev, bit);
    DTRG_HIP(hipGetLastError());
}

}  // namespace dtrg
