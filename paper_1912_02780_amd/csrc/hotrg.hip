// HOTRG forward pass, hand-written reverse pass and the C ABI (gfx950).
//
// Layouts (row-major, X = horizontal bond, Y = vertical bond, K = chi' kept, n = X^2, b = block):
//   T   [l][r][u][d] = [X][X][Y][Y]        step input (the paper's T_{x x' y y'})
//   A,B [a][b][j][k] = [X][X][Y][Y]        half-environments of the Gram
//   G   [(a,c)][(b,d)] = n x n             Gram of the (x1, x2) unfolding, then sym / trace
//   U   [n][b]                             eigenvectors (first K columns are w[x1][x2][alpha])
//   P1  [alpha][y][i][b][j]                upper copy times the left isometry
//   Q2  [alpha][y][z][i][m]                P1 joined with the lower copy over (b, j)  (chi^7)
//   T'  [alpha][beta][y][z]                step output; the next input is T'/c permuted (2,3,0,1)
// Every contraction is one call of the MFMA kernel, whose scatter epilogue writes each result
// directly in the layout its consumer reads (index maps written next to each call).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"

using namespace dtrg;

namespace {

thread_local std::string g_last_error;

struct StepShape {
    int X = 0, Y = 0, K = 0, n = 0, b = 0;
    int e = 0;          // leading eigenpairs resolved to full accuracy: the kept K plus the
                        // discarded ones nearest the cut (the rest of the block is a guard)
    bool full = false;
    bool mixed = false; // projection contractions of this step in the mixed precision
    double join_flops() const { return 2.0 * K * Y * X * (double)(Y * X) * (X * Y); }
};

struct StepCk {
    StepShape sh;
    DevBuf<double> T;      // normalised input [X][X][Y][Y]
    DevBuf<double> A, B;   // half-environments
    DevBuf<double> G;      // normalised Gram (kept for the complement solve when !full)
    DevBuf<double> U;      // [n][b]
    DevBuf<double> lam;    // b eigenvalues / Ritz values, descending
    std::vector<double> lam_h;
    double c = 0.0, t = 0.0, resid = 0.0;
    double res_next = 0.0;   // residual of the first Ritz pair beyond the resolved ones
    int iters = 0, cheb = 0;
};

double ldexp1(int e) { return std::ldexp(1.0, e); }

PermDesc pd4(i64 d0, i64 d1, i64 d2, i64 d3, int p0, int p1, int p2, int p3) {
    PermDesc d;
    d.rank = 4;
    d.in_dims[0] = d0; d.in_dims[1] = d1; d.in_dims[2] = d2; d.in_dims[3] = d3;
    d.perm[0] = p0; d.perm[1] = p1; d.perm[2] = p2; d.perm[3] = p3;
    return d;
}

PermDesc pd3(i64 d0, i64 d1, i64 d2, int p0, int p1, int p2) {
    PermDesc d;
    d.rank = 3;
    d.in_dims[0] = d0; d.in_dims[1] = d1; d.in_dims[2] = d2;
    d.perm[0] = p0; d.perm[1] = p1; d.perm[2] = p2;
    return d;
}

PermDesc pd5(const i64* dims, const int* perm) {
    PermDesc d;
    d.rank = 5;
    for (int i = 0; i < 5; ++i) { d.in_dims[i] = dims[i]; d.perm[i] = perm[i]; }
    return d;
}

// Chebyshev interpolation coefficients, on [lo, hi] at N = m + 1 first-kind nodes, of
//   g_j(t) = (1/2) d / (d^2 + eps),  d = lam_j - t   (the broadened inverse gap, halved),
// one column per kept eigenvalue: c[q][j], q = 0..m.
void cheb_coeffs(const std::vector<double>& lamK, double eps, double lo, double hi, int m,
                 std::vector<double>& c /* (m+1) x K */) {
    const int K = (int)lamK.size();
    const int N = m + 1;
    c.assign((size_t)N * K, 0.0);
    std::vector<double> fv((size_t)N * K), ct((size_t)N * N);
    for (int k = 0; k < N; ++k) {
        const double x = std::cos(M_PI * (k + 0.5) / N);
        const double t = 0.5 * (hi - lo) * x + 0.5 * (hi + lo);
        for (int j = 0; j < K; ++j) {
            const double d = lamK[j] - t;
            fv[(size_t)k * K + j] = 0.5 * d / (d * d + eps);
        }
    }
    for (int q = 0; q < N; ++q)
        for (int k = 0; k < N; ++k) ct[(size_t)q * N + k] = std::cos(M_PI * q * (k + 0.5) / N);
    for (int q = 0; q < N; ++q) {
        double* cq = &c[(size_t)q * K];
        const double w = (q == 0 ? 1.0 : 2.0) / N;
        for (int k = 0; k < N; ++k) {
            const double a = w * ct[(size_t)q * N + k];
            const double* f = &fv[(size_t)k * K];
            for (int j = 0; j < K; ++j) cq[j] += a * f[j];
        }
    }
}

}  // namespace

struct dtrg_plan {
    int D = 0, chi = 0, nsteps = 0;
    dtrg_options opt{};
    Prec prec = Prec::F64;
    hipStream_t s = nullptr;
    std::vector<StepCk> steps;
    bool fwd_ok = false;
    double lnZ = 0.0, c0 = 0.0, final_trace = 0.0;
    int Xf = 0, Yf = 0;
    // device scalars: 0 L, 1 c (current), 2 1/c, 3 trace of Gram, 4 final trace, 5 dot, 6 c0, 7 1/c0
    DevBuf<double> scal;
    DevBuf<int> flags;
    Scratch ws;
    // workspaces
    DevBuf<double> TA, TB, Tp, Tb, Tb2, Wt, Wt2, Tn, Tbar, Tbar2, Tpbar;
    DevBuf<double> P1, Q2, X5;
    DevBuf<double> Gw, Gt, Ub, Xe, Xc, Re, Om, Sm, Vc, Vp, Vn, Ye, We;
    DevBuf<double> V1, V2, Y1, Y2, H, Z, Rinv, Sg, th, res, nrm, coef;
    // contraction operands in FP32 (FP32 and split-bf16 paths)
    DevBuf<float> Tpf, Tbf, Tb2f, Wtf, Wt2f, Uf, P1f, Q2f, X5f, Tpbarf;
    DevBuf<int> iflag;
    bool mixed() const { return prec != Prec::F64; }
    std::vector<StepShape> shape;
    // HIP-event timing of the chi^7 projection contractions (when opt.profile is set)
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_flops = 0.0;
    ~dtrg_plan() {
        for (auto e : ev_pool) (void)hipEventDestroy(e);
    }
    // bytes left in the plan-owned buffer that contains p (-1 if p is not plan memory)
    i64 cap_bytes(const void* p) const {
        const char* q = (const char*)p;
        auto chk = [&](const void* base, size_t nbytes) -> i64 {
            const char* b = (const char*)base;
            if (b && q >= b && q < b + nbytes) return (i64)nbytes - (i64)(q - b);
            return -1;
        };
        const DevBuf<double>* w[] = {&TA, &TB, &Tp, &Tb, &Tb2, &Wt, &Wt2, &Tn, &Tbar, &Tbar2, &Tpbar, &P1, &Q2, &X5,
                                     &Gw, &Gt, &Ub, &Xe, &Xc, &Re, &Om, &Sm, &Vc, &Vp, &Vn, &Ye, &We, &V1, &V2,
                                     &Y1, &Y2, &H, &Z, &Rinv, &Sg, &th, &res, &nrm, &coef, &scal};
        for (auto* b : w) { const i64 r = chk(b->p, b->bytes()); if (r >= 0) return r; }
        const DevBuf<float>* f[] = {&Tpf, &Tbf, &Tb2f, &Wtf, &Wt2f, &Uf, &P1f, &Q2f, &X5f, &Tpbarf};
        for (auto* b : f) { const i64 r = chk(b->p, b->bytes()); if (r >= 0) return r; }
        for (auto& st : steps) {
            const DevBuf<double>* v[] = {&st.T, &st.A, &st.B, &st.G, &st.U, &st.lam};
            for (auto* b : v) { const i64 r = chk(b->p, b->bytes()); if (r >= 0) return r; }
        }
        return -1;
    }
    i64 cap_of(const void* p, int elem = 8) const {
        const i64 b = cap_bytes(p);
        return b < 0 ? -1 : b / elem;
    }
    size_t bytes() const {
        size_t t = 0;
        for (auto& st : steps) t += st.T.bytes() + st.A.bytes() + st.B.bytes() + st.G.bytes() + st.U.bytes() + st.lam.bytes();
        const DevBuf<double>* w[] = {&TA, &TB, &Tp, &Tb, &Tb2, &Wt, &Wt2, &Tn, &Tbar, &Tbar2, &Tpbar, &P1, &Q2, &X5,
                                     &Gw, &Gt, &Ub, &Xe, &Xc, &Re, &Om, &Sm, &Vc, &Vp, &Vn, &Ye, &We, &V1, &V2,
                                     &Y1, &Y2, &H, &Z, &Rinv, &Sg, &th, &res, &nrm, &coef, &scal, &ws.splitk, &ws.red};
        for (auto* b : w) t += b->bytes();
        const DevBuf<float>* f[] = {&Tpf, &Tbf, &Tb2f, &Wtf, &Wt2f, &Uf, &P1f, &Q2f, &X5f, &Tpbarf};
        for (auto* b : f) t += b->bytes();
        return t;
    }
};

namespace {

// -------------------------------------------------------------------------------------------
// contractions of the step (FP64)
// -------------------------------------------------------------------------------------------
struct Ctx {
    dtrg_plan* P;
    hipStream_t s;
    // one contraction in precision `pr`; operands of 8 (FP64) or 4 (FP32) bytes, output FP64 or FP32
    void run(const GemmOp& op, Prec pr, bool out_f64) {
        GemmOp g = op;
        const int ein = pr == Prec::F64 ? 8 : 4, eout = out_f64 ? 8 : 4;
        if (g.a_cap < 0) g.a_cap = P->cap_of(g.A, ein);
        if (g.b_cap < 0) g.b_cap = P->cap_of(g.B, ein);
        if (g.c_cap < 0) g.c_cap = P->cap_of(g.C, eout);
        const bool timed = P->opt.profile && g.tag == 7;
        if (timed) {
            while (P->ev_pool.size() < P->ev_used + 2) {
                hipEvent_t e;
                DTRG_HIP(hipEventCreate(&e));
                P->ev_pool.push_back(e);
            }
            DTRG_HIP(hipEventRecord(P->ev_pool[P->ev_used], s));
        }
        dtrg::gemm(pr, out_f64, g, s, P->ws);
        if (timed) {
            DTRG_HIP(hipEventRecord(P->ev_pool[P->ev_used + 1], s));
            P->ev_used += 2;
            P->prof_flops += 2.0 * g.M * (double)g.N * g.K * g.batch;
        }
    }
    // FP64 contraction (Gram, eigensolver, eigen-adjoint)
    void gemm(const GemmOp& op) { run(op, Prec::F64, true); }
    // projection contraction in precision pr (FP64 operands always write FP64)
    void gemmc(const GemmOp& op, Prec pr, bool out_f64) { run(op, pr, pr == Prec::F64 ? true : out_f64); }
};

// permute with the capacities of plan-owned buffers checked on the host
void permute_checked(dtrg_plan* P, const double* in, double* out, PermDesc d, double alpha, double beta,
                     const double* scale_dev, hipStream_t s) {
    if (d.in_cap < 0) d.in_cap = P->cap_of(in);
    if (d.out_cap < 0) d.out_cap = P->cap_of(out);
    dtrg::permute(in, out, d, alpha, beta, scale_dev, s);
}

void permute_f32_checked(dtrg_plan* P, const double* in, float* out, PermDesc d, hipStream_t s) {
    if (d.in_cap < 0) d.in_cap = P->cap_of(in, 8);
    if (d.out_cap < 0) d.out_cap = P->cap_of(out, 4);
    dtrg::permute_to_f32(in, out, d, s);
}

void permute_ff_checked(dtrg_plan* P, const float* in, float* out, PermDesc d, hipStream_t s) {
    if (d.in_cap < 0) d.in_cap = P->cap_of(in, 4);
    if (d.out_cap < 0) d.out_cap = P->cap_of(out, 4);
    dtrg::permute_f32(in, out, d, s);
}

// A[a][b][j][k] = sum_{x,y} TA[(a,j)][(x,y)] TA[(b,k)][(x,y)]  (also B with TB)
void half_env(Ctx& c, const double* Tperm, double* out, int X, int Y) {
    GemmOp g;
    g.M = g.N = X * Y; g.K = X * Y;
    g.A = Tperm; g.lda = X * Y;
    g.B = Tperm; g.ldb = X * Y;
    g.C = out;
    g.rmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
    g.cmap = IdxMap::split(Y, (i64)Y * Y, 1);
    c.gemm(g);
}

// G[(a,c)][(b,d)] = sum_{(j,k)} A[(a,b),(j,k)] B[(c,d),(j,k)]
void gram(Ctx& c, const double* A, const double* B, double* G, int X, int Y) {
    GemmOp g;
    g.M = g.N = X * X; g.K = Y * Y;
    g.A = A; g.lda = Y * Y;
    g.B = B; g.ldb = Y * Y;
    g.C = G;
    g.rmap = IdxMap::split(X, (i64)X * X * X, X);
    g.cmap = IdxMap::split(X, (i64)X * X, 1);
    c.gemm(g);
}

// P1[alpha][y][i][b][j] = sum_a Wt[(alpha,b)][a] Tp[y][(i,j)][a]   (batched over y)
void proj1(Ctx& c, Prec pr, const void* Wt, const void* Tp, void* P1, int X, int Y, int K) {
    GemmOp g;
    g.M = K * X; g.N = X * Y; g.K = X; g.batch = Y;
    g.A = Wt; g.lda = X; g.a_bs = 0;
    g.B = Tp; g.ldb = X; g.b_bs = (i64)X * Y * X;
    g.C = P1; g.c_bs = (i64)X * X * Y;
    g.rmap = IdxMap::split(X, (i64)Y * X * X * Y, Y);
    g.cmap = IdxMap::split(Y, (i64)X * Y, 1);
    c.gemmc(g, pr, false);
}

// Q2[alpha][y][z][i][m] = sum_{(b,j)} P1[(alpha,y,i)][(b,j)] Tb[(z,m)][(b,j)]      (the chi^7 term)
void proj2(Ctx& c, Prec pr, const void* P1, const void* Tb, void* Q2, int X, int Y, int K) {
    GemmOp g;
    g.tag = 7;
    g.M = K * Y * X; g.N = Y * X; g.K = X * Y;
    g.A = P1; g.lda = X * Y;
    g.B = Tb; g.ldb = X * Y;
    g.C = Q2;
    g.rmap = IdxMap::split(X, (i64)Y * X * X, X);
    g.cmap = IdxMap::split(X, (i64)X * X, 1);
    c.gemmc(g, pr, false);
}

// T'[alpha][beta][y][z] = sum_{(i,m)} Q2[(alpha,y,z)][(i,m)] w[(i,m)][beta]
void proj3(Ctx& c, Prec pr, const void* Q2, const void* U, int ldu, double* Tn, int X, int Y, int K) {
    GemmOp g;
    g.M = K * Y * Y; g.N = K; g.K = X * X;
    g.A = Q2; g.lda = X * X;
    g.B = U; g.ldb = ldu; g.b_kmajor = true;
    g.C = Tn;
    g.rmap = IdxMap::split((i64)Y * Y, (i64)K * Y * Y, 1);
    g.cmap = IdxMap::linear((i64)Y * Y);
    c.gemmc(g, pr, true);
}

// Contraction operands of one step, in the contraction precision.
struct Ops {
    const void *Tp, *Tb, *Tb2, *Wt, *Wt2, *U;
    void *P1, *Q2, *X5, *Tpbar;
    Prec pr;    // precision of this step's contractions (FP64, FP32 or split-bf16)
    int mask;   // with split-bf16: bit 0 join, 1 adjoint w.r.t. P, 2 w.r.t. the lower copy, 3 chi^6
    // precision of contraction `bit`: split-bf16 only where the mask selects it, FP32 otherwise
    Prec at(int bit) const { return (pr == Prec::BF16X3 && !(mask & (1 << bit))) ? Prec::F32 : pr; }
};

// Operand layouts of one step from its input T and its eigenvectors U:
//   Tp [u][r][d][l], Tb [d][r][l][u], Wt [alpha][b][a], U as is (n x b); for the backward also
//   Wt2 [a][alpha][b] and Tb2 [d][r][u][l].
// FP64 path: permuted FP64 copies; mixed paths: permuted FP32 copies.
Ops prep_operands(Ctx& c, const StepCk& st, bool need_wt2) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n, b = st.sh.b;
    Ops o;
    o.pr = st.sh.mixed ? P->prec : Prec::F64;
    o.mask = P->opt.bf16x3_mask;
    if (!st.sh.mixed) {
        permute_checked(P, st.T.p, P->Tp.p, pd4(X, X, Y, Y, 2, 1, 3, 0), 1.0, 0.0, nullptr, c.s);
        permute_checked(P, st.T.p, P->Tb.p, pd4(X, X, Y, Y, 3, 1, 0, 2), 1.0, 0.0, nullptr, c.s);
        permute_checked(P, st.U.p, P->Wt.p, pd3(X, X, b, 2, 1, 0), 1.0, 0.0, nullptr, c.s);
        if (need_wt2) {
            permute_checked(P, st.U.p, P->Wt2.p, pd3(X, X, b, 0, 2, 1), 1.0, 0.0, nullptr, c.s);
            permute_checked(P, st.T.p, P->Tb2.p, pd4(X, X, Y, Y, 3, 1, 2, 0), 1.0, 0.0, nullptr, c.s);
        }
        o.Tp = P->Tp.p; o.Tb = P->Tb.p; o.Tb2 = P->Tb2.p; o.Wt = P->Wt.p; o.Wt2 = P->Wt2.p; o.U = st.U.p;
        o.P1 = P->P1.p; o.Q2 = P->Q2.p; o.X5 = P->X5.p; o.Tpbar = P->Tpbar.p;
    } else {
        permute_f32_checked(P, st.T.p, P->Tpf.p, pd4(X, X, Y, Y, 2, 1, 3, 0), c.s);
        permute_f32_checked(P, st.T.p, P->Tbf.p, pd4(X, X, Y, Y, 3, 1, 0, 2), c.s);
        permute_f32_checked(P, st.U.p, P->Wtf.p, pd3(X, X, b, 2, 1, 0), c.s);
        if (need_wt2) {
            permute_f32_checked(P, st.U.p, P->Wt2f.p, pd3(X, X, b, 0, 2, 1), c.s);
            permute_f32_checked(P, st.T.p, P->Tb2f.p, pd4(X, X, Y, Y, 3, 1, 2, 0), c.s);
        }
        DTRG_REQUIRE((i64)P->Uf.n >= (i64)n * b, DTRG_EINVAL, "FP32 isometry buffer too small");
        convert_f64_to_f32(st.U.p, P->Uf.p, (i64)n * b, c.s);
        o.Tp = P->Tpf.p; o.Tb = P->Tbf.p; o.Tb2 = P->Tb2f.p; o.Wt = P->Wtf.p; o.Wt2 = P->Wt2f.p; o.U = P->Uf.p;
        o.P1 = P->P1f.p; o.Q2 = P->Q2f.p; o.X5 = P->X5f.p; o.Tpbar = P->Tpbarf.p;
    }
    return o;
}

// -------------------------------------------------------------------------------------------
// truncated eigensolve
// -------------------------------------------------------------------------------------------

// Orthonormalise the n x b block V in place: a shifted CholeskyQR pass (stable for any condition
// number up to 1/u, which the normalised iterate can reach when the Gram has a cluster of noise-level
// eigenvalues) followed by two plain passes.
void orthonormalise(Ctx& c, double* V, double* Vtmp, int n, int b, bool shifted = true) {
    dtrg_plan* P = c.P;
    double* cur = V;
    double* oth = Vtmp;
    const int first = shifted ? 0 : 1;
    for (int pass = first; pass < 3; ++pass) {
        GemmOp g;
        g.M = g.N = b; g.K = n;
        g.A = cur; g.lda = b; g.a_kmajor = true;
        g.B = cur; g.ldb = b; g.b_kmajor = true;
        g.C = P->Sg.p;
        g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
        c.gemm(g);
        const double shift = pass == 0 ? 11.0 * ((double)n * b + (double)b * (b + 1)) * std::ldexp(1.0, -53) : 0.0;
        chol_inverse(P->Sg.p, b, shift, P->Rinv.p, P->iflag.p, c.s);
        GemmOp h;
        h.M = n; h.N = b; h.K = b;
        h.A = cur; h.lda = b;
        h.B = P->Rinv.p; h.ldb = b; h.b_kmajor = true;
        h.C = oth;
        h.rmap = IdxMap::linear(b); h.cmap = IdxMap::linear(1);
        c.gemm(h);
        std::swap(cur, oth);
    }
    if (cur != V) copy2d(cur, b, V, b, n, b, c.s);
}

// C (n x b) = G (n x n) V (n x b)
void gemm_GV(Ctx& c, const double* G, const double* V, double* C, int n, int b, int ldv) {
    GemmOp g;
    g.M = n; g.N = b; g.K = n;
    g.A = G; g.lda = n;
    g.B = V; g.ldb = ldv; g.b_kmajor = true;
    g.C = C;
    g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
    c.gemm(g);
}

void int_flags_check(dtrg_plan* P, const char* where) {
    int f = 0;
    DTRG_HIP(hipMemcpyAsync(&f, P->iflag.p, sizeof(int), hipMemcpyDeviceToHost, P->s));
    DTRG_HIP(hipStreamSynchronize(P->s));
    if (f & 1) throw Error(DTRG_ENONPOS, std::string(where) + ": a norm or trace is not positive and finite");
}

void eigensolve(Ctx& c, StepCk& st, const StepCk* warm, uint64_t seed) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n, b = st.sh.b, K = st.sh.K, E = st.sh.e;
    const double* G = P->Gw.p;
    if (st.sh.full) {
        int* sw = P->iflag.p + 1;
        jacobi_eig(G, n, n, st.lam.p, st.U.p, n, 40, sw, c.s);
        st.lam_h.resize(n);
        DTRG_HIP(hipMemcpyAsync(st.lam_h.data(), st.lam.p, n * sizeof(double), hipMemcpyDeviceToHost, c.s));
        DTRG_HIP(hipStreamSynchronize(c.s));
        st.iters = 0;
        st.resid = 0.0;
        return;
    }
    // block subspace iteration with Rayleigh-Ritz on the (kept) normalised Gram
    double* V = P->V1.p;
    double* Y = P->Y1.p;
    // warm start: the Ritz vectors of the previous step in the same direction (orthonormal already)
    const bool warm_used = warm && warm->sh.n == n && warm->sh.b == b;
    if (warm_used) {
        copy2d(warm->U.p, b, V, b, n, b, c.s);
    } else {
        hash_fill(V, (i64)n * b, seed, c.s);
        orthonormalise(c, V, P->V2.p, n, b, true);
    }
    const double tol = P->opt.subspace_tol;
    double prev = INFINITY;
    int stall = 0;
    std::vector<double> resh(E);
    int it = 0;
    double best = INFINITY;
    for (it = 1; it <= P->opt.max_subspace_iters; ++it) {
        gemm_GV(c, G, V, Y, n, b, b);
        // H = V^T Y
        GemmOp g;
        g.M = g.N = b; g.K = n;
        g.A = V; g.lda = b; g.a_kmajor = true;
        g.B = Y; g.ldb = b; g.b_kmajor = true;
        g.C = P->H.p;
        g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
        c.gemm(g);
        jacobi_eig(P->H.p, b, b, P->th.p, P->Z.p, b, 40, P->iflag.p + 1, c.s);
        // V <- V Z, Y <- Y Z
        GemmOp r;
        r.M = n; r.N = b; r.K = b;
        r.B = P->Z.p; r.ldb = b; r.b_kmajor = true;
        r.rmap = IdxMap::linear(b); r.cmap = IdxMap::linear(1);
        r.A = V; r.lda = b; r.C = P->V2.p; c.gemm(r);
        r.A = Y; r.lda = b; r.C = P->Y2.p; c.gemm(r);
        std::swap(P->V1, P->V2);
        std::swap(P->Y1, P->Y2);
        V = P->V1.p;
        Y = P->Y1.p;
        ritz_residuals(V, Y, n, E, b, P->th.p, P->res.p, c.s);
        DTRG_HIP(hipMemcpyAsync(resh.data(), P->res.p, E * sizeof(double), hipMemcpyDeviceToHost, c.s));
        DTRG_HIP(hipStreamSynchronize(c.s));
        double mx = 0.0;
        for (double v : resh) mx = std::max(mx, std::isfinite(v) ? v : INFINITY);
        best = std::min(best, mx);
        if (mx <= tol) break;
        if (mx > 0.5 * prev) ++stall; else stall = 0;
        prev = mx;
        if (stall >= 3 && mx <= 1e-12) break;      // rounding floor reached
        if (it == P->opt.max_subspace_iters) break;
        // next block: G V with columns rescaled to unit norm, re-orthonormalised
        col_norms(Y, n, b, b, P->nrm.p, c.s);
        col_normalise(Y, n, b, b, P->nrm.p, seed + 7919ULL * it, c.s);
        std::swap(P->V1, P->Y1);
        V = P->V1.p;
        Y = P->Y1.p;
        orthonormalise(c, V, P->V2.p, n, b, true);
    }
    if (!(best <= 1e-12))
        throw Error(DTRG_ENOCONV, "truncated eigensolve: residual " + std::to_string(best) + " after " +
                                      std::to_string(it) + " iterations");
    copy2d(V, b, st.U.p, b, n, b, c.s);
    if (E < b) {
        ritz_residuals(V, Y, n, E + 1, b, P->th.p, P->res.p, c.s);
        DTRG_HIP(hipMemcpyAsync(&st.res_next, P->res.p + E, sizeof(double), hipMemcpyDeviceToHost, c.s));
    }
    DTRG_HIP(hipMemcpyAsync(st.lam.p, P->th.p, b * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    st.lam_h.resize(b);
    DTRG_HIP(hipMemcpyAsync(st.lam_h.data(), P->th.p, b * sizeof(double), hipMemcpyDeviceToHost, c.s));
    DTRG_HIP(hipStreamSynchronize(c.s));
    st.iters = std::min(it, P->opt.max_subspace_iters);
    st.resid = best;
}

// -------------------------------------------------------------------------------------------
// plan set-up
// -------------------------------------------------------------------------------------------
// Steps whose join contraction costs less than this fraction of the largest step's stay FP64 on
// the mixed paths: their cost is negligible and they carry the largest weights 2^-k in ln Z / N.
constexpr double kMixedMinFraction = 0.05;

std::vector<StepShape> shapes(int D, int chi, int nsteps, int block, bool mixed) {
    std::vector<StepShape> v;
    int X = D, Y = D;
    for (int k = 1; k <= nsteps; ++k) {
        StepShape s;
        s.X = X; s.Y = Y; s.n = X * X;
        s.K = std::min(chi, s.n);
        if (s.n <= kJacobiMax) { s.full = true; s.b = s.n; s.e = s.n; }
        else {
            int b = block > 0 ? block : std::max(s.K + 16, 2 * s.K);
            b = std::min(b, kJacobiMax);
            b = std::min(b, s.n - 1);
            DTRG_REQUIRE(b >= s.K, DTRG_EINVAL, "block size smaller than chi'");
            s.b = b;
            s.e = s.K + (b - s.K) / 2;
        }
        v.push_back(s);
        X = Y;
        Y = s.K;
    }
    if (mixed) {
        double mx = 0.0;
        for (auto& s : v) mx = std::max(mx, s.join_flops());
        for (auto& s : v) s.mixed = s.join_flops() >= kMixedMinFraction * mx;
    }
    return v;
}

void alloc_plan(dtrg_plan* P, const std::vector<StepShape>& sh) {
    i64 t4 = (i64)P->D * P->D * P->D * P->D, n2 = 0, nb = 0, bmax = 1;
    i64 t4d = 1, t5d = 1, bX2d = 1, t4f = 1, t5f = 1, bX2f = 1, nbf = 1;   // per-precision operand sizes
    bool any_d = false, any_f = false;
    for (auto& s : sh) {
        const i64 a4 = std::max<i64>((i64)s.X * s.X * s.Y * s.Y, (i64)s.K * s.K * s.Y * s.Y);
        const i64 a5 = (i64)s.K * s.Y * s.X * s.X * s.Y, ab = (i64)s.b * s.X * s.X;
        t4 = std::max(t4, a4);
        n2 = std::max<i64>(n2, (i64)s.n * s.n);
        nb = std::max<i64>(nb, (i64)s.n * s.b);
        bmax = std::max<i64>(bmax, s.b);
        if (s.mixed) {
            any_f = true;
            t4f = std::max(t4f, a4); t5f = std::max(t5f, a5); bX2f = std::max(bX2f, ab);
            nbf = std::max<i64>(nbf, (i64)s.n * s.b);
        } else {
            any_d = true;
            t4d = std::max(t4d, a4); t5d = std::max(t5d, a5); bX2d = std::max(bX2d, ab);
        }
    }
    P->TA.alloc(t4); P->TB.alloc(t4);
    P->Tn.alloc(t4); P->Tbar.alloc(t4); P->Tbar2.alloc(t4); P->Tpbar.alloc(t4);
    if (any_d) {
        P->Tp.alloc(t4d); P->Tb.alloc(t4d); P->Tb2.alloc(t4d);
        P->Wt.alloc(bX2d); P->Wt2.alloc(bX2d);
        P->P1.alloc(t5d); P->Q2.alloc(t5d); P->X5.alloc(t5d);
    }
    if (any_f) {
        P->Tpf.alloc(t4f); P->Tbf.alloc(t4f); P->Tb2f.alloc(t4f); P->Tpbarf.alloc(t4f);
        P->Wtf.alloc(bX2f); P->Wt2f.alloc(bX2f); P->Uf.alloc(nbf);
        P->P1f.alloc(t5f); P->Q2f.alloc(t5f); P->X5f.alloc(t5f);
    }
    P->Gw.alloc(n2); P->Gt.alloc(n2);
    P->V1.alloc(nb); P->V2.alloc(nb); P->Y1.alloc(nb); P->Y2.alloc(nb);
    P->H.alloc(bmax * bmax); P->Z.alloc(bmax * bmax); P->Rinv.alloc(bmax * bmax); P->Sg.alloc(bmax * bmax);
    P->th.alloc(bmax); P->res.alloc(bmax); P->nrm.alloc(bmax);
    P->scal.alloc(16);
    P->flags.alloc(4);
    P->iflag.alloc(4);
    P->steps.clear();
    P->steps.resize(sh.size());
    for (size_t k = 0; k < sh.size(); ++k) {
        StepCk& st = P->steps[k];
        st.sh = sh[k];
        const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n, b = st.sh.b;
        st.T.alloc((i64)X * X * Y * Y);
        st.A.alloc((i64)X * X * Y * Y);
        st.B.alloc((i64)X * X * Y * Y);
        st.U.alloc((i64)n * b);
        st.lam.alloc(b);
        if (!st.sh.full) st.G.alloc((i64)n * n);
    }
}

void alloc_backward(dtrg_plan* P) {
    i64 t5 = 0, nK = 0, bK = 0, KK = 0, n2 = 0;
    for (auto& st : P->steps) {
        const auto& s = st.sh;
        t5 = std::max<i64>(t5, (i64)s.K * s.Y * s.X * s.X * s.Y);
        nK = std::max<i64>(nK, (i64)s.n * s.K);
        bK = std::max<i64>(bK, (i64)s.b * s.K);
        KK = std::max<i64>(KK, (i64)s.K * s.K);
        n2 = std::max<i64>(n2, (i64)s.n * s.n);
    }
    P->Ub.ensure(nK); P->Xe.ensure(nK); P->Xc.ensure(nK); P->Re.ensure(nK); P->Vc.ensure(nK); P->Vp.ensure(nK);
    P->Vn.ensure(nK); P->Ye.ensure(nK); P->We.ensure(std::max(bK, nK));
    P->Om.ensure(bK); P->Sm.ensure(std::max(KK, bK));
    i64 Kmax = 1;
    for (auto& st : P->steps) Kmax = std::max<i64>(Kmax, st.sh.K);
    P->coef.ensure(1025 * Kmax);   // largest Chebyshev expansion (degree 1024)
}

// -------------------------------------------------------------------------------------------
// forward
// -------------------------------------------------------------------------------------------
void setup(dtrg_plan* P) {
    P->shape = shapes(P->D, P->chi, P->nsteps, P->opt.block_size, P->mixed());
    alloc_plan(P, P->shape);
    alloc_backward(P);
}

void forward(dtrg_plan* P, const double* T0) {
    Ctx c{P, P->s};
    const int D = P->D;
    const auto& sh = P->shape;
    fill(P->scal.p, 16, 0.0, c.s);
    fill_int(P->iflag.p, 4, 0, c.s);
    // c0 = |T0|; T1 = permute(T0, (0,2,1,3)) / c0
    norm2(T0, (i64)D * D * D * D, P->scal.p + 6, c.s, P->ws);
    double c0 = 0.0;
    DTRG_HIP(hipMemcpyAsync(&c0, P->scal.p + 6, sizeof(double), hipMemcpyDeviceToHost, c.s));
    DTRG_HIP(hipStreamSynchronize(c.s));
    if (!std::isfinite(c0)) throw Error(DTRG_EINVAL, "T0 has non-finite entries");
    if (!(c0 > 0.0)) throw Error(DTRG_ENONPOS, "T0 is zero");
    P->c0 = c0;
    accum_log(P->scal.p + 6, 1.0, P->scal.p + 0, P->scal.p + 7, P->iflag.p, c.s);
    for (int k = 1; k <= P->nsteps; ++k) {
        StepCk& st = P->steps[k - 1];
        const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K, n = st.sh.n, b = st.sh.b;
        if (k == 1) permute_checked(P, T0, st.T.p, pd4(D, D, D, D, 0, 2, 1, 3), 1.0 / c0, 0.0, nullptr, c.s);
        else {
            // T_k = permute(T'_{k-1} / c_{k-1}, (2,3,0,1))
            const StepShape& ps = sh[k - 2];
            permute_checked(P, P->Tn.p, st.T.p, pd4(ps.K, ps.K, ps.Y, ps.Y, 2, 3, 0, 1), 1.0, 0.0, P->scal.p + 2, c.s);
        }
        // half-environments and Gram
        permute_checked(P, st.T.p, P->TA.p, pd4(X, X, Y, Y, 0, 3, 1, 2), 1.0, 0.0, nullptr, c.s);
        permute_checked(P, st.T.p, P->TB.p, pd4(X, X, Y, Y, 0, 2, 1, 3), 1.0, 0.0, nullptr, c.s);
        half_env(c, P->TA.p, st.A.p, X, Y);
        half_env(c, P->TB.p, st.B.p, X, Y);
        gram(c, st.A.p, st.B.p, P->Gw.p, X, Y);
        sym_normalise(P->Gw.p, n, P->scal.p + 3, c.s);
        DTRG_HIP(hipMemcpyAsync(&st.t, P->scal.p + 3, sizeof(double), hipMemcpyDeviceToHost, c.s));
        DTRG_HIP(hipStreamSynchronize(c.s));
        if (!(st.t > 0.0) || !std::isfinite(st.t))
            throw Error(DTRG_ENONPOS, "step " + std::to_string(k) + ": Gram trace is not positive and finite");
        const StepCk* warm = (k >= 3) ? &P->steps[k - 3] : nullptr;
        eigensolve(c, st, warm, 0x5eedULL * (uint64_t)k + 17ULL);
        if (!st.sh.full)
            DTRG_HIP(hipMemcpyAsync(st.G.p, P->Gw.p, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, c.s));
        // projection (contraction precision; the output T' is FP64)
        const Ops o = prep_operands(c, st, false);
        proj1(c, o.at(3), o.Wt, o.Tp, o.P1, X, Y, K);
        proj2(c, o.at(0), o.P1, o.Tb, o.Q2, X, Y, K);
        proj3(c, o.at(3), o.Q2, o.U, b, P->Tn.p, X, Y, K);
        // c_k = |T'|, L += 2^-k ln c_k, scal[2] = 1/c_k
        norm2(P->Tn.p, (i64)K * K * Y * Y, P->scal.p + 1, c.s, P->ws);
        accum_log(P->scal.p + 1, ldexp1(-k), P->scal.p + 0, P->scal.p + 2, P->iflag.p, c.s);
        DTRG_HIP(hipMemcpyAsync(&st.c, P->scal.p + 1, sizeof(double), hipMemcpyDeviceToHost, c.s));
        int_flags_check(P, ("step " + std::to_string(k)).c_str());
    }
    // final self-trace of T_{n+1} = permute(T'_n / c_n)
    const StepShape& ls = sh.back();
    P->Xf = ls.Y; P->Yf = ls.K;
    permute_checked(P, P->Tn.p, P->Tbar2.p, pd4(ls.K, ls.K, ls.Y, ls.Y, 2, 3, 0, 1), 1.0, 0.0, P->scal.p + 2, c.s);
    trace_xxyy(P->Tbar2.p, P->Xf, P->Yf, P->scal.p + 4, c.s);
    accum_log(P->scal.p + 4, ldexp1(-P->nsteps), P->scal.p + 0, nullptr, P->iflag.p, c.s);
    double out[5];
    DTRG_HIP(hipMemcpyAsync(out, P->scal.p, 5 * sizeof(double), hipMemcpyDeviceToHost, c.s));
    int_flags_check(P, "final trace");
    P->lnZ = out[0];
    P->final_trace = out[4];
    if (!std::isfinite(P->lnZ)) throw Error(DTRG_ENONPOS, "ln Z is not finite");
}

// -------------------------------------------------------------------------------------------
// backward
// -------------------------------------------------------------------------------------------

// Gradient with respect to the normalised Gram, G_bar = (W U_K^T + U_K W^T) / t, from the
// gradient U_bar (n x K, in P->Ub) with respect to the kept eigenvectors U_K, written to P->Gw.
//   kept block:    W += U_K S / 2,  S = F o (Om - Om^T) / 2,  Om = U_K^T U_bar
//   complement:    W += sum_{i discarded} u_i F(lam_j - lam_i) (u_i^T u_bar_j) / 2
// F(d) = d / (d^2 + eps).  The discarded pairs that are resolved (all of them for Jacobi steps;
// those nearest the cut, K <= i < e, for subspace steps) enter explicitly.  For subspace steps
// the remainder is f_j(G_r) P_e u_bar_j with G_r = P_e G P_e, P_e the projector off the e
// resolved vectors, evaluated by a Chebyshev expansion of f_j on an interval [lo, hi] holding
// the spectrum of G_r (which lies below the first unresolved eigenvalue, far from the poles
// lam_j +- i sqrt(eps) of f_j).
void eig_adjoint(Ctx& c, StepCk& st) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n, b = st.sh.b, K = st.sh.K, E = st.sh.e;
    const double eps = P->opt.eig_broadening;
    const double* U = st.U.p;
    // Om = U_K^T U_bar (K x K), S on the kept block
    GemmOp g;
    g.M = K; g.N = K; g.K = n;
    g.A = U; g.lda = b; g.a_kmajor = true;
    g.B = P->Ub.p; g.ldb = K; g.b_kmajor = true;
    g.C = P->Om.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
    c.gemm(g);
    kept_block_adjoint(P->Om.p, st.lam.p, K, eps, P->Sm.p, c.s);
    // R = P_K U_bar = U_bar - U_K Om
    copy2d(P->Ub.p, K, P->Re.p, K, n, K, c.s);
    GemmOp r;
    r.M = n; r.N = K; r.K = K;
    r.A = U; r.lda = b;
    r.B = P->Om.p; r.ldb = K; r.b_kmajor = true;
    r.C = P->Re.p; r.rmap = IdxMap::linear(K); r.cmap = IdxMap::linear(1);
    r.alpha = -1.0; r.beta = 1.0;
    c.gemm(r);
    fill(P->Xe.p, (i64)n * K, 0.0, c.s);
    st.cheb = 0;
    const int p = E - K;   // resolved discarded pairs
    if (p > 0) {
        // Om_D = U_D^T R (p x K);  X = U_D [F o Om_D] / 2;  R <- R - U_D Om_D
        GemmOp o;
        o.M = p; o.N = K; o.K = n;
        o.A = U + K; o.lda = b; o.a_kmajor = true;
        o.B = P->Re.p; o.ldb = K; o.b_kmajor = true;
        o.C = P->We.p; o.rmap = IdxMap::linear(K); o.cmap = IdxMap::linear(1);
        c.gemm(o);
        over_block_adjoint(P->We.p, st.lam.p + K, st.lam.p, p, K, eps, P->Vc.p, c.s);
        GemmOp x;
        x.M = n; x.N = K; x.K = p;
        x.A = U + K; x.lda = b;
        x.B = P->Vc.p; x.ldb = K; x.b_kmajor = true;
        x.C = P->Xe.p; x.rmap = IdxMap::linear(K); x.cmap = IdxMap::linear(1);
        c.gemm(x);
        if (!st.sh.full) {
            x.B = P->We.p; x.C = P->Re.p; x.alpha = -1.0; x.beta = 1.0;
            c.gemm(x);
        }
    }
    if (!st.sh.full) {
        // spectrum of G_r: below the first unresolved eigenvalue, bounded by that Ritz value plus
        // its residual (with a margin), and never narrower than the rounding noise of the Gram,
        // +-nu with nu = 64 n u lam_1 (an unconverged Ritz value of a noise cluster can sit far
        // below the noise it came from)
        const double nu = 64.0 * n * 0x1p-53 * std::max(st.lam_h[0], 0.0);
        double hi = std::max(1.1 * (std::max(st.lam_h[E], 0.0) + st.res_next), nu) + 1e-300;
        std::vector<double> lamK(st.lam_h.begin(), st.lam_h.begin() + K);
        std::vector<double> cf;
        auto apply_Gr = [&](const double* v) {
            // Ye = G v - U_e (U_e^T G v)
            GemmOp a;
            a.M = n; a.N = K; a.K = n;
            a.A = st.G.p; a.lda = n;
            a.B = v; a.ldb = K; a.b_kmajor = true;
            a.C = P->Ye.p; a.rmap = IdxMap::linear(K); a.cmap = IdxMap::linear(1);
            c.gemm(a);
            GemmOp w;
            w.M = E; w.N = K; w.K = n;
            w.A = U; w.lda = b; w.a_kmajor = true;
            w.B = P->Ye.p; w.ldb = K; w.b_kmajor = true;
            w.C = P->We.p; w.rmap = IdxMap::linear(K); w.cmap = IdxMap::linear(1);
            c.gemm(w);
            GemmOp u;
            u.M = n; u.N = K; u.K = E;
            u.A = U; u.lda = b;
            u.B = P->We.p; u.ldb = K; u.b_kmajor = true;
            u.C = P->Ye.p; u.rmap = IdxMap::linear(K); u.cmap = IdxMap::linear(1);
            u.alpha = -1.0; u.beta = 1.0;
            c.gemm(u);
        };
        double v0n = 0.0;
        norm2(P->Re.p, (i64)n * K, P->scal.p + 8, c.s, P->ws);
        DTRG_HIP(hipMemcpyAsync(&v0n, P->scal.p + 8, sizeof(double), hipMemcpyDeviceToHost, c.s));
        DTRG_HIP(hipStreamSynchronize(c.s));
        bool ok = (v0n == 0.0);
        std::string trail;
        // the explicit part stays in Xe; the expansion accumulates into Xc
        for (int attempt = 0; attempt < 4 && !ok; ++attempt, hi *= 4.0) {
            const double lo = -std::max(nu, 0.05 * hi);
            int m = 8;
            for (;; m *= 2) {
                cheb_coeffs(lamK, eps, lo, hi, m, cf);
                double mx = 0.0, tail = 0.0;
                for (int q = 0; q <= m; ++q)
                    for (int j = 0; j < K; ++j) {
                        const double a = std::fabs(cf[(size_t)q * K + j]);
                        mx = std::max(mx, a);
                        if (q >= m - 1) tail = std::max(tail, a);
                    }
                if (tail <= 1e-15 * mx || m >= 1024) break;
            }
            st.cheb = m;
            P->coef.ensure((size_t)(m + 1) * K);
            DTRG_HIP(hipMemcpyAsync(P->coef.p, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice, c.s));
            fill(P->Xc.p, (i64)n * K, 0.0, c.s);
            // v0 = R_rest (kept in Re), v1 = s(G_r) v0, v_{q+1} = 2 s(G_r) v_q - v_{q-1}
            apply_Gr(P->Re.p);
            cheb_step(P->Ye.p, P->Re.p, nullptr, P->Vn.p, P->Xc.p, n, K, lo, hi, true, P->coef.p, c.s);
            double* prv = P->Re.p;
            double* cur = P->Vn.p;
            double* nxt = P->Vc.p;
            double* spare = P->Vp.p;
            for (int q = 2; q <= m; ++q) {
                apply_Gr(cur);
                cheb_step(P->Ye.p, cur, prv, nxt, P->Xc.p, n, K, lo, hi, false, P->coef.p + (size_t)q * K, c.s);
                double* t = (prv == P->Re.p) ? spare : prv;   // R_rest is never overwritten
                prv = cur;
                cur = nxt;
                nxt = t;
            }
            // |T_m(s(G_r)) v0| <= |v0| when the spectrum lies in [lo, hi] (up to rounding)
            double vmn = 0.0;
            norm2(cur, (i64)n * K, P->scal.p + 8, c.s, P->ws);
            DTRG_HIP(hipMemcpyAsync(&vmn, P->scal.p + 8, sizeof(double), hipMemcpyDeviceToHost, c.s));
            DTRG_HIP(hipStreamSynchronize(c.s));
            ok = std::isfinite(vmn) && vmn <= 1.5 * v0n;
            trail += " [hi " + std::to_string(hi) + " m " + std::to_string(m) + " |v_m|/|v_0| " +
                     std::to_string(vmn / v0n) + "]";
        }
        if (!ok)
            throw Error(DTRG_ENOCONV, "eigen-adjoint: complement expansion diverged (theta_e " +
                                          std::to_string(st.lam_h[E]) + ", residual " + std::to_string(st.res_next) +
                                          ")" + trail);
        if (v0n != 0.0) axpy(P->Xc.p, P->Xe.p, (i64)n * K, 1.0, c.s);   // Xe += Xc
    }
    // W = X + U_K S / 2;  G_bar = (W U_K^T + U_K W^T) / t
    GemmOp w;
    w.M = n; w.N = K; w.K = K;
    w.A = U; w.lda = b;
    w.B = P->Sm.p; w.ldb = K; w.b_kmajor = true;
    w.C = P->Xe.p; w.rmap = IdxMap::linear(K); w.cmap = IdxMap::linear(1);
    w.alpha = 0.5; w.beta = 1.0;
    c.gemm(w);
    GemmOp o1;
    o1.M = n; o1.N = n; o1.K = K;
    o1.A = P->Xe.p; o1.lda = K;
    o1.B = U; o1.ldb = b;
    o1.C = P->Gw.p; o1.rmap = IdxMap::linear(n); o1.cmap = IdxMap::linear(1);
    o1.alpha = 1.0 / st.t;
    c.gemm(o1);
    o1.A = U; o1.lda = b; o1.B = P->Xe.p; o1.ldb = K; o1.beta = 1.0;
    c.gemm(o1);
}

void backward(dtrg_plan* P, double gbar, double* T0bar, const double* dT0, double* dir_out) {
    Ctx c{P, P->s};
    const int ns = P->nsteps;
    // seed: gradient w.r.t. T_{n+1} (dims [Xf][Xf][Yf][Yf])
    seed_trace_grad(P->Tbar.p, P->Xf, P->Yf, gbar * ldexp1(-ns), P->scal.p + 4, c.s);
    for (int k = ns; k >= 1; --k) {
        StepCk& st = P->steps[k - 1];
        const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K, n = st.sh.n, b = st.sh.b;
        // T'bar_p[alpha][y][z][beta] = permute(Tbar [y][z][alpha][beta]) / c_k
        permute_checked(P, P->Tbar.p, P->Tpbar.p, pd4(Y, Y, K, K, 2, 0, 1, 3), 1.0 / st.c, 0.0, nullptr, c.s);
        // recompute the projection intermediates (contraction precision)
        const Ops o = prep_operands(c, st, true);
        const Prec pr6 = o.at(3);
        proj1(c, pr6, o.Wt, o.Tp, o.P1, X, Y, K);
        proj2(c, o.at(0), o.P1, o.Tb, o.Q2, X, Y, K);
        if (st.sh.mixed) convert_f64_to_f32(P->Tpbar.p, P->Tpbarf.p, (i64)K * Y * Y * K, c.s);
        // w_bar_R[(i,m)][beta] = sum_{(alpha,y,z)} Q2[(alpha,y,z)][(i,m)] T'bar_p[(alpha,y,z)][beta]
        {
            GemmOp g;
            g.M = n; g.N = K; g.K = K * Y * Y;
            g.A = o.Q2; g.lda = n; g.a_kmajor = true;
            g.B = o.Tpbar; g.ldb = K; g.b_kmajor = true;
            g.C = P->Ub.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
            c.gemmc(g, pr6, true);
        }
        // Qbar[alpha][y][i][z][m] = sum_beta T'bar_p[(alpha,y,z)][beta] w[(i,m)][beta]   (into Q2)
        {
            GemmOp g;
            g.M = K * Y * Y; g.N = n; g.K = K;
            g.A = o.Tpbar; g.lda = K;
            g.B = o.U; g.ldb = b;
            g.C = o.Q2;
            g.rmap = IdxMap::split(Y, (i64)X * Y * X, X);
            g.cmap = IdxMap::split(X, (i64)Y * X, 1);
            c.gemmc(g, pr6, false);
        }
        fill(P->Tbar2.p, (i64)X * X * Y * Y, 0.0, c.s);
        // Pbar_p[y][i][j][alpha][b] = sum_{(z,m)} Qbar[(alpha,y,i)][(z,m)] Tb2[(z,m)][(j,b)]   (chi^7)
        // (the adjoint of the join with respect to P, written straight in the layout of its two
        // consumers below: rows (alpha,(y,i)), columns (j,b))
        {
            GemmOp g;
            g.M = K * Y * X; g.N = Y * X; g.K = Y * X;
            g.A = o.Q2; g.lda = Y * X;
            g.B = o.Tb2; g.ldb = Y * X; g.b_kmajor = true;
            g.C = o.X5;
            g.rmap = IdxMap::split((i64)Y * X, X, (i64)Y * K * X);
            g.cmap = IdxMap::split(X, (i64)K * X, 1);
            g.tag = 8;
            c.gemmc(g, o.at(1), false);
        }
        // Tbar_lower[b][m][j][z] += sum_{(alpha,y,i)} Qbar[(alpha,y,i)][(z,m)] P1[(alpha,y,i)][(b,j)]   (chi^7)
        {
            GemmOp g;
            g.M = Y * X; g.N = X * Y; g.K = K * Y * X;
            g.A = o.Q2; g.lda = Y * X; g.a_kmajor = true;
            g.B = o.P1; g.ldb = X * Y; g.b_kmajor = true;
            g.C = P->Tbar2.p;
            g.rmap = IdxMap::split(X, 1, (i64)Y * Y);
            g.cmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
            g.beta = 1.0;
            g.tag = 9;
            c.gemmc(g, o.at(2), true);
        }
        // Tbar_upper[a][i][y][j] += sum_{(alpha,b)} Pbar_p[y][(i,j)][(alpha,b)] Wt2[a][(alpha,b)]
        {
            GemmOp g;
            g.M = X * Y; g.N = X; g.K = K * X; g.batch = Y;
            g.A = o.X5; g.lda = (i64)K * X; g.a_bs = (i64)X * Y * K * X;
            g.B = o.Wt2; g.ldb = (i64)b * X; g.b_bs = 0;
            g.C = P->Tbar2.p; g.c_bs = Y;
            g.rmap = IdxMap::split(Y, (i64)Y * Y, 1);
            g.cmap = IdxMap::linear((i64)X * Y * Y);
            g.beta = 1.0;
            c.gemmc(g, pr6, true);
        }
        // w_bar_L[(a,b)][alpha] += sum_{(y,i,j)} Tp[(y,i,j)][a] Pbar_p[(y,i,j)][(alpha,b)]
        {
            GemmOp g;
            g.M = X; g.N = K * X; g.K = Y * X * Y;
            g.A = o.Tp; g.lda = X; g.a_kmajor = true;
            g.B = o.X5; g.ldb = (i64)K * X; g.b_kmajor = true;
            g.C = P->Ub.p;
            g.rmap = IdxMap::linear((i64)X * K);
            g.cmap = IdxMap::split(X, 1, K);
            g.beta = 1.0;
            c.gemmc(g, pr6, true);
        }
        // the Gram adjoint needs the FP64 half-environment operands
        permute_checked(P, st.T.p, P->TA.p, pd4(X, X, Y, Y, 0, 3, 1, 2), 1.0, 0.0, nullptr, c.s);
        permute_checked(P, st.T.p, P->TB.p, pd4(X, X, Y, Y, 0, 2, 1, 3), 1.0, 0.0, nullptr, c.s);
        // eigensolver adjoint -> G_bar (n x n) in Gw
        eig_adjoint(c, st);
        // Gt[(a,b)][(c,d)] = G_bar[(a,c)][(b,d)]
        permute_checked(P, P->Gw.p, P->Gt.p, pd4(X, X, X, X, 0, 2, 1, 3), 1.0, 0.0, nullptr, c.s);
        // Abar'[a][j][b][k] = sum_{(c,d)} Gt[(a,b)][(c,d)] B[(c,d)][(j,k)]   (into TA's partner buffers)
        double* Abar = P->Tn.p;
        double* Bbar = P->Tpbar.p;
        {
            GemmOp g;
            g.M = X * X; g.N = Y * Y; g.K = X * X;
            g.A = P->Gt.p; g.lda = X * X;
            g.B = st.B.p; g.ldb = Y * Y; g.b_kmajor = true;
            g.C = Abar;
            g.rmap = IdxMap::split(X, (i64)X * Y * Y, Y);
            g.cmap = IdxMap::split(Y, (i64)X * Y, 1);
            c.gemm(g);
            // Bbar'[c][j][d][k] = sum_{(a,b)} Gt[(a,b)][(c,d)] A[(a,b)][(j,k)]
            g.A = P->Gt.p; g.a_kmajor = true;
            g.B = st.A.p;
            g.C = Bbar;
            c.gemm(g);
        }
        // Tbar[a][x][y][j] += 2 sum_{(b,k)} Abar'[(a,j)][(b,k)] TA[(b,k)][(x,y)]
        {
            GemmOp g;
            g.M = X * Y; g.N = X * Y; g.K = X * Y;
            g.A = Abar; g.lda = X * Y;
            g.B = P->TA.p; g.ldb = X * Y; g.b_kmajor = true;
            g.C = P->Tbar2.p;
            g.rmap = IdxMap::split(Y, (i64)X * Y * Y, 1);
            g.cmap = IdxMap::split(Y, (i64)Y * Y, Y);
            g.alpha = 2.0; g.beta = 1.0;
            c.gemm(g);
            // Tbar[a][x][j][y] += 2 sum_{(b,k)} Bbar'[(a,j)][(b,k)] TB[(b,k)][(x,y)]
            g.A = Bbar;
            g.B = P->TB.p;
            g.rmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
            g.cmap = IdxMap::split(Y, (i64)Y * Y, 1);
            c.gemm(g);
        }
        std::swap(P->Tbar, P->Tbar2);   // Tbar = gradient w.r.t. T_k
    }
    // T0bar[l][u][r][d] = permute(Tbar [l][r][u][d]) / c0
    const int D = P->D;
    permute_checked(P, P->Tbar.p, T0bar, pd4(D, D, D, D, 0, 2, 1, 3), 1.0 / P->c0, 0.0, nullptr, c.s);
    if (dT0 && dir_out) {
        dot(T0bar, dT0, (i64)D * D * D * D, P->scal.p + 5, c.s, P->ws);
        DTRG_HIP(hipMemcpyAsync(dir_out, P->scal.p + 5, sizeof(double), hipMemcpyDeviceToHost, c.s));
    }
    DTRG_HIP(hipStreamSynchronize(c.s));
}

dtrg_status fail(const Error& e) {
    g_last_error = e.what();
    return e.code;
}

}  // namespace

// -------------------------------------------------------------------------------------------
// C ABI
// -------------------------------------------------------------------------------------------
extern "C" {

void dtrg_default_options(dtrg_options* o) {
    if (!o) return;
    o->contract = DTRG_FP64;
    o->gram_fp64 = 1;
    o->eig_broadening = 1e-12;
    o->max_subspace_iters = 60;
    o->subspace_tol = 1e-15;
    o->block_size = 0;
    o->keep_projections = 0;
    o->profile = 0;
    o->bf16x3_mask = 15;
}

dtrg_status dtrg_plan_create(int D, int chi, int n_steps, const dtrg_options* opt, dtrg_plan** plan_out) {
    g_last_error.clear();
    if (plan_out) *plan_out = nullptr;
    std::unique_ptr<dtrg_plan> P;
    try {
        DTRG_REQUIRE(plan_out, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(D >= 1 && D <= 64, DTRG_EINVAL, "D out of range [1, 64]");
        DTRG_REQUIRE(chi >= 1 && chi <= 80, DTRG_EINVAL, "chi out of range [1, 80]");
        DTRG_REQUIRE(n_steps >= 1 && n_steps <= 62, DTRG_EINVAL, "n_steps out of range [1, 62]");
        P.reset(new dtrg_plan());
        dtrg_default_options(&P->opt);
        if (opt) P->opt = *opt;
        DTRG_REQUIRE(P->opt.contract == DTRG_FP64 || P->opt.contract == DTRG_FP32 || P->opt.contract == DTRG_BF16X3,
                     DTRG_EINVAL, "contract must be DTRG_FP64, DTRG_FP32 or DTRG_BF16X3");
        DTRG_REQUIRE(P->opt.bf16x3_mask >= 0 && P->opt.bf16x3_mask <= 15, DTRG_EINVAL, "bf16x3_mask out of range [0, 15]");
        DTRG_REQUIRE(P->opt.gram_fp64 == 1, DTRG_EINVAL, "the Gram is always formed in FP64 (gram_fp64 must be 1)");
        P->prec = P->opt.contract == DTRG_FP64 ? Prec::F64 : (P->opt.contract == DTRG_FP32 ? Prec::F32 : Prec::BF16X3);
        DTRG_REQUIRE(P->opt.eig_broadening >= 0.0 && std::isfinite(P->opt.eig_broadening), DTRG_EINVAL,
                     "eig_broadening must be finite and >= 0");
        DTRG_REQUIRE(P->opt.max_subspace_iters >= 1, DTRG_EINVAL, "max_subspace_iters must be >= 1");
        DTRG_REQUIRE(P->opt.block_size >= 0 && P->opt.block_size <= kJacobiMax, DTRG_EINVAL,
                     "block_size out of range [0, 96]");
        P->D = D; P->chi = chi; P->nsteps = n_steps;
        setup(P.get());
        *plan_out = P.release();
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_plan_forward(dtrg_plan* plan, const double* T0_dev, void* stream, double* lnZ_per_site_host) {
    g_last_error.clear();
    try {
        DTRG_REQUIRE(plan && T0_dev && lnZ_per_site_host, DTRG_EINVAL, "NULL argument");
        plan->fwd_ok = false;
        plan->s = (hipStream_t)stream;
        forward(plan, T0_dev);
        plan->fwd_ok = true;
        *lnZ_per_site_host = plan->lnZ;
        return DTRG_OK;
    } catch (const Error& e) {
        if (plan) (void)hipStreamSynchronize(plan->s);
        return fail(e);
    } catch (const std::exception& e) {
        if (plan) (void)hipStreamSynchronize(plan->s);
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_hotrg_forward(const double* T0_dev, int D, int chi, int n_steps, const dtrg_options* opt,
                               void* stream, dtrg_plan** plan_out, double* lnZ_per_site_host) {
    g_last_error.clear();
    if (plan_out) *plan_out = nullptr;
    if (!T0_dev || !plan_out || !lnZ_per_site_host) {
        g_last_error = "NULL argument";
        return DTRG_EINVAL;
    }
    dtrg_plan* P = nullptr;
    dtrg_status st = dtrg_plan_create(D, chi, n_steps, opt, &P);
    if (st != DTRG_OK) return st;
    st = dtrg_plan_forward(P, T0_dev, stream, lnZ_per_site_host);
    if (st != DTRG_OK) {
        const std::string msg = g_last_error;
        dtrg_plan_destroy(P);
        g_last_error = msg;
        return st;
    }
    *plan_out = P;
    return DTRG_OK;
}

dtrg_status dtrg_plan_profile(dtrg_plan* plan, long long* launches, double* total_ms, double* flops, int reset) {
    g_last_error.clear();
    try {
        DTRG_REQUIRE(plan && launches && total_ms && flops, DTRG_EINVAL, "NULL argument");
        double ms = 0.0;
        for (size_t i = 0; i + 1 < plan->ev_used; i += 2) {
            DTRG_HIP(hipEventSynchronize(plan->ev_pool[i + 1]));
            float t = 0.f;
            DTRG_HIP(hipEventElapsedTime(&t, plan->ev_pool[i], plan->ev_pool[i + 1]));
            ms += t;
        }
        *launches = (long long)(plan->ev_used / 2);
        *total_ms = ms;
        *flops = plan->prof_flops;
        if (reset) {
            plan->ev_used = 0;
            plan->prof_flops = 0.0;
        }
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

dtrg_status dtrg_hotrg_backward(dtrg_plan* plan, double gbar, double* T0bar_dev, const double* dT0_dev,
                                double* dlnZ_dir_host, void* stream) {
    g_last_error.clear();
    try {
        DTRG_REQUIRE(plan && T0bar_dev, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(plan->fwd_ok, DTRG_ESTATE, "backward before a successful forward");
        DTRG_REQUIRE(std::isfinite(gbar), DTRG_EINVAL, "gbar is not finite");
        plan->s = (hipStream_t)stream;
        backward(plan, gbar, T0bar_dev, dT0_dev, dlnZ_dir_host);
        return DTRG_OK;
    } catch (const Error& e) {
        if (plan) (void)hipStreamSynchronize(plan->s);
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_plan_step_info(const dtrg_plan* plan, int k, dtrg_step_info* info) {
    g_last_error.clear();
    if (!plan || !info) { g_last_error = "NULL argument"; return DTRG_EINVAL; }
    if (!plan->fwd_ok) { g_last_error = "plan has no successful forward"; return DTRG_ESTATE; }
    if (k < 1 || k > plan->nsteps) { g_last_error = "step index out of range"; return DTRG_EINVAL; }
    const StepCk& st = plan->steps[k - 1];
    info->X = st.sh.X; info->Y = st.sh.Y; info->chi_kept = st.sh.K; info->full_eig = st.sh.full ? 1 : 0;
    info->iters = st.iters; info->c = st.c; info->trace_G = st.t;
    info->lam_last_kept = st.lam_h.empty() ? 0.0 : st.lam_h[st.sh.K - 1];
    info->lam_first_dropped = (int)st.lam_h.size() > st.sh.K ? st.lam_h[st.sh.K] : 0.0;
    info->resid = st.resid;
    info->cheb_degree = st.cheb;
    return DTRG_OK;
}

size_t dtrg_plan_device_bytes(const dtrg_plan* plan) { return plan ? plan->bytes() : 0; }

void dtrg_plan_destroy(dtrg_plan* plan) {
    if (!plan) return;
    (void)hipStreamSynchronize(plan->s);
    delete plan;
}

const char* dtrg_last_error(void) { return g_last_error.c_str(); }

const char* dtrg_version(void) { return "dtrg 0.1 (gfx950)"; }

dtrg_status dtrg_contract(int precision, int M, int N, int K, const void* A_dev, long long lda, int a_kmajor,
                          const void* B_dev, long long ldb, int b_kmajor, void* C_dev, long long ldc, int out_f64,
                          double alpha, double beta, void* stream) {
    g_last_error.clear();
    static thread_local Scratch ws;
    try {
        DTRG_REQUIRE(A_dev && B_dev && C_dev, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(M >= 0 && N >= 0 && K >= 0, DTRG_EINVAL, "negative size");
        DTRG_REQUIRE(precision >= DTRG_FP64 && precision <= DTRG_BF16X3, DTRG_EINVAL, "bad precision");
        DTRG_REQUIRE(lda >= (a_kmajor ? M : K) && ldb >= (b_kmajor ? N : K) && ldc >= N, DTRG_EINVAL,
                     "leading dimension too small");
        GemmOp g;
        g.M = M; g.N = N; g.K = K;
        g.A = A_dev; g.lda = lda; g.a_kmajor = a_kmajor != 0;
        g.B = B_dev; g.ldb = ldb; g.b_kmajor = b_kmajor != 0;
        g.C = C_dev; g.rmap = IdxMap::linear(ldc); g.cmap = IdxMap::linear(1);
        g.alpha = alpha; g.beta = beta;
        const Prec pr = precision == DTRG_FP64 ? Prec::F64 : (precision == DTRG_FP32 ? Prec::F32 : Prec::BF16X3);
        dtrg::gemm(pr, precision == DTRG_FP64 ? true : out_f64 != 0, g, (hipStream_t)stream, ws);
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

}  // extern "C"
