// HOTRG forward pass and hand-written reverse pass of nb independent instances (gfx950).
//
// Layouts per instance (row-major, X = horizontal bond, Y = vertical bond, K = chi' kept,
// n = X^2, b = block); every plan buffer holds nb instances at its instance stride:
//   T   [l][r][u][d] = [X][X][Y][Y]        step input (the paper's T_{x x' y y'})
//   A,B [a][b][j][k] = [X][X][Y][Y]        half-environments of the Gram
//   G   [(a,c)][(b,d)] = n x n             Gram of the (x1, x2) unfolding, then sym / trace
//   U   [n][b]                             eigenvectors (first K columns are w[x1][x2][alpha])
//   P1  [alpha][y][i][b][j]                upper copy times the left isometry
//   Q2  [alpha][y][z][i][m]                P1 joined with the lower copy over (b, j)  (chi^7)
//   T'  [alpha][beta][y][z]                step output; the next input is T'/c permuted (2,3,0,1)
// Every contraction is one call of the MFMA kernel (instances are its outer batch level), whose
// scatter epilogue writes each result directly in the layout its consumer reads (index maps
// written next to each call).
//
// A step's checkpoint is its normalised input T, its eigenvectors and eigenvalues and a few
// scalars; the backward recomputes everything else of the step (the half-environments, the Gram
// and the projection intermediates) from it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace dtrg;

dtrg_plan::~dtrg_plan() {
    for (auto e : ev_pool) (void)hipEventDestroy(e);
}

i64 dtrg_plan::cap_bytes(const void* ptr) const {
    const char* q = (const char*)ptr;
    auto chk = [&](const void* base, size_t nbytes) -> i64 {
        const char* b = (const char*)base;
        if (b && q >= b && q < b + nbytes) return (i64)nbytes - (i64)(q - b);
        return -1;
    };
    const DevBuf<double>* w[] = {&TA, &TB, &Tp, &Tb, &Tb2, &Wt, &Wt2, &Tn, &Tbar, &Tbar2, &Tpbar, &A, &B, &P1, &Q2,
                                 &X5, &Gw, &Gt, &Ub, &Xe, &Xc, &Re, &Om, &Sm, &Vc, &Vp, &Vn, &Ye, &We, &V1, &V2,
                                 &Y1, &Y2, &H, &Z, &Rinv, &Sg, &th, &res, &nrm, &coef, &fv, &ctab, &scal, &T0buf,
                                 &T0barbuf, &dT0buf, &tune_c};
    for (auto* b : w) { const i64 r = chk(b->p, b->bytes()); if (r >= 0) return r; }
    const DevBuf<float>* f[] = {&Tpf, &Tbf, &Tb2f, &Wtf, &Wt2f, &Uf, &P1f, &Q2f, &X5f, &Tpbarf};
    for (auto* b : f) { const i64 r = chk(b->p, b->bytes()); if (r >= 0) return r; }
    for (auto& st : steps) {
        const DevBuf<double>* v[] = {&st.T, &st.U, &st.lam};
        for (auto* b : v) { const i64 r = chk(b->p, b->bytes()); if (r >= 0) return r; }
    }
    return -1;
}

size_t dtrg_plan::bytes() const {
    size_t t = 0;
    for (auto& st : steps) t += st.T.bytes() + st.U.bytes() + st.lam.bytes();
    const DevBuf<double>* w[] = {&TA, &TB, &Tp, &Tb, &Tb2, &Wt, &Wt2, &Tn, &Tbar, &Tbar2, &Tpbar, &A, &B, &P1, &Q2,
                                 &X5, &Gw, &Gt, &Ub, &Xe, &Xc, &Re, &Om, &Sm, &Vc, &Vp, &Vn, &Ye, &We, &V1, &V2,
                                 &Y1, &Y2, &H, &Z, &Rinv, &Sg, &th, &res, &nrm, &coef, &fv, &ctab, &scal, &T0buf,
                                 &T0barbuf, &dT0buf, &tune_c, &ws.splitk, &ws.red};
    for (auto* b : w) t += b->bytes();
    const DevBuf<float>* f[] = {&Tpf, &Tbf, &Tb2f, &Wtf, &Wt2f, &Uf, &P1f, &Q2f, &X5f, &Tpbarf};
    for (auto* b : f) t += b->bytes();
    return t + flags.bytes() + misc.bytes();
}

namespace dtrg {

namespace {

double ldexp1(int e) { return std::ldexp(1.0, e); }

constexpr double kSubspaceAccept = 1e-12;   // largest accepted resolved residual (trace-normalised)
constexpr double kChebTail = 1e-15;         // relative size of the last two expansion coefficients
constexpr int kChebMaxDegree = 1024;

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

// offset of the degree-m table in the plan's table buffer (m = 8, 16, ..., 1024)
i64 ctab_offset(int m) {
    i64 off = 0;
    for (int q = 8; q < m; q *= 2) off += (i64)(q + 1) * (q + 1);
    return off;
}
i64 ctab_total() { return ctab_offset(2 * kChebMaxDegree); }

// A device operand with its instance stride.
struct Opnd {
    const void* p = nullptr;
    i64 bs = 0;
};
template <class T> Opnd op_of(const DevBuf<T>& b) { Opnd o; o.p = b.p; o.bs = b.bs; return o; }

// -------------------------------------------------------------------------------------------
// contractions
// -------------------------------------------------------------------------------------------
struct Ctx {
    dtrg_plan* P;
    hipStream_t s;
    Mode mode;
    bool adaptive() const { return mode == Mode::Adaptive; }
    // one contraction in precision `pr` over the plan's nb instances (operand instance strides
    // set by the caller in a_bs2 / b_bs2 / c_bs2); operands of 8 (FP64) or 4 (FP32) bytes,
    // output FP64 or FP32
    void run(GemmOp g, Prec pr, bool out_f64) {
        g.batch2 = P->nb;
        const int ein = pr == Prec::F64 ? 8 : 4, eout = out_f64 ? 8 : 4;
        if (g.a_cap < 0) g.a_cap = P->cap_of(g.A, ein);
        if (g.b_cap < 0) g.b_cap = P->cap_of(g.B, ein);
        if (g.c_cap < 0) g.c_cap = P->cap_of(g.C, eout);
        if (P->opt.autotune) g.cfg = tuned_cfg(pr, out_f64, g, adaptive(), s, P->ws, P->tune_c);
        const bool timed = P->opt.profile && g.tag == 7 && adaptive();
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
            P->prof_flops += 2.0 * g.M * (double)g.N * g.K * g.batch * g.batch2;
        }
    }
    // FP64 contraction (Gram, eigensolver, eigen-adjoint)
    void gemm(const GemmOp& op) { run(op, Prec::F64, true); }
    // projection contraction in precision pr (FP64 operands always write FP64)
    void gemmc(const GemmOp& op, Prec pr, bool out_f64) { run(op, pr, pr == Prec::F64 ? true : out_f64); }
};

void set_bs(GemmOp& g, i64 a, i64 b, i64 c) { g.a_bs2 = a; g.b_bs2 = b; g.c_bs2 = c; }

// permutes over all instances with the capacities of plan-owned buffers checked on the host
void permute_checked(dtrg_plan* P, const DevBuf<double>& in, double* out, i64 out_bs, PermDesc d, double alpha,
                     const double* scale_dev, hipStream_t s) {
    d.nb = P->nb;
    d.in_bs = in.bs;
    d.out_bs = out_bs;
    d.in_cap = P->cap_of(in.p);
    d.out_cap = P->cap_of(out);
    dtrg::permute(in.p, out, d, alpha, 0.0, scale_dev, P->S, s);
}

void permute_f32_checked(dtrg_plan* P, const DevBuf<double>& in, DevBuf<float>& out, PermDesc d, hipStream_t s) {
    d.nb = P->nb;
    d.in_bs = in.bs;
    d.out_bs = out.bs;
    d.in_cap = P->cap_of(in.p, 8);
    d.out_cap = P->cap_of(out.p, 4);
    dtrg::permute_to_f32(in.p, out.p, d, s);
}

// A[a][b][j][k] = sum_{x,y} TA[(a,j)][(x,y)] TA[(b,k)][(x,y)]  (also B with TB)
void half_env(Ctx& c, const DevBuf<double>& Tperm, DevBuf<double>& out, int X, int Y) {
    GemmOp g;
    g.M = g.N = X * Y; g.K = X * Y;
    g.A = Tperm.p; g.lda = X * Y;
    g.B = Tperm.p; g.ldb = X * Y;
    g.C = out.p;
    g.rmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
    g.cmap = IdxMap::split(Y, (i64)Y * Y, 1);
    set_bs(g, Tperm.bs, Tperm.bs, out.bs);
    c.gemm(g);
}

// G[(a,c)][(b,d)] = sum_{(j,k)} A[(a,b),(j,k)] B[(c,d),(j,k)]
void gram(Ctx& c, const DevBuf<double>& A, const DevBuf<double>& B, DevBuf<double>& G, int X, int Y) {
    GemmOp g;
    g.M = g.N = X * X; g.K = Y * Y;
    g.A = A.p; g.lda = Y * Y;
    g.B = B.p; g.ldb = Y * Y;
    g.C = G.p;
    g.rmap = IdxMap::split(X, (i64)X * X * X, X);
    g.cmap = IdxMap::split(X, (i64)X * X, 1);
    set_bs(g, A.bs, B.bs, G.bs);
    c.gemm(g);
}

// Gram of step input T (checkpoint), normalised: TA, TB, A, B, then G in Gw with its trace in
// sc(k, 2).  Shared by the forward pass and the backward recompute.
void gram_of_step(Ctx& c, const StepCk& st, int k) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n;
    permute_checked(P, st.T, P->TA.p, P->TA.bs, pd4(X, X, Y, Y, 0, 3, 1, 2), 1.0, nullptr, c.s);
    permute_checked(P, st.T, P->TB.p, P->TB.bs, pd4(X, X, Y, Y, 0, 2, 1, 3), 1.0, nullptr, c.s);
    half_env(c, P->TA, P->A, X, Y);
    half_env(c, P->TB, P->B, X, Y);
    gram(c, P->A, P->B, P->Gw, X, Y);
    sym_normalise(P->Gw.p, P->Gw.bs, n, P->nb, P->sc(k, 2), P->S, P->flags.p, c.s);
}

// P1[alpha][y][i][b][j] = sum_a Wt[(alpha,b)][a] Tp[y][(i,j)][a]   (batched over y)
void proj1(Ctx& c, Prec pr, Opnd Wt, Opnd Tp, Opnd P1, int X, int Y, int K) {
    GemmOp g;
    g.M = K * X; g.N = X * Y; g.K = X; g.batch = Y;
    g.A = Wt.p; g.lda = X; g.a_bs = 0;
    g.B = Tp.p; g.ldb = X; g.b_bs = (i64)X * Y * X;
    g.C = (void*)P1.p; g.c_bs = (i64)X * X * Y;
    g.rmap = IdxMap::split(X, (i64)Y * X * X * Y, Y);
    g.cmap = IdxMap::split(Y, (i64)X * Y, 1);
    set_bs(g, Wt.bs, Tp.bs, P1.bs);
    c.gemmc(g, pr, false);
}

// Q2[alpha][y][z][i][m] = sum_{(b,j)} P1[(alpha,y,i)][(b,j)] Tb[(z,m)][(b,j)]      (the chi^7 term)
void proj2(Ctx& c, Prec pr, Opnd P1, Opnd Tb, Opnd Q2, int X, int Y, int K) {
    GemmOp g;
    g.tag = 7;
    g.M = K * Y * X; g.N = Y * X; g.K = X * Y;
    g.A = P1.p; g.lda = X * Y;
    g.B = Tb.p; g.ldb = X * Y;
    g.C = (void*)Q2.p;
    g.rmap = IdxMap::split(X, (i64)Y * X * X, X);
    g.cmap = IdxMap::split(X, (i64)X * X, 1);
    set_bs(g, P1.bs, Tb.bs, Q2.bs);
    c.gemmc(g, pr, false);
}

// T'[alpha][beta][y][z] = sum_{(i,m)} Q2[(alpha,y,z)][(i,m)] w[(i,m)][beta]
void proj3(Ctx& c, Prec pr, Opnd Q2, Opnd U, int ldu, DevBuf<double>& Tn, int X, int Y, int K) {
    GemmOp g;
    g.M = K * Y * Y; g.N = K; g.K = X * X;
    g.A = Q2.p; g.lda = X * X;
    g.B = U.p; g.ldb = ldu; g.b_kmajor = true;
    g.C = Tn.p;
    g.rmap = IdxMap::split((i64)Y * Y, (i64)K * Y * Y, 1);
    g.cmap = IdxMap::linear((i64)Y * Y);
    set_bs(g, Q2.bs, U.bs, Tn.bs);
    c.gemmc(g, pr, true);
}

// Contraction operands of one step, in the contraction precision.
struct Ops {
    Opnd Tp, Tb, Tb2, Wt, Wt2, U;
    Opnd P1, Q2, X5, Tpbar;
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
        permute_checked(P, st.T, P->Tp.p, P->Tp.bs, pd4(X, X, Y, Y, 2, 1, 3, 0), 1.0, nullptr, c.s);
        permute_checked(P, st.T, P->Tb.p, P->Tb.bs, pd4(X, X, Y, Y, 3, 1, 0, 2), 1.0, nullptr, c.s);
        permute_checked(P, st.U, P->Wt.p, P->Wt.bs, pd3(X, X, b, 2, 1, 0), 1.0, nullptr, c.s);
        if (need_wt2) {
            permute_checked(P, st.U, P->Wt2.p, P->Wt2.bs, pd3(X, X, b, 0, 2, 1), 1.0, nullptr, c.s);
            permute_checked(P, st.T, P->Tb2.p, P->Tb2.bs, pd4(X, X, Y, Y, 3, 1, 2, 0), 1.0, nullptr, c.s);
        }
        o.Tp = op_of(P->Tp); o.Tb = op_of(P->Tb); o.Tb2 = op_of(P->Tb2); o.Wt = op_of(P->Wt);
        o.Wt2 = op_of(P->Wt2); o.U = op_of(st.U);
        o.P1 = op_of(P->P1); o.Q2 = op_of(P->Q2); o.X5 = op_of(P->X5); o.Tpbar = op_of(P->Tpbar);
    } else {
        permute_f32_checked(P, st.T, P->Tpf, pd4(X, X, Y, Y, 2, 1, 3, 0), c.s);
        permute_f32_checked(P, st.T, P->Tbf, pd4(X, X, Y, Y, 3, 1, 0, 2), c.s);
        permute_f32_checked(P, st.U, P->Wtf, pd3(X, X, b, 2, 1, 0), c.s);
        if (need_wt2) {
            permute_f32_checked(P, st.U, P->Wt2f, pd3(X, X, b, 0, 2, 1), c.s);
            permute_f32_checked(P, st.T, P->Tb2f, pd4(X, X, Y, Y, 3, 1, 2, 0), c.s);
        }
        DTRG_REQUIRE(P->Uf.bs >= (i64)n * b, DTRG_EINVAL, "FP32 isometry buffer too small");
        convert_f64_to_f32(st.U.p, st.U.bs, P->Uf.p, P->Uf.bs, (i64)n * b, P->nb, c.s);
        o.Tp = op_of(P->Tpf); o.Tb = op_of(P->Tbf); o.Tb2 = op_of(P->Tb2f); o.Wt = op_of(P->Wtf);
        o.Wt2 = op_of(P->Wt2f); o.U = op_of(P->Uf);
        o.P1 = op_of(P->P1f); o.Q2 = op_of(P->Q2f); o.X5 = op_of(P->X5f); o.Tpbar = op_of(P->Tpbarf);
    }
    return o;
}

// -------------------------------------------------------------------------------------------
// host read-back helpers (adaptive passes only)
// -------------------------------------------------------------------------------------------
// column `slot` of the per-instance scalars (nb values)
std::vector<double> read_scalar(dtrg_plan* P, const double* col) {
    std::vector<double> v(P->nb);
    DTRG_HIP(hipMemcpy2DAsync(v.data(), sizeof(double), col, P->S * sizeof(double), sizeof(double), P->nb,
                              hipMemcpyDeviceToHost, P->s));
    DTRG_HIP(hipStreamSynchronize(P->s));
    return v;
}

std::vector<int> read_flags(dtrg_plan* P) {
    std::vector<int> f(P->nb);
    DTRG_HIP(hipMemcpyAsync(f.data(), P->flags.p, P->nb * sizeof(int), hipMemcpyDeviceToHost, P->s));
    DTRG_HIP(hipStreamSynchronize(P->s));
    return f;
}

std::string inst_name(const dtrg_plan* P, int i) {
    return P->nb > 1 ? "instance " + std::to_string(i) + ": " : std::string();
}

// throw for the first instance whose flags intersect `mask`
void throw_flags(const dtrg_plan* P, const std::vector<int>& f, int mask, const std::string& where,
                 bool input_stage = false) {
    for (int i = 0; i < P->nb; ++i) {
        const int b = f[i] & mask;
        if (!b) continue;
        const std::string pre = inst_name(P, i) + where + ": ";
        if (b & kFlagNonFinite) {
            if (input_stage) throw Error(DTRG_EINVAL, pre + "T0 has non-finite entries");
            throw Error(DTRG_ENONPOS, pre + "a norm or trace is not finite");
        }
        if (b & kFlagNonPos) {
            if (input_stage) throw Error(DTRG_ENONPOS, pre + "T0 is zero");
            throw Error(DTRG_ENONPOS, pre + "a norm or trace is not positive and finite");
        }
        if (b & kFlagSubspace) throw Error(DTRG_ENOCONV, pre + "truncated eigensolve did not converge");
        if (b & kFlagChebTail)
            throw Error(DTRG_ENOCONV, pre + "eigen-adjoint: complement expansion coefficients did not decay");
        if (b & kFlagChebBound) throw Error(DTRG_ENOCONV, pre + "eigen-adjoint: complement expansion diverged");
        throw Error(DTRG_ENOCONV, pre + "flag " + std::to_string(b));
    }
}

void check_flags(dtrg_plan* P, int mask, const std::string& where, bool input_stage = false) {
    throw_flags(P, read_flags(P), mask, where, input_stage);
}

constexpr int kFlagErrors = kFlagNonPos | kFlagNonFinite | kFlagSubspace | kFlagChebTail | kFlagChebBound;

// -------------------------------------------------------------------------------------------
// truncated eigensolve
// -------------------------------------------------------------------------------------------

// Orthonormalise the n x b blocks V (instance stride vbs) in place: a shifted CholeskyQR pass
// (stable for any condition number up to 1/u, which the normalised iterate can reach when the
// Gram has a cluster of noise-level eigenvalues) followed by two plain passes.
void orthonormalise(Ctx& c, double* V, double* Vtmp, i64 vbs, int n, int b) {
    dtrg_plan* P = c.P;
    double* cur = V;
    double* oth = Vtmp;
    for (int pass = 0; pass < 3; ++pass) {
        GemmOp g;
        g.M = g.N = b; g.K = n;
        g.A = cur; g.lda = b; g.a_kmajor = true;
        g.B = cur; g.ldb = b; g.b_kmajor = true;
        g.C = P->Sg.p;
        g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
        set_bs(g, vbs, vbs, P->Sg.bs);
        c.gemm(g);
        const double shift = pass == 0 ? 11.0 * ((double)n * b + (double)b * (b + 1)) * std::ldexp(1.0, -53) : 0.0;
        chol_inverse(P->Sg.p, P->Sg.bs, b, shift, P->Rinv.p, P->Rinv.bs, P->nb, P->flags.p, c.s);
        GemmOp h;
        h.M = n; h.N = b; h.K = b;
        h.A = cur; h.lda = b;
        h.B = P->Rinv.p; h.ldb = b; h.b_kmajor = true;
        h.C = oth;
        h.rmap = IdxMap::linear(b); h.cmap = IdxMap::linear(1);
        set_bs(h, vbs, P->Rinv.bs, vbs);
        c.gemm(h);
        std::swap(cur, oth);
    }
    if (cur != V) copy2d(cur, b, vbs, V, b, vbs, n, b, P->nb, c.s);
}

// C (n x b) = G (n x n) V (n x b)
void gemm_GV(Ctx& c, const DevBuf<double>& G, const double* V, double* C, i64 vbs, int n, int b) {
    GemmOp g;
    g.M = n; g.N = b; g.K = n;
    g.A = G.p; g.lda = n;
    g.B = V; g.ldb = b; g.b_kmajor = true;
    g.C = C;
    g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
    set_bs(g, G.bs, vbs, vbs);
    c.gemm(g);
}

void eigensolve(Ctx& c, StepCk& st, int k, const StepCk* warm) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n, b = st.sh.b, E = st.sh.e, nb = P->nb;
    const uint64_t seed = 0x5eedULL * (uint64_t)k + 17ULL;
    if (st.sh.full) {
        jacobi_eig(P->Gw.p, n, n, P->Gw.bs, st.lam.p, st.lam.bs, st.U.p, n, st.U.bs, nb, 40, P->misc.p, c.s);
        st.iters = 0;
        return;
    }
    // block subspace iteration with Rayleigh-Ritz on the normalised Gram
    const i64 vbs = P->V1.bs;
    // warm start: the Ritz vectors of the previous step in the same direction (orthonormal already)
    const bool warm_used = warm && warm->sh.n == n && warm->sh.b == b;
    if (warm_used) {
        copy2d(warm->U.p, b, warm->U.bs, P->V1.p, b, vbs, n, b, nb, c.s);
    } else {
        hash_fill(P->V1.p, vbs, (i64)n * b, nb, seed, c.s);
        orthonormalise(c, P->V1.p, P->V2.p, vbs, n, b);
    }
    const double tol = P->opt.subspace_tol;
    const int it_max = c.adaptive() ? P->opt.max_subspace_iters : st.iters;
    DTRG_REQUIRE(it_max >= 1, DTRG_ESTATE, "no recorded subspace iteration count for this step");
    double prev = INFINITY;
    int stall = 0, it = 0;
    std::vector<double> resh((size_t)nb * P->res.bs);
    for (it = 1; it <= it_max; ++it) {
        double* V = P->V1.p;
        double* Y = P->Y1.p;
        gemm_GV(c, P->Gw, V, Y, vbs, n, b);
        // H = V^T Y
        GemmOp g;
        g.M = g.N = b; g.K = n;
        g.A = V; g.lda = b; g.a_kmajor = true;
        g.B = Y; g.ldb = b; g.b_kmajor = true;
        g.C = P->H.p;
        g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
        set_bs(g, vbs, vbs, P->H.bs);
        c.gemm(g);
        jacobi_eig(P->H.p, b, b, P->H.bs, P->th.p, P->th.bs, P->Z.p, b, P->Z.bs, nb, 40, P->misc.p, c.s);
        // V <- V Z, Y <- Y Z
        GemmOp r;
        r.M = n; r.N = b; r.K = b;
        r.B = P->Z.p; r.ldb = b; r.b_kmajor = true;
        r.rmap = IdxMap::linear(b); r.cmap = IdxMap::linear(1);
        r.A = V; r.lda = b; r.C = P->V2.p; set_bs(r, vbs, P->Z.bs, vbs); c.gemm(r);
        r.A = Y; r.lda = b; r.C = P->Y2.p; c.gemm(r);
        std::swap(P->V1, P->V2);
        std::swap(P->Y1, P->Y2);
        ritz_residuals(P->V1.p, P->Y1.p, n, E, b, vbs, P->th.p, P->th.bs, P->res.p, P->res.bs, nb, c.s);
        if (c.adaptive()) {
            DTRG_HIP(hipMemcpyAsync(resh.data(), P->res.p, resh.size() * sizeof(double), hipMemcpyDeviceToHost, c.s));
            DTRG_HIP(hipStreamSynchronize(c.s));
            double mx = 0.0;
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < E; ++j) {
                    const double v = resh[(size_t)i * P->res.bs + j];
                    mx = std::max(mx, std::isfinite(v) ? v : INFINITY);
                }
            if (mx <= tol) break;
            if (mx > 0.5 * prev) ++stall; else stall = 0;
            prev = mx;
            if (stall >= 3 && mx <= kSubspaceAccept) break;      // rounding floor reached
        }
        if (it == it_max) break;
        // next block: G V with columns rescaled to unit norm, re-orthonormalised
        col_norms(P->Y1.p, n, b, b, vbs, P->nrm.p, P->nrm.bs, nb, c.s);
        col_normalise(P->Y1.p, n, b, b, vbs, P->nrm.p, P->nrm.bs, nb, seed + 7919ULL * it, c.s);
        std::swap(P->V1, P->Y1);
        orthonormalise(c, P->V1.p, P->V2.p, vbs, n, b);
    }
    if (c.adaptive()) st.iters = std::min(it, it_max);
    // acceptance of the resolved pairs, on the device (the fixed pass reports it afterwards)
    max_check(P->res.p, P->res.bs, E, nb, kSubspaceAccept, P->sc(k, 8), P->S, P->flags.p, kFlagSubspace, c.s);
    if (c.adaptive()) {
        const std::vector<int> f = read_flags(P);
        for (int i = 0; i < nb; ++i)
            if (f[i] & kFlagSubspace) {
                const std::vector<double> rr = read_scalar(P, P->sc(k, 8));
                throw Error(DTRG_ENOCONV, inst_name(P, i) + "step " + std::to_string(k) +
                                              ": truncated eigensolve residual " + std::to_string(rr[i]) +
                                              " after " + std::to_string(st.iters) + " iterations");
            }
    }
    copy2d(P->V1.p, b, vbs, st.U.p, b, st.U.bs, n, b, nb, c.s);
    if (E < b) {
        ritz_residuals(P->V1.p, P->Y1.p, n, E + 1, b, vbs, P->th.p, P->th.bs, P->res.p, P->res.bs, nb, c.s);
        copy2d(P->res.p + E, 1, P->res.bs, P->sc(k, 3), 1, P->S, 1, 1, nb, c.s);
    }
    copy2d(P->th.p, b, P->th.bs, st.lam.p, b, st.lam.bs, 1, b, nb, c.s);
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
            // at least one guard column beyond the kept ones: the complement expansion reads the
            // first unresolved Ritz pair (index e < b)
            DTRG_REQUIRE(b > s.K, DTRG_EINVAL, "block size must exceed chi'");
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
    const int nb = P->nb;
    const i64 D4 = (i64)P->D * P->D * P->D * P->D;
    i64 t4 = D4, n2 = 1, nbk = 1, bmax = 1, nK = 1, bK = 1, KK = 1, Kmax = 1;
    i64 t4d = 1, t5d = 1, bX2d = 1, t4f = 1, t5f = 1, bX2f = 1, nbf = 1;   // per-precision operand sizes
    bool any_d = false, any_f = false;
    for (auto& s : sh) {
        const i64 a4 = std::max<i64>((i64)s.X * s.X * s.Y * s.Y, (i64)s.K * s.K * s.Y * s.Y);
        const i64 a5 = (i64)s.K * s.Y * s.X * s.X * s.Y, ab = (i64)s.b * s.X * s.X;
        t4 = std::max(t4, a4);
        n2 = std::max<i64>(n2, (i64)s.n * s.n);
        nbk = std::max<i64>(nbk, (i64)s.n * s.b);
        bmax = std::max<i64>(bmax, s.b);
        nK = std::max<i64>(nK, (i64)s.n * s.K);
        bK = std::max<i64>(bK, (i64)s.b * s.K);
        KK = std::max<i64>(KK, (i64)s.K * s.K);
        Kmax = std::max<i64>(Kmax, s.K);
        if (s.mixed) {
            any_f = true;
            t4f = std::max(t4f, a4); t5f = std::max(t5f, a5); bX2f = std::max(bX2f, ab);
            nbf = std::max<i64>(nbf, (i64)s.n * s.b);
        } else {
            any_d = true;
            t4d = std::max(t4d, a4); t5d = std::max(t5d, a5); bX2d = std::max(bX2d, ab);
        }
    }
    P->T0buf.alloc_inst(nb, D4); P->T0barbuf.alloc_inst(nb, D4); P->dT0buf.alloc_inst(nb, D4);
    for (DevBuf<double>* b : {&P->TA, &P->TB, &P->Tn, &P->Tbar, &P->Tbar2, &P->Tpbar, &P->A, &P->B})
        b->alloc_inst(nb, t4);
    if (any_d) {
        P->Tp.alloc_inst(nb, t4d); P->Tb.alloc_inst(nb, t4d); P->Tb2.alloc_inst(nb, t4d);
        P->Wt.alloc_inst(nb, bX2d); P->Wt2.alloc_inst(nb, bX2d);
        P->P1.alloc_inst(nb, t5d); P->Q2.alloc_inst(nb, t5d); P->X5.alloc_inst(nb, t5d);
    }
    if (any_f) {
        P->Tpf.alloc_inst(nb, t4f); P->Tbf.alloc_inst(nb, t4f); P->Tb2f.alloc_inst(nb, t4f);
        P->Tpbarf.alloc_inst(nb, t4f);
        P->Wtf.alloc_inst(nb, bX2f); P->Wt2f.alloc_inst(nb, bX2f); P->Uf.alloc_inst(nb, nbf);
        P->P1f.alloc_inst(nb, t5f); P->Q2f.alloc_inst(nb, t5f); P->X5f.alloc_inst(nb, t5f);
    }
    P->Gw.alloc_inst(nb, n2); P->Gt.alloc_inst(nb, n2);
    for (DevBuf<double>* b : {&P->V1, &P->V2, &P->Y1, &P->Y2}) b->alloc_inst(nb, nbk);
    for (DevBuf<double>* b : {&P->H, &P->Z, &P->Rinv, &P->Sg}) b->alloc_inst(nb, bmax * bmax);
    for (DevBuf<double>* b : {&P->th, &P->res, &P->nrm}) b->alloc_inst(nb, bmax);
    // eigen-adjoint: every n x K block shares one instance stride (the Chebyshev step reads
    // five of them with a single stride)
    for (DevBuf<double>* b : {&P->Ub, &P->Xe, &P->Xc, &P->Re, &P->Vc, &P->Vp, &P->Vn, &P->Ye}) b->alloc_inst(nb, nK);
    P->We.alloc_inst(nb, std::max(bK, nK));
    P->Om.alloc_inst(nb, bK);
    P->Sm.alloc_inst(nb, std::max(KK, bK));
    P->coef.alloc_inst(nb, (i64)(kChebMaxDegree + 1) * Kmax);
    P->fv.alloc_inst(nb, (i64)(kChebMaxDegree + 1) * Kmax);
    P->ctab.alloc(ctab_total());
    P->ctab_ready = false;
    P->S = kScPlan + (i64)kScStep * P->nsteps;
    P->scal.alloc_inst(nb, P->S);
    P->flags.alloc_inst(nb, 1);
    P->misc.alloc(4);
    P->steps.clear();
    P->steps.resize(sh.size());
    for (size_t k = 0; k < sh.size(); ++k) {
        StepCk& st = P->steps[k];
        st.sh = sh[k];
        const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n, b = st.sh.b;
        st.T.alloc_inst(nb, (i64)X * X * Y * Y);
        st.U.alloc_inst(nb, (i64)n * b);
        st.lam.alloc_inst(nb, b);
    }
}

// -------------------------------------------------------------------------------------------
// backward helpers
// -------------------------------------------------------------------------------------------

// Gradient with respect to the normalised Gram, G_bar = (W U_K^T + U_K W^T) / t, from the
// gradient U_bar (n x K, in P->Ub) with respect to the kept eigenvectors U_K, written to P->Gt
// in the layout Gt[(a,b)][(c,d)] = G_bar[(a,c)][(b,d)] that the half-environment adjoints read.
//   kept block:    W += U_K S / 2,  S = F o (Om - Om^T) / 2,  Om = U_K^T U_bar
//   complement:    W += sum_{i discarded} u_i F(lam_j - lam_i) (u_i^T u_bar_j) / 2
// F(d) = d / (d^2 + eps).  The discarded pairs that are resolved (all of them for Jacobi steps;
// those nearest the cut, K <= i < e, for subspace steps) enter explicitly.  For subspace steps
// the remainder is f_j(G_r) P_e u_bar_j with G_r = P_e G P_e, P_e the projector off the e
// resolved vectors, evaluated by a Chebyshev expansion of f_j on an interval [lo, hi] holding
// the spectrum of G_r (which lies below the first unresolved eigenvalue, far from the poles
// lam_j +- i sqrt(eps) of f_j).  The normalised Gram G is in P->Gw.
void eig_adjoint(Ctx& c, StepCk& st, int k) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n, b = st.sh.b, K = st.sh.K, E = st.sh.e, X = st.sh.X, nb = P->nb;
    const double eps = P->opt.eig_broadening;
    const double* U = st.U.p;
    const i64 ubs = st.U.bs, vbs = P->Ub.bs;
    // Om = U_K^T U_bar (K x K), S on the kept block
    GemmOp g;
    g.M = K; g.N = K; g.K = n;
    g.A = U; g.lda = b; g.a_kmajor = true;
    g.B = P->Ub.p; g.ldb = K; g.b_kmajor = true;
    g.C = P->Om.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
    set_bs(g, ubs, vbs, P->Om.bs);
    c.gemm(g);
    kept_block_adjoint(P->Om.p, P->Om.bs, st.lam.p, st.lam.bs, K, eps, P->Sm.p, P->Sm.bs, nb, c.s);
    // R = P_K U_bar = U_bar - U_K Om
    copy2d(P->Ub.p, K, vbs, P->Re.p, K, vbs, n, K, nb, c.s);
    GemmOp r;
    r.M = n; r.N = K; r.K = K;
    r.A = U; r.lda = b;
    r.B = P->Om.p; r.ldb = K; r.b_kmajor = true;
    r.C = P->Re.p; r.rmap = IdxMap::linear(K); r.cmap = IdxMap::linear(1);
    r.alpha = -1.0; r.beta = 1.0;
    set_bs(r, ubs, P->Om.bs, vbs);
    c.gemm(r);
    fill(P->Xe.p, vbs, (i64)n * K, nb, 0.0, c.s);
    const int p = E - K;   // resolved discarded pairs
    if (p > 0) {
        // Om_D = U_D^T R (p x K);  X = U_D [F o Om_D] / 2;  R <- R - U_D Om_D
        GemmOp o;
        o.M = p; o.N = K; o.K = n;
        o.A = U + K; o.lda = b; o.a_kmajor = true;
        o.B = P->Re.p; o.ldb = K; o.b_kmajor = true;
        o.C = P->We.p; o.rmap = IdxMap::linear(K); o.cmap = IdxMap::linear(1);
        set_bs(o, ubs, vbs, P->We.bs);
        c.gemm(o);
        over_block_adjoint(P->We.p, P->We.bs, st.lam.p, st.lam.bs, p, K, eps, P->Vc.p, vbs, nb, c.s);
        GemmOp x;
        x.M = n; x.N = K; x.K = p;
        x.A = U + K; x.lda = b;
        x.B = P->Vc.p; x.ldb = K; x.b_kmajor = true;
        x.C = P->Xe.p; x.rmap = IdxMap::linear(K); x.cmap = IdxMap::linear(1);
        set_bs(x, ubs, vbs, vbs);
        c.gemm(x);
        if (!st.sh.full) {
            x.B = P->We.p; x.C = P->Re.p; x.alpha = -1.0; x.beta = 1.0;
            set_bs(x, ubs, P->We.bs, vbs);
            c.gemm(x);
        }
    }
    if (!st.sh.full) {
        auto apply_Gr = [&](const double* v) {
            // Ye = G v - U_e (U_e^T G v)
            GemmOp a;
            a.M = n; a.N = K; a.K = n;
            a.A = P->Gw.p; a.lda = n;
            a.B = v; a.ldb = K; a.b_kmajor = true;
            a.C = P->Ye.p; a.rmap = IdxMap::linear(K); a.cmap = IdxMap::linear(1);
            set_bs(a, P->Gw.bs, vbs, vbs);
            c.gemm(a);
            GemmOp w;
            w.M = E; w.N = K; w.K = n;
            w.A = U; w.lda = b; w.a_kmajor = true;
            w.B = P->Ye.p; w.ldb = K; w.b_kmajor = true;
            w.C = P->We.p; w.rmap = IdxMap::linear(K); w.cmap = IdxMap::linear(1);
            set_bs(w, ubs, vbs, P->We.bs);
            c.gemm(w);
            GemmOp u;
            u.M = n; u.N = K; u.K = E;
            u.A = U; u.lda = b;
            u.B = P->We.p; u.ldb = K; u.b_kmajor = true;
            u.C = P->Ye.p; u.rmap = IdxMap::linear(K); u.cmap = IdxMap::linear(1);
            u.alpha = -1.0; u.beta = 1.0;
            set_bs(u, ubs, P->We.bs, vbs);
            c.gemm(u);
        };
        // interval and coefficients of degree m: coef[q][j] = sum_k ct[q][k] f_j(t_k)
        auto coefficients = [&](int m, double mult) {
            cheb_interval(st.lam.p, st.lam.bs, E, P->sc(k, 3), P->S, n, mult, P->sc(k, 4), P->S, nb, c.s);
            cheb_fvals(st.lam.p, st.lam.bs, K, eps, P->sc(k, 4), P->S, m, P->fv.p, P->fv.bs, nb, c.s);
            GemmOp q;
            q.M = m + 1; q.N = K; q.K = m + 1;
            q.A = P->ctab.p + ctab_offset(m); q.lda = m + 1;
            q.B = P->fv.p; q.ldb = K; q.b_kmajor = true;
            q.C = P->coef.p; q.rmap = IdxMap::linear(K); q.cmap = IdxMap::linear(1);
            set_bs(q, 0, P->fv.bs, P->coef.bs);
            c.gemm(q);
            cheb_tail(P->coef.p, P->coef.bs, m, K, P->sc(k, 9), P->S, nb, c.s);
        };
        // Xc = sum_q c_q T_q(s(G_r)) R with s mapping [lo, hi] to [-1, 1]; |T_m(s(G_r)) R| into sc(k, 7)
        auto expansion = [&](int m) {
            fill(P->Xc.p, vbs, (i64)n * K, nb, 0.0, c.s);
            // v0 = R_rest (kept in Re), v1 = s(G_r) v0, v_{q+1} = 2 s(G_r) v_q - v_{q-1}
            apply_Gr(P->Re.p);
            cheb_step(P->Ye.p, P->Re.p, nullptr, P->Vn.p, P->Xc.p, vbs, n, K, P->sc(k, 4), P->S, true, P->coef.p,
                      P->coef.bs, nb, c.s);
            double* prv = P->Re.p;
            double* cur = P->Vn.p;
            double* nxt = P->Vc.p;
            double* spare = P->Vp.p;
            for (int q = 2; q <= m; ++q) {
                apply_Gr(cur);
                cheb_step(P->Ye.p, cur, prv, nxt, P->Xc.p, vbs, n, K, P->sc(k, 4), P->S, false,
                          P->coef.p + (size_t)q * K, P->coef.bs, nb, c.s);
                double* t = (prv == P->Re.p) ? spare : prv;   // R_rest is never overwritten
                prv = cur;
                cur = nxt;
                nxt = t;
            }
            // |T_m(s(G_r)) v0| <= |v0| when the spectrum lies in [lo, hi] (up to rounding)
            norm2(cur, vbs, (i64)n * K, nb, P->sc(k, 7), P->S, c.s, P->ws);
            cheb_bound_check(P->sc(k, 7), P->sc(k, 6), P->S, nb, P->flags.p, kFlagChebBound, c.s);
        };
        norm2(P->Re.p, vbs, (i64)n * K, nb, P->sc(k, 6), P->S, c.s, P->ws);
        if (c.adaptive()) {
            if (!P->ctab_ready) {
                for (int m = 8; m <= kChebMaxDegree; m *= 2) cheb_table(P->ctab.p + ctab_offset(m), m, c.s);
                P->ctab_ready = true;
            }
            bool ok = false;
            double mult = 1.0;
            int m = 8;
            std::string trail;
            for (int attempt = 0; attempt < 4 && !ok; ++attempt, mult *= 4.0) {
                for (m = 8;; m *= 2) {
                    coefficients(m, mult);
                    const std::vector<double> ratio = read_scalar(P, P->sc(k, 9));
                    double mx = 0.0;
                    for (double v : ratio) mx = std::max(mx, std::isfinite(v) ? v : INFINITY);
                    if (mx <= kChebTail || m >= kChebMaxDegree) break;
                }
                expansion(m);
                std::vector<int> f = read_flags(P);
                ok = true;
                for (int i = 0; i < nb; ++i) ok = ok && !(f[i] & kFlagChebBound);
                if (!ok) {
                    const std::vector<double> vm = read_scalar(P, P->sc(k, 7)), v0 = read_scalar(P, P->sc(k, 6)),
                                              lh = read_scalar(P, P->sc(k, 5));
                    for (int i = 0; i < nb; ++i)
                        if (f[i] & kFlagChebBound) {
                            trail += " [" + inst_name(P, i) + "hi " + std::to_string(lh[i]) + " m " + std::to_string(m) +
                                     " |v_m|/|v_0| " + std::to_string(vm[i] / v0[i]) + "]";
                            f[i] &= ~kFlagChebBound;
                        }
                    DTRG_HIP(hipMemcpyAsync(P->flags.p, f.data(), nb * sizeof(int), hipMemcpyHostToDevice, c.s));
                    DTRG_HIP(hipStreamSynchronize(c.s));
                } else {
                    st.cheb = m;
                    st.hi_mult = mult;
                }
            }
            if (!ok) {
                const std::vector<double> th_e = read_scalar(P, P->sc(k, 3));
                throw Error(DTRG_ENOCONV, "step " + std::to_string(k) +
                                              ": eigen-adjoint: complement expansion diverged (residual of the "
                                              "first unresolved pair " + std::to_string(th_e[0]) + ")" + trail);
            }
        } else {
            DTRG_REQUIRE(st.cheb >= 8 && P->ctab_ready, DTRG_ESTATE, "no recorded complement expansion for this step");
            coefficients(st.cheb, st.hi_mult);
            if (st.cheb < kChebMaxDegree)
                max_check(P->sc(k, 9), P->S, 1, nb, kChebTail, nullptr, 0, P->flags.p, kFlagChebTail, c.s);
            expansion(st.cheb);
        }
        axpy(P->Xc.p, P->Xe.p, vbs, (i64)n * K, nb, 1.0, c.s);   // Xe += Xc
    }
    // W = X + U_K S / 2, then W / t
    GemmOp w;
    w.M = n; w.N = K; w.K = K;
    w.A = U; w.lda = b;
    w.B = P->Sm.p; w.ldb = K; w.b_kmajor = true;
    w.C = P->Xe.p; w.rmap = IdxMap::linear(K); w.cmap = IdxMap::linear(1);
    w.alpha = 0.5; w.beta = 1.0;
    set_bs(w, ubs, P->Sm.bs, vbs);
    c.gemm(w);
    scale_inplace(P->Xe.p, vbs, (i64)n * K, nb, 1.0, P->sc(k, 2), P->S, true, c.s);
    // G_bar = W U_K^T + U_K W^T, rows (a,c) and columns (b,d) scattered to Gt[a][b][c][d]
    GemmOp o1;
    o1.M = n; o1.N = n; o1.K = K;
    o1.A = P->Xe.p; o1.lda = K;
    o1.B = U; o1.ldb = b;
    o1.C = P->Gt.p;
    o1.rmap = IdxMap::split(X, (i64)X * X * X, X);
    o1.cmap = IdxMap::split(X, (i64)X * X, 1);
    set_bs(o1, vbs, ubs, P->Gt.bs);
    c.gemm(o1);
    o1.A = U; o1.lda = b; o1.B = P->Xe.p; o1.ldb = K; o1.beta = 1.0;
    set_bs(o1, ubs, vbs, P->Gt.bs);
    c.gemm(o1);
}

}  // namespace

// -------------------------------------------------------------------------------------------
// engine entry points
// -------------------------------------------------------------------------------------------
void plan_setup(dtrg_plan* P) {
    P->shape = shapes(P->D, P->chi, P->nsteps, P->opt.block_size, P->mixed());
    alloc_plan(P, P->shape);
}

void plan_read_back(dtrg_plan* P) {
    P->scal_h.resize((size_t)P->nb * P->S);
    P->flags_h.resize(P->nb);
    DTRG_HIP(hipMemcpyAsync(P->scal_h.data(), P->scal.p, P->scal_h.size() * sizeof(double), hipMemcpyDeviceToHost,
                            P->s));
    DTRG_HIP(hipMemcpyAsync(P->flags_h.data(), P->flags.p, P->nb * sizeof(int), hipMemcpyDeviceToHost, P->s));
    DTRG_HIP(hipStreamSynchronize(P->s));
}

void plan_throw_flags(const dtrg_plan* P, int mask, const std::string& where) {
    throw_flags(P, P->flags_h, mask, where);
}

void plan_forward(dtrg_plan* P, Mode mode) {
    Ctx c{P, P->s, mode};
    const int D = P->D, nb = P->nb;
    const i64 D4 = (i64)D * D * D * D;
    const auto& sh = P->shape;
    DTRG_REQUIRE(mode == Mode::Adaptive || P->sched_fwd, DTRG_ESTATE, "fixed forward pass without a recorded schedule");
    P->fwd_ok = false;
    if (mode == Mode::Adaptive) P->sched_fwd = P->sched_bwd = false;
    fill(P->scal.p, 0, (i64)P->scal.n, 1, 0.0, c.s);
    fill_int(P->flags.p, nb, 0, c.s);
    fill_int(P->misc.p, 4, 0, c.s);
    // c0 = |T0|; T1 = permute(T0, (0,2,1,3)) / c0
    norm2(P->T0buf.p, D4, D4, nb, P->sp(6), P->S, c.s, P->ws);
    accum_log(P->sp(6), 1.0, P->sp(0), P->sp(7), P->S, nb, P->flags.p, c.s);
    if (c.adaptive()) check_flags(P, kFlagNonPos | kFlagNonFinite, "input", true);
    for (int k = 1; k <= P->nsteps; ++k) {
        StepCk& st = P->steps[k - 1];
        const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K;
        if (k == 1) {
            permute_checked(P, P->T0buf, st.T.p, st.T.bs, pd4(D, D, D, D, 0, 2, 1, 3), 1.0, P->sp(7), c.s);
        } else {
            // T_k = permute(T'_{k-1} / c_{k-1}, (2,3,0,1))
            const StepShape& ps = sh[k - 2];
            permute_checked(P, P->Tn, st.T.p, st.T.bs, pd4(ps.K, ps.K, ps.Y, ps.Y, 2, 3, 0, 1), 1.0,
                            P->sc(k - 1, 1), c.s);
        }
        gram_of_step(c, st, k);
        if (c.adaptive()) check_flags(P, kFlagNonPos | kFlagNonFinite, "step " + std::to_string(k) + ": Gram trace");
        const StepCk* warm = (k >= 3) ? &P->steps[k - 3] : nullptr;
        eigensolve(c, st, k, warm);
        // projection (contraction precision; the output T' is FP64)
        const Ops o = prep_operands(c, st, false);
        proj1(c, o.at(3), o.Wt, o.Tp, o.P1, X, Y, K);
        proj2(c, o.at(0), o.P1, o.Tb, o.Q2, X, Y, K);
        proj3(c, o.at(3), o.Q2, o.U, st.sh.b, P->Tn, X, Y, K);
        // c_k = |T'|, L += 2^-k ln c_k, 1/c_k
        norm2(P->Tn.p, P->Tn.bs, (i64)K * K * Y * Y, nb, P->sc(k, 0), P->S, c.s, P->ws);
        accum_log(P->sc(k, 0), ldexp1(-k), P->sp(0), P->sc(k, 1), P->S, nb, P->flags.p, c.s);
        if (c.adaptive()) check_flags(P, kFlagErrors, "step " + std::to_string(k));
    }
    // final self-trace of T_{n+1} = permute(T'_n / c_n)
    const StepShape& ls = sh.back();
    P->Xf = ls.Y; P->Yf = ls.K;
    permute_checked(P, P->Tn, P->Tbar2.p, P->Tbar2.bs, pd4(ls.K, ls.K, ls.Y, ls.Y, 2, 3, 0, 1), 1.0,
                    P->sc(P->nsteps, 1), c.s);
    trace_xxyy(P->Tbar2.p, P->Tbar2.bs, P->Xf, P->Yf, nb, P->sp(4), P->S, c.s);
    accum_log(P->sp(4), ldexp1(-P->nsteps), P->sp(0), nullptr, P->S, nb, P->flags.p, c.s);
    if (c.adaptive()) {
        plan_read_back(P);
        plan_throw_flags(P, kFlagErrors, "final trace");
        for (int i = 0; i < nb; ++i)
            if (!std::isfinite(P->scal_h[(size_t)i * P->S])) throw Error(DTRG_ENONPOS, inst_name(P, i) + "ln Z is not finite");
        P->sched_fwd = true;
        P->fwd_ok = true;
    }
}

void plan_backward(dtrg_plan* P, double gbar, bool with_dir, Mode mode) {
    Ctx c{P, P->s, mode};
    const int ns = P->nsteps, nb = P->nb;
    DTRG_REQUIRE(P->sched_fwd, DTRG_ESTATE, "backward before a successful forward");
    DTRG_REQUIRE(mode == Mode::Adaptive || P->sched_bwd, DTRG_ESTATE, "fixed backward pass without a recorded schedule");
    // seed: gradient w.r.t. T_{n+1} (dims [Xf][Xf][Yf][Yf])
    seed_trace_grad(P->Tbar.p, P->Tbar.bs, P->Xf, P->Yf, nb, gbar * ldexp1(-ns), P->sp(4), P->S, c.s);
    for (int k = ns; k >= 1; --k) {
        StepCk& st = P->steps[k - 1];
        const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K, n = st.sh.n, b = st.sh.b;
        // T'bar_p[alpha][y][z][beta] = permute(Tbar [y][z][alpha][beta]) / c_k
        permute_checked(P, P->Tbar, P->Tpbar.p, P->Tpbar.bs, pd4(Y, Y, K, K, 2, 0, 1, 3), 1.0, P->sc(k, 1), c.s);
        // recompute the projection intermediates (contraction precision)
        const Ops o = prep_operands(c, st, true);
        const Prec pr6 = o.at(3);
        proj1(c, pr6, o.Wt, o.Tp, o.P1, X, Y, K);
        proj2(c, o.at(0), o.P1, o.Tb, o.Q2, X, Y, K);
        if (st.sh.mixed)
            convert_f64_to_f32(P->Tpbar.p, P->Tpbar.bs, P->Tpbarf.p, P->Tpbarf.bs, (i64)K * Y * Y * K, nb, c.s);
        // w_bar_R[(i,m)][beta] = sum_{(alpha,y,z)} Q2[(alpha,y,z)][(i,m)] T'bar_p[(alpha,y,z)][beta]
        {
            GemmOp g;
            g.M = n; g.N = K; g.K = K * Y * Y;
            g.A = o.Q2.p; g.lda = n; g.a_kmajor = true;
            g.B = o.Tpbar.p; g.ldb = K; g.b_kmajor = true;
            g.C = P->Ub.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
            set_bs(g, o.Q2.bs, o.Tpbar.bs, P->Ub.bs);
            c.gemmc(g, pr6, true);
        }
        // Qbar[alpha][y][i][z][m] = sum_beta T'bar_p[(alpha,y,z)][beta] w[(i,m)][beta]   (into Q2)
        {
            GemmOp g;
            g.M = K * Y * Y; g.N = n; g.K = K;
            g.A = o.Tpbar.p; g.lda = K;
            g.B = o.U.p; g.ldb = b;
            g.C = (void*)o.Q2.p;
            g.rmap = IdxMap::split(Y, (i64)X * Y * X, X);
            g.cmap = IdxMap::split(X, (i64)Y * X, 1);
            set_bs(g, o.Tpbar.bs, o.U.bs, o.Q2.bs);
            c.gemmc(g, pr6, false);
        }
        fill(P->Tbar2.p, P->Tbar2.bs, (i64)X * X * Y * Y, nb, 0.0, c.s);
        // Pbar_p[y][i][j][alpha][b] = sum_{(z,m)} Qbar[(alpha,y,i)][(z,m)] Tb2[(z,m)][(j,b)]   (chi^7)
        // (the adjoint of the join with respect to P, written straight in the layout of its two
        // consumers below: rows (alpha,(y,i)), columns (j,b))
        {
            GemmOp g;
            g.M = K * Y * X; g.N = Y * X; g.K = Y * X;
            g.A = o.Q2.p; g.lda = Y * X;
            g.B = o.Tb2.p; g.ldb = Y * X; g.b_kmajor = true;
            g.C = (void*)o.X5.p;
            g.rmap = IdxMap::split((i64)Y * X, X, (i64)Y * K * X);
            g.cmap = IdxMap::split(X, (i64)K * X, 1);
            g.tag = 8;
            set_bs(g, o.Q2.bs, o.Tb2.bs, o.X5.bs);
            c.gemmc(g, o.at(1), false);
        }
        // Tbar_lower[b][m][j][z] += sum_{(alpha,y,i)} Qbar[(alpha,y,i)][(z,m)] P1[(alpha,y,i)][(b,j)]   (chi^7)
        {
            GemmOp g;
            g.M = Y * X; g.N = X * Y; g.K = K * Y * X;
            g.A = o.Q2.p; g.lda = Y * X; g.a_kmajor = true;
            g.B = o.P1.p; g.ldb = X * Y; g.b_kmajor = true;
            g.C = P->Tbar2.p;
            g.rmap = IdxMap::split(X, 1, (i64)Y * Y);
            g.cmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
            g.beta = 1.0;
            g.tag = 9;
            set_bs(g, o.Q2.bs, o.P1.bs, P->Tbar2.bs);
            c.gemmc(g, o.at(2), true);
        }
        // Tbar_upper[a][i][y][j] += sum_{(alpha,b)} Pbar_p[y][(i,j)][(alpha,b)] Wt2[a][(alpha,b)]
        {
            GemmOp g;
            g.M = X * Y; g.N = X; g.K = K * X; g.batch = Y;
            g.A = o.X5.p; g.lda = (i64)K * X; g.a_bs = (i64)X * Y * K * X;
            g.B = o.Wt2.p; g.ldb = (i64)b * X; g.b_bs = 0;
            g.C = P->Tbar2.p; g.c_bs = Y;
            g.rmap = IdxMap::split(Y, (i64)Y * Y, 1);
            g.cmap = IdxMap::linear((i64)X * Y * Y);
            g.beta = 1.0;
            set_bs(g, o.X5.bs, o.Wt2.bs, P->Tbar2.bs);
            c.gemmc(g, pr6, true);
        }
        // w_bar_L[(a,b)][alpha] += sum_{(y,i,j)} Tp[(y,i,j)][a] Pbar_p[(y,i,j)][(alpha,b)]
        {
            GemmOp g;
            g.M = X; g.N = K * X; g.K = Y * X * Y;
            g.A = o.Tp.p; g.lda = X; g.a_kmajor = true;
            g.B = o.X5.p; g.ldb = (i64)K * X; g.b_kmajor = true;
            g.C = P->Ub.p;
            g.rmap = IdxMap::linear((i64)X * K);
            g.cmap = IdxMap::split(X, 1, K);
            g.beta = 1.0;
            set_bs(g, o.Tp.bs, o.X5.bs, P->Ub.bs);
            c.gemmc(g, pr6, true);
        }
        // recompute the step's half-environments and normalised Gram from its checkpoint
        gram_of_step(c, st, k);
        // eigensolver adjoint -> G_bar, in Gt[(a,b)][(c,d)]
        eig_adjoint(c, st, k);
        // Abar'[a][j][b][k] = sum_{(c,d)} Gt[(a,b)][(c,d)] B[(c,d)][(j,k)]   (into Tn)
        // Bbar'[c][j][d][k] = sum_{(a,b)} Gt[(a,b)][(c,d)] A[(a,b)][(j,k)]   (into Tpbar)
        DevBuf<double>& Abar = P->Tn;
        DevBuf<double>& Bbar = P->Tpbar;
        {
            GemmOp g;
            g.M = X * X; g.N = Y * Y; g.K = X * X;
            g.A = P->Gt.p; g.lda = X * X;
            g.B = P->B.p; g.ldb = Y * Y; g.b_kmajor = true;
            g.C = Abar.p;
            g.rmap = IdxMap::split(X, (i64)X * Y * Y, Y);
            g.cmap = IdxMap::split(Y, (i64)X * Y, 1);
            set_bs(g, P->Gt.bs, P->B.bs, Abar.bs);
            c.gemm(g);
            g.A = P->Gt.p; g.a_kmajor = true;
            g.B = P->A.p;
            g.C = Bbar.p;
            set_bs(g, P->Gt.bs, P->A.bs, Bbar.bs);
            c.gemm(g);
        }
        // Tbar[a][x][y][j] += 2 sum_{(b,k)} Abar'[(a,j)][(b,k)] TA[(b,k)][(x,y)]
        {
            GemmOp g;
            g.M = X * Y; g.N = X * Y; g.K = X * Y;
            g.A = Abar.p; g.lda = X * Y;
            g.B = P->TA.p; g.ldb = X * Y; g.b_kmajor = true;
            g.C = P->Tbar2.p;
            g.rmap = IdxMap::split(Y, (i64)X * Y * Y, 1);
            g.cmap = IdxMap::split(Y, (i64)Y * Y, Y);
            g.alpha = 2.0; g.beta = 1.0;
            set_bs(g, Abar.bs, P->TA.bs, P->Tbar2.bs);
            c.gemm(g);
            // Tbar[a][x][j][y] += 2 sum_{(b,k)} Bbar'[(a,j)][(b,k)] TB[(b,k)][(x,y)]
            g.A = Bbar.p;
            g.B = P->TB.p;
            g.rmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
            g.cmap = IdxMap::split(Y, (i64)Y * Y, 1);
            set_bs(g, Bbar.bs, P->TB.bs, P->Tbar2.bs);
            c.gemm(g);
        }
        std::swap(P->Tbar, P->Tbar2);   // Tbar = gradient w.r.t. T_k
        if (c.adaptive()) check_flags(P, kFlagErrors, "backward step " + std::to_string(k));
    }
    // T0bar[l][u][r][d] = permute(Tbar [l][r][u][d]) / c0
    const int D = P->D;
    const i64 D4 = (i64)D * D * D * D;
    permute_checked(P, P->Tbar, P->T0barbuf.p, P->T0barbuf.bs, pd4(D, D, D, D, 0, 2, 1, 3), 1.0, P->sp(7), c.s);
    if (with_dir) dot(P->T0barbuf.p, P->dT0buf.p, D4, D4, nb, P->sp(5), P->S, c.s, P->ws);
    if (c.adaptive()) {
        plan_read_back(P);
        plan_throw_flags(P, kFlagErrors, "backward");
        P->sched_bwd = true;
    }
}

}  // namespace dtrg
