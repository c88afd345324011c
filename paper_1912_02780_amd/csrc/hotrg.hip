// HOTRG forward pass and hand-written reverse pass of nb independent instances (gfx950).
//
// Layouts per instance (row-major, X = horizontal bond, Y = vertical bond, K = chi' kept,
// n = X^2, b = block); every plan buffer holds nb instances at its instance stride:
//   T   [l][r][u][d] = [X][X][Y][Y]        step input (the paper's T_{x x' y y'})
//   A,B [a][b][j][k] = [X][X][Y][Y]        half-environments of the Gram
//   G   [(a,c)][(b,d)] = n x n             Gram of the (x1, x2) unfolding, then sym / trace
//   U   [n][b]                             eigenvectors (first K columns are w[x1][x2][alpha])
// The operands of the projection contractions and of their adjoints are stored in the step's
// contraction format (FP64, FP32 or bf16 planes), rows padded to a multiple of 8 elements:
// permutations of T, U and the incoming gradient write them from FP64, and each contraction's
// scatter epilogue writes its result in the layout of its first consumer, for which it is
// K-contiguous; a second consumer that contracts it over the other indices reads the same buffer as
// a K-major operand.  The layouts are written next to their producers.
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

namespace {

template <class F>
void for_each_buf(const dtrg_plan& P, F f) {
    const DevBuf<double>* w[] = {&P.TA, &P.TB, &P.Tn, &P.Tbar, &P.Tbar2, &P.Wk, &P.A, &P.B, &P.Gw, &P.Gt, &P.Ub,
                                 &P.Xe, &P.Xc, &P.Re, &P.Om, &P.Sm, &P.Vc, &P.Vp, &P.Vn, &P.Ye, &P.We, &P.V1, &P.V2,
                                 &P.Y1, &P.Y2, &P.H, &P.Z, &P.Rinv, &P.Sg, &P.th, &P.res, &P.nrm, &P.coef, &P.fv,
                                 &P.ctab, &P.scal, &P.T0buf, &P.T0barbuf, &P.dT0buf, &P.tune_c, &P.ws.splitk, &P.ws.red,
                                 &P.polS, &P.polV, &P.pollam, &P.chain_lr, &P.side_U, &P.side_lam, &P.lockW,
                                 &P.kronW, &P.Akr};
    for (auto* b : w) f(b->p, b->bytes());
    for (const OpSet& o : P.ops) {
        const OpBuf* v[] = {&o.Wt, &o.Wt2, &o.UT, &o.Us, &o.Tp, &o.Tb, &o.Tb2, &o.TpT, &o.Tpb, &o.Tpb2,
                            &o.X1, &o.X2};
        for (auto* b : v) f(b->mem.p, b->mem.bytes());
    }
    for (auto& st : P.steps) {
        const DevBuf<double>* v[] = {&st.T, &st.U, &st.lam, &st.Ak, &st.Bk, &st.Gk, &st.wbar};
        for (auto* b : v) f(b->p, b->bytes());
        f(st.P1k.mem.p, st.P1k.mem.bytes());
        f(st.Q2k.mem.p, st.Q2k.mem.bytes());
    }
}

}  // namespace

i64 dtrg_plan::cap_bytes(const void* ptr) const {
    const char* q = (const char*)ptr;
    i64 r = -1;
    for_each_buf(*this, [&](const void* base, size_t nbytes) {
        const char* b = (const char*)base;
        if (r < 0 && b && q >= b && q < b + nbytes) r = (i64)nbytes - (i64)(q - b);
    });
    return r;
}

size_t dtrg_plan::bytes() const {
    size_t t = 0;
    for_each_buf(*this, [&](const void*, size_t nbytes) { t += nbytes; });
    return t + flags.bytes() + misc.bytes() + orth.bytes();
}

namespace dtrg {

namespace {

double ldexp1(int e) { return std::ldexp(1.0, e); }

constexpr double kSubspaceAccept = 1e-12;   // largest accepted resolved residual (trace-normalised)
// Rayleigh-Ritz after every (rr_skip + 1)-th Gram product only where the first solve's Ritz values
// span less than this ratio (smallest over largest, every instance)
constexpr double kRrSkipRatio = 1e-8;
constexpr double kChebTail = 1e-15;         // relative size of the last two expansion coefficients
constexpr int kChebMaxDegree = 1024;
// at the largest degree the expansion is accepted down to this tail (a relative error of the
// complement term far below the FP64 parity of the gradient); above it the step fails
constexpr double kChebTailAccept = 1e-12;
constexpr int kJacobiSweeps = 40;

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

i64 pad8(i64 x) { return (x + 7) / 8 * 8; }

// A device operand: base, instance stride, plane stride and (for operand buffers) row stride.
struct Opnd {
    const void* p = nullptr;
    i64 bs = 0, ps = 0, ld = 0;
};
Opnd op_of(const DevBuf<double>& b, i64 ld = 0) { Opnd o; o.p = b.p; o.bs = b.bs; o.ld = ld; return o; }
Opnd op_of(const OpBuf& b, i64 ld) { Opnd o; o.p = b.p(); o.bs = b.per; o.ps = b.ps(); o.ld = ld; return o; }

int esize(Prec pr) { return pr == Prec::F64 ? 8 : (pr == Prec::F32 ? 4 : 2); }
int esize(Prec pr, Out o) { return o == Out::F64 ? 8 : (o == Out::F32 ? 4 : 2); }
// the contraction format's own output kind
Out own_out(Prec pr) { return pr == Prec::F64 ? Out::F64 : (pr == Prec::F32 ? Out::F32 : Out::Split); }
int out_code(Prec pr) { return pr == Prec::F64 ? 0 : (pr == Prec::F32 ? 1 : prec_planes(pr)); }

// -------------------------------------------------------------------------------------------
// contractions
// -------------------------------------------------------------------------------------------
struct Ctx {
    dtrg_plan* P;
    hipStream_t s;
    Mode mode;
    bool adaptive() const { return mode == Mode::Adaptive; }
    // one contraction in precision `pr` over the plan's nb instances (operand instance strides
    // set by the caller in a_bs2 / b_bs2 / c_bs2), output kind `out`
    void run(GemmOp g, Prec pr, Out out) {
        g.batch2 = P->nb;
        // the join and its adjoint with respect to P (chi^5 outputs) have their own chain cap
        g.max_chain = (g.tag == 7 || g.tag == 8) ? P->opt.max_fp32_chain_wide : P->opt.max_fp32_chain;
        const int ein = esize(pr), eout = esize(pr, out);
        if (g.a_cap < 0) g.a_cap = P->cap_of(g.A, ein);
        if (g.b_cap < 0) g.b_cap = P->cap_of(g.B, ein);
        if (g.c_cap < 0) g.c_cap = P->cap_of(g.C, eout);
        if (P->opt.autotune) g.cfg = tuned_cfg(pr, out, g, adaptive(), s, P->ws, P->tune_c);
        // timed: the joins in the plan's contraction precision on the large tiles, i.e. every
        // launch of that one kernel symbol (the small early steps stay FP64 on mixed plans); for
        // scheme (b), whose passes the eigensolver dominates, the Gram products instead (tag 10)
        const bool timed = P->opt.profile && adaptive() &&
                           (P->chain() ? g.tag == 10
                                       : (g.tag == 7 && pr == P->prec && gemm_resolve(pr, g).tile >= 2));
        if (timed) {
            while (P->ev_pool.size() < P->ev_used + 2) {
                hipEvent_t e;
                DTRG_HIP(hipEventCreate(&e));
                P->ev_pool.push_back(e);
            }
            DTRG_HIP(hipEventRecord(P->ev_pool[P->ev_used], s));
        }
        dtrg::gemm(pr, out, g, s, P->ws);
        if (timed) {
            DTRG_HIP(hipEventRecord(P->ev_pool[P->ev_used + 1], s));
            P->ev_used += 2;
            P->prof_flops += 2.0 * g.M * (double)g.N * g.K * g.batch * g.batch2;
        }
    }
    // FP64 contraction (Gram, eigensolver, eigen-adjoint)
    void gemm(const GemmOp& op) { run(op, Prec::F64, Out::F64); }
};

void set_bs(GemmOp& g, i64 a, i64 b, i64 c) { g.a_bs2 = a; g.b_bs2 = b; g.c_bs2 = c; }

// Scheme (b) steps that iterate keep their Gram in the Kronecker form G = sum_{j,k} A_jk (x) B_jk
// (G[(a,c),(b,d)] = sum_{jk} A[a,b,j,k] B[c,d,j,k]): its products and its adjoint are contractions
// of 4 X^3 d^2 work per column against 2 X^4 for the formed Gram, and nothing of size X^4 is formed.
// That pays from X > 2 d^2 on (below, the formed Gram's single product per column is cheaper to
// launch).  Scheme (a) steps, and the small steps solved by the full Jacobi eigensolve, form the Gram.
bool implicit_gram(const dtrg_plan* P, const StepShape& s) {
    return P->chain() && !s.full && s.X > 2 * s.Y * s.Y;
}
void set_ops(GemmOp& g, const Opnd& A, const Opnd& B) {
    g.A = A.p; g.lda = A.ld; g.a_bs2 = A.bs; g.a_ps = A.ps;
    g.B = B.p; g.ldb = B.ld; g.b_bs2 = B.bs; g.b_ps = B.ps;
}
void set_out(GemmOp& g, const Opnd& C) { g.C = (void*)C.p; g.c_bs2 = C.bs; g.c_ps = C.ps; }

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

// permute an FP64 tensor into an operand buffer: rows of the last `inner` output dims, row stride ld
void permute_op(dtrg_plan* P, Prec pr, const DevBuf<double>& in, const OpBuf& out, PermDesc d, int inner, i64 ld,
                const double* scale_dev, hipStream_t s) {
    d.nb = P->nb;
    d.in_bs = in.bs;
    d.out_bs = out.per;
    d.out_inner = inner;
    d.out_ld = ld;
    d.out_ps = out.ps();
    d.in_cap = P->cap_of(in.p);
    d.out_cap = P->cap_of(out.p(), esize(pr));
    dtrg::permute_out(in.p, out.p(), out_code(pr), d, 1.0, scale_dev, P->S, s);
}

// A[a][b][j][k] = sum_{x,y} TA[(a,j)][(x,y)] TA[(b,k)][(x,y)]  (also B with TB): TA TA^T, so only
// the tiles on or below its diagonal are computed and mirrored
void half_env(Ctx& c, const DevBuf<double>& Tperm, DevBuf<double>& out, int X, int Y) {
    GemmOp g;
    g.M = g.N = X * Y; g.K = X * Y;
    g.sym = 1;
    g.A = Tperm.p; g.lda = X * Y;
    g.B = Tperm.p; g.ldb = X * Y;
    g.C = out.p;
    g.rmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
    g.cmap = IdxMap::split(Y, (i64)Y * Y, 1);
    set_bs(g, Tperm.bs, Tperm.bs, out.bs);
    c.gemm(g);
}

// G[(a,c)][(b,d)] = sum_{(j,k)} A[(a,b),(j,k)] B[(c,d),(j,k)].  A and B are symmetric under
// (a,j) <-> (b,k), so G[(b,d)][(a,c)] = G[(a,c)][(b,d)]: in the rows (a,b) and columns (c,d) of the
// contraction, the element of row (b,a) and column (d,c) equals that of (a,b), (c,d).  Only the rows
// with a >= b are computed; the others are written as their mirror images.
void gram(Ctx& c, const DevBuf<double>& A, const DevBuf<double>& B, DevBuf<double>& G, int X, int Y) {
    GemmOp g;
    g.M = X * (X + 1) / 2; g.N = X * X; g.K = Y * Y;
    g.sym = 2; g.rdig = X; g.cdig = X;
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
// TA and TB, the two layouts of the step input that the half-environments contract:
// TA[(a,j)][(x,y)] = T[a][x][y][j] and TB[(a,j)][(x,y)] = T[a][x][j][y] for the left unfolding;
// the right unfolding (right = true) is the left one of the mirrored input T[x'][x][y][y'], so
// TA[(a,j)][(x,y)] = T[x][a][y][j] and TB[(a,j)][(x,y)] = T[x][a][j][y]
void step_operands_TA_TB(Ctx& c, const StepCk& st, bool right) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y;
    permute_checked(P, st.T, P->TA.p, P->TA.bs, right ? pd4(X, X, Y, Y, 1, 3, 0, 2) : pd4(X, X, Y, Y, 0, 3, 1, 2),
                    1.0, nullptr, c.s);
    permute_checked(P, st.T, P->TB.p, P->TB.bs, right ? pd4(X, X, Y, Y, 1, 2, 0, 3) : pd4(X, X, Y, Y, 0, 2, 1, 3),
                    1.0, nullptr, c.s);
}

// copy A, B and the normalised Gram of a step into its kept buffers (save) or back (!save)
void keep_gram(Ctx& c, const StepCk& st, bool save) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n;
    const DevBuf<double>* w[3] = {&P->A, &P->B, &P->Gw};
    const DevBuf<double>* k[3] = {&st.Ak, &st.Bk, &st.Gk};
    const int rows[3] = {X * X, X * X, n}, cols[3] = {Y * Y, Y * Y, n};
    const int nk = implicit_gram(P, st.sh) ? 2 : 3;   // the Kronecker form keeps no Gram
    for (int i = 0; i < nk; ++i) {
        const DevBuf<double>& src = save ? *w[i] : *k[i];
        const DevBuf<double>& dst = save ? *k[i] : *w[i];
        copy2d(src.p, cols[i], src.bs, dst.p, cols[i], dst.bs, rows[i], cols[i], P->nb, c.s);
    }
}

void gram_of_step(Ctx& c, const StepCk& st, int k, bool right) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n;
    step_operands_TA_TB(c, st, right);
    half_env(c, P->TA, P->A, X, Y);
    half_env(c, P->TB, P->B, X, Y);
    if (implicit_gram(P, st.sh)) {
        // scheme (b): the Gram stays in its Kronecker form; only its trace is formed
        kron_trace(P->A.p, P->A.bs, P->B.p, P->B.bs, X, Y, P->nb, P->sc(k, 2), P->S, P->flags.p, c.s);
        return;
    }
    gram(c, P->A, P->B, P->Gw, X, Y);
    sym_normalise(P->Gw.p, P->Gw.bs, n, P->nb, P->sc(k, 2), P->S, P->flags.p, c.s);
}

// Row strides of the operand layouts of one step (every row padded to a multiple of 8).
struct Lds {
    i64 Wt, Wt2, UT, Us, Tp, Tb, Tb2, TpT, Tpb, Tpb2;      // chi^4 / n x b class
    i64 P1, Q2, QbA, X5A;                                  // chi^5 class
    explicit Lds(const StepShape& s) {
        const i64 X = s.X, Y = s.Y, K = s.K, b = s.b, n = s.n;
        Wt = pad8(X); Wt2 = pad8(b * X); UT = pad8(n); Us = pad8(b);
        Tp = pad8(X); Tb = pad8(X * Y); Tb2 = pad8(Y * X); TpT = pad8(Y * X * Y);
        Tpb = pad8(K * Y * Y); Tpb2 = pad8(K);
        P1 = pad8(X * Y); Q2 = pad8(X * X); QbA = pad8(Y * X); X5A = pad8(K * X);
    }
    // per-instance element counts of the buffers (rows x row stride)
    static void sizes(const StepShape& s, i64 out[12]) {
        const Lds l(s);
        const i64 X = s.X, Y = s.Y, K = s.K, b = s.b, n = s.n;
        out[0] = b * X * l.Wt; out[1] = X * l.Wt2; out[2] = b * l.UT; out[3] = n * l.Us;
        out[4] = Y * X * Y * l.Tp; out[5] = Y * X * l.Tb; out[6] = Y * X * l.Tb2; out[7] = X * l.TpT;
        out[8] = K * l.Tpb; out[9] = K * Y * Y * l.Tpb2;
        out[10] = std::max(K * Y * X * l.P1, Y * X * Y * l.X5A);   // X1
        out[11] = std::max(K * Y * Y * l.Q2, K * Y * X * l.QbA);   // X2
    }
};

// forward operands of a step: Wt [(alpha,b)][a], Tp [(y,i,j)][a], Tb [(z,m)][(b,j)], UT [beta][(i,m)]
// (for the backward also Wt2 [a][(alpha,b)], Tb2 [(j,b)][(z,m)], TpT [a][(y,i,j)], Us [(i,m)][beta];
// a backward that does not recompute the first projection and the join skips Wt, Tp and Tb)
void prep_operands(Ctx& c, const StepCk& st, const OpSet& o, bool backward, bool forward_ops = true) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y, n = st.sh.n, b = st.sh.b;
    const Lds l(st.sh);
    const Prec pr = o.pr;
    if (forward_ops) {
        permute_op(P, pr, st.U, o.Wt, pd3(X, X, b, 2, 1, 0), 1, l.Wt, nullptr, c.s);
        permute_op(P, pr, st.T, o.Tp, pd4(X, X, Y, Y, 2, 1, 3, 0), 1, l.Tp, nullptr, c.s);
        permute_op(P, pr, st.T, o.Tb, pd4(X, X, Y, Y, 3, 1, 0, 2), 2, l.Tb, nullptr, c.s);
    }
    if (!backward) {
        PermDesc u;
        u.rank = 2; u.in_dims[0] = n; u.in_dims[1] = b; u.perm[0] = 1; u.perm[1] = 0;
        permute_op(P, pr, st.U, o.UT, u, 1, l.UT, nullptr, c.s);
    } else {
        permute_op(P, pr, st.U, o.Wt2, pd3(X, X, b, 0, 2, 1), 2, l.Wt2, nullptr, c.s);
        permute_op(P, pr, st.T, o.Tb2, pd4(X, X, Y, Y, 2, 0, 3, 1), 2, l.Tb2, nullptr, c.s);
        permute_op(P, pr, st.T, o.TpT, pd4(X, X, Y, Y, 0, 2, 1, 3), 3, l.TpT, nullptr, c.s);
        PermDesc u;
        u.rank = 2; u.in_dims[0] = n; u.in_dims[1] = b; u.perm[0] = 0; u.perm[1] = 1;
        permute_op(P, pr, st.U, o.Us, u, 1, l.Us, nullptr, c.s);
    }
}

// P1[(alpha,y,i)][(b,j)] = sum_a Wt[(alpha,b)][a] Tp[y][(i,j)][a]   (batched over y), into P1
// (X1, or the step's kept buffer)
void proj1(Ctx& c, const StepCk& st, const OpSet& o, const OpBuf& P1) {
    const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K;
    const Lds l(st.sh);
    GemmOp g;
    g.M = K * X; g.N = X * Y; g.K = X; g.batch = Y;
    set_ops(g, op_of(o.Wt, l.Wt), op_of(o.Tp, l.Tp));
    g.a_bs = 0;
    g.b_bs = (i64)X * Y * l.Tp;
    set_out(g, op_of(P1, l.P1));
    g.c_bs = (i64)X * l.P1;
    g.rmap = IdxMap::split(X, (i64)Y * X * l.P1, Y);
    g.cmap = IdxMap::split(Y, l.P1, 1);
    c.run(g, o.pr, own_out(o.pr));
}

// the join (the chi^7 term): Q2[(alpha,y,z)][(i,m)] = sum_{(b,j)} P1[(alpha,y,i)][(b,j)] Tb[(z,m)][(b,j)],
// from P1 into Q2 (X1 into X2, or the step's kept buffers)
void join(Ctx& c, const StepCk& st, const OpSet& o, const OpBuf& P1, const OpBuf& Q2) {
    const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K;
    const Lds l(st.sh);
    GemmOp g;
    g.tag = 7;
    g.M = K * Y * X; g.N = Y * X; g.K = X * Y;
    set_ops(g, op_of(P1, l.P1), op_of(o.Tb, l.Tb));
    set_out(g, op_of(Q2, l.Q2));
    g.rmap = IdxMap::split(X, (i64)Y * l.Q2, X);
    g.cmap = IdxMap::split(X, l.Q2, 1);
    c.run(g, o.pr, own_out(o.pr));
}

// T'[alpha][beta][y][z] = sum_{(i,m)} Q2[(alpha,y,z)][(i,m)] UT[beta][(i,m)]   (FP64 out)
void proj3(Ctx& c, const StepCk& st, const OpSet& o, const OpBuf& Q2, DevBuf<double>& Tn) {
    const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K;
    const Lds l(st.sh);
    GemmOp g;
    g.M = K * Y * Y; g.N = K; g.K = X * X;
    set_ops(g, op_of(Q2, l.Q2), op_of(o.UT, l.UT));
    g.C = Tn.p; g.c_bs2 = Tn.bs;
    g.rmap = IdxMap::split((i64)Y * Y, (i64)K * Y * Y, 1);
    g.cmap = IdxMap::linear((i64)Y * Y);
    c.run(g, o.pr, Out::F64);
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
        if (b & kFlagJacobi) throw Error(DTRG_ENOCONV, pre + "Jacobi eigensolve did not converge");
        if (b & kFlagTransfer)
            throw Error(DTRG_ENOCONV, pre + "dominant eigenvalue of the chain's transfer matrix not resolved (not "
                                            "positive, or not separated from the next)");
        throw Error(DTRG_ENOCONV, pre + "flag " + std::to_string(b));
    }
}

void check_flags(dtrg_plan* P, int mask, const std::string& where, bool input_stage = false) {
    throw_flags(P, read_flags(P), mask, where, input_stage);
}

constexpr int kFlagErrors = kFlagErrorMask;

// rewrite the plan's persisted tuning table when an adaptive pass has added shapes to the table
void persist_tuning(dtrg_plan* P) {
    if (P->tile_table.empty() || !P->opt.autotune) return;
    const int n = tuned_count();
    if (n == P->tuned_seen) return;
    tune_save(P->tile_table);
    P->tuned_seen = n;
}

// -------------------------------------------------------------------------------------------
// truncated eigensolve
// -------------------------------------------------------------------------------------------

// Orthonormalise the n x b blocks V (instance stride vbs) in place: a shifted CholeskyQR pass
// (stable for any condition number up to 1/u, which the normalised iterate can reach when the
// Gram has a cluster of noise-level eigenvalues) followed by two plain passes.  The third pass is
// skipped, on the device and per instance, when the second finds its input orthonormal to within
// kOrthNear (an input that close has condition number below 1 + b kOrthNear, so that one pass
// leaves it orthonormal to working accuracy); this is the usual case once the iteration converges.
constexpr double kOrthNear = 1e-6;
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
        chol_inverse(P->Sg.p, P->Sg.bs, b, shift, P->Rinv.p, P->Rinv.bs, P->nb, P->flags.p, c.s,
                     pass == 2 ? P->orth.p : nullptr, pass == 1 ? P->orth.p : nullptr, kOrthNear);
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
    g.tag = 10;
    g.M = n; g.N = b; g.K = n;
    g.A = G.p; g.lda = n;
    g.B = V; g.ldb = b; g.b_kmajor = true;
    g.C = C;
    g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
    set_bs(g, G.bs, vbs, vbs);
    c.gemm(g);
}

// C = G_hat V for V (n x w, ld w, instance stride vbs) with the step's normalised Gram: the formed
// Gram in Gw, or (implicit_gram) its Kronecker form from the half-environments in A and B,
//   W1[a][alpha][d][jk] = sum_b A'[b][(a,jk)] V[(b,d)][alpha]      (A'[b][a][jk] = A[a][b][jk])
//   C[(a,c)][alpha]     = sum_{d,jk} W1[a][alpha][d][jk] B[c][d][jk] / tr G,
// two contractions of 2 X^3 Y^2 w flops each (the formed Gram: 2 X^4 w), both with every dimension
// at least X (the first contraction's rows are (a, jk), not jk alone per a, which would leave most
// rows of each MFMA tile empty).
void product_G(Ctx& c, const StepCk& st, int k, const double* V, double* C, i64 vbs, int w) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n;
    if (!implicit_gram(P, st.sh)) {
        gemm_GV(c, P->Gw, V, C, vbs, n, w);
        return;
    }
    const int X = st.sh.X, YY = st.sh.Y * st.sh.Y;
    const i64 xyy = (i64)X * YY;
    permute_checked(P, P->A, P->Akr.p, P->Akr.bs, pd3(X, X, YY, 1, 0, 2), 1.0, nullptr, c.s);
    GemmOp g;   // W1 (rows (a, jk), columns (d, alpha))
    g.tag = 10;
    g.M = (int)xyy; g.N = X * w; g.K = X;
    g.A = P->Akr.p; g.lda = xyy; g.a_kmajor = true;
    g.B = V; g.ldb = (i64)X * w; g.b_kmajor = true;
    g.C = P->kronW.p;
    g.rmap = IdxMap::split(YY, (i64)w * xyy, 1);
    g.cmap = IdxMap::split(w, YY, xyy);
    set_bs(g, P->Akr.bs, vbs, P->kronW.bs);
    c.gemm(g);
    GemmOp h;   // C (rows (a, alpha), columns c)
    h.tag = 10;
    h.M = X * w; h.N = X; h.K = (int)xyy;
    h.A = P->kronW.p; h.lda = xyy;
    h.B = P->B.p; h.ldb = xyy;
    h.C = C;
    h.rmap = IdxMap::split(w, (i64)X * w, 1);
    h.cmap = IdxMap::linear(w);
    set_bs(h, P->kronW.bs, P->B.bs, vbs);
    c.gemm(h);
    scale_inplace(C, vbs, (i64)n * w, P->nb, 1.0, P->sc(k, 2), P->S, true, c.s);
}

// V -= U_L (U_L^T V) with U_L the first `cols` columns of U (n rows, ld ldu) and V n x w (ld w),
// twice, so that V leaves the locked vectors' span to working accuracy whatever its start
void deflate(Ctx& c, const double* U, int ldu, i64 ubs, int cols, double* V, int w, i64 vbs, int n) {
    if (cols == 0) return;
    dtrg_plan* P = c.P;
    for (int pass = 0; pass < 2; ++pass) {
        GemmOp g;   // W = U_L^T V  (cols x w, in lockW)
        g.M = cols; g.N = w; g.K = n;
        g.A = U; g.lda = ldu; g.a_kmajor = true;
        g.B = V; g.ldb = w; g.b_kmajor = true;
        g.C = P->lockW.p; g.rmap = IdxMap::linear(w); g.cmap = IdxMap::linear(1);
        set_bs(g, ubs, vbs, P->lockW.bs);
        c.gemm(g);
        GemmOp h;   // V -= U_L W
        h.M = n; h.N = w; h.K = cols;
        h.A = U; h.lda = ldu;
        h.B = P->lockW.p; h.ldb = w; h.b_kmajor = true;
        h.C = V; h.rmap = IdxMap::linear(w); h.cmap = IdxMap::linear(1);
        h.alpha = -1.0; h.beta = 1.0;
        set_bs(h, ubs, P->lockW.bs, vbs);
        c.gemm(h);
    }
}

// Truncated eigensolve for chi' beyond one Rayleigh-Ritz block (scheme (b) at large bond
// dimension): the leading eigenpairs are found lock_n blocks at a time by the block subspace
// iteration of eigensolve, each block of lock_bw columns deflated against the eigenvectors that the
// blocks before it resolved (they are eigenvectors of the Gram, so the deflated Gram has the
// remaining spectrum).  Each block resolves lock_r pairs to the tolerance; the last block's guard
// columns complete U, its first unresolved pair bounds the complement of the eigen-adjoint.
// Adaptive passes only (scheme (b) plans are not batched).
void eigensolve_locked(Ctx& c, StepCk& st, int k, const StepCk* warm) {
    dtrg_plan* P = c.P;
    const StepShape& s = st.sh;
    const int n = s.n, bw = s.lock_bw, er = s.lock_r, nblk = s.lock_n, b = s.b, nb = P->nb;
    DTRG_REQUIRE(c.adaptive(), DTRG_EINVAL, "the block-locked eigensolve runs in adaptive passes only");
    const i64 vbs = P->V1.bs, ubs = st.U.bs;
    const uint64_t seed = 0x5eedULL * (uint64_t)k + 17ULL;
    const bool warm_used = warm && warm->sh.n == n && warm->sh.b == b && warm->sh.lock_bw == bw;
    const double tol = P->opt.subspace_tol;
    const int it_max = P->opt.max_subspace_iters;
    std::vector<double> resh((size_t)nb * P->res.bs);
    int total = 0;
    for (int blk = 0; blk < nblk; ++blk) {
        const int c0 = blk * er;
        const bool last = blk == nblk - 1;
        const int res_n = last ? s.e - c0 : er;   // pairs this block resolves
        if (warm_used)
            copy2d(warm->U.p + c0, b, warm->U.bs, P->V1.p, bw, vbs, n, bw, nb, c.s);
        else
            hash_fill(P->V1.p, vbs, (i64)n * bw, nb, seed + 977ULL * (uint64_t)(blk + 1), c.s);
        deflate(c, st.U.p, b, ubs, c0, P->V1.p, bw, vbs, n);
        orthonormalise(c, P->V1.p, P->V2.p, vbs, n, bw);
        double prev = INFINITY, mx = INFINITY;
        int stall = 0, it = 0;
        for (it = 1; it <= it_max; ++it) {
            product_G(c, st, k, P->V1.p, P->Y1.p, vbs, bw);
            deflate(c, st.U.p, b, ubs, c0, P->Y1.p, bw, vbs, n);
            // H = V^T Y, its eigenvectors Z, V <- V Z, Y <- Y Z, residuals of the resolved pairs
            GemmOp g;
            g.M = g.N = bw; g.K = n;
            g.A = P->V1.p; g.lda = bw; g.a_kmajor = true;
            g.B = P->Y1.p; g.ldb = bw; g.b_kmajor = true;
            g.C = P->H.p;
            g.rmap = IdxMap::linear(bw); g.cmap = IdxMap::linear(1);
            set_bs(g, vbs, vbs, P->H.bs);
            c.gemm(g);
            jacobi_eig(P->H.p, bw, bw, P->H.bs, P->th.p, P->th.bs, P->Z.p, bw, P->Z.bs, nb, kJacobiSweeps, P->misc.p,
                       c.s);
            GemmOp r;
            r.M = n; r.N = bw; r.K = bw;
            r.B = P->Z.p; r.ldb = bw; r.b_kmajor = true;
            r.rmap = IdxMap::linear(bw); r.cmap = IdxMap::linear(1);
            r.A = P->V1.p; r.lda = bw; r.C = P->V2.p; set_bs(r, vbs, P->Z.bs, vbs); c.gemm(r);
            r.A = P->Y1.p; r.lda = bw; r.C = P->Y2.p; c.gemm(r);
            std::swap(P->V1, P->V2);
            std::swap(P->Y1, P->Y2);
            ritz_residuals(P->V1.p, P->Y1.p, n, res_n, bw, vbs, P->th.p, P->th.bs, P->res.p, P->res.bs, nb, c.s);
            DTRG_HIP(hipMemcpyAsync(resh.data(), P->res.p, resh.size() * sizeof(double), hipMemcpyDeviceToHost,
                                    c.s));
            DTRG_HIP(hipStreamSynchronize(c.s));
            mx = 0.0;
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < res_n; ++j) {
                    const double v = resh[(size_t)i * P->res.bs + j];
                    mx = std::max(mx, std::isfinite(v) ? v : INFINITY);
                }
            if (mx <= tol) break;
            if (mx > 0.5 * prev) ++stall; else stall = 0;
            prev = mx;
            if (stall >= 3 && mx <= kSubspaceAccept) break;      // rounding floor reached
            if (it == it_max) break;
            // next block: (G + s I) V with columns rescaled to unit norm (the shift of eigensolve),
            // deflated and re-orthonormalised
            axpy(P->V1.p, P->Y1.p, vbs, (i64)n * bw, nb, kChainGramShift, c.s);
            col_norms(P->Y1.p, n, bw, bw, vbs, P->nrm.p, P->nrm.bs, nb, c.s);
            col_normalise(P->Y1.p, n, bw, bw, vbs, P->nrm.p, P->nrm.bs, nb,
                          seed + 7919ULL * it + 104729ULL * (uint64_t)blk, c.s);
            std::swap(P->V1, P->Y1);
            deflate(c, st.U.p, b, ubs, c0, P->V1.p, bw, vbs, n);
            orthonormalise(c, P->V1.p, P->V2.p, vbs, n, bw);
        }
        total += std::min(it, it_max);
        // lock the resolved pairs (and, for the last block, its guard) into U and lam
        const int keep = last ? bw : er;
        copy2d(P->V1.p, bw, vbs, st.U.p + c0, b, ubs, n, keep, nb, c.s);
        copy2d(P->th.p, bw, P->th.bs, st.lam.p + c0, b, st.lam.bs, 1, keep, nb, c.s);
        if (last) {
            // residual of the first unresolved pair (it bounds the complement of the eigen-adjoint)
            ritz_residuals(P->V1.p, P->Y1.p, n, res_n + 1, bw, vbs, P->th.p, P->th.bs, P->res.p, P->res.bs, nb,
                           c.s);
            copy2d(P->res.p + res_n, 1, P->res.bs, P->sc(k, 3), 1, P->S, 1, 1, nb, c.s);
        }
        max_check(P->res.p, P->res.bs, res_n, nb, kSubspaceAccept, P->sc(k, 8), P->S, P->flags.p, kFlagSubspace,
                  c.s);
        const std::vector<int> f = read_flags(P);
        for (int i = 0; i < nb; ++i)
            if (f[i] & kFlagSubspace)
                throw Error(DTRG_ENOCONV, inst_name(P, i) + "step " + std::to_string(k) + ", locked block " +
                                              std::to_string(blk) + ": truncated eigensolve residual " +
                                              std::to_string(mx) + " after " + std::to_string(it) + " iterations");
    }
    st.iters = total;
}

// The next block of the scheme (a) subspace iteration from V1 and Y1 = G V1: G V with columns
// rescaled to unit norm, re-orthonormalised.  Scheme (b): (G + s I) V (s = 2^-45 of the unit trace),
// because the Grams of a squared Trotter operator have far fewer non-negligible eigenvalues than chi'
// (rank 6 of 256 at tau = 5e-5), and G V alone would collapse the block onto that range and break its
// Cholesky factorisation; the shift leaves the eigenvectors unchanged and keeps the block's
// null-space directions at norm s.  With subspace_shift: (G - s I) V, s = theta_{b-1} / 2 from the
// last Rayleigh-Ritz solve's values on the device.
void next_block(Ctx& c, const StepShape& sh, int it, uint64_t seed) {
    dtrg_plan* P = c.P;
    const int n = sh.n, b = sh.b, nb = P->nb;
    const i64 vbs = P->V1.bs;
    if (P->chain()) axpy(P->V1.p, P->Y1.p, vbs, (i64)n * b, nb, kChainGramShift, c.s);
    else if (P->opt.subspace_shift) axpy(P->V1.p, P->Y1.p, vbs, (i64)n * b, nb, -0.5, c.s, P->th.p + (b - 1), P->th.bs);
    col_norms(P->Y1.p, n, b, b, vbs, P->nrm.p, P->nrm.bs, nb, c.s);
    col_normalise(P->Y1.p, n, b, b, vbs, P->nrm.p, P->nrm.bs, nb, seed + 7919ULL * it, c.s);
    std::swap(P->V1, P->Y1);
    orthonormalise(c, P->V1.p, P->V2.p, vbs, n, b);
}

void eigensolve(Ctx& c, StepCk& st, int k, const StepCk* warm) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n, b = st.sh.b, E = st.sh.e, nb = P->nb;
    const uint64_t seed = 0x5eedULL * (uint64_t)k + 17ULL;
    if (st.sh.full) {
        // the whole spectrum: nothing downstream checks it, so a sweep cap reached is an error (the
        // Rayleigh-Ritz solves below are checked through the Ritz residuals instead)
        jacobi_eig(P->Gw.p, n, n, P->Gw.bs, st.lam.p, st.lam.bs, st.U.p, n, st.U.bs, nb, kJacobiSweeps, P->misc.p,
                   c.s, P->flags.p, kFlagJacobi);
        st.iters = 0;
        return;
    }
    if (st.sh.lock_n) {
        eigensolve_locked(c, st, k, warm);
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
    // Rayleigh-Ritz after every stride-th product (and after the first and the last): the adaptive
    // pass starts at 1 and may raise it after the first solve; fixed passes replay it
    int stride = c.adaptive() ? 1 : st.rr_stride;
    for (it = 1; it <= it_max; ++it) {
        double* V = P->V1.p;
        double* Y = P->Y1.p;
        product_G(c, st, k, V, Y, vbs, b);
        if ((it - 1) % stride != 0 && it < it_max) {
            // no Rayleigh-Ritz after this product: the next block comes from Y (and the shift of the
            // last solve's Ritz values)
            next_block(c, st.sh, it, seed);
            continue;
        }
        // H = V^T Y
        GemmOp g;
        g.M = g.N = b; g.K = n;
        g.A = V; g.lda = b; g.a_kmajor = true;
        g.B = Y; g.ldb = b; g.b_kmajor = true;
        g.C = P->H.p;
        g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
        set_bs(g, vbs, vbs, P->H.bs);
        c.gemm(g);
        jacobi_eig(P->H.p, b, b, P->H.bs, P->th.p, P->th.bs, P->Z.p, b, P->Z.bs, nb, kJacobiSweeps, P->misc.p, c.s);
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
            if (it == 1 && warm_used && P->opt.rr_skip && !P->chain()) {
                // the spread of the first solve's Ritz values decides the stride (see kRrSkipRatio); a
                // warm block is close to the Gram's eigenvectors, so they approximate its spectrum (a
                // random block's would not: its Ritz values average over the spectrum)
                std::vector<double> th((size_t)nb * P->th.bs);
                DTRG_HIP(hipMemcpyAsync(th.data(), P->th.p, th.size() * sizeof(double), hipMemcpyDeviceToHost, c.s));
                DTRG_HIP(hipStreamSynchronize(c.s));
                double ratio = INFINITY;
                for (int i = 0; i < nb; ++i) {
                    const double* t = th.data() + (size_t)i * P->th.bs;
                    ratio = std::min(ratio, t[0] > 0.0 ? t[b - 1] / t[0] : 0.0);
                }
                stride = ratio > kRrSkipRatio ? 1 + P->opt.rr_skip : 1;
            }
        }
        if (it == it_max) break;
        next_block(c, st.sh, it, seed);
    }
    if (c.adaptive()) {
        st.iters = std::min(it, it_max);
        st.rr_stride = stride;
    }
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

// Truncated weight 1 - sum of the kept eigenvalues of a step's normalised Gram, from st.lam
// (single-instance plans; synchronises the stream).
double host_trunc_weight(Ctx& c, const StepCk& st) {
    std::vector<double> lam(st.sh.K);
    DTRG_HIP(hipMemcpyAsync(lam.data(), st.lam.p, lam.size() * sizeof(double), hipMemcpyDeviceToHost, c.s));
    DTRG_HIP(hipStreamSynchronize(c.s));
    double kept = 0.0;
    for (double v : lam) kept += v;
    return st.sh.K < st.sh.n ? 1.0 - kept : 0.0;
}

// The side rule (SM B: the local HOSVD of the pair on either of its unfoldings).  Both the right
// and the left unfolding's Grams are eigensolved; the isometry comes from the one whose discarded
// eigenvalues weigh less, the right one only when lighter by more than kSideMargin.  The right
// unfolding runs first and its eigenpairs and scalars are set aside, so that the usual outcome (the
// left one, always for mirror-symmetric inputs) needs no copies back.
void eigensolve_sides(Ctx& c, StepCk& st, int k, const StepCk* warm) {
    dtrg_plan* P = c.P;
    const int n = st.sh.n, b = st.sh.b, nb = P->nb;
    DTRG_REQUIRE(nb == 1 && c.adaptive(), DTRG_EINVAL, "the side rule runs on single-instance plans");
    const std::string where = "step " + std::to_string(k) + ": Gram trace";
    gram_of_step(c, st, k, true);
    check_flags(P, kFlagNonPos | kFlagNonFinite, where + " (right unfolding)");
    eigensolve(c, st, k, warm);
    const int iters_right = st.iters;
    st.tw_right = host_trunc_weight(c, st);
    copy2d(st.U.p, b, st.U.bs, P->side_U.p, b, P->side_U.bs, n, b, nb, c.s);
    copy2d(st.lam.p, b, st.lam.bs, P->side_lam.p, b, P->side_lam.bs, 1, b, nb, c.s);
    const int slots[3] = {2, 3, 8};
    for (int i = 0; i < 3; ++i) copy2d(P->sc(k, slots[i]), 1, P->S, P->sp(9 + i), 1, P->S, 1, 1, nb, c.s);
    gram_of_step(c, st, k, false);
    check_flags(P, kFlagNonPos | kFlagNonFinite, where);
    eigensolve(c, st, k, warm);
    st.tw_left = host_trunc_weight(c, st);
    st.side = st.tw_right < st.tw_left - kSideMargin ? 1 : 0;
    if (st.side == 1) {
        copy2d(P->side_U.p, b, P->side_U.bs, st.U.p, b, st.U.bs, n, b, nb, c.s);
        copy2d(P->side_lam.p, b, P->side_lam.bs, st.lam.p, b, st.lam.bs, 1, b, nb, c.s);
        for (int i = 0; i < 3; ++i) copy2d(P->sp(9 + i), 1, P->S, P->sc(k, slots[i]), 1, P->S, 1, 1, nb, c.s);
        st.iters = iters_right;
        if (st.keep_gram) gram_of_step(c, st, k, true);
    }
    if (st.keep_gram) keep_gram(c, st, true);
}

// Scheme (b): close the chain after step k.  E = transfer matrix of T'_k / c_k (Tn, [K][K][Y][Y]) in
// Gw; its powers E^(2^j), each rescaled by its largest entry, alternate between Gt and Sm (FP64 MFMA
// products); the dominant eigenvalue goes to sc(k, 11) and [r | l] to chain_lr, and ln Z per cell per
// slice of the chain closed here, L_k + 2^-k ln lambda_k, to sc(k, 10).
void chain_close(Ctx& c, int k) {
    dtrg_plan* P = c.P;
    const StepShape& s = P->shape[k - 1];
    const int K = s.K, Y = s.Y, nb = P->nb;
    chain_transfer(P->Tn.p, P->Tn.bs, K, Y, P->sc(k, 1), P->S, P->Gw.p, P->Gw.bs, nb, c.s);
    copy2d(P->Gw.p, K, P->Gw.bs, P->Gt.p, K, P->Gt.bs, K, K, nb, c.s);
    chain_normalise(P->Gt.p, P->Gt.bs, (i64)K * K, nb, P->flags.p, kFlagTransfer, c.s);
    DevBuf<double>* a = &P->Gt;
    DevBuf<double>* b = &P->Sm;
    for (int j = 0; j < kChainSquarings; ++j) {
        // b = a a:  C(r, c) = sum_q A(r, q) B(c, q) with B(c, q) = a(q, c), a K-major operand
        GemmOp g;
        g.M = K; g.N = K; g.K = K;
        g.A = a->p; g.lda = K;
        g.B = a->p; g.ldb = K; g.b_kmajor = true;
        g.C = b->p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
        set_bs(g, a->bs, a->bs, b->bs);
        c.gemm(g);
        chain_normalise(b->p, b->bs, (i64)K * K, nb, P->flags.p, kFlagTransfer, c.s);
        std::swap(a, b);
    }
    chain_dominant_finish(P->Gw.p, P->Gw.bs, a->p, a->bs, K, nb, P->chain_lr.p, P->chain_lr.bs, P->sc(k, 11), P->S,
                          P->flags.p, kFlagTransfer, c.s);
    chain_lnZ_at(P->sp(0), P->sc(k, 11), ldexp1(-k), P->sc(k, 10), P->S, nb, c.s);
}

// -------------------------------------------------------------------------------------------
// plan set-up
// -------------------------------------------------------------------------------------------
// Steps whose join contraction costs less than this fraction of the largest step's stay FP64 on
// the mixed paths: their cost is negligible and they carry the largest weights 2^-k in ln Z / N.
constexpr double kMixedMinFraction = 0.05;

// phys > 0: scheme (b), the vertical legs keep dimension phys and every step merges vertically
std::vector<StepShape> shapes(int D, int chi, int nsteps, int block, int oversample, bool mixed, int phys) {
    std::vector<StepShape> v;
    int X = D, Y = phys > 0 ? phys : D;
    for (int k = 1; k <= nsteps; ++k) {
        StepShape s;
        s.X = X; s.Y = Y; s.n = X * X;
        s.K = std::min(chi, s.n);
        if (s.n <= kJacobiMax) { s.full = true; s.b = s.n; s.e = s.n; }
        else if (phys > 0 && s.K == s.n) { s.ident = true; s.b = s.n; s.e = s.n; }
        else if (phys > 0 && (s.K + 16 > kJacobiMax || (block > 0 && block <= s.K + 8))) {
            // scheme (b) beyond one Rayleigh-Ritz block: the eigenpairs are found lock_n blocks at a
            // time, each block deflated against the ones before (block_size, when set, is the
            // block width)
            s.lock_bw = block > 0 ? std::min(block, kJacobiMax) : kJacobiMax;
            DTRG_REQUIRE(s.lock_bw >= 16, DTRG_EINVAL, "block size too small for the locked eigensolve");
            // Resolved pairs beyond the cut: max(8, chi'/2), so that the complement of the
            // eigen-adjoint starts well below the kept eigenvalues (a gapless chain's spectrum is flat
            // near the cut: with 16 beyond it the complement expansion needed degrees beyond 1024 at
            // chi' = 128).  A block converges at the ratio lam_bw / lam_r of its width to the pairs it
            // resolves, so each keeps a guard of max(8, bw/4) columns; the last block resolves what
            // remains and keeps its whole width, so U has b = (lock_n - 1) lock_r + lock_bw < n
            // columns.  Where the Gram is too small for that (chi' near X^2), the guard shrinks to
            // 8 and the pairs beyond the cut to what fits, at least 8.
            const int e_want = s.K + std::max(8, s.K / 2);
            int best_e = -1;
            for (int g = std::max(8, s.lock_bw / 4); g >= 8 && best_e < e_want; --g) {
                const int r = s.lock_bw - g;
                for (int m = 1;; ++m) {
                    if ((m - 1) * r + s.lock_bw >= s.n) break;
                    const int e = std::min(e_want, m * r);
                    if (e > best_e) { best_e = e; s.lock_r = r; s.lock_n = m; }
                    if (m * r >= e_want) break;
                }
            }
            DTRG_REQUIRE(best_e >= s.K + 8, DTRG_EINVAL, "chi' too close to X^2 for the locked eigensolve");
            s.e = best_e;
            s.b = (s.lock_n - 1) * s.lock_r + s.lock_bw;
        } else {
            int b = block > 0 ? block : (oversample > 0 ? s.K + oversample : std::max(s.K + 16, 2 * s.K));
            b = std::min(b, kJacobiMax);
            b = std::min(b, s.n - 1);
            // at least one guard column beyond the kept ones: the complement expansion reads the
            // first unresolved Ritz pair (index e < b)
            DTRG_REQUIRE(b > s.K, DTRG_EINVAL, "block size must exceed chi'");
            s.b = b;
            s.e = s.K + (b - s.K) / 2;
        }
        v.push_back(s);
        if (phys > 0) {
            X = s.K;
        } else {
            X = Y;
            Y = s.K;
        }
    }
    if (mixed) {
        double mx = 0.0;
        for (auto& s : v) mx = std::max(mx, s.join_flops());
        for (auto& s : v) s.mixed = s.join_flops() >= kMixedMinFraction * mx;
    }
    return v;
}

// Forward intermediates kept for the backward pass, within P->ck_budget bytes: first the FP64
// half-environments and Gram of every step (from the last step back), then the first projection
// and the join of each step (from the last step back; the forward pass writes them there).  Steps that do not fit recompute
// them in the backward pass.
void alloc_kept(dtrg_plan* P) {
    const int nb = P->nb;
    i64 left = P->ck_budget;
    const int ns = (int)P->steps.size();
    for (int k = ns - 1; k >= 0; --k) {
        StepCk& st = P->steps[k];
        const i64 X = st.sh.X, Y = st.sh.Y, n = st.sh.n;
        const i64 gn = implicit_gram(P, st.sh) ? 0 : n * n;
        const i64 bytes = (i64)nb * (2 * X * X * Y * Y + gn) * 8;
        if (bytes > left) continue;
        st.Ak.alloc_inst(nb, X * X * Y * Y);
        st.Bk.alloc_inst(nb, X * X * Y * Y);
        if (gn) st.Gk.alloc_inst(nb, gn);
        st.keep_gram = true;
        left -= bytes;
    }
    for (int k = ns - 1; k >= 0; --k) {
        StepCk& st = P->steps[k];
        const OpSet& o = P->ops[st.sh.mixed ? 1 : 0];
        const Lds l(st.sh);
        const i64 X = st.sh.X, Y = st.sh.Y, K = st.sh.K;
        const int np = prec_planes(o.pr), esz = o.pr == Prec::F64 ? 8 : (o.pr == Prec::F32 ? 4 : 2);
        const i64 e1 = K * Y * X * l.P1, e2 = K * Y * Y * l.Q2;
        const i64 bytes = (i64)np * nb * (pad8(e1) + pad8(e2)) * esz;
        if (bytes > left) continue;
        st.P1k.alloc(o.pr, nb, e1);
        st.Q2k.alloc(o.pr, nb, e2);
        st.keep_join = true;
        left -= bytes;
    }
}

void alloc_plan(dtrg_plan* P, const std::vector<StepShape>& sh) {
    const int nb = P->nb;
    const i64 D4 = P->t0_elems();
    i64 t4 = D4, n2 = 1, nbk = 1, bmax = 1, nK = 1, bK = 1, KK = 1, Kmax = 1, lockw = 1, kronw = 1;
    i64 osz[2][12] = {};   // operand buffer sizes per format (FP64 steps, steps in the plan's format)
    bool used[2] = {false, false};
    for (auto& s : sh) {
        const i64 a4 = std::max<i64>((i64)s.X * s.X * s.Y * s.Y, (i64)s.K * s.K * s.Y * s.Y);
        t4 = std::max(t4, a4);
        // scheme (b) keeps explicit Grams only for the full eigensolves (n <= 96); its Gw and Gt also
        // hold the K x K transfer matrix and its powers
        if (!implicit_gram(P, s)) n2 = std::max<i64>(n2, (i64)s.n * s.n);
        else kronw = std::max<i64>(kronw, (i64)s.n * std::max(s.rr(), s.K) * s.Y * s.Y);
        if (P->chain()) n2 = std::max<i64>(n2, (i64)s.K * s.K);
        nbk = std::max<i64>(nbk, (i64)s.n * s.rr());
        bmax = std::max<i64>(bmax, s.rr());
        lockw = std::max<i64>(lockw, s.lock_n ? (i64)s.b * s.lock_bw : 1);
        nK = std::max<i64>(nK, (i64)s.n * s.K);
        bK = std::max<i64>(bK, (i64)s.b * s.K);
        KK = std::max<i64>(KK, (i64)s.K * s.K);
        Kmax = std::max<i64>(Kmax, s.K);
        const int f = s.mixed ? 1 : 0;
        used[f] = true;
        i64 z[12];
        Lds::sizes(s, z);
        for (int i = 0; i < 12; ++i) osz[f][i] = std::max(osz[f][i], z[i]);
    }
    P->T0buf.alloc_inst(nb, D4); P->T0barbuf.alloc_inst(nb, D4); P->dT0buf.alloc_inst(nb, D4);
    if (P->chain()) {
        // the closing squarings use Gw (E), Gt and Sm (the powers): K x K fits in each
        DTRG_REQUIRE(Kmax <= kChainMaxK, DTRG_EINVAL, "chain: chi' above the closing kernel's limit");
        P->chain_lr.alloc_inst(nb, 2 * Kmax);
    }
    for (DevBuf<double>* b : {&P->TA, &P->TB, &P->Tn, &P->Tbar, &P->Tbar2, &P->Wk, &P->A, &P->B})
        b->alloc_inst(nb, t4);
    for (int f = 0; f < 2; ++f) {
        OpSet& o = P->ops[f];
        o.pr = f == 0 ? Prec::F64 : P->prec;
        if (!used[f]) continue;
        OpBuf* v[] = {&o.Wt, &o.Wt2, &o.UT, &o.Us, &o.Tp, &o.Tb, &o.Tb2, &o.TpT, &o.Tpb, &o.Tpb2, &o.X1, &o.X2};
        for (int i = 0; i < 12; ++i) v[i]->alloc(o.pr, nb, std::max<i64>(osz[f][i], 8));
    }
    P->Gw.alloc_inst(nb, n2); P->Gt.alloc_inst(nb, n2);
    for (DevBuf<double>* b : {&P->V1, &P->V2, &P->Y1, &P->Y2}) b->alloc_inst(nb, nbk);
    if (P->side_rule()) {
        P->side_U.alloc_inst(nb, nbk);
        P->side_lam.alloc_inst(nb, bmax);
    }
    if (lockw > 1) P->lockW.alloc_inst(nb, lockw);
    if (kronw > 1) {
        P->kronW.alloc_inst(nb, kronw);
        P->Akr.alloc_inst(nb, t4);
    }
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
    P->orth.alloc_inst(nb, 1);
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
    alloc_kept(P);
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
            product_G(c, st, k, v, P->Ye.p, vbs, K);
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
                    if (mx <= kChebTail) break;
                    if (m >= kChebMaxDegree) {
                        if (mx <= kChebTailAccept) break;
                        throw Error(DTRG_ENOCONV, "step " + std::to_string(k) +
                                                      ": eigen-adjoint: complement expansion coefficients did not "
                                                      "decay by degree " + std::to_string(m) + " (tail ratio " +
                                                      std::to_string(mx) + ")");
                    }
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
            max_check(P->sc(k, 9), P->S, 1, nb, st.cheb < kChebMaxDegree ? kChebTail : kChebTailAccept, nullptr, 0,
                      P->flags.p, kFlagChebTail, c.s);
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
    if (implicit_gram(P, st.sh)) return;   // scheme (b): G_bar stays factored (kron_gram_adjoint)
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

// The half-environment adjoints of a Kronecker-form Gram (implicit_gram), in the layouts of the
// formed path, Abar'[a][j][b][k] and Bbar'[c][j][d][k], from G_bar = W U_K^T + U_K W^T kept factored
// (W in Xe, n x K, already divided by tr G; U_K the step's kept eigenvectors):
//   Abar' = F(W, U_K; B) + F(U_K, W; B),   Bbar' = F(W~, U_K~; A) + F(U_K~, W~; A),
//   F(P, Q; M)[a][j][b][k] = sum_alpha sum_{c,d} P[(a,c),alpha] M[c][d][jk] Q[(b,d),alpha],
// with ~ the exchange of the two bond indices of a row, (a,c) -> (c,a).  Each F is two contractions
// of 2 X^3 K Y^2 flops, through Z'[(d,alpha)][(a,jk)] (kronW) into F'[(a,jk)][b] (Akr), whose rows
// (a, jk) keep every dimension at least X; nothing n x n is formed.
void kron_gram_adjoint(Ctx& c, const StepCk& st, DevBuf<double>& Abar, DevBuf<double>& Bbar) {
    dtrg_plan* P = c.P;
    const int X = st.sh.X, Y = st.sh.Y, YY = Y * Y, K = st.sh.K, n = st.sh.n, b = st.sh.b, nb = P->nb;
    const i64 vbs = P->Xe.bs, xyy = (i64)X * YY;
    // U_K with leading dimension K (Vc); W~ (Vp) and U_K~ (Vn)
    copy2d(st.U.p, b, st.U.bs, P->Vc.p, K, vbs, n, K, nb, c.s);
    permute_checked(P, P->Xe, P->Vp.p, vbs, pd3(X, X, K, 1, 0, 2), 1.0, nullptr, c.s);
    permute_checked(P, P->Vc, P->Vn.p, vbs, pd3(X, X, K, 1, 0, 2), 1.0, nullptr, c.s);
    auto F = [&](const double* Pm, const double* Q, const DevBuf<double>& M, double beta) {
        GemmOp g;   // Z'[(d,alpha)][(a,jk)] = sum_c P[(a,c),alpha] M[c][(d,jk)]   (batched over a)
        g.M = K; g.N = (int)xyy; g.K = X; g.batch = X;
        g.A = Pm; g.lda = K; g.a_kmajor = true; g.a_bs = (i64)X * K;
        g.B = M.p; g.ldb = xyy; g.b_kmajor = true; g.b_bs = 0;
        g.C = P->kronW.p; g.c_bs = YY;
        g.rmap = IdxMap::linear(xyy);
        g.cmap = IdxMap::split(YY, (i64)K * xyy, 1);
        set_bs(g, vbs, M.bs, P->kronW.bs);
        c.gemm(g);
        GemmOp h;   // F'[(a,jk)][b] (+)= sum_{(d,alpha)} Z'[(d,alpha)][(a,jk)] Q[b][(d,alpha)]
        h.M = (int)xyy; h.N = X; h.K = X * K;
        h.A = P->kronW.p; h.lda = xyy; h.a_kmajor = true;
        h.B = Q; h.ldb = (i64)X * K;
        h.C = P->Akr.p;
        h.rmap = IdxMap::linear(X);
        h.cmap = IdxMap::linear(1);
        h.beta = beta;
        set_bs(h, P->kronW.bs, vbs, P->Akr.bs);
        c.gemm(h);
    };
    // F'[a][j][k][b] -> out[a][j][b][k]
    const PermDesc to_out = pd4(X, Y, Y, X, 0, 1, 3, 2);
    F(P->Xe.p, P->Vc.p, P->B, 0.0);
    F(P->Vc.p, P->Xe.p, P->B, 1.0);
    permute_checked(P, P->Akr, Abar.p, Abar.bs, to_out, 1.0, nullptr, c.s);
    F(P->Vp.p, P->Vn.p, P->A, 0.0);
    F(P->Vn.p, P->Vp.p, P->A, 1.0);
    permute_checked(P, P->Akr, Bbar.p, Bbar.bs, to_out, 1.0, nullptr, c.s);
}

// -------------------------------------------------------------------------------------------
// engine entry points
// -------------------------------------------------------------------------------------------
void plan_setup(dtrg_plan* P) {
    P->shape = shapes(P->D, P->chi, P->nsteps, P->opt.block_size, P->opt.oversample, P->mixed(), P->phys);
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
    const int D = P->D, nb = P->nb, d = P->phys;
    const i64 D4 = P->t0_elems();
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
            // [l][u][r][d] -> [l][r][u][d] (an MPO: D x d x D x d)
            permute_checked(P, P->T0buf, st.T.p, st.T.bs,
                            P->chain() ? pd4(D, d, D, d, 0, 2, 1, 3) : pd4(D, D, D, D, 0, 2, 1, 3), 1.0, P->sp(7), c.s);
        } else if (P->chain()) {
            // scheme (b): T_k = T'_{k-1} / c_{k-1} (every step merges vertically)
            const StepShape& ps = sh[k - 2];
            permute_checked(P, P->Tn, st.T.p, st.T.bs, pd4(ps.K, ps.K, ps.Y, ps.Y, 0, 1, 2, 3), 1.0,
                            P->sc(k - 1, 1), c.s);
        } else {
            // T_k = permute(T'_{k-1} / c_{k-1}, (2,3,0,1))
            const StepShape& ps = sh[k - 2];
            permute_checked(P, P->Tn, st.T.p, st.T.bs, pd4(ps.K, ps.K, ps.Y, ps.Y, 2, 3, 0, 1), 1.0,
                            P->sc(k - 1, 1), c.s);
        }
        if (st.sh.ident) {
            eye(st.U.p, st.U.bs, st.sh.n, st.sh.b, nb, c.s);
            fill(st.lam.p, st.lam.bs, st.sh.b, nb, 0.0, c.s);
        }
        if (!st.fixed && !st.sh.ident) {
            // warm start from the previous step in the same direction
            const int kw = P->chain() ? k - 1 : k - 2;
            const StepCk* warm =
                (kw >= 1 && !P->steps[kw - 1].fixed && !P->steps[kw - 1].sh.ident) ? &P->steps[kw - 1] : nullptr;
            if (P->side_rule()) {
                eigensolve_sides(c, st, k, warm);
            } else {
                gram_of_step(c, st, k, false);
                if (st.keep_gram) keep_gram(c, st, true);
                if (c.adaptive())
                    check_flags(P, kFlagNonPos | kFlagNonFinite, "step " + std::to_string(k) + ": Gram trace");
                eigensolve(c, st, k, warm);
            }
        }
        // projection (in the step's contraction format; the output T' is FP64)
        const OpSet& o = P->ops[st.sh.mixed ? 1 : 0];
        const Lds l(st.sh);
        prep_operands(c, st, o, false);
        // P and the join go straight into the step's kept buffers when the plan keeps them
        const OpBuf& P1 = st.keep_join ? st.P1k : o.X1;
        const OpBuf& Q2 = st.keep_join ? st.Q2k : o.X2;
        proj1(c, st, o, P1);
        join(c, st, o, P1, Q2);
        proj3(c, st, o, Q2, P->Tn);
        // c_k = |T'|, L += 2^-k ln c_k, 1/c_k
        norm2(P->Tn.p, P->Tn.bs, (i64)K * K * Y * Y, nb, P->sc(k, 0), P->S, c.s, P->ws);
        accum_log(P->sc(k, 0), ldexp1(-k), P->sp(0), P->sc(k, 1), P->S, nb, P->flags.p, c.s);
        if (P->chain()) chain_close(c, k);
        if (c.adaptive()) check_flags(P, kFlagErrors, "step " + std::to_string(k));
    }
    const StepShape& ls = sh.back();
    if (P->chain()) {
        // scheme (b): the infinite chain of the last step's cells, L += 2^-n ln lambda_n
        P->Xf = ls.K; P->Yf = ls.Y;
        accum_log(P->sc(P->nsteps, 11), ldexp1(-P->nsteps), P->sp(0), nullptr, P->S, nb, P->flags.p, c.s);
    } else {
        // final self-trace of T_{n+1} = permute(T'_n / c_n)
        P->Xf = ls.Y; P->Yf = ls.K;
        permute_checked(P, P->Tn, P->Tbar2.p, P->Tbar2.bs, pd4(ls.K, ls.K, ls.Y, ls.Y, 2, 3, 0, 1), 1.0,
                        P->sc(P->nsteps, 1), c.s);
        trace_xxyy(P->Tbar2.p, P->Tbar2.bs, P->Xf, P->Yf, nb, P->sp(4), P->S, c.s);
        accum_log(P->sp(4), ldexp1(-P->nsteps), P->sp(0), nullptr, P->S, nb, P->flags.p, c.s);
    }
    if (c.adaptive()) {
        plan_read_back(P);
        plan_throw_flags(P, kFlagErrors, "final trace");
        for (int i = 0; i < nb; ++i)
            if (!std::isfinite(P->scal_h[(size_t)i * P->S])) throw Error(DTRG_ENONPOS, inst_name(P, i) + "ln Z is not finite");
        P->sched_fwd = true;
        P->fwd_ok = true;
        persist_tuning(P);
    }
}

void plan_backward(dtrg_plan* P, double gbar, bool with_dir, Mode mode) {
    Ctx c{P, P->s, mode};
    const int ns = P->nsteps, nb = P->nb;
    DTRG_REQUIRE(P->sched_fwd, DTRG_ESTATE, "backward before a successful forward");
    DTRG_REQUIRE(mode == Mode::Adaptive || P->sched_bwd, DTRG_ESTATE, "fixed backward pass without a recorded schedule");
    // seed: gradient w.r.t. the last step's normalised output, in the layout [y][z][alpha][beta] the
    // step adjoint reads (scheme (a): T_{n+1} = permute(T'_n / c_n), dims [Xf][Xf][Yf][Yf], through its
    // self-trace; scheme (b): T'_n / c_n through ln lambda of its transfer matrix)
    if (P->chain())
        chain_seed(P->Tbar.p, P->Tbar.bs, P->Xf, P->Yf, P->chain_lr.p, P->chain_lr.bs, gbar * ldexp1(-ns),
                   P->sc(ns, 11), P->S, nb, c.s);
    else
        seed_trace_grad(P->Tbar.p, P->Tbar.bs, P->Xf, P->Yf, nb, gbar * ldexp1(-ns), P->sp(4), P->S, c.s);
    for (int k = ns; k >= 1; --k) {
        StepCk& st = P->steps[k - 1];
        const int X = st.sh.X, Y = st.sh.Y, K = st.sh.K, n = st.sh.n, b = st.sh.b;
        const OpSet& o = P->ops[st.sh.mixed ? 1 : 0];
        const Prec pr = o.pr;
        const Lds l(st.sh);
        if (P->chain() && k < ns) {
            // scheme (b): the gradient w.r.t. T_{k+1} = T'_k / c_k is in [l][r][u][d]; the step
            // adjoint reads it as [y][z][alpha][beta]
            permute_checked(P, P->Tbar, P->Tbar2.p, P->Tbar2.bs, pd4(K, K, Y, Y, 2, 3, 0, 1), 1.0, nullptr, c.s);
            std::swap(P->Tbar, P->Tbar2);
        }
        // incoming gradient / c_k in the two layouts it is contracted in:
        //   Tpb [beta][(alpha,y,z)] and Tpb2 [(alpha,y,z)][beta]  (from Tbar [y][z][alpha][beta])
        permute_op(P, pr, P->Tbar, o.Tpb, pd4(Y, Y, K, K, 3, 2, 0, 1), 3, l.Tpb, P->sc(k, 1), c.s);
        permute_op(P, pr, P->Tbar, o.Tpb2, pd4(Y, Y, K, K, 2, 0, 1, 3), 1, l.Tpb2, P->sc(k, 1), c.s);
        // P1 [(alpha,y,i)][(b,j)] and Q2 [(alpha,y,z)][(i,m)]: kept by the forward pass, or
        // recomputed into X1 and X2.  The adjoint contractions read them, and Q_bar and P_bar below,
        // in their producers' layouts as K-major operands (no transposed copies)
        prep_operands(c, st, o, true, !st.keep_join);
        const OpBuf& P1 = st.keep_join ? st.P1k : o.X1;
        const OpBuf& Q2 = st.keep_join ? st.Q2k : o.X2;
        if (!st.keep_join) {
            proj1(c, st, o, P1);
            join(c, st, o, P1, Q2);
        }
        // w_bar_R[(i,m)][beta] = sum_{(alpha,y,z)} Q2[(alpha,y,z)][(i,m)] Tpb[beta][(alpha,y,z)]
        {
            GemmOp g;
            g.M = n; g.N = K; g.K = K * Y * Y;
            set_ops(g, op_of(Q2, l.Q2), op_of(o.Tpb, l.Tpb));
            g.a_kmajor = true;
            g.C = P->Ub.p; g.c_bs2 = P->Ub.bs;
            g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
            c.run(g, pr, Out::F64);
        }
        // QbA[(alpha,y,i)][(z,m)] = sum_beta Tpb2[(alpha,y,z)][beta] Us[(i,m)][beta]   (X2; a
        // recomputed Q2 there is consumed)
        {
            GemmOp g;
            g.M = K * Y * Y; g.N = n; g.K = K;
            set_ops(g, op_of(o.Tpb2, l.Tpb2), op_of(o.Us, l.Us));
            set_out(g, op_of(o.X2, l.QbA));
            g.rmap = IdxMap::split(Y, (i64)X * l.QbA, X);
            g.cmap = IdxMap::split(X, l.QbA, 1);
            c.run(g, pr, own_out(pr));
        }
        fill(P->Tbar2.p, P->Tbar2.bs, (i64)X * X * Y * Y, nb, 0.0, c.s);
        // Tbar_lower[b][m][j][z] = sum_{(alpha,y,i)} QbA[(alpha,y,i)][(z,m)] P1[(alpha,y,i)][(b,j)]   (chi^7)
        {
            GemmOp g;
            g.M = Y * X; g.N = X * Y; g.K = K * Y * X;
            set_ops(g, op_of(o.X2, l.QbA), op_of(P1, l.P1));
            g.a_kmajor = g.b_kmajor = true;
            g.C = P->Tbar2.p; g.c_bs2 = P->Tbar2.bs;
            g.rmap = IdxMap::split(X, 1, (i64)Y * Y);
            g.cmap = IdxMap::split(Y, (i64)X * Y * Y, Y);
            g.beta = 1.0;
            g.tag = 9;
            c.run(g, pr, Out::F64);
        }
        // X5A[(y,i,j)][(alpha,b)] = sum_{(z,m)} QbA[(alpha,y,i)][(z,m)] Tb2[(j,b)][(z,m)]   (chi^7, X1;
        // a recomputed P1 there is consumed)
        {
            GemmOp g;
            g.M = K * Y * X; g.N = Y * X; g.K = Y * X;
            set_ops(g, op_of(o.X2, l.QbA), op_of(o.Tb2, l.Tb2));
            set_out(g, op_of(o.X1, l.X5A));
            g.rmap = IdxMap::split((i64)Y * X, X, (i64)Y * l.X5A);
            g.cmap = IdxMap::split(X, l.X5A, 1);
            g.tag = 8;
            c.run(g, pr, own_out(pr));
        }
        // Tbar_upper[a][i][y][j] += sum_{(alpha,b)} X5A[y][(i,j)][(alpha,b)] Wt2[a][(alpha,b)]   (batched over y)
        {
            GemmOp g;
            g.M = X * Y; g.N = X; g.K = K * X; g.batch = Y;
            set_ops(g, op_of(o.X1, l.X5A), op_of(o.Wt2, l.Wt2));
            g.a_bs = (i64)X * Y * l.X5A; g.b_bs = 0;
            g.C = P->Tbar2.p; g.c_bs = Y; g.c_bs2 = P->Tbar2.bs;
            g.rmap = IdxMap::split(Y, (i64)Y * Y, 1);
            g.cmap = IdxMap::linear((i64)X * Y * Y);
            g.beta = 1.0;
            c.run(g, pr, Out::F64);
        }
        // w_bar_L[(a,b)][alpha] += sum_{(y,i,j)} TpT[a][(y,i,j)] X5A[(y,i,j)][(alpha,b)]
        {
            GemmOp g;
            g.M = X; g.N = K * X; g.K = Y * X * Y;
            set_ops(g, op_of(o.TpT, l.TpT), op_of(o.X1, l.X5A));
            g.b_kmajor = true;
            g.C = P->Ub.p; g.c_bs2 = P->Ub.bs;
            g.rmap = IdxMap::linear((i64)X * K);
            g.cmap = IdxMap::split(X, 1, K);
            g.beta = 1.0;
            c.run(g, pr, Out::F64);
        }
        if (st.fixed || st.sh.ident) {
            // the isometry is a parameter of its own: its gradient is kept, and nothing flows
            // through the Gram of the step (an untruncated step's identity has no gradient at all)
            if (st.fixed) copy2d(P->Ub.p, K, P->Ub.bs, st.wbar.p, K, st.wbar.bs, n, K, nb, c.s);
            std::swap(P->Tbar, P->Tbar2);
            if (c.adaptive()) check_flags(P, kFlagErrors, "backward step " + std::to_string(k));
            continue;
        }
        // the step's half-environments and normalised Gram: kept, or recomputed from its checkpoint
        const bool right = st.side == 1;
        if (st.keep_gram) {
            step_operands_TA_TB(c, st, right);
            keep_gram(c, st, false);
        } else {
            gram_of_step(c, st, k, right);
        }
        // eigensolver adjoint -> G_bar, in Gt[(a,b)][(c,d)]
        eig_adjoint(c, st, k);
        // Abar'[a][j][b][k] = sum_{(c,d)} Gt[(a,b)][(c,d)] B[(c,d)][(j,k)]   (into Tn)
        // Bbar'[c][j][d][k] = sum_{(a,b)} Gt[(a,b)][(c,d)] A[(a,b)][(j,k)]   (into Wk)
        DevBuf<double>& Abar = P->Tn;
        DevBuf<double>& Bbar = P->Wk;
        if (implicit_gram(P, st.sh)) {
            kron_gram_adjoint(c, st, Abar, Bbar);
        } else {
            // G_bar and the half-environments are symmetric, so Abar' is symmetric under
            // (a,j) <-> (b,k) and Bbar' under (c,j) <-> (d,k): only the rows (a,b) (and (c,d)) with
            // a >= b are computed, the others are their mirror images
            GemmOp g;
            g.M = X * (X + 1) / 2; g.N = Y * Y; g.K = X * X;
            g.sym = 2; g.rdig = X; g.cdig = Y;
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
        // Tbar[a][x][y][j] += 2 sum_{(b,k)} Abar'[(a,j)][(b,k)] TA[(b,k)][(x,y)]   (the right
        // unfolding's tensor is the mirrored input: its gradient lands on Tbar[x][a][y][j])
        const i64 s1 = (i64)X * Y * Y, s0 = (i64)Y * Y;
        // Tbar += 2 Hbar' T_H for one half-environment H (A with TA, B with TB): in FP64, or on the steps
        // whose projections run in the plan's split-bf16 format, in that format (the two operands
        // converted into the step's chi^5 work buffers, which are free at this point of the step),
        // with FP64 accumulation into Tbar.  Like the projection contractions, this product comes
        // after the eigensolve and its adjoint, which stay FP64.
        const bool split_tbar = st.sh.mixed && !P->chain() && prec_planes(P->prec) > 1;
        auto tbar_update = [&](const DevBuf<double>& Hbar, const DevBuf<double>& TH, IdxMap rmap, IdxMap cmap) {
            GemmOp g;
            g.M = X * Y; g.N = X * Y; g.K = X * Y;
            g.b_kmajor = true;
            g.C = P->Tbar2.p;
            g.rmap = rmap;
            g.cmap = cmap;
            g.alpha = 2.0; g.beta = 1.0;
            if (split_tbar) {
                const OpSet& o = P->ops[1];
                const i64 ld = pad8((i64)X * Y);
                // Hbar'[(a,j)][(b,k)] rows (a,j), K-contiguous; T_H[(b,k)][(x,y)] K-major rows (b,k)
                permute_op(P, P->prec, Hbar, o.X1, pd4(X, Y, X, Y, 0, 1, 2, 3), 2, ld, nullptr, c.s);
                permute_op(P, P->prec, TH, o.X2, pd4(X, Y, X, Y, 0, 1, 2, 3), 2, ld, nullptr, c.s);
                set_ops(g, op_of(o.X1, ld), op_of(o.X2, ld));
                g.c_bs2 = P->Tbar2.bs;
                c.run(g, P->prec, Out::F64);
            } else {
                g.A = Hbar.p; g.lda = X * Y;
                g.B = TH.p; g.ldb = X * Y;
                set_bs(g, Hbar.bs, TH.bs, P->Tbar2.bs);
                c.gemm(g);
            }
        };
        tbar_update(Abar, P->TA, IdxMap::split(Y, right ? s0 : s1, 1), IdxMap::split(Y, right ? s1 : s0, Y));
        // Tbar[a][x][j][y] += 2 sum_{(b,k)} Bbar'[(a,j)][(b,k)] TB[(b,k)][(x,y)]   (right: Tbar[x][a][j][y])
        tbar_update(Bbar, P->TB, IdxMap::split(Y, right ? s0 : s1, Y), IdxMap::split(Y, right ? s1 : s0, 1));
        std::swap(P->Tbar, P->Tbar2);   // Tbar = gradient w.r.t. T_k
        if (c.adaptive()) check_flags(P, kFlagErrors, "backward step " + std::to_string(k));
    }
    // T0bar[l][u][r][d] = permute(Tbar [l][r][u][d]) / c0
    const int D = P->D, Yd = P->chain() ? P->phys : P->D;
    const i64 D4 = P->t0_elems();
    permute_checked(P, P->Tbar, P->T0barbuf.p, P->T0barbuf.bs, pd4(D, D, Yd, Yd, 0, 2, 1, 3), 1.0, P->sp(7), c.s);
    if (with_dir) dot(P->T0barbuf.p, P->dT0buf.p, D4, D4, nb, P->sp(5), P->S, c.s, P->ws);
    if (c.adaptive()) {
        plan_read_back(P);
        plan_throw_flags(P, kFlagErrors, "backward");
        P->sched_bwd = true;
        persist_tuning(P);
    }
}

// polar(R) of the K x K matrix R in P->H into P->Rinv by the Newton-Schulz iteration
// X_0 = R / |R|_F, X <- X (3 I - X^T X) / 2: every singular value below 1 grows by a factor of up to
// 3/2 a step and they converge quadratically once near 1, while the singular vectors stay those of
// R.  Stops when |X^T X - I|_F <= 1e-13 (checked every 8 steps), at most 256 steps (then
// DTRG_ENOCONV: R numerically rank deficient).
void polar_newton(Ctx& c, int K) {
    dtrg_plan* P = c.P;
    const int nb = P->nb;
    const i64 kk = (i64)K * K;
    norm2(P->H.p, P->H.bs, kk, nb, P->sp(12), P->S, c.s, P->ws);
    copy2d(P->H.p, K, P->H.bs, P->Rinv.p, K, P->Rinv.bs, K, K, nb, c.s);
    scale_inplace(P->Rinv.p, P->Rinv.bs, kk, nb, 1.0, P->sp(12), P->S, true, c.s);
    auto gram = [&]() {   // polS = X^T X
        GemmOp g;
        g.M = g.N = K; g.K = K;
        g.A = P->Rinv.p; g.lda = K; g.a_kmajor = true;
        g.B = P->Rinv.p; g.ldb = K; g.b_kmajor = true;
        g.C = P->polS.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
        set_bs(g, P->Rinv.bs, P->Rinv.bs, P->polS.bs);
        c.gemm(g);
    };
    for (int it = 1;; ++it) {
        gram();
        // polV = 1.5 X - 0.5 X (X^T X), then X = polV
        copy2d(P->Rinv.p, K, P->Rinv.bs, P->polV.p, K, P->polV.bs, K, K, nb, c.s);
        GemmOp h;
        h.M = h.N = K; h.K = K;
        h.A = P->Rinv.p; h.lda = K;
        h.B = P->polS.p; h.ldb = K; h.b_kmajor = true;
        h.C = P->polV.p; h.rmap = IdxMap::linear(K); h.cmap = IdxMap::linear(1);
        h.alpha = -0.5; h.beta = 1.5;
        set_bs(h, P->Rinv.bs, P->polS.bs, P->polV.bs);
        c.gemm(h);
        copy2d(P->polV.p, K, P->polV.bs, P->Rinv.p, K, P->Rinv.bs, K, K, nb, c.s);
        if (it % 8 != 0) continue;
        gram();
        eye(P->polV.p, P->polV.bs, K, K, nb, c.s);
        axpy(P->polV.p, P->polS.p, P->polS.bs, kk, nb, -1.0, c.s);   // polS = X^T X - I
        norm2(P->polS.p, P->polS.bs, kk, nb, P->sp(13), P->S, c.s, P->ws);
        const std::vector<double> dev = read_scalar(P, P->sp(13));
        double mx = 0.0;
        for (double v : dev) mx = std::max(mx, std::isfinite(v) ? v : INFINITY);
        if (mx <= 1e-13) break;
        DTRG_REQUIRE(it < 256, DTRG_ENOCONV,
                     "polar factor: Newton-Schulz iteration did not converge (environment numerically rank "
                     "deficient, |X^T X - I| = " + std::to_string(mx) + ")");
    }
}

// MERA update of step k's fixed isometry (paper, main text: the SVD E = U S V^T of the environment
// and w <- U V^T, which maximises Tr(E^T w)) from the gradient in st.wbar, which is E up to a
// positive factor.  The polar factor is formed without squaring E's condition number (the
// environments reach condition numbers of 1e8): E = Q R with the shifted CholeskyQR3 of the
// eigensolver (orthonormal to working accuracy for condition numbers up to ~1/u), R = Q^T E, and
// polar(R) = sum_j u_j v_j^T from the positive eigenpairs of [[0, R], [R^T, 0]] (Jacobi), whose
// eigenvectors are (u_j, v_j) / sqrt 2; then w = Q polar(R).  For K > 48 (2K beyond the Jacobi kernel),
// or with the polar_newton option, polar(R) comes from the Newton-Schulz iteration instead.
void polar_update(dtrg_plan* P, int k) {
    StepCk& st = P->steps[k - 1];
    const int n = st.sh.n, K = st.sh.K, b = st.sh.b, nb = P->nb, m = 2 * K;
    DTRG_REQUIRE(st.fixed, DTRG_ESTATE, "polar update of a step without a fixed isometry");
    DTRG_REQUIRE(K <= kJacobiMax && !st.sh.lock_n && !st.sh.ident, DTRG_EINVAL,
                 "isometry optimisation needs chi' <= 80 (one Rayleigh-Ritz block) on the optimised steps");
    const bool newton = m > kJacobiMax || P->opt.polar_newton;
    Ctx c{P, P->s, Mode::Adaptive};
    if (P->polS.n < (size_t)m * m * nb) {
        P->polS.alloc_inst(nb, (i64)m * m);
        P->polV.alloc_inst(nb, (i64)m * m);
        P->pollam.alloc_inst(nb, m);
    }
    const i64 vbs = P->V1.bs;
    // the environment E = w_bar; scheme (b): E + mu |E|_F w with the step's current isometry w (the
    // last layer's environment has rank <= 2, the derivative of the transfer matrix's eigenvalue
    // being l r^T, so the maximisers of Tr(E^T w) leave the rest of w free: the term keeps it)
    const double* E = st.wbar.p;
    i64 ebs = st.wbar.bs;
    if (P->chain()) {
        norm2(st.wbar.p, st.wbar.bs, (i64)n * K, nb, P->sp(8), P->S, c.s, P->ws);
        copy2d(st.U.p, b, st.U.bs, P->We.p, K, P->We.bs, n, K, nb, c.s);
        scale_inplace(P->We.p, P->We.bs, (i64)n * K, nb, kPolarTieBreak, P->sp(8), P->S, false, c.s);
        DTRG_REQUIRE(nb == 1, DTRG_EINVAL, "isometry optimisation needs a single-instance plan");
        axpy(st.wbar.p, P->We.p, 0, (i64)n * K, 1, 1.0, c.s);
        E = P->We.p;
        ebs = P->We.bs;
    }
    // Q: E orthonormalised (in V1, ld K)
    copy2d(E, K, ebs, P->V1.p, K, vbs, n, K, nb, c.s);
    orthonormalise(c, P->V1.p, P->V2.p, vbs, n, K);
    // R = Q^T E (K x K, in H)
    {
        GemmOp g;
        g.M = K; g.N = K; g.K = n;
        g.A = P->V1.p; g.lda = K; g.a_kmajor = true;
        g.B = E; g.ldb = K; g.b_kmajor = true;
        g.C = P->H.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
        set_bs(g, vbs, ebs, P->H.bs);
        c.gemm(g);
    }
    if (newton) {
        polar_newton(c, K);
    } else {
        sym_augment(P->H.p, P->H.bs, K, P->polS.p, P->polS.bs, nb, c.s);
        // floor at the rounding level of [[0, R], [R^T, 0]]: the polar factor needs the singular vectors
        // to working accuracy only, and rotations among its large entries leave residues of about u |R|
        // next to the small singular values, which a lower floor keeps rotating
        jacobi_eig(P->polS.p, m, m, P->polS.bs, P->pollam.p, P->pollam.bs, P->polV.p, m, P->polV.bs, nb, kJacobiSweeps,
                   P->misc.p, c.s, P->flags.p, kFlagJacobi, 0x1p-50);
        // polar(R)[r][c] = 2 sum_{j < K} V[r][j] V[K + c][j]   (into Rinv, K x K)
        {
            GemmOp g;
            g.M = K; g.N = K; g.K = K;
            g.A = P->polV.p; g.lda = m;
            g.B = P->polV.p + (i64)K * m; g.ldb = m;
            g.C = P->Rinv.p; g.rmap = IdxMap::linear(K); g.cmap = IdxMap::linear(1);
            g.alpha = 2.0;
            set_bs(g, P->polV.bs, P->polV.bs, P->Rinv.bs);
            c.gemm(g);
        }
    }
    // w = Q polar(R), into the first K columns of U (ld b)
    {
        GemmOp g;
        g.M = n; g.N = K; g.K = K;
        g.A = P->V1.p; g.lda = K;
        g.B = P->Rinv.p; g.ldb = K; g.b_kmajor = true;
        g.C = st.U.p; g.rmap = IdxMap::linear(b); g.cmap = IdxMap::linear(1);
        set_bs(g, vbs, P->Rinv.bs, st.U.bs);
        c.gemm(g);
    }
    check_flags(P, kFlagJacobi, "step " + std::to_string(k) + ": polar factor of the isometry gradient");
}

void plan_isometry_optimize(dtrg_plan* P, int layers, int n_inner, int n_sweeps, double* lnZ_hotrg,
                            std::vector<double>* history) {
    DTRG_REQUIRE(P->nb == 1, DTRG_EINVAL, "isometry optimisation needs a single-instance plan");
    DTRG_REQUIRE(layers >= 1 && n_inner >= 1 && n_sweeps >= 0, DTRG_EINVAL, "layers, n_inner >= 1 and n_sweeps >= 0");
    for (auto& st : P->steps) st.fixed = false;
    plan_forward(P, Mode::Adaptive);   // plain HOTRG: its isometries start the optimisation
    if (lnZ_hotrg) *lnZ_hotrg = P->scal_h[0];
    // scheme (a): the first `layers` truncating steps; scheme (b): the last `layers` (the optimisation
    // depth n_d below the target temperature), visited from the lowest up
    std::vector<int> opt;
    if (P->chain()) {
        for (int k = P->nsteps; k >= 1 && (int)opt.size() < layers; --k)
            if (P->steps[k - 1].sh.K < P->steps[k - 1].sh.n) opt.insert(opt.begin(), k);
    } else {
        for (int k = 1; k <= P->nsteps && (int)opt.size() < layers; ++k)
            if (P->steps[k - 1].sh.K < P->steps[k - 1].sh.n) opt.push_back(k);
    }
    DTRG_REQUIRE((int)opt.size() == layers, DTRG_EINVAL, "fewer truncating steps than layers to optimise");
    for (int k : opt) {
        StepCk& st = P->steps[k - 1];
        DTRG_REQUIRE(st.sh.K <= kJacobiMax && !st.sh.lock_n && !st.sh.ident, DTRG_EINVAL,
                     "isometry optimisation needs chi' <= 80 (one Rayleigh-Ritz block) on the optimised steps");
        if (st.wbar.n == 0) st.wbar.alloc_inst(1, (i64)st.sh.n * st.sh.K);
        st.fixed = true;   // U already holds HOTRG's isometry of the step
    }
    for (int s = 0; s < n_sweeps; ++s)
        for (int k : opt)
            for (int it = 0; it < n_inner; ++it) {
                plan_backward(P, 1.0, false, Mode::Adaptive);
                polar_update(P, k);
                plan_forward(P, Mode::Adaptive);
                if (history) history->push_back(P->scal_h[0]);
            }
}

}  // namespace dtrg
