// C ABI of the library: single-instance plans, mixed-chi batches replayed from a HIP graph, the
// standalone contraction, diagnostics and errors.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace dtrg;

namespace {

thread_local std::string g_last_error;

dtrg_status fail(const Error& e) {
    g_last_error = e.what();
    return e.code;
}

Prec prec_of(int contract) {
    switch (contract) {
        case DTRG_FP32: return Prec::F32;
        case DTRG_BF16X3: return Prec::BF16X3;
        case DTRG_BF16X6: return Prec::BF16X6;
        default: return Prec::F64;
    }
}

void validate_options(const dtrg_options& o) {
    DTRG_REQUIRE(o.contract >= DTRG_FP64 && o.contract <= DTRG_BF16X6, DTRG_EINVAL,
                 "contract must be DTRG_FP64, DTRG_FP32, DTRG_BF16X3 or DTRG_BF16X6");
    DTRG_REQUIRE(o.gram_fp64 == 1, DTRG_EINVAL, "the Gram is always formed in FP64 (gram_fp64 must be 1)");
    DTRG_REQUIRE(o.eig_broadening >= 0.0 && std::isfinite(o.eig_broadening), DTRG_EINVAL,
                 "eig_broadening must be finite and >= 0");
    DTRG_REQUIRE(o.max_subspace_iters >= 1, DTRG_EINVAL, "max_subspace_iters must be >= 1");
    DTRG_REQUIRE(o.block_size >= 0 && o.block_size <= kJacobiMax, DTRG_EINVAL, "block_size out of range [0, 96]");
    DTRG_REQUIRE(o.autotune == 0 || o.autotune == 1, DTRG_EINVAL, "autotune must be 0 or 1");
    DTRG_REQUIRE(o.checkpoint_gib >= 0.0 && std::isfinite(o.checkpoint_gib), DTRG_EINVAL,
                 "checkpoint_gib must be finite and >= 0");
    DTRG_REQUIRE(o.oversample >= 0 && o.oversample < kJacobiMax, DTRG_EINVAL, "oversample out of range [0, 95]");
    DTRG_REQUIRE(o.max_fp32_chain >= 32 && o.max_fp32_chain <= (1 << 20), DTRG_EINVAL,
                 "max_fp32_chain out of range [32, 2^20]");
    DTRG_REQUIRE(o.max_fp32_chain_wide >= 32 && o.max_fp32_chain_wide <= (1 << 20), DTRG_EINVAL,
                 "max_fp32_chain_wide out of range [32, 2^20]");
    DTRG_REQUIRE((o.alloc_fn == nullptr) == (o.free_fn == nullptr), DTRG_EINVAL,
                 "alloc_fn and free_fn must both be set or both be NULL");
    DTRG_REQUIRE(o.chain_phys >= 0 && o.chain_phys <= 16, DTRG_EINVAL, "chain_phys out of range [0, 16]");
    DTRG_REQUIRE(o.side_rule == 0 || o.side_rule == 1, DTRG_EINVAL, "side_rule must be 0 or 1");
    DTRG_REQUIRE(o.polar_newton == 0 || o.polar_newton == 1, DTRG_EINVAL, "polar_newton must be 0 or 1");
    DTRG_REQUIRE(o.subspace_shift == 0 || o.subspace_shift == 1, DTRG_EINVAL, "subspace_shift must be 0 or 1");
    DTRG_REQUIRE(o.rr_skip >= 0 && o.rr_skip <= 3, DTRG_EINVAL, "rr_skip must be 0 to 3");
    DTRG_REQUIRE(o.side_rule == 0 || o.chain_phys == 0, DTRG_EINVAL, "the side rule is for scheme (a) (chain_phys 0)");
}

void validate_sizes(int D, int chi, int n_steps, bool chain = false) {
    DTRG_REQUIRE(D >= 1 && D <= 64, DTRG_EINVAL, "D out of range [1, 64]");
    if (chain)
        DTRG_REQUIRE(chi >= 1 && chi <= kChainMaxChi, DTRG_EINVAL,
                     "chi out of range [1, " + std::to_string(kChainMaxChi) + "] for scheme (b)");
    else
        DTRG_REQUIRE(chi >= 1 && chi <= 80, DTRG_EINVAL, "chi out of range [1, 80]");
    DTRG_REQUIRE(n_steps >= 1 && n_steps <= 62, DTRG_EINVAL, "n_steps out of range [1, 62]");
}

Allocator allocator_of(const dtrg_options* opt, hipStream_t s) {
    Allocator a;
    if (opt) {
        a.alloc_fn = opt->alloc_fn;
        a.free_fn = opt->free_fn;
        a.user = opt->alloc_user;
    }
    a.stream = s;
    return a;
}

// share: the fraction of the checkpoint budget this plan may use (a batch divides it); s: the
// stream handed to the caller's allocator
std::unique_ptr<dtrg_plan> make_plan(int D, int chi, int n_steps, int nb, const dtrg_options* opt,
                                     double share = 1.0, hipStream_t s = nullptr) {
    validate_sizes(D, chi, n_steps, opt && opt->chain_phys > 0);
    std::unique_ptr<dtrg_plan> P(new dtrg_plan());
    dtrg_default_options(&P->opt);
    if (opt) P->opt = *opt;
    validate_options(P->opt);
    P->alloc = allocator_of(&P->opt, s);
    AllocScope scope(&P->alloc);
    if (P->opt.tile_table) P->tile_table = P->opt.tile_table;   // the plan keeps its own copy
    P->opt.tile_table = nullptr;
    if (!P->tile_table.empty()) {
        tune_load(P->tile_table);
        P->tuned_seen = tuned_count();   // rewritten only when a pass tunes something new
    }
    P->ck_budget = (dtrg::i64)std::min(P->opt.checkpoint_gib * share * 1073741824.0, 9.0e18);
    P->prec = prec_of(P->opt.contract);
    P->D = D; P->chi = chi; P->nsteps = n_steps; P->nb = nb;
    P->phys = P->opt.chain_phys;
    plan_setup(P.get());
    return P;
}

// diagnostics of step k of instance i (reads the device)
void step_info(const dtrg_plan* P, int i, int k, dtrg_step_info* info) {
    const StepCk& st = P->steps[k - 1];
    std::vector<double> row(P->S), lam(st.sh.b);
    DTRG_HIP(hipMemcpyAsync(row.data(), P->scal.p + (i64)i * P->S, P->S * sizeof(double), hipMemcpyDeviceToHost,
                            P->s));
    DTRG_HIP(hipMemcpyAsync(lam.data(), st.lam.p + (i64)i * st.lam.bs, st.sh.b * sizeof(double),
                            hipMemcpyDeviceToHost, P->s));
    DTRG_HIP(hipStreamSynchronize(P->s));
    const double* sc = row.data() + kScPlan + (i64)kScStep * (k - 1);
    info->X = st.sh.X; info->Y = st.sh.Y; info->chi_kept = st.sh.K; info->full_eig = st.sh.full ? 1 : 0;
    info->iters = st.iters; info->c = sc[0]; info->trace_G = sc[2];
    info->lam_last_kept = lam[st.sh.K - 1];
    info->lam_first_dropped = st.sh.b > st.sh.K ? lam[st.sh.K] : 0.0;
    info->resid = st.sh.full ? 0.0 : sc[8];
    info->cheb_degree = st.cheb;
    // the normalised Gram has trace 1, so the discarded weight is 1 - the kept eigenvalues
    double kept = 0.0, gmin = INFINITY;
    for (int j = 0; j < st.sh.K; ++j) {
        kept += lam[j];
        if (j + 1 < st.sh.K) gmin = std::min(gmin, lam[j] - lam[j + 1]);
    }
    info->trunc_weight = st.sh.K < st.sh.n ? std::max(0.0, 1.0 - kept) : 0.0;
    info->cut_gap = st.sh.b > st.sh.K ? lam[st.sh.K - 1] - lam[st.sh.K] : 0.0;
    info->min_kept_gap = st.sh.K > 1 ? gmin : 0.0;
    info->mixed = st.sh.mixed ? 1 : 0;
    info->lnZ_at_step = P->chain() ? sc[10] : NAN;
    info->side = st.side;
    info->trunc_weight_left = st.tw_left;
    info->trunc_weight_right = st.tw_right;
    info->rr_stride = st.sh.full ? 0 : st.rr_stride;
    if (st.fixed || st.sh.ident) {   // a given isometry (or the identity): no Gram, no spectrum
        info->full_eig = 0;
        info->iters = -1;
        info->trace_G = info->lam_last_kept = info->lam_first_dropped = info->resid = 0.0;
        info->trunc_weight = info->cut_gap = info->min_kept_gap = 0.0;
        info->cheb_degree = 0;
        info->trunc_weight_left = info->trunc_weight_right = NAN;
        info->rr_stride = 0;
    }
}

// step k of a single-instance plan, checked
StepCk& plan_step(dtrg_plan* P, int k) {
    DTRG_REQUIRE(P, DTRG_EINVAL, "NULL argument");
    DTRG_REQUIRE(P->nb == 1, DTRG_EINVAL, "not a single-instance plan");
    DTRG_REQUIRE(k >= 1 && k <= P->nsteps, DTRG_EINVAL, "step index out of range");
    return P->steps[k - 1];
}

}  // namespace

// A batch of problem instances with their own bond dimensions: one plan per distinct chi (its
// instances share every shape), run one after the other on the caller's stream in adaptive
// passes, and as parallel branches of one captured HIP graph in replays.
struct dtrg_batch {
    int n_inst = 0, D = 0, nsteps = 0;
    Allocator alloc;   // the caller's device allocator, shared by the batch's plans
    std::vector<std::unique_ptr<dtrg_plan>> plans;
    std::vector<std::vector<int>> members;
    std::vector<DevBuf<int>> idx;
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr, ev_in = nullptr;
    hipStream_t origin = nullptr;   // graphs are captured and launched on this stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // arguments the captured graph was recorded with
    const double* g_T0 = nullptr;
    const double* g_dT0 = nullptr;
    double* g_T0bar = nullptr;
    double g_gbar = 0.0;
    bool sched = false, sched_bwd = false;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~dtrg_batch() {
        drop_graph();
        for (auto s : branch) (void)hipStreamDestroy(s);
        for (auto e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (origin) (void)hipStreamDestroy(origin);
    }
};

namespace {

// one plan's share of a batch run: gather its inputs, forward, backward, scatter its gradient
void batch_group(dtrg_batch* Bt, size_t g, const double* T0s, const double* dT0s, double gbar, double* T0bar,
                 Mode mode, hipStream_t s) {
    dtrg_plan* P = Bt->plans[g].get();
    const int nb = P->nb;
    const i64 D4 = (i64)P->D * P->D * P->D * P->D;
    P->s = s;
    gather_rows(T0s, D4, Bt->idx[g].p, P->T0buf.p, D4, D4, nb, false, s);
    if (dT0s) gather_rows(dT0s, D4, Bt->idx[g].p, P->dT0buf.p, D4, D4, nb, false, s);
    plan_forward(P, mode);
    if (T0bar) {
        plan_backward(P, gbar, dT0s != nullptr, mode);
        gather_rows(P->T0barbuf.p, D4, Bt->idx[g].p, T0bar, D4, D4, nb, true, s);
    }
}

void batch_results(dtrg_batch* Bt, double* lnZ, double* dir, bool with_dir) {
    for (size_t g = 0; g < Bt->plans.size(); ++g) {
        const dtrg_plan* P = Bt->plans[g].get();
        for (int i = 0; i < P->nb; ++i) {
            const int id = Bt->members[g][i];
            if (lnZ) lnZ[id] = P->scal_h[(size_t)i * P->S + 0];
            if (with_dir && dir) dir[id] = P->scal_h[(size_t)i * P->S + 5];
        }
    }
}

void capture(dtrg_batch* Bt, const double* T0s, const double* dT0s, double gbar, double* T0bar, hipStream_t s) {
    Bt->drop_graph();
    DTRG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        DTRG_HIP(hipEventRecord(Bt->fork, s));
        for (size_t g = 0; g < Bt->plans.size(); ++g) {
            DTRG_HIP(hipStreamWaitEvent(Bt->branch[g], Bt->fork, 0));
            batch_group(Bt, g, T0s, dT0s, gbar, T0bar, Mode::Fixed, Bt->branch[g]);
            DTRG_HIP(hipEventRecord(Bt->join[g], Bt->branch[g]));
            DTRG_HIP(hipStreamWaitEvent(s, Bt->join[g], 0));
        }
    } catch (...) {
        hipGraph_t partial = nullptr;
        (void)hipStreamEndCapture(s, &partial);
        if (partial) (void)hipGraphDestroy(partial);
        throw;
    }
    DTRG_HIP(hipStreamEndCapture(s, &Bt->graph));
    DTRG_HIP(hipGraphInstantiate(&Bt->exec, Bt->graph, nullptr, nullptr, 0));
    Bt->g_T0 = T0s; Bt->g_dT0 = dT0s; Bt->g_T0bar = T0bar; Bt->g_gbar = gbar;
}

}  // namespace

namespace {

// One standalone contraction (dtrg_contract and its variants), validated, with its operand layouts
// resolved; the FP32 operands of the split-bf16 precisions are split into planes at launch.
struct ContractCall {
    Prec pr = Prec::F64;
    Out out = Out::F64;
    int np = 1;
    GemmOp g;
    const void* A = nullptr;
    const void* B = nullptr;
    i64 lda = 0, ldb = 0;
    bool akm = false, bkm = false;
    i64 lda_p = 0, ldb_p = 0, a_ps = 0, b_ps = 0;   // plane layouts (np > 1)
    // doubles of plane storage (0 when the operands are used as given)
    i64 plane_doubles() const { return np > 1 ? (np * (a_ps + b_ps) * 2 + 7) / 8 + 2 : 0; }
};

ContractCall contract_call(int precision, int M, int N, int K, const void* A_dev, long long lda, int a_kmajor,
                           const void* B_dev, long long ldb, int b_kmajor, void* C_dev, long long ldc, int out_f64,
                           double alpha, double beta, int tile, int splits) {
    DTRG_REQUIRE(A_dev && B_dev && C_dev, DTRG_EINVAL, "NULL argument");
    DTRG_REQUIRE(M >= 0 && N >= 0 && K >= 0, DTRG_EINVAL, "negative size");
    DTRG_REQUIRE(precision >= DTRG_FP64 && precision <= DTRG_BF16X6, DTRG_EINVAL, "bad precision");
    DTRG_REQUIRE(lda >= (a_kmajor ? M : K) && ldb >= (b_kmajor ? N : K) && ldc >= N, DTRG_EINVAL,
                 "leading dimension too small");
    ContractCall c;
    c.pr = prec_of(precision);
    DTRG_REQUIRE(tile >= 0 && tile <= (prec_planes(c.pr) > 1 ? 6 : 2), DTRG_EINVAL, "bad tile code");
    DTRG_REQUIRE(tile != 6 || (!a_kmajor && !b_kmajor && K % 16 == 0), DTRG_EINVAL,
                 "tile code 6 takes K-contiguous operands and K a multiple of 16 only");
    DTRG_REQUIRE(splits >= 0 && splits <= 64, DTRG_EINVAL, "split-K count out of range (0 to 64)");
    c.out = precision == DTRG_FP64 || out_f64 ? Out::F64 : Out::F32;
    c.np = prec_planes(c.pr);
    c.A = A_dev; c.B = B_dev; c.lda = lda; c.ldb = ldb; c.akm = a_kmajor != 0; c.bkm = b_kmajor != 0;
    GemmOp& g = c.g;
    g.M = M; g.N = N; g.K = K;
    g.C = C_dev; g.rmap = IdxMap::linear(ldc); g.cmap = IdxMap::linear(1);
    g.alpha = alpha; g.beta = beta;
    g.cfg.tile = tile;
    g.cfg.splits = splits;
    g.a_kmajor = c.akm;
    g.b_kmajor = c.bkm;
    if (c.np == 1) {
        g.A = A_dev; g.lda = lda;
        g.B = B_dev; g.ldb = ldb;
    } else {
        // FP32 operands split into bf16 planes in their own layout (K-contiguous or K-major, rows
        // padded to 8 elements)
        auto r8 = [](i64 x) { return (x + 7) / 8 * 8; };
        c.lda_p = r8(c.akm ? M : K);
        c.ldb_p = r8(c.bkm ? N : K);
        c.a_ps = (i64)(c.akm ? K : M) * c.lda_p;
        c.b_ps = (i64)(c.bkm ? K : N) * c.ldb_p;
        g.lda = c.lda_p; g.a_ps = c.a_ps;
        g.ldb = c.ldb_p; g.b_ps = c.b_ps;
    }
    return c;
}

// planes: at least c.plane_doubles() doubles (unused when the operands are used as given)
void contract_launch(ContractCall& c, double* planes, hipStream_t s, Scratch& ws) {
    GemmOp& g = c.g;
    if (c.np > 1) {
        const int M = g.M, N = g.N, K = g.K;
        __bf16* pa = (__bf16*)planes;
        __bf16* pb = pa + c.np * c.a_ps;
        // a K-major matrix is split as the row-major K x M matrix it is stored as
        if (c.akm) split_matrix((const float*)c.A, c.lda, false, K, M, pa, c.lda_p, c.a_ps, c.np, s);
        else split_matrix((const float*)c.A, c.lda, false, M, K, pa, c.lda_p, c.a_ps, c.np, s);
        if (c.bkm) split_matrix((const float*)c.B, c.ldb, false, K, N, pb, c.ldb_p, c.b_ps, c.np, s);
        else split_matrix((const float*)c.B, c.ldb, false, N, K, pb, c.ldb_p, c.b_ps, c.np, s);
        g.A = pa;
        g.B = pb;
    }
    dtrg::gemm(c.pr, c.out, g, s, ws);
}

// Device scratch of dtrg_contract_noalloc: the bf16 planes and split-K partials of one contraction.
// Each device holds its own copy for the life of the process; host code reaches it only through
// the device address hipGetSymbolAddress returns for the current device.
constexpr i64 kNoAllocScratchBytes = 128LL << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch` (looked up once per device)
void* noalloc_scratch_ptr() {
    int dev = -1;
    DTRG_HIP(hipGetDevice(&dev));
    DTRG_REQUIRE(dev >= 0 && dev < kMaxDevices, DTRG_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw Error(DTRG_EHIP, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                       hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
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
    o->autotune = 0;
    o->profile = 0;
    o->checkpoint_gib = 64.0;
    o->oversample = 0;
    o->max_fp32_chain = 4096;
    o->max_fp32_chain_wide = 4096;
    o->tile_table = nullptr;
    o->alloc_fn = nullptr;
    o->free_fn = nullptr;
    o->alloc_user = nullptr;
    o->chain_phys = 0;
    o->side_rule = 0;
    o->polar_newton = 0;
    o->subspace_shift = 1;
    o->rr_skip = 3;
}

dtrg_status dtrg_plan_create(int D, int chi, int n_steps, const dtrg_options* opt, dtrg_plan** plan_out) {
    g_last_error.clear();
    if (plan_out) *plan_out = nullptr;
    try {
        DTRG_REQUIRE(plan_out, DTRG_EINVAL, "NULL argument");
        *plan_out = make_plan(D, chi, n_steps, 1, opt).release();
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
        DTRG_REQUIRE(plan->nb == 1, DTRG_EINVAL, "not a single-instance plan");
        plan->fwd_ok = false;
        plan->s = (hipStream_t)stream;
        plan->alloc.stream = plan->s;
        AllocScope scope(&plan->alloc);
        const i64 D4 = plan->t0_elems();
        DTRG_HIP(hipMemcpyAsync(plan->T0buf.p, T0_dev, D4 * sizeof(double), hipMemcpyDeviceToDevice, plan->s));
        plan_forward(plan, Mode::Adaptive);
        *lnZ_per_site_host = plan->scal_h[0];
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
    try {
        P = make_plan(D, chi, n_steps, 1, opt, 1.0, (hipStream_t)stream).release();
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
    dtrg_status st = dtrg_plan_forward(P, T0_dev, stream, lnZ_per_site_host);
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
        DTRG_REQUIRE(plan->nb == 1, DTRG_EINVAL, "not a single-instance plan");
        DTRG_REQUIRE(plan->fwd_ok, DTRG_ESTATE, "backward before a successful forward");
        DTRG_REQUIRE(std::isfinite(gbar), DTRG_EINVAL, "gbar is not finite");
        plan->s = (hipStream_t)stream;
        plan->alloc.stream = plan->s;
        AllocScope scope(&plan->alloc);
        const i64 D4 = plan->t0_elems();
        const bool with_dir = dT0_dev && dlnZ_dir_host;
        if (with_dir)
            DTRG_HIP(hipMemcpyAsync(plan->dT0buf.p, dT0_dev, D4 * sizeof(double), hipMemcpyDeviceToDevice, plan->s));
        plan_backward(plan, gbar, with_dir, Mode::Adaptive);
        DTRG_HIP(hipMemcpyAsync(T0bar_dev, plan->T0barbuf.p, D4 * sizeof(double), hipMemcpyDeviceToDevice, plan->s));
        if (with_dir) *dlnZ_dir_host = plan->scal_h[5];
        DTRG_HIP(hipStreamSynchronize(plan->s));
        return DTRG_OK;
    } catch (const Error& e) {
        if (plan) (void)hipStreamSynchronize(plan->s);
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_plan_isometry(dtrg_plan* plan, int k, double* w_dev, void* stream) {
    g_last_error.clear();
    try {
        StepCk& st = plan_step(plan, k);
        DTRG_REQUIRE(w_dev, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(plan->fwd_ok, DTRG_ESTATE, "plan has no successful forward");
        plan->s = (hipStream_t)stream;
        copy2d(st.U.p, st.sh.b, st.U.bs, w_dev, st.sh.K, 0, st.sh.n, st.sh.K, 1, plan->s);
        DTRG_HIP(hipStreamSynchronize(plan->s));
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

dtrg_status dtrg_plan_fix_isometry(dtrg_plan* plan, int k, const double* w_dev, void* stream) {
    g_last_error.clear();
    try {
        StepCk& st = plan_step(plan, k);
        DTRG_REQUIRE(!st.sh.ident, DTRG_EINVAL, "step keeps everything (chi' = X^2): its isometry is the identity");
        plan->s = (hipStream_t)stream;
        plan->alloc.stream = plan->s;
        AllocScope scope(&plan->alloc);
        plan->fwd_ok = false;
        plan->sched_fwd = plan->sched_bwd = false;
        if (!w_dev) {
            st.fixed = false;
            return DTRG_OK;
        }
        if (st.wbar.n == 0) st.wbar.alloc_inst(1, (i64)st.sh.n * st.sh.K);
        copy2d(w_dev, st.sh.K, 0, st.U.p, st.sh.b, st.U.bs, st.sh.n, st.sh.K, 1, plan->s);
        DTRG_HIP(hipStreamSynchronize(plan->s));
        st.fixed = true;
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_plan_isometry_grad(dtrg_plan* plan, int k, double* wbar_dev, void* stream) {
    g_last_error.clear();
    try {
        StepCk& st = plan_step(plan, k);
        DTRG_REQUIRE(wbar_dev, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(st.fixed, DTRG_EINVAL, "step has no fixed isometry");
        DTRG_REQUIRE(plan->fwd_ok && plan->sched_bwd, DTRG_ESTATE, "no backward pass since the forward");
        plan->s = (hipStream_t)stream;
        copy2d(st.wbar.p, st.sh.K, 0, wbar_dev, st.sh.K, 0, st.sh.n, st.sh.K, 1, plan->s);
        DTRG_HIP(hipStreamSynchronize(plan->s));
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

dtrg_status dtrg_isometry_optimize(dtrg_plan* plan, const double* T0_dev, int layers, int n_inner, int n_sweeps,
                                   void* stream, double* lnZ_hotrg_host, double* lnZ_host, double* history_host) {
    g_last_error.clear();
    try {
        DTRG_REQUIRE(plan && T0_dev && lnZ_host, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(plan->nb == 1, DTRG_EINVAL, "not a single-instance plan");
        plan->fwd_ok = false;
        plan->s = (hipStream_t)stream;
        plan->alloc.stream = plan->s;
        AllocScope scope(&plan->alloc);
        const i64 D4 = plan->t0_elems();
        DTRG_HIP(hipMemcpyAsync(plan->T0buf.p, T0_dev, D4 * sizeof(double), hipMemcpyDeviceToDevice, plan->s));
        std::vector<double> hist;
        plan_isometry_optimize(plan, layers, n_inner, n_sweeps, lnZ_hotrg_host, &hist);
        *lnZ_host = plan->scal_h[0];
        if (history_host) std::copy(hist.begin(), hist.end(), history_host);
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

dtrg_status dtrg_plan_step_info(const dtrg_plan* plan, int k, dtrg_step_info* info) {
    g_last_error.clear();
    if (!plan || !info) { g_last_error = "NULL argument"; return DTRG_EINVAL; }
    if (!plan->fwd_ok) { g_last_error = "plan has no successful forward"; return DTRG_ESTATE; }
    if (k < 1 || k > plan->nsteps) { g_last_error = "step index out of range"; return DTRG_EINVAL; }
    try {
        step_info(plan, 0, k, info);
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

size_t dtrg_plan_device_bytes(const dtrg_plan* plan) { return plan ? plan->bytes() : 0; }

void dtrg_plan_destroy(dtrg_plan* plan) {
    if (!plan) return;
    (void)hipStreamSynchronize(plan->s);
    delete plan;
}

dtrg_status dtrg_batch_create(int n_inst, int D, const int* chi_host, int n_steps, const dtrg_options* opt,
                              dtrg_batch** batch_out) {
    g_last_error.clear();
    if (batch_out) *batch_out = nullptr;
    try {
        DTRG_REQUIRE(batch_out && chi_host, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(n_inst >= 1 && n_inst <= 65535, DTRG_EINVAL, "n_inst out of range [1, 65535]");
        std::unique_ptr<dtrg_batch> Bt(new dtrg_batch());
        Bt->n_inst = n_inst; Bt->D = D; Bt->nsteps = n_steps;
        if (opt) validate_options(*opt);
        DTRG_REQUIRE(!opt || opt->chain_phys == 0, DTRG_EINVAL, "batches run scheme (a) only (chain_phys must be 0)");
        DTRG_REQUIRE(!opt || opt->side_rule == 0, DTRG_EINVAL, "batches take the left unfolding only (side_rule must be 0)");
        Bt->alloc = allocator_of(opt, nullptr);
        AllocScope scope(&Bt->alloc);
        std::map<int, size_t> group_of;
        std::vector<int> order;
        for (int i = 0; i < n_inst; ++i) {
            validate_sizes(D, chi_host[i], n_steps);
            auto it = group_of.find(chi_host[i]);
            if (it == group_of.end()) {
                group_of[chi_host[i]] = Bt->members.size();
                Bt->members.emplace_back();
                order.push_back(chi_host[i]);
            }
            Bt->members[group_of[chi_host[i]]].push_back(i);
        }
        for (size_t g = 0; g < order.size(); ++g) {
            Bt->plans.push_back(make_plan(D, order[g], n_steps, (int)Bt->members[g].size(), opt,
                                          (double)Bt->members[g].size() / n_inst));
            Bt->idx.emplace_back();
            Bt->idx.back().alloc(Bt->members[g].size());
            DTRG_HIP(hipMemcpy(Bt->idx.back().p, Bt->members[g].data(), Bt->members[g].size() * sizeof(int),
                               hipMemcpyHostToDevice));
            hipStream_t s;
            DTRG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            Bt->branch.push_back(s);
            hipEvent_t e;
            DTRG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            Bt->join.push_back(e);
        }
        DTRG_HIP(hipEventCreateWithFlags(&Bt->fork, hipEventDisableTiming));
        DTRG_HIP(hipEventCreateWithFlags(&Bt->ev_in, hipEventDisableTiming));
        DTRG_HIP(hipStreamCreateWithFlags(&Bt->origin, hipStreamNonBlocking));
        *batch_out = Bt.release();
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_batch_run(dtrg_batch* batch, const double* T0s_dev, const double* dT0s_dev, double gbar,
                           double* lnZ_host, double* T0bar_dev, double* dlnZ_dir_host, int replay, void* stream) {
    g_last_error.clear();
    hipStream_t s = (hipStream_t)stream;
    try {
        DTRG_REQUIRE(batch && T0s_dev && lnZ_host, DTRG_EINVAL, "NULL argument");
        DTRG_REQUIRE(std::isfinite(gbar), DTRG_EINVAL, "gbar is not finite");
        DTRG_REQUIRE(replay == 0 || replay == 1, DTRG_EINVAL, "replay must be 0 or 1");
        batch->alloc.stream = s;
        AllocScope scope(&batch->alloc);
        const bool with_dir = dT0s_dev && dlnZ_dir_host && T0bar_dev;
        const double* dT0 = with_dir ? dT0s_dev : nullptr;
        if (!replay) {
            batch->drop_graph();
            batch->sched = batch->sched_bwd = false;
            for (size_t g = 0; g < batch->plans.size(); ++g) {
                batch_group(batch, g, T0s_dev, dT0, gbar, T0bar_dev, Mode::Adaptive, s);
                batch->plans[g]->fwd_ok = true;
            }
            DTRG_HIP(hipStreamSynchronize(s));
            batch->sched = true;
            batch->sched_bwd = T0bar_dev != nullptr;
        } else {
            DTRG_REQUIRE(batch->sched && (batch->sched_bwd || !T0bar_dev), DTRG_ESTATE,
                         "replay without a recorded schedule (run once with replay = 0 first)");
            // the graph runs on the batch's own stream, after the work already queued on `stream`
            hipStream_t o = batch->origin;
            DTRG_HIP(hipEventRecord(batch->ev_in, s));
            DTRG_HIP(hipStreamWaitEvent(o, batch->ev_in, 0));
            if (!batch->exec || batch->g_T0 != T0s_dev || batch->g_dT0 != dT0 || batch->g_T0bar != T0bar_dev ||
                batch->g_gbar != gbar)
                capture(batch, T0s_dev, dT0, gbar, T0bar_dev, o);
            DTRG_HIP(hipGraphLaunch(batch->exec, o));
            s = o;
            for (auto& P : batch->plans) {
                P->s = s;
                plan_read_back(P.get());
            }
            for (size_t g = 0; g < batch->plans.size(); ++g) {
                dtrg_plan* P = batch->plans[g].get();
                P->fwd_ok = false;
                for (int i = 0; i < P->nb; ++i)
                    if (P->flags_h[i] & kFlagErrorMask) {
                        try {
                            plan_throw_flags(P, kFlagErrorMask, "replay");
                        } catch (const Error& e) {
                            throw Error(e.code, "batch instance " + std::to_string(batch->members[g][i]) + " (chi " +
                                                    std::to_string(P->chi) + "): " + e.what() +
                                                    "; the recorded schedule does not fit these inputs, run with "
                                                    "replay = 0 to record a new one");
                        }
                    }
                P->fwd_ok = true;
            }
        }
        batch_results(batch, lnZ_host, dlnZ_dir_host, with_dir);
        return DTRG_OK;
    } catch (const Error& e) {
        if (batch) (void)hipStreamSynchronize(s);
        return fail(e);
    } catch (const std::exception& e) {
        if (batch) (void)hipStreamSynchronize(s);
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_batch_step_info(const dtrg_batch* batch, int inst, int k, dtrg_step_info* info) {
    g_last_error.clear();
    if (!batch || !info) { g_last_error = "NULL argument"; return DTRG_EINVAL; }
    if (inst < 0 || inst >= batch->n_inst) { g_last_error = "instance index out of range"; return DTRG_EINVAL; }
    if (k < 1 || k > batch->nsteps) { g_last_error = "step index out of range"; return DTRG_EINVAL; }
    try {
        for (size_t g = 0; g < batch->plans.size(); ++g) {
            const auto& mem = batch->members[g];
            auto it = std::find(mem.begin(), mem.end(), inst);
            if (it == mem.end()) continue;
            const dtrg_plan* P = batch->plans[g].get();
            if (!P->fwd_ok) { g_last_error = "batch has no successful run"; return DTRG_ESTATE; }
            step_info(P, (int)(it - mem.begin()), k, info);
            return DTRG_OK;
        }
        g_last_error = "instance not found";
        return DTRG_EINVAL;
    } catch (const Error& e) {
        return fail(e);
    }
}

dtrg_status dtrg_batch_profile(dtrg_batch* batch, long long* launches, double* total_ms, double* flops, int reset) {
    g_last_error.clear();
    if (!batch || !launches || !total_ms || !flops) { g_last_error = "NULL argument"; return DTRG_EINVAL; }
    long long n = 0;
    double ms = 0.0, fl = 0.0;
    for (auto& P : batch->plans) {
        long long a = 0;
        double b = 0.0, c = 0.0;
        const dtrg_status st = dtrg_plan_profile(P.get(), &a, &b, &c, reset);
        if (st != DTRG_OK) return st;
        n += a; ms += b; fl += c;
    }
    *launches = n; *total_ms = ms; *flops = fl;
    return DTRG_OK;
}

dtrg_status dtrg_hotrg_batched(const double* T0s_dev, int D, const int* chi_host, int n_inst, int n_steps,
                               const double* gbar_host, const dtrg_options* opt, void* stream, double* lnZ_host,
                               double* T0bar_dev, const double* dT0s_dev, double* dlnZ_dir_host) {
    g_last_error.clear();
    if (!T0s_dev || !chi_host || !lnZ_host || (gbar_host && !T0bar_dev) || (!gbar_host && T0bar_dev)) {
        g_last_error = "NULL argument (gbar_host and T0bar_dev are both given or both NULL)";
        return DTRG_EINVAL;
    }
    dtrg_batch* Bt = nullptr;
    dtrg_status st = dtrg_batch_create(n_inst, D, chi_host, n_steps, opt, &Bt);
    if (st != DTRG_OK) return st;
    st = dtrg_batch_run(Bt, T0s_dev, dT0s_dev, gbar_host ? *gbar_host : 1.0, lnZ_host, T0bar_dev, dlnZ_dir_host, 0,
                        stream);
    const std::string msg = g_last_error;
    dtrg_batch_destroy(Bt);
    g_last_error = msg;
    return st;
}

size_t dtrg_batch_device_bytes(const dtrg_batch* batch) {
    if (!batch) return 0;
    size_t t = 0;
    for (auto& P : batch->plans) t += P->bytes();
    return t;
}

void dtrg_batch_destroy(dtrg_batch* batch) {
    if (!batch) return;
    for (auto& P : batch->plans) (void)hipStreamSynchronize(P->s);
    for (auto s : batch->branch) (void)hipStreamSynchronize(s);
    delete batch;
}

const char* dtrg_last_error(void) { return g_last_error.c_str(); }

const char* dtrg_version(void) { return "dtrg 0.2 (gfx950)"; }

int dtrg_tuned_shapes(void) { return tuned_count(); }

dtrg_status dtrg_contract(int precision, int M, int N, int K, const void* A_dev, long long lda, int a_kmajor,
                          const void* B_dev, long long ldb, int b_kmajor, void* C_dev, long long ldc, int out_f64,
                          double alpha, double beta, void* stream) {
    return dtrg_contract_config(precision, M, N, K, A_dev, lda, a_kmajor, B_dev, ldb, b_kmajor, C_dev, ldc, out_f64,
                                alpha, beta, 0, 0, stream);
}

dtrg_status dtrg_contract_config(int precision, int M, int N, int K, const void* A_dev, long long lda, int a_kmajor,
                                 const void* B_dev, long long ldb, int b_kmajor, void* C_dev, long long ldc,
                                 int out_f64, double alpha, double beta, int tile, int splits, void* stream) {
    g_last_error.clear();
    // scratch (split-K partials and bf16 planes) per thread and stream: calls on one stream run in
    // order and may share it; calls on different streams must not
    struct CallScratch {
        Scratch ws;
        DevBuf<double> planes;
    };
    static thread_local std::map<hipStream_t, CallScratch> scratch_of;
    try {
        ContractCall c = contract_call(precision, M, N, K, A_dev, lda, a_kmajor, B_dev, ldb, b_kmajor, C_dev, ldc,
                                       out_f64, alpha, beta, tile, splits);
        const hipStream_t s = (hipStream_t)stream;
        CallScratch& sc = scratch_of[s];
        sc.planes.ensure((size_t)c.plane_doubles());
        contract_launch(c, sc.planes.p, s, sc.ws);
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

dtrg_status dtrg_contract_noalloc(int precision, int M, int N, int K, const void* A_dev, long long lda, int a_kmajor,
                                  const void* B_dev, long long ldb, int b_kmajor, void* C_dev, long long ldc,
                                  int out_f64, double alpha, double beta, void* stream) {
    g_last_error.clear();
    try {
        ContractCall c = contract_call(precision, M, N, K, A_dev, lda, a_kmajor, B_dev, ldb, b_kmajor, C_dev, ldc,
                                       out_f64, alpha, beta, 0, 0);
        // the whole need, checked before any work is issued: planes first, split-K partials after
        const i64 plane_bytes = (c.plane_doubles() * 8 + 255) / 256 * 256;
        const i64 splitk_bytes = gemm_workspace(c.pr, c.g) * 8;
        DTRG_REQUIRE(plane_bytes + splitk_bytes <= kNoAllocScratchBytes, DTRG_EINVAL,
                     "dtrg_contract_noalloc: the contraction needs " + std::to_string(plane_bytes + splitk_bytes) +
                         " bytes of scratch, more than the library's static " +
                         std::to_string(kNoAllocScratchBytes) + " bytes");
        char* base = (char*)noalloc_scratch_ptr();
        Scratch ws;   // borrowed views of the static array: never freed or grown
        ws.splitk.borrow((double*)(base + plane_bytes), (size_t)((kNoAllocScratchBytes - plane_bytes) / 8));
        contract_launch(c, (double*)base, (hipStream_t)stream, ws);
        return DTRG_OK;
    } catch (const Error& e) {
        return fail(e);
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return DTRG_EHIP;
    }
}

}  // extern "C"
