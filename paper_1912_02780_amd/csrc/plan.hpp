// The HOTRG plan: checkpoints, workspaces and the per-step schedule of nb independent problem
// instances that share (D, chi, n_steps), and the engine that runs their forward and backward
// passes.
//
// Two modes.  An adaptive pass reads small results back to the host to take its data-dependent
// decisions (subspace iterations to convergence, the degree and interval of the complement
// expansion, the tile autotuner) and records them in the schedule.  A fixed pass replays the
// recorded schedule without any host read-back or allocation, so it can be captured into a HIP
// graph; its acceptance tests run on the device and leave per-instance flags that the caller
// reads afterwards.
#pragma once

#include <string>
#include <vector>

#include "common.hpp"

namespace dtrg {

enum class Mode { Adaptive, Fixed };

// Per-instance error flags (device int per instance).
enum : int {
    kFlagNonPos = 1,      // a norm or trace is not positive
    kFlagChol = 2,        // non-positive pivot in CholeskyQR (diagnostic only)
    kFlagNonFinite = 4,   // a norm or trace is not finite
    kFlagSubspace = 8,    // subspace iteration residual above the acceptance bound
    kFlagChebTail = 16,   // complement expansion coefficients not decayed at the recorded degree
    kFlagChebBound = 32,  // complement expansion not bounded (spectrum outside its interval)
    kFlagJacobi = 64,     // full Jacobi eigensolve still rotating at its sweep cap
    kFlagTransfer = 128,  // scheme (b): dominant eigenvalue of the transfer matrix not resolved
};
// the flags that fail a pass (kFlagChol is a diagnostic: the shifted pass absorbs it)
constexpr int kFlagErrorMask =
    kFlagNonPos | kFlagNonFinite | kFlagSubspace | kFlagChebTail | kFlagChebBound | kFlagJacobi | kFlagTransfer;

// Per-instance FP64 scalars: one row of kScPlan + kScStep * n_steps doubles per instance.
// scheme (b): weight of the current isometry added to its environment before the polar factor
constexpr double kPolarTieBreak = 1e-6;
// scheme (b): shift of the trace-normalised Gram in the subspace iteration's block update
constexpr double kChainGramShift = 0x1p-45;
// side rule: the right unfolding wins only when its truncated weight is below the left one's by
// more than this (absolute, on the trace-normalised spectrum): ties decided by rounding go left
constexpr double kSideMargin = 1e-12;
constexpr int kScPlan = 16;   // 0 L (ln Z / N), 4 final trace (scheme (b): the final transfer matrix's
                              // dominant eigenvalue), 5 <T0bar, dT0>, 6 c0, 7 1/c0, 8 polar tie-break
                              // norm; 9-11 the side rule's copy of a step's slots 2, 3 and 8
constexpr int kScStep = 12;   // per step: 0 c_k, 1 1/c_k, 2 trace of the Gram, 3 residual of the first
                              // unresolved Ritz pair, 4 lo, 5 hi (complement interval), 6 |v_0|,
                              // 7 |v_m|, 8 largest resolved residual, 9 coefficient tail ratio;
                              // scheme (b): 10 ln Z per cell per slice closed after the step,
                              // 11 the dominant eigenvalue of that step's transfer matrix

struct StepShape {
    int X = 0, Y = 0, K = 0, n = 0, b = 0;
    int e = 0;          // leading eigenpairs resolved to full accuracy: the kept K plus the
                        // discarded ones nearest the cut (the rest of the block is a guard)
    bool full = false;
    bool mixed = false; // projection contractions of this step in the mixed precision
    // block-locked eigensolve (scheme (b) with chi' beyond one Rayleigh-Ritz block): lock_n blocks
    // of lock_bw columns, each resolving lock_r eigenpairs; then e = lock_n * lock_r and the last
    // block's lock_bw - lock_r guard columns complete U (b = e + guard)
    int lock_bw = 0, lock_r = 0, lock_n = 0;
    int rr() const { return lock_n ? lock_bw : b; }   // width of the Rayleigh-Ritz problems
    // scheme (b): an untruncated step (chi' = X^2 > 96) projects with the identity: Z does not depend
    // on an orthogonal isometry that keeps everything, so no Gram is needed, forward or backward
    bool ident = false;
    double join_flops() const { return 2.0 * K * Y * X * (double)(Y * X) * (X * Y); }
};

// A contraction operand of nb instances in a contraction format (FP64, FP32 or bf16 planes):
// per instance `per` elements (rows x padded row stride, a multiple of 8); bf16 planes outermost,
// plane q of instance i at (q * nb + i) * per elements.
struct OpBuf {
    DevBuf<double> mem;   // raw storage
    i64 per = 0;
    int esz = 8, np = 1, nb = 1;
    void alloc(Prec pr, int n_inst, i64 per_elems) {
        np = prec_planes(pr);
        esz = pr == Prec::F64 ? 8 : (pr == Prec::F32 ? 4 : 2);
        nb = n_inst;
        per = (per_elems + 7) / 8 * 8;
        const i64 bytes = (i64)np * nb * per * esz;
        mem.alloc((size_t)((bytes + 7) / 8));
    }
    void* p() const { return mem.p; }
    i64 ps() const { return per * nb; }
};

// Operands of the projection contractions and their adjoints in one format, every one stored
// K-contiguous for the contraction that reads it (names: the layouts written next to their producers).
struct OpSet {
    Prec pr = Prec::F64;
    OpBuf Wt, Wt2, UT, Us, Tp, Tb, Tb2, TpT, Tpb, Tpb2;   // chi^4 / n x b class
    OpBuf X1, X2;                                          // chi^5 class
};

struct StepCk {
    StepShape sh;
    DevBuf<double> T;      // normalised input [X][X][Y][Y] (checkpoint)
    DevBuf<double> U;      // [n][b] eigenvectors / Ritz vectors (first K columns: w)
    DevBuf<double> lam;    // b eigenvalues / Ritz values, descending
    // forward intermediates kept for the backward pass (within the plan's checkpoint budget)
    bool keep_gram = false;          // Ak, Bk, Gk: half-environments and normalised Gram
    bool keep_join = false;          // P1k, Q2k: first projection and join (written there by the
                                     // forward pass, read by the backward)
    DevBuf<double> Ak, Bk, Gk;
    OpBuf P1k, Q2k;
    // schedule (written by adaptive passes, replayed by fixed passes)
    int iters = 0;         // subspace iterations
    int rr_stride = 1;     // Gram products per Rayleigh-Ritz solve of the subspace iteration
    int cheb = 0;          // degree of the complement expansion (0: none)
    double hi_mult = 1.0;  // widening factor of the complement interval
    // a given isometry (the first K columns of U, set by the caller or by the isometry optimiser):
    // the forward projects with it instead of the leading eigenvectors of the step's Gram, and the
    // backward stops at the projection adjoint and leaves d(gbar lnZ/N)/dw in wbar [n][K]
    bool fixed = false;
    DevBuf<double> wbar;
    // side rule: the unfolding the isometry came from (0: left legs (x1, x2), 1: right legs
    // (x1', x2')) and the truncated weights of both (NaN unless the rule ran on this step)
    int side = 0;
    double tw_left = NAN, tw_right = NAN;
};

}  // namespace dtrg

struct dtrg_plan {
    int D = 0, chi = 0, nsteps = 0, nb = 1;
    int phys = 0;               // scheme (b): physical dimension of the MPO input (0: scheme (a))
    bool chain() const { return phys > 0; }
    // elements of one instance's input (D^4, or D^2 d^2 for an MPO)
    dtrg::i64 t0_elems() const { return chain() ? (dtrg::i64)D * D * phys * phys : (dtrg::i64)D * D * D * D; }
    dtrg_options opt{};
    dtrg::Prec prec = dtrg::Prec::F64;
    hipStream_t s = nullptr;
    dtrg::Allocator alloc;      // the caller's device allocator (empty: hipMalloc)
    std::vector<dtrg::StepCk> steps;
    std::vector<dtrg::StepShape> shape;
    bool fwd_ok = false;        // a forward pass succeeded (checkpoints valid)
    bool sched_fwd = false;     // the schedule of the forward pass is recorded
    bool sched_bwd = false;     // the schedule of the backward pass is recorded
    int Xf = 0, Yf = 0;
    dtrg::i64 S = 0;            // scalar row length per instance (kScPlan + kScStep * nsteps)
    dtrg::DevBuf<double> scal;  // nb x S
    dtrg::DevBuf<int> flags;    // nb error flags
    dtrg::DevBuf<int> misc;     // 4 ints: Jacobi sweep counter
    dtrg::DevBuf<int> orth;     // nb ints: the second CholeskyQR pass found its input orthonormal
                                // to within 1e-6, so that its output is orthonormal to working
                                // accuracy and the third pass is skipped
    std::vector<double> scal_h; // host copy of scal after a pass (adaptive passes, or on demand)
    std::vector<int> flags_h;
    dtrg::Scratch ws;
    // inputs and outputs of the nb instances ([nb][D^4])
    dtrg::DevBuf<double> T0buf, T0barbuf, dT0buf;
    // workspaces (instance stride bs)
    dtrg::DevBuf<double> TA, TB, Tn, Tbar, Tbar2, Wk;
    dtrg::DevBuf<double> A, B;
    // contraction operands: [0] for steps in FP64, [1] for steps in the plan's contraction format
    dtrg::OpSet ops[2];
    dtrg::DevBuf<double> Gw, Gt, Ub, Xe, Xc, Re, Om, Sm, Vc, Vp, Vn, Ye, We;
    dtrg::DevBuf<double> V1, V2, Y1, Y2, H, Z, Rinv, Sg, th, res, nrm, coef, fv;
    dtrg::DevBuf<double> ctab;  // Chebyshev DCT tables of degree 8, 16, ..., 1024
    bool ctab_ready = false;
    dtrg::DevBuf<double> tune_c;  // autotuner output scratch
    dtrg::DevBuf<double> polS, polV, pollam;   // polar factor of an isometry gradient (2K x 2K, 2K)
    dtrg::DevBuf<double> chain_lr;             // scheme (b): right and left dominant eigenvectors [r | l]
    dtrg::DevBuf<double> side_U, side_lam;     // side rule: the other unfolding's eigenvectors and values
    dtrg::DevBuf<double> lockW;                // block-locked eigensolve: projections on the locked vectors
    dtrg::DevBuf<double> kronW;                // scheme (b): intermediates of the Kronecker-form Gram products
    dtrg::DevBuf<double> Akr;                  // ... and the permuted half-environment / adjoint (X^2 Y^2)
    bool side_rule() const { return opt.side_rule != 0; }
    dtrg::i64 ck_budget = 0;      // bytes the kept forward intermediates may take
    std::string tile_table;       // persisted autotuning table ("" = none)
    int tuned_seen = -1;          // size of the process table when the file was last written
    bool mixed() const { return prec != dtrg::Prec::F64; }
    // HIP-event timing of the chi^7 join contractions (adaptive passes with opt.profile)
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_flops = 0.0;
    ~dtrg_plan();
    double* sc(int k, int slot) { return scal.p + dtrg::kScPlan + (dtrg::i64)dtrg::kScStep * (k - 1) + slot; }
    double* sp(int slot) { return scal.p + slot; }
    dtrg::i64 cap_bytes(const void* p) const;
    dtrg::i64 cap_of(const void* p, int elem = 8) const {
        const dtrg::i64 b = cap_bytes(p);
        return b < 0 ? -1 : b / elem;
    }
    size_t bytes() const;
};

namespace dtrg {

// Allocate the plan of nb instances of (D, chi, nsteps) with options opt (validated by the caller).
void plan_setup(dtrg_plan* P);
// Forward pass of the nb instances in P->T0buf (adaptive or fixed); in adaptive mode throws on
// the first failed instance and leaves ln Z / N in P->scal_h.
void plan_forward(dtrg_plan* P, Mode mode);
// Backward pass into P->T0barbuf (and <T0bar, dT0> with dT0 from P->dT0buf if with_dir).
void plan_backward(dtrg_plan* P, double gbar, bool with_dir, Mode mode);
// Read scalars and flags back (synchronises the plan's stream); throw the error of the first
// flagged instance (bits in mask).
void plan_read_back(dtrg_plan* P);
// Differentiable-TRG isometry optimisation of the first `layers` truncating steps of a
// single-instance plan (T0 already in P->T0buf): n_sweeps sweeps over the layers from the finest
// scale up, n_inner MERA updates per layer and sweep (a backward pass for the isometry gradient E,
// w <- U V^T from E = U S V^T, a forward pass).  history (nullable): ln Z / N after every update.
// Leaves the optimised isometries fixed in the plan and its last forward pass valid.
void plan_isometry_optimize(dtrg_plan* P, int layers, int n_inner, int n_sweeps, double* lnZ_hotrg,
                            std::vector<double>* history);
// The MERA update of step k's fixed isometry from the gradient in its wbar: w <- polar factor.
void polar_update(dtrg_plan* P, int k);
void plan_throw_flags(const dtrg_plan* P, int mask, const std::string& where);

// tune.hip: the tile configuration for op, measured once per shape when tuning is allowed
// (adaptive passes with the autotuner on) and reused afterwards; `scratch` receives the trial
// outputs.
GemmCfg tuned_cfg(Prec prec, Out out, const GemmOp& op, bool allow_tune, hipStream_t s, Scratch& ws,
                  DevBuf<double>& scratch);
// Number of shapes in the tuning table (for tests and diagnostics).
int tuned_count();
// Merge a persisted table into the process table (a missing file loads nothing; returns the number
// of entries added), and write the process table to a file.
int tune_load(const std::string& path);
void tune_save(const std::string& path);

}  // namespace dtrg
