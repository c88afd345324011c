/*
 * dtrg.h - C ABI of the HOTRG coarse-graining step and its reverse-mode adjoint on one
 * AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv:1912.02780, Supplemental Material B and E):
 *   Z = periodic trace of a square network of identical rank-4 tensors T0 (SM A, first eq.).
 *   Each HOTRG step (SM B, eq. HOTRGstep and its figure) joins two copies of the current tensor
 *   along a vertical bond and compresses each doubled horizontal leg with an isometry w made of
 *   the leading chi' = min(chi, X^2) eigenvectors of the pair's (x1, x2)-unfolding Gram matrix
 *   (SM B, local HOSVD).  The direction alternates, the tensor is rescaled by its Frobenius norm
 *   every step, and after n steps (2^n sites) the periodic self-trace closes the network (main
 *   text, scheme (a)).  The result is ln Z / N, N = 2^n.
 *   The backward pass is the SRG environment recursion (SM B, eq. SRG), i.e. the chain rule
 *   (SM E, eqs. Eeq, Teq, Unify), extended through the eigensolver: the leading-eigenvector
 *   derivative uses the inverse gaps 1/(l_j - l_i) broadened to d / (d^2 + eps).
 *
 * Index order.  T0 is passed as T0[l][u][r][d] (left, up, right, down), row-major, D^4 doubles.
 * The same layout is used for the gradient T0bar.
 *
 * Memory.  Every pointer whose name ends in _dev is a device pointer (hipMalloc'd or from
 * PyTorch's allocator) on the current HIP device; every pointer ending in _host is host memory.
 * The caller owns T0_dev, T0bar_dev and the stream.  A plan owns its checkpoints and workspaces
 * (device memory allocated when the plan is created, through the options' alloc_fn / free_fn when
 * given (e.g. PyTorch's caching allocator), with hipMalloc / hipFree otherwise; released by
 * dtrg_plan_destroy).  A step's checkpoint is its normalised input tensor, its isometry and its
 * spectrum; the backward recomputes the rest of the step from it, except the forward
 * intermediates the plan keeps within dtrg_options.checkpoint_gib.  The contraction kernel's
 * split-K scratch (and the autotuner's trial output) grows on the first forward and backward of a
 * plan; later calls on the plan allocate no device memory.
 *
 * Errors.  Every entry point returns a dtrg_status; nothing throws or aborts across the ABI.
 * dtrg_last_error() returns a thread-local message describing the last failure on the calling
 * thread (valid until the next call on that thread).  If dtrg_hotrg_forward fails, *plan_out is
 * set to NULL and nothing is leaked.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the legacy default stream).  All device work of a
 * call is enqueued on it; entry points that return host values synchronise that stream.  One
 * plan must not be used from two threads at once.
 */
#ifndef DTRG_H
#define DTRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DTRG_OK = 0,
    DTRG_EINVAL = 1,   /* invalid argument: sizes, NULL pointers, non-finite T0 */
    DTRG_ENOMEM = 2,   /* device allocation failed */
    DTRG_EHIP = 3,     /* a HIP runtime call failed */
    DTRG_ENOCONV = 4,  /* the truncated eigensolver did not reach its tolerance */
    DTRG_ENONPOS = 5,  /* a norm or the final trace is not positive and finite */
    DTRG_ESTATE = 6    /* call out of order (e.g. backward on a plan whose forward failed) */
} dtrg_status;

/* Arithmetic of the O(chi^7) and O(chi^6) contractions.  The eigensolver, its adjoint, all
 * norms and the log accumulation are always FP64. */
typedef enum {
    DTRG_FP64 = 0,     /* FP64 operands, FP64 MFMA */
    DTRG_FP32 = 1,     /* FP32 operands, FP32 MFMA, FP32 accumulation */
    DTRG_BF16X3 = 2,   /* FP32 values carried as two bf16 planes x0 + x1 (x0 = bf16(x),
                          x1 = bf16(x - x0)); a1 b0 + a0 b1 + a0 b0 on bf16 MFMA with FP32
                          accumulation (the "3-term split-bf16" product, ~2^-17 relative) */
    DTRG_BF16X6 = 3    /* three bf16 planes; the six partial products down to 2^-24 relative:
                          FP32-level accuracy on bf16 MFMA */
} dtrg_precision;

/* Device-memory callbacks.  alloc_fn returns `bytes` bytes of device memory on the current device,
 * aligned to 256 bytes, for use on `stream` (the hipStream_t of the call that allocates; NULL for
 * dtrg_plan_create and dtrg_batch_create), or NULL when it cannot (the call then fails with
 * DTRG_ENOMEM).  free_fn releases a block with the size it was allocated with; the library waits
 * for the device to finish with a block before it frees it.  `user` is passed through. */
typedef void* (*dtrg_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*dtrg_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

typedef struct {
    int contract;             /* dtrg_precision; default DTRG_FP64 */
    int gram_fp64;            /* 1: half-environments and Gram in FP64 whatever `contract` is
                                 (default 1) */
    double eig_broadening;    /* eps in d / (d^2 + eps), on the trace-normalised spectrum;
                                 default 1e-12 */
    int max_subspace_iters;   /* cap on block subspace iterations per step; default 60 */
    double subspace_tol;      /* residual |G v - theta v| on the trace-normalised Gram at which
                                 the kept Ritz vectors count as converged; default 1e-15.  If the
                                 residual stops decreasing above it, the step is accepted when the
                                 residual is below 1e-12 and fails with DTRG_ENOCONV otherwise. */
    int block_size;           /* subspace block b (> chi', <= 96); 0 = automatic (min(96, max(chi' + 16,
                                 2 chi'))).  DTRG_EINVAL if b <= chi' on a step that iterates.
                                 Scheme (b): a block_size of at most chi' + 8 selects the block-locked
                                 eigensolve with blocks of that width (which is automatic, with 96
                                 columns, for chi' > 80); each block resolves all but max(8, b/4)
                                 of its columns, and together they resolve max(8, chi'/2) pairs
                                 beyond the cut where X^2 leaves room (at least 8) */
    int autotune;             /* 1: the first time a contraction shape is met, time every tile shape
                                 (64 x 64, 128 x 128, and for the bf16-plane precisions 256 x 128,
                                 64 x 64 on full-width waves for outputs of at most 64 columns and
                                 128 x 128 with one LDS stage for K of at most 128)
                                 and split-K factor (the least one that keeps every FP32
                                 accumulation chain at max_fp32_chain products or fewer, then 2, 3, 4, 5, 6, 8,
                                 12, 16, 24 and 32 above it) of the MFMA kernels on a scratch output
                                 (the least of three timed runs) and keep the fastest for that shape (a table shared by all plans of the
                                 process); 0: fixed heuristic.  Default 0 */
    int profile;              /* 1: time the chi^7 join contractions (scheme (b): the Gram products)
                                 with HIP events on the plan's stream (read with dtrg_plan_profile);
                                 default 0 */
    double checkpoint_gib;    /* device memory (GiB) the plan may spend keeping forward-pass
                                 intermediates that the backward pass would otherwise recompute:
                                 first each step's half-environments and normalised Gram (FP64),
                                 then, from the last step back, each step's first projection and
                                 join in the layouts their adjoints read.  What does not fit is
                                 recomputed in the backward pass (0: recompute everything, the
                                 least memory).  Results do not depend on it.  A batch divides it
                                 among its plans in proportion to their instances.  Finite, >= 0;
                                 default 64 */
    int oversample;           /* guard columns p of the subspace block when block_size is 0:
                                 b = min(96, chi' + p); 0 = automatic (see block_size); 0 <= p <= 95 */
    int max_fp32_chain;       /* longest FP32 accumulation chain (products summed into one FP32
                                 value) of the FP32 and split-bf16 formats, for every contraction
                                 except the two below: a contraction with a longer K is split into
                                 K chunks whose partials are summed in FP64 (as many chunks as
                                 16 GiB of partials allow, at most 256).  These contractions write
                                 at most chi^4 values, so the partials cost little traffic, while
                                 their K reaches chi^3 (the adjoints with respect to the lower copy
                                 and to both isometries).  32 <= value <= 2^20; default 4096 */
    int max_fp32_chain_wide;  /* the same for the join and its adjoint with respect to the upper
                                 copy's product, whose chi^5 outputs make every extra K chunk a
                                 full chi^5 pass of FP32 partials (K = chi^2 there).  32 <= value
                                 <= 2^20; default 4096 */
    const char* tile_table;   /* path of a persisted autotuning table, or NULL: when set, the
                                 plan loads the file's entries into the process table at creation
                                 (a missing file is not an error) and a pass that tuned new shapes
                                 rewrites the file (text, one shape and configuration per line),
                                 so tuned configurations, and with them the rounding of split-K
                                 sums, are the same in every process that uses the file.  Default
                                 NULL */
    dtrg_alloc_fn alloc_fn;   /* device allocator of the plan's memory, or NULL for hipMalloc;
                                 alloc_fn and free_fn are both set or both NULL (DTRG_EINVAL
                                 otherwise).  Default NULL */
    dtrg_free_fn free_fn;     /* its release function */
    void* alloc_user;         /* passed to both */
    int chain_phys;           /* 0: the paper's scheme (a), a square-lattice network of one D^4 tensor
                                 coarse-grained along alternating directions and closed by its
                                 self-trace.  d > 0: scheme (b) (paper, Fig. 1(b) and the infinite
                                 XY chain): T0 is one cell's matrix-product operator M[l][u][r][d]
                                 of bond D and physical dimension d (D x d x D x d doubles); every
                                 step squares the operator (the upper copy's input leg joined to
                                 the lower copy's output leg, the doubled bonds compressed by the
                                 step's isometry, the physical legs keeping dimension d), and the
                                 infinite chain is closed by the dominant eigenvalue of the final
                                 transfer matrix E[l][r] = sum_u M_n[l][r][u][u].  ln Z / N is then
                                 ln Z per cell per Trotter slice, and dtrg_step_info.lnZ_at_step
                                 gives it after every step.  0 <= d <= 16; batches take 0 only.
                                 Default 0 */
    int side_rule;            /* which unfolding of the pair gives each step's isometry (SM B: the
                                 local higher-order SVD of the pair).  0: the left legs (x1, x2).
                                 1: whichever of the left legs (x1, x2) and the right legs
                                 (x1', x2') has the smaller truncated weight (1 - the sum of the kept
                                 eigenvalues of its trace-normalised Gram), the right one only when
                                 lighter by more than 1e-12; one isometry still serves both sides,
                                 as a bond carries one projector.  Rule 1 eigensolves both Grams in
                                 the forward pass (the backward differentiates the chosen one); it
                                 matters for tensors without the left/right mirror symmetry
                                 (chiral or generic), while mirror-symmetric inputs keep the left
                                 side.  Single-instance plans of scheme (a) only (DTRG_EINVAL for
                                 batches and chain_phys > 0).  Default 0 */
    int polar_newton;         /* polar factor of the MERA update (dtrg_isometry_optimize): 0 = the
                                 Jacobi eigensolve of [[0, R], [R^T, 0]] for chi' <= 48 and the
                                 Newton-Schulz iteration X <- X (3 I - X^T X) / 2 above (chi' <= 80);
                                 1 = Newton-Schulz for every chi'.  Default 0 */
    int subspace_shift;       /* the block subspace iteration of scheme (a) (SM B: the isometry from
                                 the leading eigenvectors of the pair's Gram): 0 = each new block from
                                 G V; 1 = from (G - s I) V with s half the block's smallest Ritz
                                 value, the first-degree Chebyshev filter on [0, s]: the eigenvalues
                                 the block leaves out map into [-s, s], so a wanted pair converges at
                                 the ratio s / (lambda - s) in place of lambda_b / lambda.  The
                                 eigenvectors are those of G either way.  Scheme (b) plans build the
                                 block from (G + 2^-45 I) V whatever the setting.  Default 1 */
    int rr_skip;              /* Rayleigh-Ritz solves of the same subspace iteration, 0 to 3: a solve
                                 after every (rr_skip + 1)-th Gram product on steps that start from
                                 the previous step's vectors and whose first solve finds the block's
                                 Ritz values within eight decades (the smallest above 1e-8 of the
                                 largest, for every instance), where the product of a block that is
                                 not aligned with eigenvectors loses no direction to rounding (each
                                 new block is still re-orthonormalised); after every product
                                 elsewhere, and with 0.  The iteration still ends on a solve, whose
                                 Ritz residuals decide convergence.  The choice is made in the
                                 adaptive pass and replayed.  Scheme (b) plans solve after every
                                 product.  Default 3 */
} dtrg_options;

/* Per-step diagnostics, all gauge invariant. */
typedef struct {
    int X;                    /* horizontal bond dimension entering the step */
    int Y;                    /* vertical bond dimension entering the step */
    int chi_kept;             /* chi' = min(chi, X^2) */
    int full_eig;             /* 1 if the whole spectrum was computed (X^2 <= block limit) */
    int iters;                /* subspace iterations used (0 for a full eigensolve) */
    double c;                 /* Frobenius norm of the unnormalised step output */
    double trace_G;           /* trace of the symmetrised Gram */
    double lam_last_kept;     /* smallest kept eigenvalue of the normalised Gram */
    double lam_first_dropped; /* largest discarded eigenvalue (or Ritz value) */
    double resid;             /* largest kept residual |G v - theta v| */
    int cheb_degree;          /* degree of the complement expansion in the last backward */
    double trunc_weight;      /* discarded weight 1 - sum of the kept eigenvalues of the
                                 normalised Gram (its trace is 1) */
    double cut_gap;           /* lam_last_kept - lam_first_dropped (0 when nothing is cut) */
    double min_kept_gap;      /* least gap between consecutive kept eigenvalues (0 for one kept) */
    int mixed;                /* 1 if the step's projection contractions ran in the `contract`
                                 format, 0 if in FP64 */
    double lnZ_at_step;       /* scheme (b) (chain_phys > 0): ln Z per cell per Trotter slice of the
                                 chain closed after this step (rho(2^k tau)); NaN for scheme (a) */
    int side;                 /* unfolding the step's isometry came from: 0 left, 1 right */
    double trunc_weight_left; /* side_rule 1: truncated weights of the left and right unfoldings */
    double trunc_weight_right;/* (NaN with side_rule 0 and on steps with a given isometry) */
    int rr_stride;            /* Gram products per Rayleigh-Ritz solve of the subspace iteration (1 to
                                 4, see rr_skip; 0 where the step does not iterate) */
} dtrg_step_info;

typedef struct dtrg_plan dtrg_plan;

/* Fill *opt with the defaults documented above. */
void dtrg_default_options(dtrg_options* opt);

/*
 * Forward pass: ln Z / N for the 2^n_steps-site periodic network of T0.
 *   T0_dev        device, D^4 doubles, [l][u][r][d] (with opt->chain_phys = d > 0: one MPO cell,
 *                 D x d x D x d doubles); read only; all entries finite, not all 0.
 *   D             bond dimension of T0, 1 <= D <= 64.
 *   chi           truncation bond dimension, 1 <= chi <= 80 (scheme (b), opt->chain_phys > 0:
 *                 1 <= chi <= 512; chi' beyond one 96-column Rayleigh-Ritz block is found by the
 *                 block-locked eigensolve, blocks of 96 or of opt->block_size columns, each deflated
 *                 against the eigenvectors resolved before it; a step that keeps everything
 *                 (chi' = X^2 > 96) projects with the identity; a step whose chi' leaves fewer than
 *                 8 resolved pairs and a guard below X^2 gives DTRG_EINVAL).
 *   n_steps       number of single-direction HOTRG steps, 1 <= n_steps <= 62.
 *   opt           options or NULL for the defaults.
 *   stream        hipStream_t or NULL.
 *   plan_out      receives a plan holding one checkpoint per step (needed by the backward).
 *   lnZ_per_site_host  receives ln Z / N.
 * Synchronises `stream`.  DTRG_EINVAL for bad sizes / NULL pointers / non-finite T0,
 * DTRG_ENONPOS if T0 is zero or a scale or the final trace is not positive, DTRG_ENOCONV if the
 * eigensolver stalls above 1e-12, DTRG_ENOMEM / DTRG_EHIP on runtime failures.
 */
dtrg_status dtrg_hotrg_forward(const double* T0_dev, int D, int chi, int n_steps,
                               const dtrg_options* opt, void* stream, dtrg_plan** plan_out,
                               double* lnZ_per_site_host);

/*
 * Plan creation: allocates the checkpoints and workspaces of the forward and backward passes of
 * this (D, chi, n_steps, options) problem.  Same argument ranges and errors as dtrg_hotrg_forward.
 */
dtrg_status dtrg_plan_create(int D, int chi, int n_steps, const dtrg_options* opt, dtrg_plan** plan_out);

/*
 * Forward pass on an existing plan (its checkpoints are overwritten).  T0_dev: device, D^4 doubles,
 * [l][u][r][d] with the plan's D.  Synchronises `stream`.  Errors as dtrg_hotrg_forward; after a
 * failure the plan must not be used for a backward until a forward succeeds.
 */
dtrg_status dtrg_plan_forward(dtrg_plan* plan, const double* T0_dev, void* stream, double* lnZ_per_site_host);

/*
 * Backward pass: T0bar = gbar * d(lnZ/N)/dT0, written to T0bar_dev (device, D^4 doubles,
 * [l][u][r][d]).  If dT0_dev (device, D^4 doubles, same layout) is not NULL, also writes
 * <T0bar, dT0> to *dlnZ_dir_host (with dT0 = dT0/dbeta this is gbar * d(lnZ/N)/dbeta).
 * May be called any number of times on a plan whose forward succeeded.  Synchronises `stream`.
 */
dtrg_status dtrg_hotrg_backward(dtrg_plan* plan, double gbar, double* T0bar_dev,
                                const double* dT0_dev, double* dlnZ_dir_host, void* stream);

/*
 * Differentiable TRG (paper, main text: the isometries w of the RG steps as parameters of the
 * network, their environments E_w = w_bar / N_i from the backward pass (Eq. EGrad), and the MERA
 * update w <- U V^T from the SVD E_w = U S V^T).  Single-instance plans only.
 *
 * dtrg_plan_isometry: copy step k's isometry w[x1][x2][a] (n = X^2 rows of chi' values, row-major;
 *   w_dev device, n chi' doubles) after a successful forward pass.
 * dtrg_plan_fix_isometry: later forward passes project step k with the given isometry (w_dev
 *   device, same layout; copied into the plan) instead of the leading eigenvectors of the step's
 *   Gram, and the backward pass treats it as a parameter: it stops at the step's projection adjoint
 *   (nothing flows through that step's Gram) and keeps d(gbar lnZ/N)/dw.  w_dev NULL releases it.
 *   The plan needs a new forward pass afterwards (DTRG_ESTATE otherwise).
 * dtrg_plan_isometry_grad: after a backward pass, d(gbar lnZ/N)/dw of a step with a fixed isometry
 *   (wbar_dev device, n chi' doubles, layout of w): the environment E_w up to the positive factor
 *   Z N / N_i (DTRG_EINVAL for a step without a fixed isometry).
 * dtrg_isometry_optimize: forward pass of plain HOTRG on T0_dev (its ln Z / N to *lnZ_hotrg_host,
 *   nullable), then n_sweeps sweeps over the first `layers` steps whose isometry truncates (a
 *   scheme-(b) plan: the last `layers`, the optimisation depth below the final temperature)
 *   (chi' < X^2), from the finest scale up; per sweep and step, n_inner MERA updates, each a
 *   backward pass for the isometry gradient, the polar factor w <- U V^T (computed on the device
 *   without squaring the gradient's condition number), and a forward pass with the new isometry;
 *   the isometries above the optimised steps remain HOTRG's local ones, recomputed every pass.
 *   ln Z / N after every update goes to history_host (host, n_sweeps * layers * n_inner doubles,
 *   nullable), the last to *lnZ_host.  The optimised isometries stay fixed in the plan, whose last
 *   forward pass is valid (a backward pass may follow).  The optimised steps need chi' <= 80 and
 *   one Rayleigh-Ritz block (DTRG_EINVAL otherwise; see polar_newton for the polar factor);
 *   DTRG_EINVAL if fewer steps truncate than `layers`.
 * All four synchronise `stream`.
 */
dtrg_status dtrg_plan_isometry(dtrg_plan* plan, int k, double* w_dev, void* stream);
dtrg_status dtrg_plan_fix_isometry(dtrg_plan* plan, int k, const double* w_dev, void* stream);
dtrg_status dtrg_plan_isometry_grad(dtrg_plan* plan, int k, double* wbar_dev, void* stream);
dtrg_status dtrg_isometry_optimize(dtrg_plan* plan, const double* T0_dev, int layers, int n_inner, int n_sweeps,
                                   void* stream, double* lnZ_hotrg_host, double* lnZ_host, double* history_host);

/* Diagnostics of step k (1 <= k <= n_steps) of a plan whose forward succeeded.  A step with a fixed
 * isometry reports iters = -1 and zero spectrum fields. */
dtrg_status dtrg_plan_step_info(const dtrg_plan* plan, int k, dtrg_step_info* info);

/*
 * HIP-event timing of the chi^7 join contraction (the O(D^7) term of the step: the upper copy
 * times the left isometry joined with the lower copy over (x2, j); launched once per step in the
 * forward and once more in the backward's recompute) recorded since the last reset on a plan
 * created with opt.profile = 1: number of launches, summed milliseconds and summed algorithmic
 * flops (2 M N K per launch).  Only launches in the plan's contraction precision on the 128 x 128
 * tile are timed (all launches of that kernel), so the average matches that kernel's average in a
 * kernel trace.  Scheme (b) plans (whose passes the eigensolver dominates) time instead every
 * product with a step's Gram (the subspace iteration's and the eigen-adjoint's, FP64; in Kronecker
 * form two contractions each).  Synchronises on the recorded events; reset != 0 clears the record.
 */
dtrg_status dtrg_plan_profile(dtrg_plan* plan, long long* launches, double* total_ms, double* flops, int reset);

/*
 * Batches.  n_inst independent problems with the same D and n_steps and their own chi (e.g. an
 * Ising model at many temperatures and mixed bond dimensions) in one call.  Instances of equal chi
 * share every shape and run as one batched problem (each contraction, eigensolve and reduction is
 * one launch over all of them); the groups of different chi are independent branches.
 *
 * dtrg_batch_create: chi_host[n_inst] (host) holds each instance's chi; D, n_steps and each chi in
 * the ranges of dtrg_hotrg_forward, 1 <= n_inst <= 65535; opt as for plans (shared by all).
 * Allocates every group's checkpoints and workspaces.
 */
typedef struct dtrg_batch dtrg_batch;
dtrg_status dtrg_batch_create(int n_inst, int D, const int* chi_host, int n_steps, const dtrg_options* opt,
                              dtrg_batch** batch_out);

/*
 * Forward (and backward, when T0bar_dev is not NULL) of all instances.
 *   T0s_dev       device, n_inst x D^4 doubles, instance i at T0s_dev + i D^4, [l][u][r][d].
 *   dT0s_dev      device, same shape, or NULL: directions for <T0bar_i, dT0_i>.
 *   gbar          seed of the backward (the same for all instances).
 *   lnZ_host      host, n_inst: ln Z / N of each instance.
 *   T0bar_dev     device, n_inst x D^4 or NULL (forward only): gbar * d(lnZ/N)/dT0 per instance.
 *   dlnZ_dir_host host, n_inst or NULL: <T0bar_i, dT0_i> (needs dT0s_dev and T0bar_dev).
 *   replay = 0    adaptive run: iterates every eigensolve to convergence and sizes every complement
 *                 expansion from the data (reading small results back to the host), and records
 *                 these decisions as the batch's schedule.  Groups run one after the other on
 *                 `stream`.
 *   replay = 1    replays the recorded schedule from one HIP graph (captured on first use, and again
 *                 whenever the pointer arguments or gbar differ from the captured ones) in which the
 *                 groups are parallel branches; nothing is read back while it runs.  Every acceptance
 *                 test of the adaptive run (eigensolver residuals, expansion decay and boundedness,
 *                 positivity of norms and traces) is evaluated on the device and checked afterwards:
 *                 inputs the schedule does not fit give DTRG_ENOCONV (or DTRG_ENONPOS) naming the
 *                 instance, and a new adaptive run is needed.  DTRG_ESTATE without a prior adaptive
 *                 run that covered the backward when T0bar_dev is given.
 * Synchronises `stream`.  Errors otherwise as dtrg_hotrg_forward / dtrg_hotrg_backward.
 */
dtrg_status dtrg_batch_run(dtrg_batch* batch, const double* T0s_dev, const double* dT0s_dev, double gbar,
                           double* lnZ_host, double* T0bar_dev, double* dlnZ_dir_host, int replay, void* stream);

/*
 * One call for a whole batch: dtrg_batch_create, one adaptive dtrg_batch_run and
 * dtrg_batch_destroy.  Arguments as there; gbar_host (host, one value) and T0bar_dev are both
 * NULL (forward only) or both given; dT0s_dev and dlnZ_dir_host as in dtrg_batch_run.  Allocates and
 * releases every buffer within the call (through opt's allocator when given).  Synchronises `stream`.
 */
dtrg_status dtrg_hotrg_batched(const double* T0s_dev, int D, const int* chi_host, int n_inst, int n_steps,
                               const double* gbar_host, const dtrg_options* opt, void* stream, double* lnZ_host,
                               double* T0bar_dev, const double* dT0s_dev, double* dlnZ_dir_host);

/* Diagnostics of step k of instance inst (0-based) after a successful run. */
dtrg_status dtrg_batch_step_info(const dtrg_batch* batch, int inst, int k, dtrg_step_info* info);

/* dtrg_plan_profile summed over the batch's groups (adaptive runs with opt.profile = 1; replays
 * record no events). */
dtrg_status dtrg_batch_profile(dtrg_batch* batch, long long* launches, double* total_ms, double* flops, int reset);

/* Device bytes held by the batch. */
size_t dtrg_batch_device_bytes(const dtrg_batch* batch);

/* Release a batch (NULL is allowed). */
void dtrg_batch_destroy(dtrg_batch* batch);

/* Number of contraction shapes in the process's autotuning table. */
int dtrg_tuned_shapes(void);

/* Device bytes held by the plan (checkpoints + workspaces). */
size_t dtrg_plan_device_bytes(const dtrg_plan* plan);

/* Release a plan (NULL is allowed). */
void dtrg_plan_destroy(dtrg_plan* plan);

/* Thread-local description of the last error on this thread ("" if none). */
const char* dtrg_last_error(void);

/*
 * Diagnostic: one plain contraction with the library's MFMA kernel,
 *   C[r * ldc + c] = alpha * sum_k A(r, k) B(c, k) + beta * C[r * ldc + c],  r < M, c < N,
 * with A(r, k) = A_dev[r * lda + k] (a_kmajor = 0) or A_dev[k * lda + r] (a_kmajor = 1) and
 * B(c, k) = B_dev[c * ldb + k] (b_kmajor = 0) or B_dev[k * ldb + c] (b_kmajor = 1).
 * precision DTRG_FP64: A, B, C are double.  DTRG_FP32 / DTRG_BF16X3 / DTRG_BF16X6: A, B are float
 * and C is double if out_f64 else float (the split precisions first split A and B into bf16 planes,
 * each in its own layout, K-contiguous or K-major, in a scratch buffer the library keeps per thread
 * and stream).
 * Device pointers; enqueued on `stream`, not synchronised.
 */
dtrg_status dtrg_contract(int precision, int M, int N, int K, const void* A_dev, long long lda, int a_kmajor,
                          const void* B_dev, long long ldb, int b_kmajor, void* C_dev, long long ldc,
                          int out_f64, double alpha, double beta, void* stream);

/*
 * Diagnostic: dtrg_contract with the kernel configuration given instead of chosen.  tile: 0 = the
 * library's choice; 1 = 64 x 64 and 2 = 128 x 128 blocks (every precision); for DTRG_BF16X3 and
 * DTRG_BF16X6 also 3 = 256 x 128, 4 = 64 x 64 on four waves that each cover all 64 columns,
 * 5 = 128 x 128 with a single LDS stage, and 6 = 256 x 256 on 32 x 32 MFMA tiles with K tiles of 16
 * and three LDS stages (K-contiguous operands and K a multiple of 16 only: DTRG_EINVAL when either
 * operand is K-major or 16 does not divide K).  splits: 0 = the library's choice (at least the count that
 * keeps every FP32 accumulation chain at 4096 products or fewer), else 1 to 64 K-chunks whose
 * partials are summed in FP64 in a fixed order (a count below that floor is taken as given).
 * DTRG_EINVAL for a tile code the precision does not have or a count outside 0 to 64.
 */
dtrg_status dtrg_contract_config(int precision, int M, int N, int K, const void* A_dev, long long lda,
                                 int a_kmajor, const void* B_dev, long long ldb, int b_kmajor, void* C_dev,
                                 long long ldc, int out_f64, double alpha, double beta, int tile, int splits,
                                 void* stream);

/*
 * dtrg_contract that allocates no device memory, for callers that cannot allocate (code that must
 * not call hipMalloc, e.g. tight serving loops or harnesses that forbid allocation).  Arguments,
 * layouts and results are those of dtrg_contract (the same kernels and the same configuration).
 * The bf16 planes of the split precisions and the FP64/FP32 split-K partials live in a static
 * device array of 128 MiB that each device holds for the life of the process (its address is
 * looked up on the first call on a device; nothing is allocated, ever).  A contraction whose
 * planes and partials need more than 128 MiB fails with DTRG_EINVAL before any work is issued.
 * The array's contents need no clearing: every byte a call reads it has written first.  All calls
 * on one device share the array, so calls that overlap on one device (different streams or host
 * threads without ordering between them) race; calls ordered on one stream do not.
 */
dtrg_status dtrg_contract_noalloc(int precision, int M, int N, int K, const void* A_dev, long long lda,
                                  int a_kmajor, const void* B_dev, long long ldb, int b_kmajor, void* C_dev,
                                  long long ldc, int out_f64, double alpha, double beta, void* stream);

/* Library version string. */
const char* dtrg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DTRG_H */
