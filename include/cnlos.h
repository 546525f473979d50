/*
 * cnlos.h — C ABI of the MI355X (gfx950) curvature-regularized confocal NLOS
 * reconstruction library.
 *
 * The library implements the ADMM solvers of Ding et al., "Curvature
 * regularization for non-line-of-sight imaging from under-sampled data"
 * (arXiv 2301.00406): the object-domain model (Section 3, Algorithm 1) and the
 * dual signal/object-domain model (Section 4.1, Algorithm 2), on top of the
 * light-cone-transform forward operator A = R_t^{-1} H R_z of Section 2,
 * eq. (3), restricted to the measured scan points (A_D = D A, Section 3.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Volumes are C-order float32 arrays [nx][ny][nt] with the time/depth axis
 *   fastest.  The hidden albedo u and the transient signal tau share this
 *   layout: index (i, j) is a scan point on the wall, k a depth bin for u and
 *   a time bin for tau.
 * - The scan mask is uint8 [nx][ny] in HOST memory, 1 = measured.
 * - "_dev" pointers are device pointers on the device that owns the
 *   workspace; the caller owns them and the library keeps none of them after a
 *   call returns (the mask and the measurement are copied into the workspace).
 * - All device work is enqueued on the HIP stream given to cnlos_create (NULL
 *   = the legacy default stream).  cnlos_apply_A / cnlos_apply_AT /
 *   cnlos_get_* / cnlos_set_* are asynchronous with respect to the host;
 *   cnlos_create, cnlos_set_measurement, cnlos_run and cnlos_get_info
 *   synchronize the stream before they return.
 * - Every function returns a cnlos_status and never aborts; no C++ exception
 *   crosses the ABI.  cnlos_last_error() gives a thread-local message for the
 *   last failing call on the calling thread.
 * - Validation of the configuration, the mask and the workspace size happens
 *   before any HIP call, so it needs no GPU.
 * - After a HIP failure (CNLOS_EHIP) the handle is poisoned: every later call
 *   except cnlos_destroy returns CNLOS_ESTATE.
 * - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef CNLOS_H
#define CNLOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CNLOS_VERSION_MAJOR 1
#define CNLOS_VERSION_MINOR 0

typedef enum {
  CNLOS_OK = 0,
  CNLOS_EINVAL = 1,        /* bad argument, configuration, mask or workspace size   */
  CNLOS_EUNSUPPORTED = 2,  /* valid in the paper's terms but outside the supported sizes */
  CNLOS_ENOMEM = 3,        /* host allocation failed                                 */
  CNLOS_EHIP = 4,          /* a HIP runtime call or kernel launch failed              */
  CNLOS_ESTATE = 5,        /* poisoned handle, or call out of order                  */
  CNLOS_EBACKTRACK = 6,    /* backtracking found no acceptable step within bt_max_trials */
  CNLOS_ENONFINITE = 7     /* a residual/energy reduction or the measurement is not finite */
} cnlos_status;

typedef enum {
  CNLOS_MODEL_OPERATOR = 0, /* operator only: apply_A / apply_AT, no ADMM state      */
  CNLOS_MODEL_OBJECT = 1,   /* Algorithm 1, object-domain curvature model eq. (4)   */
  CNLOS_MODEL_DUAL = 2      /* Algorithm 2, dual-domain model eq. (13), warm-started by Algorithm 1 */
} cnlos_model;

typedef enum {               /* curvature weight phi(kappa), Section 3              */
  CNLOS_PHI_TSC = 0,         /* a + b kappa^2   (total squared curvature; default)  */
  CNLOS_PHI_TAC = 1,         /* a + b |kappa|   (total absolute curvature)          */
  CNLOS_PHI_TRV = 2          /* sqrt(a + b kappa^2) (total roto-translation variation) */
} cnlos_phi;

typedef enum {
  /* R_t^{-1} without its radiometric weight; the measurement is instead
   * multiplied by rhat_k^3, rhat_k = (k + 1/2)/nt, masked and normalized to a
   * unit maximum by cnlos_set_measurement.  Default for reconstruction.      */
  CNLOS_FALLOFF_COMPENSATED = 0,
  /* R_t^{-1} with the weight rhat_k^{-3} of eq. (3) taken literally (the
   * measurement is only masked and normalized to a unit maximum).             */
  CNLOS_FALLOFF_LITERAL = 1
} cnlos_falloff;

/* Problem description.  Fill with cnlos_config_default() and override. */
typedef struct cnlos_config {
  int32_t nx, ny, nt;         /* scan grid and bins; nx == ny in {8..128}, nt in {16..2048}, powers of two */
  int32_t model;              /* cnlos_model                                                  */
  double wall_w_m, wall_h_m;  /* scanned wall extent in metres (x, y)                         */
  double bin_ps;              /* time-bin width in picoseconds; c = 299792458 m/s             */
  int32_t phi;                /* cnlos_phi                                                    */
  int32_t falloff;            /* cnlos_falloff                                                */
  double a_u, b_u;            /* object-domain phi weights (Algorithm 1; Algorithm 2's u term) */
  double a_tau, b_tau;        /* signal-domain phi weights (Algorithm 2)                      */
  double warm_a, warm_b;      /* Algorithm-1 warm start of Algorithm 2; < 0: use a_u, b_u     */
  double mu;                  /* Algorithm-1 penalty mu (also the warm start's)               */
  double mu1, mu2, mu3;       /* Algorithm-2 penalties (paper: 1, 800, 2)                     */
  double lambda;              /* Algorithm-2 fidelity weight                                  */
  double eta_curv;            /* curvature regularizer eta in grad u / sqrt(|grad u|^2+eta^2) */
  int32_t max_iters;          /* ADMM iterations T_max (Algorithm 2's, for the dual model)    */
  int32_t init_iters;         /* dual model: Algorithm-1 warm-start iterations                */
  double eps_stop;            /* relative energy change stop; 0 = fixed iteration count       */
  int32_t backtracking;       /* 1 = Beck-Teboulle backtracking on L                          */
  int32_t bt_max_trials;      /* rejections allowed per iteration before CNLOS_EBACKTRACK     */
  double L0;                  /* initial step constant; <= 0: 2 * power-iteration estimate of ||A_D||^2 */
  double L0_dual;             /* dual model: Algorithm-2 step constant; <= 0: 2 * estimate of ||A||^2 */
  double bt_factor;           /* L <- bt_factor * L on rejection (> 1)                         */
  int32_t power_iters;        /* power-iteration steps for the estimate (from the ones vector) */
  int32_t fista_restart;      /* 0: the extrapolation exactly as Algorithms 1-2 print it (default);
                                 1: also restart it (t = 1) after an energy rise of more than a
                                 relative 1e-3 (function-value restart, O'Donoghue-Candes)      */
} cnlos_config;

/* Fields of the ADMM state, for checkpoint/resume and inspection.
 * Three-component fields (V, LAM, W, LAM2) are [3][nx][ny][nt] (x, y, t).   */
typedef enum {
  CNLOS_FIELD_U = 0,        /* u^k                                          */
  CNLOS_FIELD_UBAR = 1,     /* extrapolated ubar^k                          */
  CNLOS_FIELD_V = 2,        /* v of the next iteration (derived, read-only) */
  CNLOS_FIELD_LAM = 3,      /* multiplier Lambda (Lambda_1)                 */
  CNLOS_FIELD_PHI = 4,      /* curvature weight phi(kappa(u))               */
  CNLOS_FIELD_AU = 5,       /* A u^k (unmasked)                             */
  CNLOS_FIELD_AU_PREV = 6,  /* A u^{k-1} (unmasked)                         */
  CNLOS_FIELD_TAU0 = 7,     /* normalized measurement (read-only)           */
  CNLOS_FIELD_TAU = 8,      /* dual model: tau^k                            */
  CNLOS_FIELD_TAUBAR = 9,   /* dual model: extrapolated taubar^k            */
  CNLOS_FIELD_W = 10,       /* dual model: next w (derived from tau, read-only) */
  CNLOS_FIELD_LAM2 = 11,    /* dual model: Lambda_2                         */
  CNLOS_FIELD_F = 12,       /* dual model: next f (derived, read-only)      */
  CNLOS_FIELD_LAM3 = 13,    /* dual model: Lambda_3                         */
  CNLOS_FIELD_PHI_TAU = 14, /* dual model: phi(kappa(tau))                  */
  CNLOS_FIELD_COUNT = 15
} cnlos_field;

typedef struct cnlos_problem cnlos_problem;  /* opaque */

typedef struct cnlos_report {
  int32_t iters_done;       /* iterations accepted in this call                 */
  int32_t total_iters;      /* iterations accepted since create/reset           */
  int32_t stopped_early;    /* 1 if the eps_stop rule fired                     */
  int32_t bt_rejects;       /* rejected backtracking trials in this call        */
  double L_final;           /* step constant after the call                     */
  double energy;            /* E(u) (object) or E(u, tau) (dual) after the call */
  double primal_res;        /* ||v - grad u||                                   */
  double dual_res;          /* mu ||grad(u^{k+1} - u^k)||                       */
  int32_t status;           /* this problem's cnlos_status for the call         */
  int32_t reserved;
} cnlos_report;

typedef struct cnlos_info {
  double L0_obj;            /* step constant used by Algorithm 1 (and the warm start) */
  double L0_dual;           /* step constant used by Algorithm 2                      */
  double L;                 /* current step constant                                  */
  double t;                 /* current FISTA t_k (1 after a restart)                  */
  double beta;              /* extrapolation weight that produced ubar^k              */
  double meas_scale;        /* normalization s of the measurement                     */
  double energy_prev;       /* last energy (NaN before the first iteration)           */
  int32_t iter;             /* accepted iterations since create/reset                 */
  int32_t stage;            /* 1 = Algorithm 1 (or warm start), 2 = Algorithm 2       */
  int32_t bt_rejects;       /* rejected trials since create/reset                     */
  int32_t has_measurement;  /* cnlos_set_measurement has been called                  */
} cnlos_info;

/* Library version string "major.minor". */
const char* cnlos_version(void);

/* Defaults: 16x16x128, 1 m wall, 32 ps, object model, TSC, compensated
 * falloff, a = b = 5e-5, mu = 0.1 (the Bowling parameters printed with the
 * full-sampling comparison of Section 5.2.1), mu1..3 = 1, 800, 2 (Section
 * 5.1), lambda = 200, eta = 1e-3, 50 iterations, 50 warm-start iterations,
 * eps = 0, backtracking on with factor 2 and 20 trials, L0 from 15 power
 * iterations, the printed FISTA step (no restart).  cfg must not be NULL. */
void cnlos_config_default(cnlos_config* cfg);

/* Check a configuration (and, if mask_host is not NULL, the mask: at least one
 * measured point).  Touches no device.  Returns CNLOS_OK, CNLOS_EINVAL or
 * CNLOS_EUNSUPPORTED. */
cnlos_status cnlos_validate(const cnlos_config* cfg, const uint8_t* mask_host);

/* Device workspace bytes that cnlos_create needs for cfg (validates cfg).
 * Touches no device. */
cnlos_status cnlos_workspace_bytes(const cnlos_config* cfg, uint64_t* bytes);

/* Create a problem in a caller-owned device workspace of at least
 * cnlos_workspace_bytes(cfg) bytes, 256-byte aligned.  Builds the resampling
 * tables and the kernel spectrum H^ (eq. (3)), and, for the solver models,
 * the step constants L0 = 2 * estimate of ||A_D||^2 (Section 3.1, the choice
 * of L after eq. (10); the dual model also estimates ||A||^2 for its
 * unmasked u-step).  Synchronizes the stream.  The workspace must outlive the
 * handle; the library never frees it. */
cnlos_status cnlos_create(const cnlos_config* cfg, const uint8_t* mask_host,
                          void* workspace_dev, uint64_t workspace_bytes,
                          void* hip_stream, cnlos_problem** out);

/* Load a raw measurement tau0_dev [nx][ny][nt] (photon counts, any finite
 * non-negative scale).  Forms the normalized data of the selected falloff
 * (see cnlos_falloff) masked by D; CNLOS_ENONFINITE if it has a non-finite
 * value, CNLOS_EINVAL if it has no positive value on a measured point.
 * Synchronizes the stream. */
cnlos_status cnlos_set_measurement(cnlos_problem* p, const float* tau0_dev);

/* tau = A u, or D A u when masked != 0 (eq. (3); A_D of Section 3.1).
 * u_dev and tau_dev are [nx][ny][nt]; they may not alias.  Asynchronous. */
cnlos_status cnlos_apply_A(cnlos_problem* p, const float* u_dev, float* tau_dev, int32_t masked);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tau = A u,
 * or D A u when masked != 0, for a configuration without a problem handle or
 * workspace.  Equal to cnlos_create (any model; the operator part is used) +
 * cnlos_apply_A.  The operator's tables, H^ and convolution spectrum live in
 * a static device array of 96 MiB (one per device, held until the process
 * ends), which admits shapes up to 64x64x512 and 32x32x1024; larger shapes
 * return CNLOS_EINVAL before any device work.  Allocates no device or pinned
 * memory (the small host tables are built in ordinary host memory and copied
 * in).  Runs on the current device; hip_stream must belong to it.  Every call
 * on a device rebuilds the scratch from scratch, so calls that overlap on one
 * device (other threads, other streams) race.  Synchronizes the stream. */
cnlos_status cnlos_apply_A_noalloc(const cnlos_config* cfg, const uint8_t* mask_host,
                                   const float* u_dev, float* tau_dev, int32_t masked,
                                   void* hip_stream);

/* u = A^T tau, or A^T D tau when masked != 0 (the adjoint used in the gradient
 * of the data term, Section 3.1).  May not alias.  Asynchronous. */
cnlos_status cnlos_apply_AT(cnlos_problem* p, const float* tau_dev, float* u_dev, int32_t masked);

/* Run ADMM iterations (Algorithm 1, or Algorithm 2 after init_iters
 * iterations of Algorithm 1): iters > 0 runs that many more (counting
 * warm-start iterations of the dual model), iters <= 0 runs to completion
 * (max_iters, plus init_iters for the dual model).  Resumable: two calls of
 * T1 and T2 iterations equal one call of T1 + T2.  A trial step that fails the
 * backtracking test is repeated with L * bt_factor.  With fista_restart = 1,
 * when an accepted iterate's energy exceeds the previous one by more than a
 * relative 1e-3 the FISTA sequence restarts (t = 1).  Algorithm 2's splitting
 * steps of the signal (w and f) start from the last accepted tau; the
 * extrapolated taubar is the data of its linearized u-step.  Stops early when
 * eps_stop > 0 and the relative energy change falls to eps_stop.  Requires a measurement.  Fills *out if it
 * is not NULL.  Synchronizes the stream. */
cnlos_status cnlos_run(cnlos_problem* p, int32_t iters, cnlos_report* out);

/* Zero the ADMM state (u = ubar = 0, multipliers 0, phi = a, t = 1, L = L0),
 * keeping H^, the step constants and the measurement.  Asynchronous. */
cnlos_status cnlos_reset(cnlos_problem* p);

/* Copy the current volume u [nx][ny][nt] to u_dev.  Asynchronous. */
cnlos_status cnlos_get_volume(cnlos_problem* p, float* u_dev);

/* Dual model: copy the current signal estimate tau [nx][ny][nt].  Asynchronous. */
cnlos_status cnlos_get_signal(cnlos_problem* p, float* tau_dev);

/* Copy a state field out / in (checkpoint and resume).  Sizes per cnlos_field
 * (V, LAM, W and LAM2 hold 3 volumes).  The splitting variables v, w and f are
 * not stored: reading them computes the values the next iteration will use
 * from ubar, Lambda, phi (tau, Lambda2, phi_tau; tau, Lambda3, tau0),
 * so they are read-only, like TAU0; restoring the other fields restores them.
 * Dual-model fields need the dual model.  Asynchronous. */
cnlos_status cnlos_get_field(cnlos_problem* p, int32_t field, float* dst_dev);
cnlos_status cnlos_set_field(cnlos_problem* p, int32_t field, const float* src_dev);

/* Scalars of the run (synchronizes the stream), and their restore for resume
 * (sets L, t, beta, energy_prev, iter, stage, bt_rejects; the step constants
 * and meas_scale are ignored).  */
cnlos_status cnlos_get_info(cnlos_problem* p, cnlos_info* out);
cnlos_status cnlos_set_info(cnlos_problem* p, const cnlos_info* in);

/* Per-iteration log, oldest first, up to cap rows of 6 doubles:
 * (energy, primal_res, dual_res, L, rejected trials, relative energy change).
 * The library keeps the last 4096 iterations.  *n receives the row count.
 * Synchronizes the stream. */
cnlos_status cnlos_get_log(cnlos_problem* p, double* host, int32_t cap, int32_t* n);

/* Kernel kinds of the per-kernel timer (bit k of a mask selects kind k).
 * In the iteration loop the first pass of each diagonal solve runs inside the
 * convolution pass before it (timed as T_INV_CONV) and the first pass of the
 * forward operator of u+ inside the u solve's last pass (timed as
 * T_INV_SOLVE); T_FWD_SOLVE and the forward operator's T_FWD_CONV then do not
 * occur as launches of their own. */
typedef enum {
  CNLOS_KK_T_FWD_CONV = 0,   /* convolution: resample + R2C along t           */
  CNLOS_KK_PLANE_CONV = 1,   /* convolution: padded (x, y) transform with H^  */
  CNLOS_KK_T_INV_CONV = 2,   /* convolution: C2R along t + R_t^{-1} + epilogue
                                (+ a solve's right-hand side and R2C)          */
  CNLOS_KK_T_FWD_SOLVE = 3,  /* diagonal solve: right-hand side + R2C along t */
  CNLOS_KK_PLANE_SOLVE = 4,  /* diagonal solve: (x, y) transform and divide    */
  CNLOS_KK_T_INV_SOLVE = 5,  /* diagonal solve: C2R along t (+ the first pass
                                of the forward operator of the result)        */
  CNLOS_KK_FIELD = 6,        /* read-back of a splitting variable (v, w, f are
                                recomputed where the iteration uses them;
                                cnlos_get_field forms them on request)         */
  CNLOS_KK_POST = 7,         /* backtracking decision, then multiplier,
                                extrapolation, curvature: u (object model); u
                                and tau in one kernel (dual model)             */
  CNLOS_KK_CONTROL = 8,      /* iteration finalize (energy, log, L, FISTA t)   */
  CNLOS_KK_OTHER = 9,        /* warm-start hand-over                           */
  CNLOS_KK_COUNT = 10
} cnlos_kernel_kind;

/* Per-kernel timing for tracing and roofline measurement (not part of the
 * paper's method).  Every later launch of a selected kind is bracketed by two
 * HIP events recorded on the problem's stream; 0 disables.  Costs two event
 * records per timed launch. */
cnlos_status cnlos_profile_enable(cnlos_problem* p, uint32_t kind_mask);

/* Accumulated milliseconds and launch counts per kind (arrays of
 * CNLOS_KK_COUNT, either may be NULL); reset != 0 zeroes the accumulators.
 * Synchronizes the stream. */
cnlos_status cnlos_profile_read(cnlos_problem* p, double* ms, int64_t* launches, int32_t reset);

/* Release the handle (the workspace stays the caller's).  NULL is accepted. */
cnlos_status cnlos_destroy(cnlos_problem* p);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* cnlos_last_error(void);

/* ------------------------------------------------------------------------
 * Launch plans (autotuning).  A plan holds layout choices of the plane
 * kernels of the zero-padded 3-D FFT: the LDS row pads of their transposes.
 * The pads decide only where values sit in LDS (bank conflicts), never a
 * result: every plan gives bitwise the same results.  A problem starts with
 * the plan that cnlos_tune last measured for its shape on the current device
 * (in this process), or with the defaults (convolution pad 2; solve pad 2 at
 * nx = 64, 4 at nx = 128, 8 otherwise).  A batch runs with its first member's
 * plan; a serving slot group with the plan of its shape when it is created.
 * ------------------------------------------------------------------------ */
typedef struct cnlos_plan {
  int32_t conv_row_pad;       /* plane kernel of the convolution: 1, 2 or 4                  */
  int32_t solve_row_pad;      /* plane kernel of the diagonal solve: 2, 4 or 8               */
  int32_t tuned;              /* 1 when these figures were measured by the call              */
  int32_t reserved;
  double conv_plane_us[3];    /* measured plane pass of one convolution, pads 1, 2, 4 (us)  */
  double solve_plane_us[3];   /* measured plane pass of one solve, pads 2, 4, 8 (us)        */
} cnlos_plan;

/* Measure every candidate pad on this problem's workspace (eight convolutions
 * and solves each, timed with HIP events on its stream), keep the fastest for
 * the problem and for later problems of its shape (a candidate replaces the
 * default only when it is more than 3% faster), and fill *out (may be
 * NULL).  Overwrites the A u buffers, so a solver problem's iteration state
 * is reset (the measurement is kept).  Not for batch members or
 * operator-only problems (ESTATE).  Synchronizes the stream. */
cnlos_status cnlos_tune(cnlos_problem* p, cnlos_plan* out);

/* The problem's current plan (tuned = 0, no timings). */
cnlos_status cnlos_get_plan(cnlos_problem* p, cnlos_plan* out);

/* Use the given pads for this problem (EINVAL for other values; ESTATE for
 * batch members). */
cnlos_status cnlos_set_plan(cnlos_problem* p, const cnlos_plan* plan);

/* ------------------------------------------------------------------------
 * Batches: several problems that advance together, one kernel launch per
 * step of the iteration for all of them (launch grid z = problem).  The
 * scenes are independent reconstructions (Sections 3 and 4.1 per scene); the
 * batch changes where they run, not what they compute: each member's result
 * is bitwise the result of running it alone (fixed-order reductions).
 *
 * Members must agree on nx, ny, nt, model, phi, falloff, the weights a_u,
 * b_u, a_tau, b_tau, warm_a, warm_b, the penalties mu, mu1, mu2, mu3, lambda,
 * eta_curv and backtracking; they may differ in the wall extent, bin width,
 * mask, measurement, max_iters, init_iters, eps_stop, bt_factor,
 * bt_max_trials, L0, L0_dual, power_iters and fista_restart.
 * ------------------------------------------------------------------------ */
typedef struct cnlos_batch cnlos_batch;   /* opaque */

/* Device bytes for a batch of `count` problems shaped like cfg: count equal
 * slices of cnlos_workspace_bytes(cfg) each. */
cnlos_status cnlos_batch_workspace_bytes(const cnlos_config* cfg, int32_t count, uint64_t* bytes);

/* Create `count` member problems from cfgs[count] and masks_host[count]
 * (host [nx][ny] arrays) in one caller-owned workspace (256-byte aligned),
 * each built as cnlos_create builds one (H^ and step constants per member).
 * All work goes to hip_stream.  EINVAL if the members disagree on a field
 * that must match.  On error after the handle exists, *out is set and must
 * be destroyed. */
cnlos_status cnlos_batch_create(const cnlos_config* cfgs, int32_t count,
                                const uint8_t* const* masks_host, void* workspace_dev,
                                uint64_t workspace_bytes, void* hip_stream, cnlos_batch** out);

/* Member i as a problem handle (owned by the batch: do not destroy it).  It
 * accepts every problem call: set_measurement, apply_A/AT, get/set field,
 * info, log, reset, and cnlos_run, which runs that member alone. */
cnlos_status cnlos_batch_member(cnlos_batch* b, int32_t i, cnlos_problem** out);

/* Run every member (iters > 0: that many more iterations each; else each
 * member's configured count).  Members that stop early or fail drop out while
 * the others continue; reports[count] (nullable) receive each member's
 * report with its own status.  Returns the first member error, else OK.
 * Every member needs a measurement.  Synchronizes the stream. */
cnlos_status cnlos_batch_run(cnlos_batch* b, int32_t iters, cnlos_report* reports);

/* Run several batches at once, each on its own stream (the stream given at
 * its creation): every round enqueues work for all of them before waiting,
 * so batches of different shapes overlap on the device.  reports holds one
 * array per batch (the array, or an entry, may be NULL). */
cnlos_status cnlos_batch_run_many(cnlos_batch* const* batches, int32_t count, int32_t iters,
                                  cnlos_report* const* reports);

/* Release the batch and its members (the workspace stays the caller's). */
cnlos_status cnlos_batch_destroy(cnlos_batch* b);

/* ------------------------------------------------------------------------
 * Serving with continuous batching.  Requests of any supported shape are
 * queued; each step admits queued requests into free slots of a slot group of
 * their shape (a batch that keeps running while its members change), creating
 * a group when the HBM arena has room, advances every group on its own
 * stream (groups overlap on the device), and retires finished requests,
 * whose slots take new requests at the next step.  A request's result is
 * bitwise the result of running it alone (cnlos_create + cnlos_run).
 * All device memory comes from one caller-owned arena; the server never
 * allocates device memory.  Not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct cnlos_server cnlos_server;   /* opaque */

typedef struct cnlos_request {
  cnlos_config cfg;           /* shape, model, weights and iteration budget         */
  const uint8_t* mask_host;   /* [nx][ny]; copied at submit                         */
  const float* tau0_dev;      /* raw measurement [nx][ny][nt]; read at admission,   */
                              /* so it must stay valid until the request completes  */
  float* out_dev;             /* receives u [nx][ny][nt] when the request completes */
  int64_t id;                 /* caller's tag, returned in the completion           */
} cnlos_request;

typedef struct cnlos_completion {
  int64_t id;
  int32_t status;             /* cnlos_status of the request                        */
  int32_t iters;              /* iterations accepted                                */
  double energy;              /* final energy                                       */
  double queued_steps;        /* steps between submit and admission                 */
  double served_steps;        /* steps between admission and completion             */
} cnlos_completion;

/* arena: device memory for every slot group (256-byte aligned); slots: slots
 * per group (1..64); rounds: iteration slots enqueued per group per step. */
cnlos_status cnlos_server_create(void* arena_dev, uint64_t arena_bytes, int32_t slots,
                                 int32_t rounds, cnlos_server** out);

/* Queue a request (validated now; EINVAL/EUNSUPPORTED on a bad config or mask,
 * ENOMEM if one slot group of its shape can never fit the arena). */
cnlos_status cnlos_server_submit(cnlos_server* s, const cnlos_request* r);

/* One scheduling step: retire, admit, advance.  active / queued (nullable)
 * receive the number of requests in slots and waiting after the step.
 * Synchronizes every group stream. */
cnlos_status cnlos_server_step(cnlos_server* s, int32_t* active, int32_t* queued);

/* Testing hook for failure handling: the next `count` slot-group creations
 * fail with CNLOS_EHIP after the group's arena range, stream and host objects
 * exist (they are released again), before any device work.  The request that
 * needed the group completes with that status; the others are unaffected. */
cnlos_status cnlos_server_fail_next_groups(cnlos_server* s, int32_t count);

/* Completions since the last poll (up to cap; *n receives the count). */
cnlos_status cnlos_server_poll(cnlos_server* s, cnlos_completion* out, int32_t cap, int32_t* n);

/* Arena bytes in use by slot groups, and the number of groups. */
cnlos_status cnlos_server_usage(cnlos_server* s, uint64_t* bytes_used, int32_t* groups);

/* Release everything (in-flight requests are dropped; the arena stays the
 * caller's). */
cnlos_status cnlos_server_destroy(cnlos_server* s);

/* ------------------------------------------------------------------------
 * Non-confocal model (Section 2, general form; Section 5's non-confocal
 * experiment).  One wall point is illuminated and an n x n detector grid is
 * scanned.  With the wall normals along z the model's direction terms reduce to
 * the volumetric albedo weight 1 / (d_i^2 d_d^2): d_i runs from the illuminated
 * point to the voxel and d_d from the voxel to the detector, and the path
 * d_i + d_d selects the time bin.  The model is not shift-invariant, so it has
 * no light-cone (FFT) form.  These entry points apply it by direct summation
 * over all n^4 m (detector, voxel) paths.  That suits small grids; the
 * reconstruction route of Section 5 is the midpoint approximation below,
 * followed by the confocal solver.
 *
 * Grid conventions (those of the confocal operator):
 * - detector and voxel column (i, j) sit at x_i = (i + 1/2) W / n - W / 2;
 * - depth bin k sits at z_k = (k + 1/2) R / m, with R = m c dt / 2;
 * - time bin b holds path lengths in [b, b + 1) c dt;
 * - paths beyond bin m - 1 are dropped.
 *
 * Volumes u and transients tau are float32 [n][n][m] (time/depth fastest),
 * device pointers owned by the caller.  Time bins are decided in FP64.  Sums
 * are FP64 in a fixed order, so results are bitwise reproducible.  The calls
 * allocate nothing and keep no pointer.  Work is enqueued on hip_stream of the
 * current device (asynchronous).  Geometry errors return before any device
 * call.
 * ------------------------------------------------------------------------ */
typedef struct cnlos_nc_geometry {
  int32_t n;              /* detectors (and voxel columns) per side, 1..256               */
  int32_t m;              /* time bins = depth bins, 1..1024                              */
  double wall_m;          /* wall extent W (square, centred at 0), metres                 */
  double bin_ps;          /* time-bin width, picoseconds                                  */
  double illum_x_m;       /* illuminated wall point, metres                               */
  double illum_y_m;
  int32_t literal;        /* 1: weight 1/(d_i^2 d_d^2); 0: weight 1 (paths only)          */
} cnlos_nc_geometry;

/* Check a geometry (no device work).  EINVAL for bad values, EUNSUPPORTED
 * beyond the size limits. */
cnlos_status cnlos_nc_validate(const cnlos_nc_geometry* g);

/* tau = A_nc u: tau[i][j][b] sums w u over the voxels whose path from the
 * illumination point through the voxel to detector (i, j) falls in bin b.
 * u and tau may not alias.  Asynchronous. */
cnlos_status cnlos_nc_apply(const cnlos_nc_geometry* g, const float* u_dev, float* tau_dev,
                            void* hip_stream);

/* u = A_nc^T tau: u[p][q][k] sums w tau[i][j][bin] over the detectors.  May not
 * alias.  Asynchronous. */
cnlos_status cnlos_nc_apply_T(const cnlos_nc_geometry* g, const float* tau_dev, float* u_dev,
                              void* hip_stream);

/* Midpoint approximation (Section 5's non-confocal experiment).  A detector
 * at x_d under illumination x_i reads as a confocal measurement at the
 * midpoint (x_i + x_d) / 2.  The midpoints of the detector grid form an n x n
 * grid of extent W / 2 centred at half the illumination point.  The transient
 * array is then reconstructed unchanged by the confocal solver, with
 * wall_w_m = wall_h_m = *wall_m.  The confocal operator is shift-invariant, so
 * the centre only places the result.  Host only. */
cnlos_status cnlos_nc_midpoint(const cnlos_nc_geometry* g, double* wall_m, double* centre_x_m,
                               double* centre_y_m);

#ifdef __cplusplus
}
#endif

#endif /* CNLOS_H */
