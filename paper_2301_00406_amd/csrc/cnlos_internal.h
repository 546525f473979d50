// Internal interfaces between the host driver and the kernel translation units.
#pragma once
#include <cstddef>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

namespace cnlos {

// Kernel kinds for event timing (mirrors cnlos_kernel_kind of the ABI).
enum KernelKind : int {
  KK_T_FWD_CONV = 0,
  KK_PLANE_CONV = 1,
  KK_T_INV_CONV = 2,
  KK_T_FWD_SOLVE = 3,
  KK_PLANE_SOLVE = 4,
  KK_T_INV_SOLVE = 5,
  KK_FIELD = 6,
  KK_POST = 7,
  KK_CONTROL = 8,
  KK_OTHER = 9,
  KK_COUNT = 10
};

// HIP-event timer around launches of selected kernel kinds, on the launch
// stream.  Pairs are harvested after the stream has been synchronized.
struct Prof {
  uint32_t mask = 0;
  double ms[KK_COUNT] = {};
  long long launches[KK_COUNT] = {};
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  bool on(int kind) const { return (mask >> kind) & 1u; }
  hipError_t begin(int kind, hipStream_t st);
  hipError_t end(int kind, hipStream_t st);
  void harvest();     // stream must be idle
  void release();
};

// Reduction slots of the FP64 partials buffer.
enum Slot : int {
  SL_CHECK = 0,     // ||D A (u+ - ubar)||^2 (object) or ||A (u+ - ubar)||^2 (dual)
  SL_DATA = 1,      // ||D A u+ - tau0||^2 (object energy data term)
  SL_STEP = 2,      // ||u+ - ubar||^2
  SL_TV_U = 3,      // sum phi_u |grad u+|
  SL_PRIMAL = 4,    // ||v - grad u+||^2
  SL_DUAL = 5,      // ||grad (u+ - u)||^2
  SL_FIT = 6,       // ||A u+ - tau+||^2 (dual energy)
  SL_FID = 7,       // ||D (tau+ - tau0)||^2 (dual energy)
  SL_TV_TAU = 8,    // sum phi_tau |grad tau+|
  SL_NORM = 9,      // ||x||^2 (power iteration)
  SL_MAX = 10,      // measurement maximum (stored as double)
  SL_BAD = 11,      // count of non-finite measurement values
  SL_COUNT = 12
};

constexpr int kMaxBlocks = 4096;     // partial-sum capacity per slot
// relative energy rise that restarts the FISTA sequence (t = 1) when the
// optional function-value restart is on
constexpr double kRestartTol = 1e-3;
constexpr int kLogRows = 4096;       // per-iteration log ring
constexpr int kLogCols = 6;

enum HaltReason : int { HR_NONE = 0, HR_REJECT = 1, HR_STOP = 2, HR_BACKTRACK = 3, HR_NONFINITE = 4 };

// Volumes whose role rotates with the accepted-iteration count.  Each role
// draws from a small set of buffers (u, ubar, tau, taubar: 2; A u: 3); the controller
// keeps which buffer currently plays each role (rotated by the finalize
// kernel), so a kernel resolves it on the device and scenes at different
// iteration counts can share one launch.
enum Role : int {
  R_U_CUR = 0,    // u^k
  R_U_TR = 1,     // u^{k+1} trial
  R_AU_CUR = 2,   // A u^k
  R_AU_PREV = 3,  // A u^{k-1}
  R_AU_TR = 4,    // A u^{k+1} trial
  R_T_CUR = 5,    // tau^k
  R_T_TR = 6,     // tau^{k+1} trial
  R_UB_CUR = 7,   // ubar^k (read by the iteration)
  R_UB_NEW = 8,   // ubar^{k+1} (written by the post step)
  R_TB_CUR = 9,   // taubar^k
  R_TB_NEW = 10,  // taubar^{k+1}
  R_COUNT = 11
};

// Phase gate of an iteration kernel (bits): which stage it belongs to, and
// whether it is the first kernel of an iteration slot (it clears the previous
// slot's rejection).
enum Gate : int { G_NONE = 0, G_STAGE1 = 1, G_STAGE2 = 2, G_FIRST = 8 };

// Scalars shared by the host driver and the kernels, resident in the workspace.
// Every kernel of the ADMM iteration returns at once while `halt` is set, so a
// batch of enqueued iterations stops cleanly at an error or a stop.  The post
// kernel takes the backtracking decision; a rejected trial sets `reject`, the
// post kernel stops, k_finalize doubles L instead of advancing, and the next
// slot retries the iteration.
struct DevCtl {
  // the fields every kernel's phase gate reads, in one 32-byte block at the
  // start (one scalar load at kernel start)
  int32_t halt;
  int32_t iter;        // accepted iterations
  int32_t stage;       // 1 = Algorithm 1, 2 = Algorithm 2
  int32_t target;      // iteration kernels return once iter >= target
  int32_t reject;      // the current slot's trial was rejected
  int32_t stage1_end;  // dual model: iterations of the warm start; object: a large value
  int32_t reason;
  int32_t trials;      // rejections in the current iteration
  int32_t slot[R_COUNT];   // buffer index per role
  int32_t slot_pad;
  double L;            // current step constant
  double t;            // FISTA t_k
  double beta;         // extrapolation weight that produced ubar^k
  double energy_prev;  // last energy (NaN before the first iteration)
  double L0_obj, L0_dual;
  double meas_scale;
  double pow_est;
  double last_energy, last_primal, last_dual;
  double restart_tol;  // > 0: function-value FISTA restart at this relative rise; 0: off
  int32_t bt_rejects;  // rejections since create/reset
  int32_t log_count;   // rows written to the log ring
  int32_t bt_max_trials;
  double bt_factor;
  double eps_stop;
  double mu_dual;      // mu (object) or mu1 (dual) for the dual residual
  double lambda;
};
static_assert(offsetof(DevCtl, slot) == 32, "the gate fields fill the first 32 bytes");

// The controller's head (gate fields and buffer slots), read once at kernel
// start: one memory round trip for the phase gate and every role operand.
struct CtlHead {
  int32_t halt, iter, stage, target, reject, stage1_end, reason, trials;
  int32_t slot[R_COUNT];
  bool valid;                // false: no controller (plain operator launches)
};
__device__ __forceinline__ CtlHead ctl_head(const DevCtl* c) {
  CtlHead h{};
  h.valid = c != nullptr;
  if (c) {
    h.halt = c->halt;
    h.iter = c->iter;
    h.stage = c->stage;
    h.target = c->target;
    h.reject = c->reject;
    h.stage1_end = c->stage1_end;
    h.reason = c->reason;
    h.trials = c->trials;
#pragma unroll
    for (int r = 0; r < R_COUNT; ++r) h.slot[r] = c->slot[r];
  }
  return h;
}
__device__ __forceinline__ bool gated_off(const CtlHead& h, int gate) {
  const bool s1 = (gate & G_STAGE1) != 0, s2 = (gate & G_STAGE2) != 0;
  return h.valid & ((h.halt != 0) | ((gate != G_NONE) & (h.iter >= h.target)) |
                    (s1 & ((h.stage != 1) | (h.iter >= h.stage1_end))) | (s2 & (h.stage != 2)));
}

// true when a kernel with phase gate `gate` has nothing to do for this scene
// (every field is loaded before the first decision, so the test costs one
// memory round trip at kernel start instead of a chain of dependent ones)
__device__ __forceinline__ bool gated_off(const DevCtl* c, int gate) {
  if (c == nullptr) return false;
  const int halt = c->halt, iter = c->iter, target = c->target, stage = c->stage;
  const int s1end = c->stage1_end;
  const bool s1 = (gate & G_STAGE1) != 0, s2 = (gate & G_STAGE2) != 0;
  return (halt != 0) | ((gate != G_NONE) & (iter >= target)) |
         (s1 & ((stage != 1) | (iter >= s1end))) | (s2 & (stage != 2));
}

// A volume operand: the fixed pointer p[0] (role < 0), or the buffer p[slot]
// that the controller currently assigns to the role.
struct Vol {
  float* p[3] = {nullptr, nullptr, nullptr};
  int role = -1;
};

// Scenes of a batch live in equal workspaces at a fixed byte stride; a kernel
// launched over a batch (grid z = scene) shifts every workspace pointer by
// blockIdx.z * stride.  Role pointers read from a shifted controller are the
// scene's own already.
template <typename T>
__device__ __forceinline__ T* zsh(T* p, size_t off) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + off) : p;
}

// the buffer behind v for the scene whose controller is c (zo: its offset)
__device__ __forceinline__ float* vol_resolve(const Vol& v, const DevCtl* c, size_t zo) {
  if (v.role < 0) return zsh(v.p[0], zo);
  const int k = c->slot[v.role];
  float* q = k == 0 ? v.p[0] : (k == 1 ? v.p[1] : v.p[2]);
  return zsh(q, zo);
}
__device__ __forceinline__ float* vol_resolve(const Vol& v, const CtlHead& h, size_t zo) {
  // select chain over the roles (a runtime index would put the head in scratch)
  int k = 0;
#pragma unroll
  for (int r = 0; r < R_COUNT; ++r) k = v.role == r ? h.slot[r] : k;
  float* q = k == 0 ? v.p[0] : (k == 1 ? v.p[1] : v.p[2]);
  return zsh(q, zo);
}

// Sparse resampling table S (depth bin k -> squared-distance bin q) in both
// orientations; ranges are contiguous so each row/column is (start, count, off).
struct ResampleTables {
  const int4* rows;    // [m]: (k_start, count, value_offset, 0)
  const float* rvals;
  const int4* cols;    // [m]: (q_start, count, value_offset, 0)
  const float* cvals;
};

// Source of the t-axis forward pass of a convolution:
//   x[k] = mask[col] * w[k] * inv_scale * (ca * a[k] + cb * b[k] - c[k]),
// with (ca, cb) = (1, 0) or, in the linearity-cache mode, (1 + beta, -beta)
// with beta read from the controller.  Null pointers drop their factor.
struct ConvSrc {
  Vol a;
  Vol b;
  Vol c;
  const float* w;
  const uint8_t* mask;
  const double* scale_div;   // divide by *scale_div (power iteration)
  int lincache;
};

enum Epi : int { EPI_PLAIN = 0, EPI_FWD_OBJ = 1, EPI_FWD_DUAL = 2, EPI_NORM = 3 };

// Epilogue of the t-axis inverse pass of a convolution.
struct ConvEpi {
  Vol out;                 // [n][n][m]
  const float* w;          // per-bin output weight (nullable)
  const uint8_t* mask;     // output mask (EPI_PLAIN) / fidelity mask (EPI_FWD_OBJ)
  Vol au;                  // A u^k       (check)
  Vol au_prev;             // A u^{k-1}   (check)
  const float* tau0;       // data (EPI_FWD_OBJ)
  double* partials;
};

// Right-hand side of a diagonal solve computed where the solve's t pass reads
// it, instead of being stored:
//   RHS_U   : L ubar - grad f + nabla^*(mu v + Lambda)          (eqs. (10), (11))
//   RHS_TAU : A u+ + mu3 f + Lambda3 + nabla^*(mu2 w + Lambda2) (tau-subproblem)
// with v (w) and f recomputed from xbar, Lambda, phi (and Lambda3, tau0).
enum RhsMode : int { RHS_LOAD = 0, RHS_U = 1, RHS_TAU = 2 };
struct RhsSrc {
  int mode = RHS_LOAD;
  Vol xb;                    // ubar / taubar
  Vol au;                    // A u+ (RHS_TAU)
  const float* gf = nullptr;     // grad f (RHS_U)
  const float* lam = nullptr;    // Lambda / Lambda2
  const float* phi = nullptr;    // phi / phi_tau
  const float* lam3 = nullptr;   // RHS_TAU
  const float* tau0 = nullptr;
  const uint8_t* mask = nullptr;
  float mu = 1.f, lambda = 0.f, mu3 = 0.f;
  int logn = 0;
};

// Epilogue of the t-axis inverse pass of a diagonal solve.
struct SolveEpi {
  Vol out;
  Vol ref;                 // ||out - ref||^2 into SL_STEP when not null
  double* partials;
};

// Launch plan: layout choices of the plane kernels, the LDS row pads of their
// transposes (bank conflicts only: no choice changes a result), picked per
// shape from measured timings (cnlos_tune) or the defaults below.
constexpr int kConvPads[3] = {1, 2, 4};
constexpr int kSolvePads[3] = {2, 4, 8};
inline int default_solve_pad(int logn) { return logn == 6 ? 2 : (logn == 7 ? 4 : 8); }
struct Plan {
  int conv_pad = 2;
  int solve_pad = 0;      // 0: default_solve_pad(logn)
};

struct Tables {
  const float2* tw_t;     // exp(-2 pi i j / (2m)), j < m
  const float2* tw_xy;    // exp(-2 pi i j / (2n)), j < n
  const float2* twc_t;    // per-span butterfly twiddles: [d + k] = exp(-pi i k / d), size m
  const float2* twc_xy;   // the same for the (x, y) transforms, size 2n
  ResampleTables S;
  const float* sig_xy;    // 4 sin^2(pi k / n), k < n
  const float* sig_t;     // 4 sin^2(pi k / m), k <= m/2
  const float2* hq;       // H^: [m+1] planes of 4 n^2 entries, lane-ordered for the
                          // plane kernel that reads them (hq_lane_index)
  Plan plan;
};

// ---------------------------------------------------------------- launchers
// All launchers return hipGetLastError() of their launch.
// Launch geometry of a batch: nz scenes at a workspace stride of zs bytes
// (nz = 1, zs = 0 for a single problem), and the phase gate of the launch.
// Lane-rows of a t-pass column (G lanes, m / G rows) whose prefix sums the
// R_z rows of more than 3 taps use: those rows end below m/4 + 8 (the table
// builder checks it).
constexpr int resample_scan_rows(int M, int G) {
  const int r = (M / 4 + 8 + G - 1) / G;
  return r < M / G ? r : M / G;
}

// XCD-aware block order.  Workgroups are dealt round-robin over the 8 XCDs,
// each with its own L2; logical block xcd_block(b, nb) places nb / 8
// consecutive logical blocks on one XCD, so blocks that read each other's
// neighbour columns share an L2 (identity when nb is not a multiple of 8).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

struct Batch {
  int nz;
  size_t zs;
  int gate;
  bool hq_shared = false;   // every scene reads the lead's H^ (one geometry)
};
constexpr Batch kSingle{1, 0, G_NONE};

// tfwd_done: the forward t pass already ran (fused into the preceding solve);
// rhs_next: the inverse t pass (plain epilogue) also runs the forward t pass
// of the u solve with this right-hand side (RHS_U, grad f kept on chip; its
// output is not stored), and launch_solve follows with tfwd_done
hipError_t launch_conv(int logn, int logm, const Tables& tb, const ConvSrc& src, float2* spec,
                       bool adjoint, int epi, const ConvEpi& ep, const DevCtl* ctl,
                       const Batch& bt, hipStream_t st, Prof* prof, bool tfwd_done = false,
                       const RhsSrc* rhs_next = nullptr);
// fwd_next: the last pass also runs the forward t pass of the convolution of
// the result (no weight, mask or offset); its step partials then come from
// fused_solve_blocks blocks, and launch_conv follows with tfwd_done
hipError_t launch_solve(int logn, int logm, const Tables& tb, const float* rhs, const RhsSrc& rs,
                        float2* spec, const double* c_dev, double c_val, double mu,
                        const SolveEpi& ep, const DevCtl* ctl, const Batch& bt, hipStream_t st,
                        Prof* prof, bool fwd_next = false, bool tfwd_done = false);
hipError_t launch_build_hq(int logn, int logm, float2* hq, const int* dq, const double2* etab,
                           const double* cosn, double invZ, hipStream_t st);
int conv_blocks(int logn, int logm);          // blocks of the convolution t passes
int solve_blocks(int logn, int logm);         // blocks of the diagonal-solve t passes
int fused_solve_blocks(int logn, int logm);   // blocks of the solve pass fused with a conv t pass

// ADMM stencils and control (k_admm.hip)
struct PhiArgs {
  double a, b;
  int kind;
  float eta;
};
// derived fields: v (or w) and f from the current state, single problem
hipError_t launch_vstep(int logn, int logm, const float* xbar, const float* lam, const float* phi,
                        float* v, double mu, hipStream_t st);
hipError_t launch_fstep(int logn, int logm, const float* taubar, const float* lam3,
                        const float* tau0, const uint8_t* mask, float* f, double lambda,
                        double mu3, hipStream_t st);
// one side (u or tau) of the post-step update
struct PostArgs {
  Vol xn;            // x+ (accepted)
  Vol xo;            // x^k
  Vol xb;            // xbar^k (the iteration's v / w are recomputed from it)
  Vol xbn;           // xbar^{k+1}, written
  float* lam;        // Lambda or Lambda2, updated in place
  float* phi;        // curvature weight, updated in place
  float mu;
  PhiArgs pa;
};

// Inputs of the backtracking decision that the post kernels take: the block
// counts of the check (forward pass) and step (u solve) partial sums, and
// whether backtracking is on.
struct CheckArgs {
  int nb_conv;
  int nb_step;
  int bt_on;
};
hipError_t launch_post_dual(int logn, int logm, const PostArgs& pu, const PostArgs& pt,
                            float* lam3, double mu3, double lambda, Vol au, const float* tau0,
                            const uint8_t* mask, double* partials, const CheckArgs& ck,
                            const DevCtl* ctl, const Batch& bt, hipStream_t st);
hipError_t launch_post(int logn, int logm, const PostArgs& pa, double* partials,
                       const CheckArgs& ck, const DevCtl* ctl, const Batch& bt, hipStream_t st);
int stencil_blocks(int logn, int logm);
hipError_t launch_finalize(DevCtl* ctl, double* log, const double* partials, int nb_conv,
                           int nb_sten, int dual, double lambda, double mu_res, const Batch& bt,
                           hipStream_t st);
hipError_t launch_transition(int logn, int logm, DevCtl* ctl, Vol u, Vol ubar,
                             float* phi_u, const PhiArgs& pa_u, float* phi_tau, double phi_tau0,
                             float* const* zero_fields, const size_t* zero_counts, int nzero,
                             const Batch& bt, hipStream_t st);
hipError_t launch_fill(float* x, size_t n, float val, hipStream_t st);
hipError_t launch_copy(float* dst, const float* src, size_t n, hipStream_t st);
hipError_t launch_phi_of_u(int logn, int logm, const float* u, float* phi, const PhiArgs& pa,
                           hipStream_t st);
hipError_t launch_meas_prep(int logn, int logm, const float* raw, const uint8_t* mask,
                            const float* r3, float* out, double* partials, hipStream_t st);
hipError_t launch_meas_finish(int logn, int logm, float* out, DevCtl* ctl, double* partials,
                              hipStream_t st);
hipError_t launch_pow_finalize(DevCtl* ctl, const double* partials, int nb, const Batch& bt,
                               hipStream_t st);
hipError_t launch_ctl_clear_halt(DevCtl* ctl, hipStream_t st);

// Non-confocal direct-sum operator (k_nonconfocal.hip): n x n detectors and
// voxel columns, m time/depth bins, wall extent W, depth range R = m c dt / 2,
// path length per bin c dt, illumination point (ix, iy) on the wall.
struct NcGeo {
  int n, m;
  double wall, range, cdt, ix, iy;
  int literal;
};
size_t nc_forward_lds_bytes(int m);
hipError_t launch_nc_forward(const NcGeo& g, const float* u, float* tau, hipStream_t st);
hipError_t launch_nc_transpose(const NcGeo& g, const float* tau, float* u, hipStream_t st);

}  // namespace cnlos
