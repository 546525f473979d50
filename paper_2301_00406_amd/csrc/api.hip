// Host side of the C ABI: validation, workspace carving, table construction,
// problem set-up (H^, step constants) and the ADMM driver of Algorithms 1 and 2.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "cnlos.h"
#include "cnlos_internal.h"

using namespace cnlos;

namespace {

constexpr double kC = 299792458.0;
constexpr int kNcMaxGrid = 256;     // non-confocal operator: detectors per side
constexpr int kNcMaxBins = 1024;    // and time bins (the forward kernel's LDS histograms)
thread_local std::string g_err;

// Launch plans measured by cnlos_tune, per device and shape; problems
// created later on that device with that shape start with the plan.
std::mutex g_plan_mu;
std::map<std::tuple<int, int, int>, Plan> g_plans;

Plan plan_for(int logn, int logm) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::lock_guard<std::mutex> lock(g_plan_mu);
  auto it = g_plans.find(std::make_tuple(dev, logn, logm));
  return it == g_plans.end() ? Plan{} : it->second;
}

cnlos_status fail(cnlos_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}
bool finite_pos(double x) { return isfinite(x) && x > 0.0; }
bool finite_nonneg(double x) { return isfinite(x) && x >= 0.0; }

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Workspace carving.  With base == nullptr only the size is computed.
struct Carver {
  uint8_t* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// defer_steps: return once the tables and H^ are built; the caller estimates
// the step constants (possibly for several problems at once) and calls
// finish_create
cnlos_status create_into(const cnlos_config* cfg, const uint8_t* mask_host, void* workspace_dev,
                         uint64_t workspace_bytes, void* hip_stream, cnlos_problem** out,
                         float2* shared_hq = nullptr, bool own_hq = true, bool defer_steps = false);
cnlos_status finish_create(cnlos_problem* p, double est_masked, double est_unmasked);
cnlos_status destroy_problem(cnlos_problem* p);

}  // namespace

namespace {
// progress of one scene within a run
struct SceneRun {
  int start = 0, goal = 0, rejects0 = 0;
  bool active = false, stopped = false;
  cnlos_status status = CNLOS_OK;
};
}  // namespace

struct cnlos_batch {
  std::vector<cnlos_problem*> mem;
  size_t stride = 0;
  hipStream_t st = nullptr;
  bool hq_shared = false;     // one geometry: every member reads member 0's H^
};

// ------------------------------------------------------------ serving state
namespace {

// First-fit allocator over the caller's device arena (offsets only).
struct Arena {
  uint8_t* base = nullptr;
  uint64_t bytes = 0, used = 0;
  std::vector<std::pair<uint64_t, uint64_t>> holes;   // (offset, size), sorted by offset
  bool take(uint64_t n, uint64_t* off) {
    for (size_t i = 0; i < holes.size(); ++i) {
      if (holes[i].second < n) continue;
      *off = holes[i].first;
      holes[i].first += n;
      holes[i].second -= n;
      if (holes[i].second == 0) holes.erase(holes.begin() + i);
      used += n;
      return true;
    }
    return false;
  }
  void give(uint64_t off, uint64_t n) {
    used -= n;
    size_t i = 0;
    while (i < holes.size() && holes[i].first < off) ++i;
    holes.insert(holes.begin() + i, {off, n});
    if (i + 1 < holes.size() && holes[i].first + holes[i].second == holes[i + 1].first) {
      holes[i].second += holes[i + 1].second;
      holes.erase(holes.begin() + i + 1);
    }
    if (i > 0 && holes[i - 1].first + holes[i - 1].second == holes[i].first) {
      holes[i - 1].second += holes[i].second;
      holes.erase(holes.begin() + i);
    }
  }
};

struct SrvReq {
  cnlos_request r;
  std::vector<uint8_t> mask;
  long long submitted = 0;
};

// A group of scenes advanced by the same launches (one scene, or a batch at
// a workspace stride), on the stream of its first scene.
struct Group {
  cnlos_problem* lead = nullptr;
  std::vector<cnlos_problem*> mem;
  Batch bt = kSingle;
};

// A slot group: a batch whose members change while it runs.
struct SrvGroup {
  cnlos_config proto;
  size_t stride = 0;
  int K = 0;
  uint64_t off = 0;            // arena range: [off, off + bytes)
  uint64_t bytes = 0;
  float2* hq = nullptr;        // the group's H^, at the start of its range
  // ||A||^2 estimate of the group's geometry (unmasked: the dual model's step
  // constant), measured at the first admission that needs it, for power_iters
  double est_unmasked = 0.0;
  int est_unmasked_iters = 0;
  uint64_t slots_off = 0;      // slot i's workspace at slots_off + i * stride
  hipStream_t st = nullptr;
  cnlos_problem* layout = nullptr;       // buffer layout of slot 0 (no device state of its own)
  std::vector<cnlos_problem*> slot;      // occupant per slot, or null
  std::vector<SrvReq> req;
  std::vector<SceneRun> run;
  std::vector<long long> admitted;
  // rounds in flight: the members and runs they advance, and the event
  // recorded after them on the group's stream
  hipEvent_t done = nullptr;
  bool busy = false;
  long long busy_since = 0;
  Group view;
  std::vector<SceneRun> vruns;
  std::vector<int> vidx;
  int occupied() const {
    int k = 0;
    for (cnlos_problem* m : slot) k += m != nullptr;
    return k;
  }
};

}  // namespace

struct cnlos_server {
  Arena arena;
  int K = 8, rounds = 8;
  long long step_no = 0;
  long long enqueues = 0;     // order of the groups' rounds in flight
  int fail_next_groups = 0;   // test hook: slot-group creations to fail on purpose
  std::vector<SrvReq> queue;
  std::vector<SrvGroup*> groups;
  std::vector<cnlos_completion> done;
};

struct cnlos_problem {
  cnlos_config cfg;
  int logn = 0, logm = 0;
  size_t V = 0;
  int nn = 0;
  hipStream_t st = nullptr;
  uint8_t* ws = nullptr;
  uint64_t ws_bytes = 0;
  bool poisoned = false;
  bool has_meas = false;
  bool in_batch = false;      // owned by a cnlos_batch
  size_t carve_bytes = 0;
  int iter_host = 0;
  DevCtl* ctl = nullptr;
  DevCtl* ctl_host = nullptr;   // pinned mirror
  double* partials = nullptr;
  double* logbuf = nullptr;
  float2* spec = nullptr;
  float2* hq = nullptr;
  bool hq_shared = false;     // hq belongs to the batch or slot group, built once
  float2* tw_t = nullptr;
  float2* tw_xy = nullptr;
  float2* twc_t = nullptr;
  float2* twc_xy = nullptr;
  int4* srows = nullptr;
  float* srvals = nullptr;
  int4* scols = nullptr;
  float* scvals = nullptr;
  float* wk = nullptr;
  float* r3 = nullptr;
  float* sig_xy = nullptr;
  float* sig_t = nullptr;
  uint8_t* mask = nullptr;
  float* tau0 = nullptr;
  float* U[2] = {nullptr, nullptr};
  float* UB[2] = {nullptr, nullptr};   // ubar^k and ubar^{k+1}
  float* lam = nullptr;
  float* phi = nullptr;
  float* AU[3] = {nullptr, nullptr, nullptr};
  float* gf = nullptr;
  float* T[2] = {nullptr, nullptr};
  float* TB[2] = {nullptr, nullptr};   // taubar^k and taubar^{k+1}
  float* lam2 = nullptr;
  float* lam3 = nullptr;
  float* phi_tau = nullptr;
  Tables tb;
  int nb_conv = 0, nb_solve = 0, nb_sten = 0;
  int nb_step = 0;          // blocks writing the u solve's step partials (fused pass)
  Prof prof;
};

// ---------------------------------------------------------------- event timer
namespace cnlos {

hipError_t Prof::begin(int kind, hipStream_t st) {
  Pending pd;
  pd.kind = kind;
  hipError_t e = hipSuccess;
  for (hipEvent_t* ev : {&pd.a, &pd.b}) {
    if (!pool.empty()) {
      *ev = pool.back();
      pool.pop_back();
    } else {
      // timing-only events: no system-scope fence (no cache write-back between
      // the bracketed kernel and its neighbours)
      e = hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
      if (e != hipSuccess) return e;
    }
  }
  pending.push_back(pd);
  return hipEventRecord(pd.a, st);
}

hipError_t Prof::end(int kind, hipStream_t st) {
  for (auto it = pending.rbegin(); it != pending.rend(); ++it)
    if (it->kind == kind) return hipEventRecord(it->b, st);
  return hipErrorInvalidValue;
}

void Prof::harvest() {
  for (const Pending& pd : pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pd.a, pd.b) == hipSuccess) {
      ms[pd.kind] += t;
      launches[pd.kind] += 1;
    }
    pool.push_back(pd.a);
    pool.push_back(pd.b);
  }
  pending.clear();
}

void Prof::release() {
  for (const Pending& pd : pending) {
    pool.push_back(pd.a);
    pool.push_back(pd.b);
  }
  pending.clear();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

}  // namespace cnlos

namespace {

int resample_nnz(int m) {
  // counted exactly when the tables are built; this bound sizes the buffer
  return 3 * m + 64;
}

// bytes of one lane-ordered H^ (every kt plane's full 2n x 2n spectrum)
size_t hq_bytes(const cnlos_config& c) {
  return align_up((size_t)(c.nt + 1) * 4 * c.nx * c.nx * sizeof(float2));
}

// With own_hq == false the problem reads an H^ held elsewhere (a slot group
// of one geometry keeps one copy) and its workspace has no room for one.
size_t carve(cnlos_problem* p, const cnlos_config& c, uint8_t* base, bool own_hq = true) {
  Carver cv{base};
  const int n = c.nx, m = c.nt;
  const size_t V = (size_t)n * n * m;
  const size_t nn = (size_t)n * n;
  const size_t nspec = (size_t)(m + 1) * nn;
  // H^: the full 2n x 2n spectrum of every kt plane, lane-ordered
  const size_t nhq = (size_t)(m + 1) * 4 * n * n;
  DevCtl* ctl = cv.take<DevCtl>(1);
  double* partials = cv.take<double>((size_t)SL_COUNT * kMaxBlocks);
  double* logbuf = cv.take<double>((size_t)kLogRows * kLogCols);
  float2* spec = cv.take<float2>(nspec);
  float2* hq = own_hq ? cv.take<float2>(nhq) : nullptr;
  float2* tw_t = cv.take<float2>(m);
  float2* tw_xy = cv.take<float2>(n);
  float2* twc_t = cv.take<float2>(m);
  float2* twc_xy = cv.take<float2>(2 * n);
  int4* srows = cv.take<int4>(m);
  float* srvals = cv.take<float>(resample_nnz(m));
  int4* scols = cv.take<int4>(m);
  float* scvals = cv.take<float>(resample_nnz(m));
  float* wk = cv.take<float>(m);
  float* r3 = cv.take<float>(m);
  float* sig_xy = cv.take<float>(n);
  float* sig_t = cv.take<float>(m / 2 + 1);
  uint8_t* mask = cv.take<uint8_t>(nn);
  if (p) {
    p->ctl = ctl;
    p->partials = partials;
    p->logbuf = logbuf;
    p->spec = spec;
    if (own_hq) p->hq = hq;
    p->tw_t = tw_t;
    p->tw_xy = tw_xy;
    p->twc_t = twc_t;
    p->twc_xy = twc_xy;
    p->srows = srows;
    p->srvals = srvals;
    p->scols = scols;
    p->scvals = scvals;
    p->wk = wk;
    p->r3 = r3;
    p->sig_xy = sig_xy;
    p->sig_t = sig_t;
    p->mask = mask;
  }
  if (c.model == CNLOS_MODEL_OPERATOR) return align_up(cv.off);
  float* tau0 = cv.take<float>(V);
  float* U0 = cv.take<float>(V);
  float* U1 = cv.take<float>(V);
  float* UB0 = cv.take<float>(V);
  float* UB1 = cv.take<float>(V);
  float* lam = cv.take<float>(3 * V);
  float* phi = cv.take<float>(V);
  float* A0 = cv.take<float>(V);
  float* A1 = cv.take<float>(V);
  float* A2 = cv.take<float>(V);
  float* gf = cv.take<float>(V);
  if (p) {
    p->tau0 = tau0;
    p->U[0] = U0;
    p->U[1] = U1;
    p->UB[0] = UB0;
    p->UB[1] = UB1;
    p->lam = lam;
    p->phi = phi;
    p->AU[0] = A0;
    p->AU[1] = A1;
    p->AU[2] = A2;
    p->gf = gf;
  }
  if (c.model == CNLOS_MODEL_DUAL) {
    float* T0 = cv.take<float>(V);
    float* T1 = cv.take<float>(V);
    float* TB0 = cv.take<float>(V);
    float* TB1 = cv.take<float>(V);
    float* lam2 = cv.take<float>(3 * V);
    float* lam3 = cv.take<float>(V);
    float* phi_tau = cv.take<float>(V);
    if (p) {
      p->T[0] = T0;
      p->T[1] = T1;
      p->TB[0] = TB0;
      p->TB[1] = TB1;
      p->lam2 = lam2;
      p->lam3 = lam3;
      p->phi_tau = phi_tau;
    }
  }
  return align_up(cv.off);
}

cnlos_status validate_cfg(const cnlos_config* c) {
  if (!c) return fail(CNLOS_EINVAL, "config is NULL");
  if (c->nx <= 0 || c->ny <= 0 || c->nt <= 0) return fail(CNLOS_EINVAL, "nx, ny, nt must be positive");
  if (c->nx != c->ny) return fail(CNLOS_EUNSUPPORTED, "only square scan grids (nx == ny) are supported");
  if (!is_pow2(c->nx) || c->nx < 8 || c->nx > 128)
    return fail(CNLOS_EUNSUPPORTED, "nx must be a power of two in [8, 128]");
  if (!is_pow2(c->nt) || c->nt < 16 || c->nt > 2048)
    return fail(CNLOS_EUNSUPPORTED, "nt must be a power of two in [16, 2048]");
  if (!finite_pos(c->wall_w_m) || !finite_pos(c->wall_h_m)) return fail(CNLOS_EINVAL, "wall extent must be positive");
  if (!finite_pos(c->bin_ps)) return fail(CNLOS_EINVAL, "bin_ps must be positive");
  if (c->model < 0 || c->model > 2) return fail(CNLOS_EINVAL, "unknown model");
  if (c->phi < 0 || c->phi > 2) return fail(CNLOS_EINVAL, "unknown phi kind");
  if (c->falloff < 0 || c->falloff > 1) return fail(CNLOS_EINVAL, "unknown falloff mode");
  if (c->model == CNLOS_MODEL_OPERATOR) return CNLOS_OK;
  if (!finite_nonneg(c->a_u) || !finite_nonneg(c->b_u)) return fail(CNLOS_EINVAL, "a_u, b_u must be >= 0");
  if (!finite_pos(c->mu)) return fail(CNLOS_EINVAL, "mu must be > 0");
  if (!finite_pos(c->eta_curv)) return fail(CNLOS_EINVAL, "eta_curv must be > 0");
  if (c->max_iters < 0 || c->init_iters < 0) return fail(CNLOS_EINVAL, "iteration counts must be >= 0");
  if (!finite_nonneg(c->eps_stop)) return fail(CNLOS_EINVAL, "eps_stop must be >= 0");
  if (!(isfinite(c->bt_factor) && c->bt_factor > 1.0)) return fail(CNLOS_EINVAL, "bt_factor must be > 1");
  if (c->bt_max_trials < 0) return fail(CNLOS_EINVAL, "bt_max_trials must be >= 0");
  if (!isfinite(c->L0) || !isfinite(c->L0_dual)) return fail(CNLOS_EINVAL, "L0, L0_dual must be finite");
  if (c->fista_restart != 0 && c->fista_restart != 1) return fail(CNLOS_EINVAL, "fista_restart must be 0 or 1");
  if ((c->L0 <= 0.0 || (c->model == CNLOS_MODEL_DUAL && c->L0_dual <= 0.0)) && c->power_iters < 1)
    return fail(CNLOS_EINVAL, "power_iters must be >= 1 when a step constant is estimated");
  if (c->model == CNLOS_MODEL_DUAL) {
    if (!finite_nonneg(c->a_tau) || !finite_nonneg(c->b_tau)) return fail(CNLOS_EINVAL, "a_tau, b_tau must be >= 0");
    if (!finite_pos(c->mu1) || !finite_pos(c->mu2) || !finite_pos(c->mu3))
      return fail(CNLOS_EINVAL, "mu1, mu2, mu3 must be > 0");
    if (!finite_pos(c->lambda)) return fail(CNLOS_EINVAL, "lambda must be > 0");
    if (!isfinite(c->warm_a) || !isfinite(c->warm_b)) return fail(CNLOS_EINVAL, "warm_a, warm_b must be finite");
  }
  return CNLOS_OK;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      p->poisoned = true;                                                              \
      return fail(CNLOS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    }                                                                                  \
  } while (0)

// launch `call` with event timing when its kind is selected
#define TIMED(kind, call)                                      \
  do {                                                         \
    const bool t_ = p->prof.on(kind);                          \
    if (t_) HIPCHK(p->prof.begin(kind, p->st));                \
    HIPCHK(call);                                              \
    if (t_) HIPCHK(p->prof.end(kind, p->st));                  \
  } while (0)

PhiArgs phi_args(const cnlos_problem* p, int stage, bool tau) {
  const cnlos_config& c = p->cfg;
  PhiArgs pa;
  pa.kind = c.phi;
  pa.eta = (float)c.eta_curv;
  if (tau) {
    pa.a = c.a_tau;
    pa.b = c.b_tau;
  } else if (c.model == CNLOS_MODEL_DUAL && stage == 1) {
    pa.a = c.warm_a >= 0.0 ? c.warm_a : c.a_u;
    pa.b = c.warm_b >= 0.0 ? c.warm_b : c.b_u;
  } else {
    pa.a = c.a_u;
    pa.b = c.b_u;
  }
  return pa;
}

double phi_at_zero(const PhiArgs& pa) { return pa.kind == 2 ? sqrt(pa.a) : pa.a; }

cnlos_status ctl_pull(cnlos_problem* p) {
  HIPCHK(hipMemcpyAsync(p->ctl_host, p->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  p->prof.harvest();
  return CNLOS_OK;
}

cnlos_status ctl_push(cnlos_problem* p) {
  HIPCHK(hipMemcpyAsync(p->ctl, p->ctl_host, sizeof(DevCtl), hipMemcpyHostToDevice, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  return CNLOS_OK;
}

// fields that the kernels of one launch share across a batch
bool same_shared(const cnlos_config& b, const cnlos_config& a) {
  return b.nx == a.nx && b.ny == a.ny && b.nt == a.nt && b.model == a.model && b.phi == a.phi &&
         b.falloff == a.falloff && b.a_u == a.a_u && b.b_u == a.b_u && b.a_tau == a.a_tau &&
         b.b_tau == a.b_tau && b.warm_a == a.warm_a && b.warm_b == a.warm_b && b.mu == a.mu &&
         b.mu1 == a.mu1 && b.mu2 == a.mu2 && b.mu3 == a.mu3 && b.lambda == a.lambda &&
         b.eta_curv == a.eta_curv && b.backtracking == a.backtracking;
}

// equal H^ (eq. (3) depends on the shape, the wall extent and the bin width)
bool same_geometry(const cnlos_config& b, const cnlos_config& a) {
  return b.nx == a.nx && b.ny == a.ny && b.nt == a.nt && b.wall_w_m == a.wall_w_m &&
         b.wall_h_m == a.wall_h_m && b.bin_ps == a.bin_ps;
}

// the rotating-role operand r of problem p (its candidate buffers and role)
Vol role_of(const cnlos_problem* p, int r) {
  Vol v;
  v.role = r;
  if (r == R_U_CUR || r == R_U_TR) {
    v.p[0] = p->U[0];
    v.p[1] = p->U[1];
  } else if (r == R_T_CUR || r == R_T_TR) {
    v.p[0] = p->T[0];
    v.p[1] = p->T[1];
  } else if (r == R_UB_CUR || r == R_UB_NEW) {
    v.p[0] = p->UB[0];
    v.p[1] = p->UB[1];
  } else if (r == R_TB_CUR || r == R_TB_NEW) {
    v.p[0] = p->TB[0];
    v.p[1] = p->TB[1];
  } else {
    v.p[0] = p->AU[0];
    v.p[1] = p->AU[1];
    v.p[2] = p->AU[2];
  }
  return v;
}

inline Vol fixed(const float* q) { return Vol{{const_cast<float*>(q), nullptr, nullptr}, -1}; }
inline float* zsh_host(float* q, size_t off) { return reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(q) + off); }

// One padded convolution of the problem (forward or adjoint).
hipError_t conv(cnlos_problem* p, const ConvSrc& src, bool adjoint, int epi, const ConvEpi& ep,
                const DevCtl* ctl) {
  return launch_conv(p->logn, p->logm, p->tb, src, p->spec, adjoint, epi, ep, ctl, kSingle, p->st,
                     &p->prof);
}

// ||B||^2 by power iteration (B = A_D when masked, else A), from the ones
// vector, for the bt.nz problems mem[0..nz) of one layout that follow p = mem[0]
// at the workspace stride bt.zs (one launch per step for all of them, each
// with its own mask and estimate); est[i] receives member i's estimate.
cnlos_status power_estimate(cnlos_problem* p, const Batch& bt, cnlos_problem* const* mem,
                            bool masked, double* est) {
  float* X = p->AU[0];
  float* Y = p->AU[1];
  for (int i = 0; i < bt.nz; ++i)
    HIPCHK(launch_fill(zsh_host(X, i * bt.zs), p->V, (float)(1.0 / sqrt((double)p->V)), p->st));
  for (int it = 0; it < p->cfg.power_iters; ++it) {
    ConvSrc s1{};
    s1.a = fixed(X);
    s1.b = fixed(nullptr);
    s1.scale_div = it > 0 ? &p->ctl->pow_est : nullptr;
    ConvEpi e1{};
    e1.out = fixed(Y);
    e1.au = fixed(nullptr);
    e1.au_prev = fixed(nullptr);
    e1.w = p->wk;
    e1.mask = masked ? p->mask : nullptr;
    HIPCHK(launch_conv(p->logn, p->logm, p->tb, s1, p->spec, false, EPI_PLAIN, e1, nullptr, bt,
                       p->st, &p->prof));
    ConvSrc s2{};
    s2.a = fixed(Y);
    s2.b = fixed(nullptr);
    s2.w = p->wk;
    s2.mask = masked ? p->mask : nullptr;
    ConvEpi e2{};
    e2.out = fixed(X);
    e2.au = fixed(nullptr);
    e2.au_prev = fixed(nullptr);
    e2.partials = p->partials;
    HIPCHK(launch_conv(p->logn, p->logm, p->tb, s2, p->spec, true, EPI_NORM, e2, nullptr, bt,
                       p->st, &p->prof));
    HIPCHK(launch_pow_finalize(p->ctl, p->partials, p->nb_conv, bt, p->st));
  }
  for (int i = 0; i < bt.nz; ++i) {
    cnlos_status s = ctl_pull(mem[i]);
    if (s != CNLOS_OK) return s;
    est[i] = mem[i]->ctl_host->pow_est;
    if (!isfinite(est[i]) || est[i] <= 0.0)
      return fail(CNLOS_ENONFINITE, "power iteration gave no positive norm estimate");
  }
  return CNLOS_OK;
}
cnlos_status power_estimate(cnlos_problem* p, bool masked, double* est) {
  return power_estimate(p, kSingle, &p, masked, est);
}

cnlos_status reset_state(cnlos_problem* p) {
  const size_t V = p->V;
  float* zero[] = {p->U[0], p->U[1], p->UB[0], p->UB[1], p->AU[0], p->AU[1], p->AU[2], p->gf};
  for (float* z : zero) HIPCHK(launch_fill(z, V, 0.f, p->st));
  HIPCHK(launch_fill(p->lam, 3 * V, 0.f, p->st));
  HIPCHK(launch_fill(p->phi, V, (float)phi_at_zero(phi_args(p, 1, false)), p->st));
  if (p->cfg.model == CNLOS_MODEL_DUAL) {
    float* zd[] = {p->T[0], p->T[1], p->TB[0], p->TB[1], p->lam3};
    for (float* z : zd) HIPCHK(launch_fill(z, V, 0.f, p->st));
    HIPCHK(launch_fill(p->lam2, 3 * V, 0.f, p->st));
    HIPCHK(launch_fill(p->phi_tau, V, (float)phi_at_zero(phi_args(p, 2, true)), p->st));
  }
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  DevCtl& c = *p->ctl_host;
  c.L = c.L0_obj;
  c.t = 1.0;
  c.beta = 0.0;
  c.energy_prev = NAN;
  c.halt = 0;
  c.reason = HR_NONE;
  c.iter = 0;
  c.trials = 0;
  c.bt_rejects = 0;
  c.stage = 1;
  c.log_count = 0;
  c.target = 0;
  c.reject = 0;
  c.stage1_end = p->cfg.model == CNLOS_MODEL_DUAL ? p->cfg.init_iters : 0x7fffffff;
  c.slot[R_U_CUR] = 0;
  c.slot[R_U_TR] = 1;
  c.slot[R_AU_CUR] = 0;
  c.slot[R_AU_PREV] = 2;
  c.slot[R_AU_TR] = 1;
  c.slot[R_T_CUR] = 0;
  c.slot[R_T_TR] = 1;
  c.slot[R_UB_CUR] = 0;
  c.slot[R_UB_NEW] = 1;
  c.slot[R_TB_CUR] = 0;
  c.slot[R_TB_NEW] = 1;
  c.slot_pad = 0;
  p->iter_host = 0;
  return ctl_push(p);
}

// Sequences of one iteration slot.  Every kernel carries a phase gate, so a
// slot may hold sequences that some (or all) scenes skip: a scene runs the
// Algorithm-1 sequence while in the warm start (or the object model), the
// hand-over once its warm start is done, and the Algorithm-2 sequence after.
enum SlotSeq : int { SEQ_S1 = 1, SEQ_TR = 2, SEQ_S2 = 4 };


// Enqueue one iteration slot for the scenes of `bt` (p: the first scene; the
// others follow at the workspace stride).
cnlos_status enqueue_slot(cnlos_problem* p, Batch bt, int seqs) {
  const cnlos_config& c = p->cfg;
  const int ln = p->logn, lm = p->logm;
  DevCtl* ctl = p->ctl;
  const size_t V = p->V;
  auto gated = [&](int g) {
    Batch b = bt;
    b.gate = g;
    return b;
  };
  // right-hand side of the u solve, computed in the solve's t pass
  auto rhs_u = [&](double mu) {
    RhsSrc r;
    r.mode = RHS_U;
    r.xb = role_of(p, R_UB_CUR);
    r.gf = p->gf;
    r.lam = p->lam;
    r.phi = p->phi;
    r.mu = (float)mu;
    r.logn = ln;
    return r;
  };
  auto role = [&](int r) { return role_of(p, r); };

  if (seqs & SEQ_S1) {
    const double mu = c.mu;
    const int G = G_STAGE1;
    ConvSrc sa{};
    sa.a = role(R_AU_CUR);
    sa.b = role(R_AU_PREV);
    sa.c = fixed(p->tau0);
    sa.w = p->wk;
    sa.mask = p->mask;
    sa.lincache = 1;
    ConvEpi ea{};
    ea.out = fixed(p->gf);
    ea.au = fixed(nullptr);
    ea.au_prev = fixed(nullptr);
    // grad f stays on chip: the adjoint's last pass also runs the u solve's
    // first (right-hand side and forward t pass); the solve's last pass also
    // starts A u+ (forward t pass of the convolution)
    const RhsSrc ru = rhs_u(mu);
    HIPCHK(launch_conv(ln, lm, p->tb, sa, p->spec, true, EPI_PLAIN, ea, ctl, gated(G | G_FIRST),
                       p->st, &p->prof, false, &ru));
    SolveEpi se{};
    se.out = role(R_U_TR);
    se.ref = role(R_UB_CUR);
    se.partials = p->partials;
    HIPCHK(launch_solve(ln, lm, p->tb, nullptr, ru, p->spec, &ctl->L, 0.0, mu, se, ctl,
                        gated(G | G_FIRST), p->st, &p->prof, true, true));
    ConvSrc sf{};
    sf.a = role(R_U_TR);
    sf.b = fixed(nullptr);
    sf.c = fixed(nullptr);
    ConvEpi ef{};
    ef.out = role(R_AU_TR);
    ef.w = p->wk;
    ef.mask = p->mask;
    ef.au = role(R_AU_CUR);
    ef.au_prev = role(R_AU_PREV);
    ef.tau0 = p->tau0;
    ef.partials = p->partials;
    HIPCHK(launch_conv(ln, lm, p->tb, sf, p->spec, false, EPI_FWD_OBJ, ef, ctl, gated(G), p->st,
                       &p->prof, true));
    // the post kernel takes the backtracking decision; k_finalize applies it
    const CheckArgs ck{p->nb_conv, p->nb_step, c.backtracking ? 1 : 0};
    const PostArgs pa{role(R_U_TR), role(R_U_CUR), role(R_UB_CUR), role(R_UB_NEW), p->lam, p->phi,
                      (float)mu, phi_args(p, 1, false)};
    TIMED(KK_POST, launch_post(ln, lm, pa, p->partials, ck, ctl, gated(G), p->st));
    // the data term of the energy comes from the forward pass (SL_DATA)
    TIMED(KK_CONTROL, launch_finalize(ctl, p->logbuf, p->partials, p->nb_conv, p->nb_sten, 0, 0.0, mu,
                                      gated(G), p->st));
  }
  if (c.model != CNLOS_MODEL_DUAL) return CNLOS_OK;

  if (seqs & SEQ_TR) {
    const PhiArgs pu = phi_args(p, 2, false), pt = phi_args(p, 2, true);
    float* zf[] = {p->T[0], p->T[1], p->TB[0], p->TB[1], p->lam3, p->lam2, p->lam};
    size_t zc[] = {V, V, V, V, V, 3 * V, 3 * V};
    TIMED(KK_OTHER, launch_transition(ln, lm, ctl, role(R_U_CUR), role(R_UB_CUR), p->phi, pu,
                                      p->phi_tau, phi_at_zero(pt), zf, zc, 7, bt, p->st));
  }

  if (seqs & SEQ_S2) {
    // Algorithm 2
    const double mu1 = c.mu1, mu2 = c.mu2, mu3 = c.mu3, lam = c.lambda;
    const int G = G_STAGE2;
    ConvSrc sa{};
    sa.a = role(R_AU_CUR);
    sa.b = role(R_AU_PREV);
    sa.c = role(R_TB_CUR);
    sa.w = p->wk;
    sa.lincache = 1;
    ConvEpi ea{};
    ea.out = fixed(p->gf);
    ea.au = fixed(nullptr);
    ea.au_prev = fixed(nullptr);
    const RhsSrc ru = rhs_u(mu1);
    HIPCHK(launch_conv(ln, lm, p->tb, sa, p->spec, true, EPI_PLAIN, ea, ctl, gated(G | G_FIRST),
                       p->st, &p->prof, false, &ru));
    SolveEpi se{};
    se.out = role(R_U_TR);
    se.ref = role(R_UB_CUR);
    se.partials = p->partials;
    HIPCHK(launch_solve(ln, lm, p->tb, nullptr, ru, p->spec, &ctl->L, 0.0, mu1, se, ctl,
                        gated(G | G_FIRST), p->st, &p->prof, true, true));
    ConvSrc sf{};
    sf.a = role(R_U_TR);
    sf.b = fixed(nullptr);
    sf.c = fixed(nullptr);
    ConvEpi ef{};
    ef.out = role(R_AU_TR);
    ef.w = p->wk;
    ef.au = role(R_AU_CUR);
    ef.au_prev = role(R_AU_PREV);
    ef.partials = p->partials;
    // the forward operator's last pass also runs the tau solve's first (its
    // right-hand side reads A u+ on chip); the tau solve writes the trial
    // buffers only, so it runs before the backtracking decision, which the
    // post kernel takes (a rejected trial's tau is recomputed in the next slot)
    RhsSrc rt;
    rt.mode = RHS_TAU;
    rt.xb = role(R_T_CUR);   // w and f start from the last accepted tau
    rt.au = role(R_AU_TR);
    rt.lam = p->lam2;
    rt.phi = p->phi_tau;
    rt.lam3 = p->lam3;
    rt.tau0 = p->tau0;
    rt.mask = p->mask;
    rt.mu = (float)mu2;
    rt.lambda = (float)lam;
    rt.mu3 = (float)mu3;
    rt.logn = ln;
    HIPCHK(launch_conv(ln, lm, p->tb, sf, p->spec, false, EPI_FWD_DUAL, ef, ctl, gated(G), p->st,
                       &p->prof, true, &rt));
    SolveEpi st2{};
    st2.out = role(R_T_TR);
    st2.ref = fixed(nullptr);
    st2.partials = p->partials;
    HIPCHK(launch_solve(ln, lm, p->tb, nullptr, rt, p->spec, nullptr, 1.0 + mu3, mu2, st2, ctl,
                        gated(G), p->st, &p->prof, false, true));
    const PostArgs pu{role(R_U_TR), role(R_U_CUR), role(R_UB_CUR), role(R_UB_NEW), p->lam, p->phi,
                      (float)mu1, phi_args(p, 2, false)};
    const PostArgs pt{role(R_T_TR), role(R_T_CUR), role(R_T_CUR), role(R_TB_NEW), p->lam2,
                      p->phi_tau, (float)mu2, phi_args(p, 2, true)};
    const CheckArgs ck{p->nb_conv, p->nb_step, c.backtracking ? 1 : 0};
    TIMED(KK_POST, launch_post_dual(ln, lm, pu, pt, p->lam3, mu3, lam, role(R_AU_TR), p->tau0,
                                      p->mask, p->partials, ck, ctl, gated(G), p->st));
    TIMED(KK_CONTROL, launch_finalize(ctl, p->logbuf, p->partials, p->nb_conv, p->nb_sten, 1, lam, mu1,
                                      gated(G), p->st));
  }
  return CNLOS_OK;
}

float* field_ptr(cnlos_problem* p, int field, size_t* count) {
  const size_t V = p->V;
  const DevCtl& h = *p->ctl_host;
  const bool dual = p->cfg.model == CNLOS_MODEL_DUAL;
  *count = V;
  switch (field) {
    case CNLOS_FIELD_U: return p->U[h.slot[R_U_CUR]];
    case CNLOS_FIELD_UBAR: return p->UB[h.slot[R_UB_CUR]];
    case CNLOS_FIELD_LAM: *count = 3 * V; return p->lam;
    case CNLOS_FIELD_PHI: return p->phi;
    case CNLOS_FIELD_AU: return p->AU[h.slot[R_AU_CUR]];
    case CNLOS_FIELD_AU_PREV: return p->AU[h.slot[R_AU_PREV]];
    case CNLOS_FIELD_TAU0: return p->tau0;
    default: break;
  }
  if (!dual) return nullptr;
  switch (field) {
    case CNLOS_FIELD_TAU: return p->T[h.slot[R_T_CUR]];
    case CNLOS_FIELD_TAUBAR: return p->TB[h.slot[R_TB_CUR]];
    case CNLOS_FIELD_LAM2: *count = 3 * V; return p->lam2;
    case CNLOS_FIELD_LAM3: return p->lam3;
    case CNLOS_FIELD_PHI_TAU: return p->phi_tau;
    default: return nullptr;
  }
}


// pull every member's controller with one stream synchronization
cnlos_status group_pull(Group& g) {
  cnlos_problem* p = g.lead;
  for (cnlos_problem* m : g.mem)
    HIPCHK(hipMemcpyAsync(m->ctl_host, m->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  p->prof.harvest();
  return CNLOS_OK;
}

cnlos_status group_push(Group& g) {
  cnlos_problem* p = g.lead;
  for (cnlos_problem* m : g.mem)
    HIPCHK(hipMemcpyAsync(m->ctl, m->ctl_host, sizeof(DevCtl), hipMemcpyHostToDevice, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  return CNLOS_OK;
}

// Start a run of a group's members: goal per member (iters > 0: that many
// more iterations; else the configured count), written to the controllers.
cnlos_status group_start(Group& g, std::vector<SceneRun>& runs, int32_t iters) {
  cnlos_status s = group_pull(g);
  if (s != CNLOS_OK) return s;
  runs.assign(g.mem.size(), SceneRun());
  for (size_t i = 0; i < g.mem.size(); ++i) {
    cnlos_problem* m = g.mem[i];
    const cnlos_config& c = m->cfg;
    DevCtl& h = *m->ctl_host;
    SceneRun& r = runs[i];
    const int planned = c.max_iters + (c.model == CNLOS_MODEL_DUAL ? c.init_iters : 0);
    r.start = h.iter;
    r.goal = iters > 0 ? h.iter + iters : planned;
    r.rejects0 = h.bt_rejects;
    r.active = h.iter < r.goal;
    h.target = r.goal;
    h.reject = 0;
    h.halt = 0;
    h.reason = HR_NONE;
    h.trials = 0;
  }
  return group_push(g);
}

// Enqueue up to `batch` iteration slots for the group's active members (the
// sequences each slot needs follow from the members' last known state).
// Sets *enqueued to whether anything was enqueued.
cnlos_status group_enqueue(Group& g, const std::vector<SceneRun>& runs, int batch, bool* enqueued) {
  cnlos_problem* p = g.lead;
  int need = 0, to_s1end = 0x7fffffff;
  bool s1 = false, s2 = false;
  for (size_t i = 0; i < g.mem.size(); ++i) {
    if (!runs[i].active) continue;
    const DevCtl& h = *g.mem[i]->ctl_host;
    need = std::max(need, runs[i].goal - h.iter);
    if (h.stage == 1 && h.iter < h.stage1_end) {
      s1 = true;
      to_s1end = std::min(to_s1end, h.stage1_end - h.iter);
    } else {
      s2 = true;
    }
  }
  *enqueued = need > 0;
  if (need <= 0) return CNLOS_OK;
  int nb = std::min(batch, need);
  // a warm-start batch ends where the first scene reaches the hand-over
  if (s1 && !s2) nb = std::min(nb, to_s1end);
  for (int j = 0; j < nb; ++j) {
    int seq = 0;
    for (size_t i = 0; i < g.mem.size(); ++i) {
      if (!runs[i].active) continue;
      const DevCtl& h = *g.mem[i]->ctl_host;
      if (h.stage == 1 && h.iter < h.stage1_end) {
        seq |= SEQ_S1;
        if (p->cfg.model == CNLOS_MODEL_DUAL && h.iter + j + 1 >= h.stage1_end) seq |= SEQ_TR | SEQ_S2;
      } else if (h.stage == 1) {
        seq |= SEQ_TR | SEQ_S2;       // warm start done, hand-over pending
      } else {
        seq |= SEQ_S2;
      }
    }
    cnlos_status s = enqueue_slot(p, g.bt, seq);
    if (s != CNLOS_OK) return s;
  }
  return CNLOS_OK;
}

// Wait for the group, then retire members that reached their goal, stopped
// early or failed (their halt is cleared for later calls).
cnlos_status group_absorb(Group& g, std::vector<SceneRun>& runs) {
  cnlos_status s = group_pull(g);
  if (s != CNLOS_OK) return s;
  bool dirty = false;
  for (size_t i = 0; i < g.mem.size(); ++i) {
    SceneRun& r = runs[i];
    cnlos_problem* m = g.mem[i];
    DevCtl& h = *m->ctl_host;
    m->iter_host = h.iter;
    if (!r.active) continue;
    if (h.halt) {
      const int reason = h.reason;
      // parked: the halt is cleared for later calls, the target keeps the
      // member out of the rest of this run's launches
      h.halt = 0;
      h.reason = HR_NONE;
      h.trials = 0;
      h.target = h.iter;
      dirty = true;
      r.active = false;
      if (reason == HR_STOP) {
        r.stopped = true;
      } else if (reason == HR_BACKTRACK) {
        r.status = fail(CNLOS_EBACKTRACK, "backtracking found no acceptable step");
      } else {
        r.status = fail(CNLOS_ENONFINITE, "non-finite residual or energy");
      }
    } else if (h.iter >= r.goal) {
      r.active = false;
    }
  }
  if (dirty) return group_push(g);
  return CNLOS_OK;
}

void fill_report(const cnlos_problem* m, const SceneRun& r, cnlos_report* out) {
  const DevCtl& h = *m->ctl_host;
  out->iters_done = h.iter - r.start;
  out->total_iters = h.iter;
  out->stopped_early = r.stopped ? 1 : 0;
  out->bt_rejects = h.bt_rejects - r.rejects0;
  out->L_final = h.L;
  out->energy = h.last_energy;
  out->primal_res = h.last_primal;
  out->dual_res = h.last_dual;
  out->status = r.status;
  out->reserved = 0;
}

// Run every scene of every group to its goal.  Groups run on their own
// streams: each round enqueues a batch of iteration slots on every group
// before it waits for any, so the groups' work overlaps on the device.
cnlos_status run_groups(std::vector<Group>& gs, int32_t iters, std::vector<cnlos_report*>* reps) {
  std::vector<std::vector<SceneRun>> runs(gs.size());
  for (size_t gi = 0; gi < gs.size(); ++gi) {
    cnlos_status s = group_start(gs[gi], runs[gi], iters);
    if (s != CNLOS_OK) return s;
  }
  int batch = 2;
  for (;;) {
    bool any = false;
    std::vector<char> busy(gs.size(), 0);
    for (size_t gi = 0; gi < gs.size(); ++gi) {
      bool e = false;
      cnlos_status s = group_enqueue(gs[gi], runs[gi], batch, &e);
      if (s != CNLOS_OK) return s;
      busy[gi] = e;
      any = any || e;
    }
    if (!any) break;
    for (size_t gi = 0; gi < gs.size(); ++gi) {
      if (!busy[gi]) continue;
      cnlos_status s = group_absorb(gs[gi], runs[gi]);
      if (s != CNLOS_OK) return s;
    }
    if (batch < 64) batch *= 2;
  }
  cnlos_status result = CNLOS_OK;
  size_t flat = 0;
  for (size_t gi = 0; gi < gs.size(); ++gi)
    for (size_t i = 0; i < gs[gi].mem.size(); ++i, ++flat) {
      const SceneRun& r = runs[gi][i];
      cnlos_problem* m = gs[gi].mem[i];
      m->iter_host = m->ctl_host->iter;
      if (result == CNLOS_OK && r.status != CNLOS_OK) result = r.status;
      cnlos_report* out = (reps && flat < reps->size()) ? (*reps)[flat] : nullptr;
      if (out) fill_report(m, r, out);
    }
  return result;
}

#define CHECK_HANDLE(p)                                                      \
  do {                                                                       \
    if (!(p)) return fail(CNLOS_EINVAL, "problem handle is NULL");           \
    if ((p)->poisoned) return fail(CNLOS_ESTATE, "handle poisoned by an earlier HIP failure"); \
  } while (0)

#define CHECK_SOLVER(p)                                                       \
  do {                                                                        \
    if ((p)->cfg.model == CNLOS_MODEL_OPERATOR)                               \
      return fail(CNLOS_ESTATE, "operator-only problem has no ADMM state");   \
  } while (0)

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* cnlos_version(void) { return "1.0"; }

const char* cnlos_last_error(void) { return g_err.c_str(); }

void cnlos_config_default(cnlos_config* c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->nx = c->ny = 16;
  c->nt = 128;
  c->model = CNLOS_MODEL_OBJECT;
  c->wall_w_m = c->wall_h_m = 1.0;
  c->bin_ps = 32.0;
  c->phi = CNLOS_PHI_TSC;
  c->falloff = CNLOS_FALLOFF_COMPENSATED;
  c->a_u = 5e-5;
  c->b_u = 5e-5;
  c->a_tau = 1e-4;
  c->b_tau = 3e-2;
  c->warm_a = -1.0;
  c->warm_b = -1.0;
  c->mu = 0.1;
  c->mu1 = 1.0;
  c->mu2 = 800.0;
  c->mu3 = 2.0;
  c->lambda = 200.0;
  c->eta_curv = 1e-3;
  c->max_iters = 50;
  c->init_iters = 50;
  c->eps_stop = 0.0;
  c->backtracking = 1;
  c->bt_max_trials = 20;
  c->L0 = 0.0;
  c->L0_dual = 0.0;
  c->bt_factor = 2.0;
  c->power_iters = 15;
  c->fista_restart = 0;
}

cnlos_status cnlos_validate(const cnlos_config* cfg, const uint8_t* mask_host) {
  cnlos_status s = validate_cfg(cfg);
  if (s != CNLOS_OK) return s;
  if (mask_host) {
    const int nn = cfg->nx * cfg->ny;
    int kept = 0;
    for (int i = 0; i < nn; ++i) kept += mask_host[i] != 0;
    if (kept == 0) return fail(CNLOS_EINVAL, "mask has no measured scan point");
  }
  return CNLOS_OK;
}

cnlos_status cnlos_workspace_bytes(const cnlos_config* cfg, uint64_t* bytes) {
  if (!bytes) return fail(CNLOS_EINVAL, "bytes is NULL");
  cnlos_status s = validate_cfg(cfg);
  if (s != CNLOS_OK) return s;
  *bytes = (uint64_t)carve(nullptr, *cfg, nullptr);
  return CNLOS_OK;
}

cnlos_status cnlos_create(const cnlos_config* cfg, const uint8_t* mask_host, void* workspace_dev,
                          uint64_t workspace_bytes, void* hip_stream, cnlos_problem** out) {
  return create_into(cfg, mask_host, workspace_dev, workspace_bytes, hip_stream, out);
}

}  // extern "C"

namespace {

// Sizes, buffer addresses and launch geometry of a problem whose workspace
// starts at ws.
// shared_hq: an H^ of this geometry held elsewhere; with own_hq false the
// workspace has no room of its own for one (slot groups), with own_hq true it
// keeps the room unused so that every slice of a batch has one layout.
void layout_problem(cnlos_problem* p, const cnlos_config& cfg, uint8_t* ws, uint64_t ws_bytes,
                    hipStream_t st, float2* shared_hq = nullptr, bool own_hq = true) {
  p->cfg = cfg;
  p->logn = ilog2(cfg.nx);
  p->logm = ilog2(cfg.nt);
  p->V = (size_t)cfg.nx * cfg.nx * cfg.nt;
  p->nn = cfg.nx * cfg.nx;
  p->st = st;
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  p->carve_bytes = carve(p, cfg, ws, own_hq);
  if (shared_hq) {
    p->hq = shared_hq;
    p->hq_shared = true;
  }
  p->nb_conv = conv_blocks(p->logn, p->logm);
  p->nb_solve = solve_blocks(p->logn, p->logm);
  p->nb_step = fused_solve_blocks(p->logn, p->logm);
  p->nb_sten = stencil_blocks(p->logn, p->logm);
}

// Operator tables of a problem laid out by carve(): twiddles, the R_z
// resampling table (eq. (3)), falloff and compensation weights, difference-
// operator symbols (eq. (11)), the mask, and H^ built on the device from the
// cone kernel's support.  Waits for the copies before the host tables go.
cnlos_status build_tables(cnlos_problem* p, const cnlos_config* cfg, const uint8_t* mask_host) {
  const int n = cfg->nx, m = cfg->nt;
  // ---------------- host tables (FP64) ----------------
  const double PI = 3.14159265358979323846;
  std::vector<float2> tw_t(m), tw_xy(n);
  for (int j = 0; j < m; ++j) {
    const double a = -2.0 * PI * j / (2.0 * m);
    tw_t[j] = make_float2((float)cos(a), (float)sin(a));
  }
  for (int j = 0; j < n; ++j) {
    const double a = -2.0 * PI * j / (2.0 * n);
    tw_xy[j] = make_float2((float)cos(a), (float)sin(a));
  }
  // per-span butterfly twiddles: entry d + k holds exp(-pi i k / d), d = 1, 2, 4, ...
  auto per_span = [&](int size) {
    std::vector<float2> t(size, make_float2(1.f, 0.f));
    for (int d = 1; d < size; d <<= 1)
      for (int k = 0; k < d; ++k) {
        const double a = -PI * k / d;
        t[d + k] = make_float2((float)cos(a), (float)sin(a));
      }
    return t;
  };
  const std::vector<float2> twc_t = per_span(m), twc_xy = per_span(2 * n);
  // R_z as overlap lengths of [sqrt(q/m), sqrt((q+1)/m)) with [k/m, (k+1)/m), times m
  std::vector<std::vector<std::pair<int, double>>> rows(m), cols(m);
  for (int q = 0; q < m; ++q) {
    const double lo = sqrt((double)q / m), hi = sqrt((double)(q + 1) / m);
    int k0 = (int)floor(lo * m) - 1;
    if (k0 < 0) k0 = 0;
    int k1 = (int)ceil(hi * m) + 1;
    if (k1 > m - 1) k1 = m - 1;
    for (int k = k0; k <= k1; ++k) {
      const double a = fmax(lo, (double)k / m), b = fmin(hi, (double)(k + 1) / m);
      if (b > a) {
        rows[q].push_back({k, m * (b - a)});
        cols[k].push_back({q, m * (b - a)});
      }
    }
  }
  std::vector<int4> srows(m), scols(m);
  std::vector<float> srv, scv;
  // the t pass computes rows of more than 3 taps from prefix sums of the first
  // resample_scan_rows lane-rows of the column and takes their interior
  // weights as 1: check both
  const int lanes = m / 2 < 64 ? m / 2 : 64;
  const int scan_end = resample_scan_rows(m, lanes) * lanes;
  for (int q = 0; q < m; ++q) {
    if (rows[q].size() > 3) {
      if (rows[q].back().first + 1 > scan_end)
        return fail(CNLOS_EINVAL, "long resampling row beyond the prefix-summed range");
      for (size_t t = 1; t + 1 < rows[q].size(); ++t)
        if ((float)rows[q][t].second != 1.f) return fail(CNLOS_EINVAL, "resampling interior weight is not 1");
    }
    srows[q] = make_int4(rows[q].empty() ? 0 : rows[q][0].first, (int)rows[q].size(), (int)srv.size(), 0);
    for (size_t t = 0; t < rows[q].size(); ++t) {
      if (rows[q][t].first != rows[q][0].first + (int)t) return fail(CNLOS_EINVAL, "resampling row not contiguous");
      srv.push_back((float)rows[q][t].second);
    }
  }
  for (int k = 0; k < m; ++k) {
    if (cols[k].size() > 3) return fail(CNLOS_EINVAL, "resampling column of more than 3 taps");
    scols[k] = make_int4(cols[k].empty() ? 0 : cols[k][0].first, (int)cols[k].size(), (int)scv.size(), 0);
    for (size_t t = 0; t < cols[k].size(); ++t) {
      if (cols[k][t].first != cols[k][0].first + (int)t) return fail(CNLOS_EINVAL, "resampling column not contiguous");
      scv.push_back((float)cols[k][t].second);
    }
  }
  if ((int)srv.size() > resample_nnz(m) || (int)scv.size() > resample_nnz(m))
    return fail(CNLOS_EINVAL, "resampling table larger than its bound");
  std::vector<float> wk(m), r3(m), sig_xy(n), sig_t(m / 2 + 1);
  for (int k = 0; k < m; ++k) {
    const double r = (k + 0.5) / m;
    wk[k] = cfg->falloff == CNLOS_FALLOFF_LITERAL ? (float)(1.0 / (r * r * r)) : 1.f;
    r3[k] = (float)(r * r * r);
  }
  for (int k = 0; k < n; ++k) {
    const double s = sin(PI * k / n);
    sig_xy[k] = (float)(4.0 * s * s);
  }
  for (int k = 0; k <= m / 2; ++k) {
    const double s = sin(PI * k / m);
    sig_t[k] = (float)(4.0 * s * s);
  }
  std::vector<uint8_t> mk(p->nn);
  for (int i = 0; i < p->nn; ++i) mk[i] = mask_host[i] ? 1 : 0;
  // cone kernel support: dq = round(m (sx dx^2 + sy dy^2)), kept when < m
  const double R = m * kC * (cfg->bin_ps * 1e-12) / 2.0;
  const double ax = cfg->wall_w_m / (n * R), ay = cfg->wall_h_m / (n * R);
  const double sx = ax * ax, sy = ay * ay;
  std::vector<int> dq((size_t)n * n);
  long long Z = 0;
  for (int dx = 0; dx < n; ++dx)
    for (int dy = 0; dy < n; ++dy) {
      const double x = (double)m * (sx * (double)(dx * dx) + sy * (double)(dy * dy));
      const long long q = (long long)floor(x + 0.5);
      dq[(size_t)dx * n + dy] = q < m ? (int)q : -1;
      if (q < m) Z += (dx ? 2 : 1) * (dy ? 2 : 1);
    }
  std::vector<double2> etab(2 * m);
  for (int j = 0; j < 2 * m; ++j) etab[j] = make_double2(cos(-PI * j / m), sin(-PI * j / m));
  std::vector<double> cosn(2 * n);
  for (int j = 0; j < 2 * n; ++j) cosn[j] = cos(PI * j / n);

  // setup-only tables live in the spectrum buffer until H^ is built
  uint8_t* scratch = reinterpret_cast<uint8_t*>(p->spec);
  int* d_dq = reinterpret_cast<int*>(scratch);
  double2* d_etab = reinterpret_cast<double2*>(scratch + align_up(dq.size() * sizeof(int)));
  double* d_cosn = reinterpret_cast<double*>(reinterpret_cast<uint8_t*>(d_etab) +
                                             align_up(etab.size() * sizeof(double2)));

  auto h2d = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, p->st);
  };
  HIPCHK(h2d(p->tw_t, tw_t.data(), m * sizeof(float2)));
  HIPCHK(h2d(p->tw_xy, tw_xy.data(), n * sizeof(float2)));
  HIPCHK(h2d(p->twc_t, twc_t.data(), m * sizeof(float2)));
  HIPCHK(h2d(p->twc_xy, twc_xy.data(), 2 * n * sizeof(float2)));
  HIPCHK(h2d(p->srows, srows.data(), m * sizeof(int4)));
  HIPCHK(h2d(p->scols, scols.data(), m * sizeof(int4)));
  HIPCHK(h2d(p->srvals, srv.data(), srv.size() * sizeof(float)));
  HIPCHK(h2d(p->scvals, scv.data(), scv.size() * sizeof(float)));
  HIPCHK(h2d(p->wk, wk.data(), m * sizeof(float)));
  HIPCHK(h2d(p->r3, r3.data(), m * sizeof(float)));
  HIPCHK(h2d(p->sig_xy, sig_xy.data(), n * sizeof(float)));
  HIPCHK(h2d(p->sig_t, sig_t.data(), (m / 2 + 1) * sizeof(float)));
  HIPCHK(h2d(p->mask, mk.data(), mk.size()));
  if (!p->hq_shared) {      // a shared H^ is built once, by its owner
    HIPCHK(h2d(d_dq, dq.data(), dq.size() * sizeof(int)));
    HIPCHK(h2d(d_etab, etab.data(), etab.size() * sizeof(double2)));
    HIPCHK(h2d(d_cosn, cosn.data(), cosn.size() * sizeof(double)));
    HIPCHK(launch_build_hq(p->logn, p->logm, p->hq, d_dq, d_etab, d_cosn, 1.0 / (double)Z, p->st));
  }

  p->tb.tw_t = p->tw_t;
  p->tb.tw_xy = p->tw_xy;
  p->tb.twc_t = p->twc_t;
  p->tb.twc_xy = p->twc_xy;
  p->tb.S.rows = p->srows;
  p->tb.S.rvals = p->srvals;
  p->tb.S.cols = p->scols;
  p->tb.S.cvals = p->scvals;
  p->tb.sig_xy = p->sig_xy;
  p->tb.sig_t = p->sig_t;
  p->tb.hq = p->hq;
  p->tb.plan = plan_for(p->logn, p->logm);
  HIPCHK(hipStreamSynchronize(p->st));
  return CNLOS_OK;
}

cnlos_status create_into(const cnlos_config* cfg, const uint8_t* mask_host, void* workspace_dev,
                         uint64_t workspace_bytes, void* hip_stream, cnlos_problem** out,
                         float2* shared_hq, bool own_hq, bool defer_steps) {
  if (!out) return fail(CNLOS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mask_host) return fail(CNLOS_EINVAL, "mask is NULL");
  cnlos_status s = cnlos_validate(cfg, mask_host);
  if (s != CNLOS_OK) return s;
  const size_t need = carve(nullptr, *cfg, nullptr, own_hq);
  if (!workspace_dev) return fail(CNLOS_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace_dev) % kAlign) return fail(CNLOS_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < need)
    return fail(CNLOS_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");

  cnlos_problem* p = new (std::nothrow) cnlos_problem();
  if (!p) return fail(CNLOS_ENOMEM, "host allocation failed");
  layout_problem(p, *cfg, (uint8_t*)workspace_dev, workspace_bytes, (hipStream_t)hip_stream,
                 shared_hq, own_hq);
  *out = p;   // from here on errors leave a handle the caller must destroy

  if (hipHostMalloc((void**)&p->ctl_host, sizeof(DevCtl), hipHostMallocDefault) != hipSuccess) {
    p->ctl_host = nullptr;
    p->poisoned = true;
    return fail(CNLOS_EHIP, "pinned host allocation failed");
  }
  memset(p->ctl_host, 0, sizeof(DevCtl));

  s = build_tables(p, cfg, mask_host);
  if (s != CNLOS_OK) return s;

  DevCtl& c = *p->ctl_host;
  memset(&c, 0, sizeof(c));
  c.L = c.L0_obj = c.L0_dual = 1.0;
  c.t = 1.0;
  c.energy_prev = NAN;
  c.stage = 1;
  c.bt_max_trials = cfg->bt_max_trials;
  c.bt_factor = cfg->bt_factor;
  c.eps_stop = cfg->eps_stop;
  c.restart_tol = cfg->fista_restart ? kRestartTol : 0.0;
  c.lambda = cfg->lambda;
  c.meas_scale = 0.0;
  s = ctl_push(p);   // also waits for the tables and H^
  if (s != CNLOS_OK) return s;
  if (cfg->model == CNLOS_MODEL_OPERATOR || defer_steps) return CNLOS_OK;

  double em = 0.0, eu = 0.0;
  if (cfg->L0 <= 0.0) {
    s = power_estimate(p, true, &em);
    if (s != CNLOS_OK) return s;
  }
  if (cfg->model == CNLOS_MODEL_DUAL && cfg->L0_dual <= 0.0) {
    s = power_estimate(p, false, &eu);
    if (s != CNLOS_OK) return s;
  }
  return finish_create(p, em, eu);
}

// Step constants L0 = 2 est ||A_D||^2 (masked) and, for the dual model,
// 2 est ||A||^2 (unmasked), unless the configuration gives them; then the
// initial state.
cnlos_status finish_create(cnlos_problem* p, double est_masked, double est_unmasked) {
  const cnlos_config* cfg = &p->cfg;
  const double L0o = cfg->L0 > 0.0 ? cfg->L0 : 2.0 * est_masked;
  const double L0d = cfg->model != CNLOS_MODEL_DUAL ? L0o
                     : (cfg->L0_dual > 0.0 ? cfg->L0_dual : 2.0 * est_unmasked);
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  p->ctl_host->L0_obj = L0o;
  p->ctl_host->L0_dual = L0d;
  s = ctl_push(p);
  if (s != CNLOS_OK) return s;
  HIPCHK(launch_fill(p->tau0, p->V, 0.f, p->st));
  return reset_state(p);
}

}  // namespace

extern "C" {

cnlos_status cnlos_set_measurement(cnlos_problem* p, const float* tau0_dev) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  if (!tau0_dev) return fail(CNLOS_EINVAL, "measurement is NULL");
  const float* r3 = p->cfg.falloff == CNLOS_FALLOFF_COMPENSATED ? p->r3 : nullptr;
  HIPCHK(launch_meas_prep(p->logn, p->logm, tau0_dev, p->mask, r3, p->tau0, p->partials, p->st));
  HIPCHK(launch_meas_finish(p->logn, p->logm, p->tau0, p->ctl, p->partials, p->st));
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  if (p->ctl_host->reason == HR_NONFINITE) {
    p->ctl_host->reason = HR_NONE;
    ctl_push(p);
    return fail(CNLOS_ENONFINITE, "measurement holds a non-finite value");
  }
  if (!(p->ctl_host->meas_scale > 0.0))
    return fail(CNLOS_EINVAL, "measurement has no positive value on a measured scan point");
  p->has_meas = true;
  return CNLOS_OK;
}

cnlos_status cnlos_apply_A(cnlos_problem* p, const float* u_dev, float* tau_dev, int32_t masked) {
  CHECK_HANDLE(p);
  if (!u_dev || !tau_dev) return fail(CNLOS_EINVAL, "NULL volume");
  if ((const void*)u_dev == (const void*)tau_dev) return fail(CNLOS_EINVAL, "input and output may not alias");
  ConvSrc s{};
  s.a = fixed(u_dev);
  s.b = fixed(nullptr);
  ConvEpi e{};
  e.out = fixed(tau_dev);
  e.au = fixed(nullptr);
  e.au_prev = fixed(nullptr);
  e.w = p->wk;
  e.mask = masked ? p->mask : nullptr;
  HIPCHK(conv(p, s, false, EPI_PLAIN, e, nullptr));
  return CNLOS_OK;
}

cnlos_status cnlos_apply_AT(cnlos_problem* p, const float* tau_dev, float* u_dev, int32_t masked) {
  CHECK_HANDLE(p);
  if (!u_dev || !tau_dev) return fail(CNLOS_EINVAL, "NULL volume");
  if ((const void*)u_dev == (const void*)tau_dev) return fail(CNLOS_EINVAL, "input and output may not alias");
  ConvSrc s{};
  s.a = fixed(tau_dev);
  s.b = fixed(nullptr);
  s.w = p->wk;
  s.mask = masked ? p->mask : nullptr;
  ConvEpi e{};
  e.out = fixed(u_dev);
  e.au = fixed(nullptr);
  e.au_prev = fixed(nullptr);
  HIPCHK(conv(p, s, true, EPI_PLAIN, e, nullptr));
  return CNLOS_OK;
}

}  // extern "C"

// ------------------------------------- the forward operator without a workspace
namespace {

// Scratch of cnlos_apply_A_noalloc: the operator's tables, H^ and convolution
// spectrum, laid out as an operator-only workspace.  Each device that runs the
// entry point holds one copy for the life of the process.  In host code the
// array's name is only a stand-in for the device symbol: its device address
// comes from hipGetSymbolAddress, once per device.
constexpr uint64_t kScratchBytes = 96ull << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kScratchDevices] = {};

// device address of the current device's scratch (looked up on first use)
cnlos_status scratch_of_current_device(uint8_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CNLOS_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(CNLOS_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CNLOS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<uint8_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return CNLOS_OK;
}

}  // namespace

extern "C" {

cnlos_status cnlos_apply_A_noalloc(const cnlos_config* cfg, const uint8_t* mask_host,
                                   const float* u_dev, float* tau_dev, int32_t masked,
                                   void* hip_stream) {
  if (!cfg) return fail(CNLOS_EINVAL, "config is NULL");
  if (!mask_host) return fail(CNLOS_EINVAL, "mask is NULL");
  if (!u_dev || !tau_dev) return fail(CNLOS_EINVAL, "NULL volume");
  if ((const void*)u_dev == (const void*)tau_dev) return fail(CNLOS_EINVAL, "input and output may not alias");
  cnlos_config oc = *cfg;
  oc.model = CNLOS_MODEL_OPERATOR;
  cnlos_status s = cnlos_validate(&oc, mask_host);
  if (s != CNLOS_OK) return s;
  const size_t need = carve(nullptr, oc, nullptr);
  if (need > kScratchBytes)
    return fail(CNLOS_EINVAL, "this shape needs " + std::to_string(need) +
                                  " bytes of operator scratch; the static scratch holds " +
                                  std::to_string(kScratchBytes));
  uint8_t* base = nullptr;
  s = scratch_of_current_device(&base);
  if (s != CNLOS_OK) return s;
  cnlos_problem prob;
  cnlos_problem* p = &prob;
  layout_problem(p, oc, base, kScratchBytes, (hipStream_t)hip_stream);
  s = build_tables(p, &oc, mask_host);
  if (s != CNLOS_OK) return s;
  ConvSrc src{};
  src.a = fixed(u_dev);
  src.b = fixed(nullptr);
  ConvEpi e{};
  e.out = fixed(tau_dev);
  e.au = fixed(nullptr);
  e.au_prev = fixed(nullptr);
  e.w = p->wk;
  e.mask = masked ? p->mask : nullptr;
  HIPCHK(conv(p, src, false, EPI_PLAIN, e, nullptr));
  HIPCHK(hipStreamSynchronize(p->st));
  return CNLOS_OK;
}

// ------------------------------------------------------------ launch plans
}  // extern "C"

namespace {

void plan_out(const Plan& pl, int logn, bool tuned, const double* conv_us, const double* solve_us,
              cnlos_plan* out) {
  out->conv_row_pad = pl.conv_pad;
  out->solve_row_pad = pl.solve_pad > 0 ? pl.solve_pad : default_solve_pad(logn);
  out->tuned = tuned ? 1 : 0;
  out->reserved = 0;
  for (int i = 0; i < 3; ++i) {
    out->conv_plane_us[i] = conv_us ? conv_us[i] : 0.0;
    out->solve_plane_us[i] = solve_us ? solve_us[i] : 0.0;
  }
}

int pad_index(const int (&pads)[3], int v) {
  for (int i = 0; i < 3; ++i)
    if (pads[i] == v) return i;
  return -1;
}

}  // namespace

extern "C" {

cnlos_status cnlos_tune(cnlos_problem* p, cnlos_plan* out) {
  CHECK_HANDLE(p);
  // the measurement runs on the solver's A u buffers, which an operator-only
  // workspace does not have
  if (p->cfg.model == CNLOS_MODEL_OPERATOR)
    return fail(CNLOS_ESTATE, "tune needs a solver problem (an operator-only workspace has no room for the measurement)");
  if (p->in_batch) return fail(CNLOS_ESTATE, "tune a standalone problem; batch members keep the batch's plan");
  // every candidate runs on this problem's buffers: a plain forward
  // convolution (A u[0] -> A u[1]) and a diagonal solve of A u[0], eight times
  // each after a warm-up; their plane kernels are timed with HIP events
  constexpr int kReps = 8;
  Prof tp;
  tp.mask = (1u << KK_PLANE_CONV) | (1u << KK_PLANE_SOLVE);
  double conv_us[3] = {0, 0, 0}, solve_us[3] = {0, 0, 0};
  const Plan keep = p->tb.plan;
  HIPCHK(launch_fill(p->AU[0], p->V, 1.0f, p->st));
  ConvSrc src{};
  src.a = fixed(p->AU[0]);
  src.b = fixed(nullptr);
  ConvEpi ep{};
  ep.out = fixed(p->AU[1]);
  ep.au = fixed(nullptr);
  ep.au_prev = fixed(nullptr);
  RhsSrc rs;
  SolveEpi se{};
  se.out = fixed(p->AU[1]);
  se.ref = fixed(nullptr);
  se.partials = p->partials;
  for (int i = 0; i < 3; ++i) {
    p->tb.plan.conv_pad = kConvPads[i];
    p->tb.plan.solve_pad = kSolvePads[i];
    HIPCHK(launch_conv(p->logn, p->logm, p->tb, src, p->spec, false, EPI_PLAIN, ep, nullptr,
                       kSingle, p->st, nullptr));   // warm-up of this variant
    HIPCHK(launch_solve(p->logn, p->logm, p->tb, p->AU[0], rs, p->spec, nullptr, 1.0, 1.0, se,
                        nullptr, kSingle, p->st, nullptr));
    for (int r = 0; r < kReps; ++r) {
      HIPCHK(launch_conv(p->logn, p->logm, p->tb, src, p->spec, false, EPI_PLAIN, ep, nullptr,
                         kSingle, p->st, &tp));
      HIPCHK(launch_solve(p->logn, p->logm, p->tb, p->AU[0], rs, p->spec, nullptr, 1.0, 1.0, se,
                          nullptr, kSingle, p->st, &tp));
    }
    const hipError_t e = hipStreamSynchronize(p->st);
    if (e != hipSuccess) {
      tp.release();
      p->tb.plan = keep;
      HIPCHK(e);
    }
    tp.harvest();
    conv_us[i] = 1e3 * tp.ms[KK_PLANE_CONV] / (double)(tp.launches[KK_PLANE_CONV] ? tp.launches[KK_PLANE_CONV] : 1);
    solve_us[i] = 1e3 * tp.ms[KK_PLANE_SOLVE] / (double)(tp.launches[KK_PLANE_SOLVE] ? tp.launches[KK_PLANE_SOLVE] : 1);
    for (int k = 0; k < KK_COUNT; ++k) {
      tp.ms[k] = 0.0;
      tp.launches[k] = 0;
    }
  }
  tp.release();
  // the fastest candidate of each kernel; it replaces the untuned default
  // only when it is faster by more than the run-to-run spread of the timing
  constexpr double kMargin = 0.97;
  Plan best;
  const int dc = pad_index(kConvPads, Plan{}.conv_pad), ds = pad_index(kSolvePads, default_solve_pad(p->logn));
  int bc = dc, bs = ds;
  for (int i = 0; i < 3; ++i) {
    if (conv_us[i] < conv_us[bc]) bc = i;
    if (solve_us[i] < solve_us[bs]) bs = i;
  }
  if (!(conv_us[bc] < kMargin * conv_us[dc])) bc = dc;
  if (!(solve_us[bs] < kMargin * solve_us[ds])) bs = ds;
  best.conv_pad = kConvPads[bc];
  best.solve_pad = kSolvePads[bs];
  p->tb.plan = best;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans[std::make_tuple(dev, p->logn, p->logm)] = best;
  }
  // the timing runs used the A u buffers: the solver starts afresh
  if (p->cfg.model != CNLOS_MODEL_OPERATOR) {
    cnlos_status s = reset_state(p);
    if (s != CNLOS_OK) return s;
  }
  if (out) plan_out(best, p->logn, true, conv_us, solve_us, out);
  return CNLOS_OK;
}

cnlos_status cnlos_get_plan(cnlos_problem* p, cnlos_plan* out) {
  CHECK_HANDLE(p);
  if (!out) return fail(CNLOS_EINVAL, "out is NULL");
  plan_out(p->tb.plan, p->logn, false, nullptr, nullptr, out);
  return CNLOS_OK;
}

cnlos_status cnlos_set_plan(cnlos_problem* p, const cnlos_plan* plan) {
  CHECK_HANDLE(p);
  if (!plan) return fail(CNLOS_EINVAL, "plan is NULL");
  if (p->in_batch) return fail(CNLOS_ESTATE, "batch members keep the batch's plan");
  if (pad_index(kConvPads, plan->conv_row_pad) < 0 || pad_index(kSolvePads, plan->solve_row_pad) < 0)
    return fail(CNLOS_EINVAL, "row pads must be 1, 2 or 4 (convolution) and 2, 4 or 8 (solve)");
  p->tb.plan.conv_pad = plan->conv_row_pad;
  p->tb.plan.solve_pad = plan->solve_row_pad;
  return CNLOS_OK;
}

// ------------------------------------------------ non-confocal operator
}  // extern "C"

namespace {

cnlos_status nc_geo(const cnlos_nc_geometry* g, NcGeo* out) {
  if (!g) return fail(CNLOS_EINVAL, "geometry is NULL");
  if (g->n < 1 || g->m < 1) return fail(CNLOS_EINVAL, "n and m must be positive");
  if (g->n > kNcMaxGrid) return fail(CNLOS_EUNSUPPORTED, "n must be at most " + std::to_string(kNcMaxGrid));
  if (g->m > kNcMaxBins) return fail(CNLOS_EUNSUPPORTED, "m must be at most " + std::to_string(kNcMaxBins));
  if (!finite_pos(g->wall_m)) return fail(CNLOS_EINVAL, "wall extent must be positive");
  if (!finite_pos(g->bin_ps)) return fail(CNLOS_EINVAL, "bin_ps must be positive");
  if (!isfinite(g->illum_x_m) || !isfinite(g->illum_y_m)) return fail(CNLOS_EINVAL, "illumination point must be finite");
  if (g->literal != 0 && g->literal != 1) return fail(CNLOS_EINVAL, "literal must be 0 or 1");
  out->n = g->n;
  out->m = g->m;
  out->wall = g->wall_m;
  out->range = g->m * kC * (g->bin_ps * 1e-12) / 2.0;
  out->cdt = kC * g->bin_ps * 1e-12;
  out->ix = g->illum_x_m;
  out->iy = g->illum_y_m;
  out->literal = g->literal;
  return CNLOS_OK;
}

cnlos_status nc_launch(const cnlos_nc_geometry* g, const float* in_dev, float* out_dev,
                       void* hip_stream, bool transpose) {
  NcGeo ng{};
  cnlos_status s = nc_geo(g, &ng);
  if (s != CNLOS_OK) return s;
  if (!in_dev || !out_dev) return fail(CNLOS_EINVAL, "NULL volume");
  if ((const void*)in_dev == (const void*)out_dev) return fail(CNLOS_EINVAL, "input and output may not alias");
  const hipStream_t st = (hipStream_t)hip_stream;
  const hipError_t e = transpose ? launch_nc_transpose(ng, in_dev, out_dev, st)
                                 : launch_nc_forward(ng, in_dev, out_dev, st);
  if (e != hipSuccess)
    return fail(CNLOS_EHIP, std::string(transpose ? "k_nc_transpose" : "k_nc_forward") + ": " +
                                hipGetErrorString(e));
  return CNLOS_OK;
}

}  // namespace

extern "C" {

cnlos_status cnlos_nc_validate(const cnlos_nc_geometry* g) {
  NcGeo ng{};
  return nc_geo(g, &ng);
}

cnlos_status cnlos_nc_apply(const cnlos_nc_geometry* g, const float* u_dev, float* tau_dev,
                            void* hip_stream) {
  return nc_launch(g, u_dev, tau_dev, hip_stream, false);
}

cnlos_status cnlos_nc_apply_T(const cnlos_nc_geometry* g, const float* tau_dev, float* u_dev,
                              void* hip_stream) {
  return nc_launch(g, tau_dev, u_dev, hip_stream, true);
}

cnlos_status cnlos_nc_midpoint(const cnlos_nc_geometry* g, double* wall_m, double* centre_x_m,
                               double* centre_y_m) {
  NcGeo ng{};
  cnlos_status s = nc_geo(g, &ng);
  if (s != CNLOS_OK) return s;
  if (!wall_m || !centre_x_m || !centre_y_m) return fail(CNLOS_EINVAL, "NULL output");
  *wall_m = g->wall_m / 2.0;
  *centre_x_m = g->illum_x_m / 2.0;
  *centre_y_m = g->illum_y_m / 2.0;
  return CNLOS_OK;
}

cnlos_status cnlos_run(cnlos_problem* p, int32_t iters, cnlos_report* out) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  if (!p->has_meas) return fail(CNLOS_ESTATE, "no measurement set");
  std::vector<Group> gs(1);
  gs[0].lead = p;
  gs[0].mem.push_back(p);
  gs[0].bt = kSingle;
  std::vector<cnlos_report*> reps{out};
  return run_groups(gs, iters, &reps);
}

cnlos_status cnlos_reset(cnlos_problem* p) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  return reset_state(p);
}

cnlos_status cnlos_get_volume(cnlos_problem* p, float* u_dev) {
  return cnlos_get_field(p, CNLOS_FIELD_U, u_dev);
}

cnlos_status cnlos_get_signal(cnlos_problem* p, float* tau_dev) {
  return cnlos_get_field(p, CNLOS_FIELD_TAU, tau_dev);
}

cnlos_status cnlos_get_field(cnlos_problem* p, int32_t field, float* dst_dev) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  if (!dst_dev) return fail(CNLOS_EINVAL, "destination is NULL");
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  const DevCtl& h = *p->ctl_host;
  const bool dual = p->cfg.model == CNLOS_MODEL_DUAL;
  const bool stage2 = dual && h.stage == 2;
  // v, w and f are not stored: computed from the state the next iteration starts from
  if (field == CNLOS_FIELD_V) {
    TIMED(KK_FIELD, launch_vstep(p->logn, p->logm, p->UB[h.slot[R_UB_CUR]], p->lam, p->phi,
                                 dst_dev, stage2 ? p->cfg.mu1 : p->cfg.mu, p->st));
    return CNLOS_OK;
  }
  if (dual && field == CNLOS_FIELD_W) {
    TIMED(KK_FIELD, launch_vstep(p->logn, p->logm, p->T[h.slot[R_T_CUR]], p->lam2, p->phi_tau,
                                 dst_dev, p->cfg.mu2, p->st));
    return CNLOS_OK;
  }
  if (dual && field == CNLOS_FIELD_F) {
    TIMED(KK_FIELD, launch_fstep(p->logn, p->logm, p->T[h.slot[R_T_CUR]], p->lam3, p->tau0,
                                 p->mask, dst_dev, p->cfg.lambda, p->cfg.mu3, p->st));
    return CNLOS_OK;
  }
  size_t n = 0;
  float* src = field_ptr(p, field, &n);
  if (!src) return fail(CNLOS_EINVAL, "field not available for this model");
  HIPCHK(hipMemcpyAsync(dst_dev, src, n * sizeof(float), hipMemcpyDeviceToDevice, p->st));
  return CNLOS_OK;
}

cnlos_status cnlos_set_field(cnlos_problem* p, int32_t field, const float* src_dev) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  if (!src_dev) return fail(CNLOS_EINVAL, "source is NULL");
  if (field == CNLOS_FIELD_TAU0) return fail(CNLOS_EINVAL, "the measurement is set by cnlos_set_measurement");
  if (field == CNLOS_FIELD_V || field == CNLOS_FIELD_W || field == CNLOS_FIELD_F)
    return fail(CNLOS_EINVAL, "v, w and f are derived from the other fields and cannot be set");
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  size_t n = 0;
  float* dst = field_ptr(p, field, &n);
  if (!dst) return fail(CNLOS_EINVAL, "field not available for this model");
  HIPCHK(hipMemcpyAsync(dst, src_dev, n * sizeof(float), hipMemcpyDeviceToDevice, p->st));
  return CNLOS_OK;
}

cnlos_status cnlos_get_info(cnlos_problem* p, cnlos_info* o) {
  CHECK_HANDLE(p);
  if (!o) return fail(CNLOS_EINVAL, "out is NULL");
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  const DevCtl& h = *p->ctl_host;
  o->L0_obj = h.L0_obj;
  o->L0_dual = h.L0_dual;
  o->L = h.L;
  o->t = h.t;
  o->beta = h.beta;
  o->meas_scale = h.meas_scale;
  o->energy_prev = h.energy_prev;
  o->iter = h.iter;
  o->stage = h.stage;
  o->bt_rejects = h.bt_rejects;
  o->has_measurement = p->has_meas ? 1 : 0;
  return CNLOS_OK;
}

cnlos_status cnlos_set_info(cnlos_problem* p, const cnlos_info* in) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  if (!in) return fail(CNLOS_EINVAL, "info is NULL");
  if (in->iter < 0 || (in->stage != 1 && in->stage != 2) || !(in->L > 0) || !(in->t >= 1.0))
    return fail(CNLOS_EINVAL, "inconsistent info");
  if (in->stage == 2 && p->cfg.model != CNLOS_MODEL_DUAL) return fail(CNLOS_EINVAL, "stage 2 needs the dual model");
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  DevCtl& h = *p->ctl_host;
  h.L = in->L;
  h.t = in->t;
  h.beta = in->beta;
  h.energy_prev = in->energy_prev;
  h.iter = in->iter;
  h.stage = in->stage;
  h.bt_rejects = in->bt_rejects;
  h.trials = 0;
  h.halt = 0;
  h.reason = HR_NONE;
  p->iter_host = in->iter;
  return ctl_push(p);
}

cnlos_status cnlos_get_log(cnlos_problem* p, double* host, int32_t cap, int32_t* n) {
  CHECK_HANDLE(p);
  CHECK_SOLVER(p);
  if (!n || (cap > 0 && !host)) return fail(CNLOS_EINVAL, "NULL output");
  cnlos_status s = ctl_pull(p);
  if (s != CNLOS_OK) return s;
  const int total = p->ctl_host->log_count;
  const int avail = total < kLogRows ? total : kLogRows;
  const int rows = cap < avail ? cap : avail;
  *n = rows;
  if (rows <= 0) return CNLOS_OK;
  std::vector<double> all((size_t)kLogRows * kLogCols);
  HIPCHK(hipMemcpyAsync(all.data(), p->logbuf, all.size() * sizeof(double), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  const int first = total - rows;
  for (int r = 0; r < rows; ++r) {
    const int src = (first + r) % kLogRows;
    memcpy(host + (size_t)r * kLogCols, all.data() + (size_t)src * kLogCols, kLogCols * sizeof(double));
  }
  return CNLOS_OK;
}

cnlos_status cnlos_profile_enable(cnlos_problem* p, uint32_t kind_mask) {
  CHECK_HANDLE(p);
  p->prof.mask = kind_mask & ((1u << KK_COUNT) - 1u);
  return CNLOS_OK;
}

cnlos_status cnlos_profile_read(cnlos_problem* p, double* ms, int64_t* launches, int32_t reset) {
  CHECK_HANDLE(p);
  HIPCHK(hipStreamSynchronize(p->st));
  p->prof.harvest();
  for (int k = 0; k < KK_COUNT; ++k) {
    if (ms) ms[k] = p->prof.ms[k];
    if (launches) launches[k] = p->prof.launches[k];
    if (reset) {
      p->prof.ms[k] = 0.0;
      p->prof.launches[k] = 0;
    }
  }
  return CNLOS_OK;
}

cnlos_status cnlos_destroy(cnlos_problem* p) {
  if (!p) return CNLOS_OK;
  if (p->in_batch) return fail(CNLOS_EINVAL, "a batch member is released with its batch");
  return destroy_problem(p);
}

// ---------------------------------------------------------------- batches
}  // extern "C"

namespace {

// Step constants of a batch's members with the batch's launches: the masked
// estimates of all members at once (each with its own mask), and the
// unmasked one (dual model) once when the members share the geometry, since
// it depends on nothing else.  Members that give their constants, or that
// differ in power_iters, estimate alone.  Every estimate is the same
// fixed-order computation as for a problem created alone, so the constants
// are bitwise the same.
cnlos_status batch_step_constants(cnlos_batch* b) {
  const int K = (int)b->mem.size();
  cnlos_problem* lead = b->mem[0];
  const Batch bt{K, b->stride, G_NONE, b->hq_shared};
  std::vector<double> em(K, 0.0), eu(K, 0.0);
  bool all_m = true, all_u = true, same_iters = true;
  const bool dual = lead->cfg.model == CNLOS_MODEL_DUAL;
  for (cnlos_problem* m : b->mem) {
    all_m = all_m && m->cfg.L0 <= 0.0;
    all_u = all_u && dual && m->cfg.L0_dual <= 0.0;
    same_iters = same_iters && m->cfg.power_iters == lead->cfg.power_iters;
  }
  cnlos_status s = CNLOS_OK;
  if (all_m && same_iters) {
    s = power_estimate(lead, bt, b->mem.data(), true, em.data());
  } else {
    for (int i = 0; i < K && s == CNLOS_OK; ++i)
      if (b->mem[i]->cfg.L0 <= 0.0) s = power_estimate(b->mem[i], true, &em[i]);
  }
  if (s != CNLOS_OK) return s;
  if (dual) {
    if (all_u && same_iters && b->hq_shared) {
      s = power_estimate(lead, false, &eu[0]);
      for (int i = 1; i < K; ++i) eu[i] = eu[0];
    } else if (all_u && same_iters) {
      s = power_estimate(lead, bt, b->mem.data(), false, eu.data());
    } else {
      for (int i = 0; i < K && s == CNLOS_OK; ++i)
        if (b->mem[i]->cfg.L0_dual <= 0.0) s = power_estimate(b->mem[i], false, &eu[i]);
    }
    if (s != CNLOS_OK) return s;
  }
  for (int i = 0; i < K; ++i) {
    s = finish_create(b->mem[i], em[i], eu[i]);
    if (s != CNLOS_OK) return s;
  }
  return CNLOS_OK;
}

}  // namespace

extern "C" {

cnlos_status cnlos_batch_workspace_bytes(const cnlos_config* cfg, int32_t count, uint64_t* bytes) {
  if (!bytes) return fail(CNLOS_EINVAL, "bytes is NULL");
  if (count < 1) return fail(CNLOS_EINVAL, "count must be >= 1");
  cnlos_status s = validate_cfg(cfg);
  if (s != CNLOS_OK) return s;
  if (cfg->model == CNLOS_MODEL_OPERATOR) return fail(CNLOS_EINVAL, "a batch needs a solver model");
  *bytes = (uint64_t)carve(nullptr, *cfg, nullptr) * (uint64_t)count;
  return CNLOS_OK;
}

cnlos_status cnlos_batch_create(const cnlos_config* cfgs, int32_t count,
                                const uint8_t* const* masks_host, void* workspace_dev,
                                uint64_t workspace_bytes, void* hip_stream, cnlos_batch** out) {
  if (!out) return fail(CNLOS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfgs || !masks_host) return fail(CNLOS_EINVAL, "configs or masks are NULL");
  if (count < 1) return fail(CNLOS_EINVAL, "count must be >= 1");
  const cnlos_config& a = cfgs[0];
  for (int i = 0; i < count; ++i) {
    cnlos_status s = cnlos_validate(&cfgs[i], masks_host[i]);
    if (s != CNLOS_OK) return s;
    if (!masks_host[i]) return fail(CNLOS_EINVAL, "mask is NULL");
    if (!same_shared(cfgs[i], a)) return fail(CNLOS_EINVAL, "batch member " + std::to_string(i) + " differs in a shared field");
  }
  if (a.model == CNLOS_MODEL_OPERATOR) return fail(CNLOS_EINVAL, "a batch needs a solver model");
  const size_t stride = carve(nullptr, a, nullptr);
  if (!workspace_dev) return fail(CNLOS_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace_dev) % kAlign) return fail(CNLOS_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < stride * (uint64_t)count)
    return fail(CNLOS_EINVAL, "workspace too small: need " + std::to_string(stride * (uint64_t)count) + " bytes");
  cnlos_batch* b = new (std::nothrow) cnlos_batch();
  if (!b) return fail(CNLOS_ENOMEM, "host allocation failed");
  b->stride = stride;
  b->st = (hipStream_t)hip_stream;
  // members of one geometry read member 0's H^ (built once); their own room
  // for it stays unused so that every slice has the same layout
  b->hq_shared = true;
  for (int i = 1; i < count; ++i) b->hq_shared = b->hq_shared && same_geometry(cfgs[i], a);
  *out = b;
  for (int i = 0; i < count; ++i) {
    cnlos_problem* m = nullptr;
    float2* shared = (b->hq_shared && i > 0) ? b->mem[0]->hq : nullptr;
    cnlos_status s = create_into(&cfgs[i], masks_host[i], (uint8_t*)workspace_dev + stride * i, stride,
                                 hip_stream, &m, shared, true, true);
    if (m) {
      m->in_batch = true;
      b->mem.push_back(m);
    }
    if (s != CNLOS_OK) return s;
  }
  return batch_step_constants(b);
}

cnlos_status cnlos_batch_member(cnlos_batch* b, int32_t i, cnlos_problem** out) {
  if (!b || !out) return fail(CNLOS_EINVAL, "NULL argument");
  if (i < 0 || i >= (int32_t)b->mem.size()) return fail(CNLOS_EINVAL, "member index out of range");
  *out = b->mem[i];
  return CNLOS_OK;
}

static cnlos_status batch_group(cnlos_batch* b, Group* g) {
  if (!b || b->mem.empty()) return fail(CNLOS_EINVAL, "empty batch");
  for (cnlos_problem* m : b->mem) {
    if (m->poisoned) return fail(CNLOS_ESTATE, "a member is poisoned by an earlier HIP failure");
    if (!m->has_meas) return fail(CNLOS_ESTATE, "a member has no measurement");
  }
  g->lead = b->mem[0];
  g->mem = b->mem;
  g->bt = Batch{(int)b->mem.size(), b->stride, G_NONE, b->hq_shared};
  return CNLOS_OK;
}

cnlos_status cnlos_batch_run(cnlos_batch* b, int32_t iters, cnlos_report* reports) {
  std::vector<Group> gs(1);
  cnlos_status s = batch_group(b, &gs[0]);
  if (s != CNLOS_OK) return s;
  std::vector<cnlos_report*> reps(b->mem.size(), nullptr);
  if (reports)
    for (size_t i = 0; i < reps.size(); ++i) reps[i] = reports + i;
  return run_groups(gs, iters, &reps);
}

cnlos_status cnlos_batch_run_many(cnlos_batch* const* batches, int32_t count, int32_t iters,
                                  cnlos_report* const* reports) {
  if (!batches || count < 1) return fail(CNLOS_EINVAL, "no batches");
  std::vector<Group> gs(count);
  std::vector<cnlos_report*> reps;
  for (int k = 0; k < count; ++k) {
    cnlos_status s = batch_group(batches[k], &gs[k]);
    if (s != CNLOS_OK) return s;
    for (int j = 0; j < k; ++j)
      if (batches[j] == batches[k]) return fail(CNLOS_EINVAL, "a batch appears twice");
    cnlos_report* r = reports ? reports[k] : nullptr;
    for (size_t i = 0; i < batches[k]->mem.size(); ++i) reps.push_back(r ? r + i : nullptr);
  }
  return run_groups(gs, iters, &reps);
}

cnlos_status cnlos_batch_destroy(cnlos_batch* b) {
  if (!b) return CNLOS_OK;
  for (cnlos_problem* m : b->mem) destroy_problem(m);
  delete b;
  return CNLOS_OK;
}

// ---------------------------------------------------------------- serving
}  // extern "C"

namespace {

cnlos_status srv_fail(cnlos_status st, const std::string& msg) { return fail(st, msg); }
void srv_group_free(cnlos_server* sv, SrvGroup* g);

// a group's device state starts parked: every slot's controller halted.  Its
// arena range holds one H^ of the group's geometry, then the K slots, whose
// workspaces have no H^ of their own.
cnlos_status srv_group_new(cnlos_server* sv, const cnlos_config& cfg, SrvGroup** out) {
  *out = nullptr;
  const size_t stride = carve(nullptr, cfg, nullptr, false);
  const size_t hqb = hq_bytes(cfg);
  const uint64_t bytes = (uint64_t)stride * sv->K + hqb;
  uint64_t off = 0;
  if (!sv->arena.take(bytes, &off)) return CNLOS_ENOMEM;
  SrvGroup* g = new (std::nothrow) SrvGroup();
  if (!g) {
    sv->arena.give(off, bytes);
    return srv_fail(CNLOS_ENOMEM, "host allocation failed");
  }
  g->proto = cfg;
  g->stride = stride;
  g->K = sv->K;
  g->off = off;
  g->bytes = bytes;
  g->hq = reinterpret_cast<float2*>(sv->arena.base + off);
  g->slots_off = off + hqb;
  g->slot.assign(g->K, nullptr);
  g->req.resize(g->K);
  g->run.resize(g->K);
  g->admitted.assign(g->K, 0);
  cnlos_problem* p = new (std::nothrow) cnlos_problem();
  if (!p || hipStreamCreate(&g->st) != hipSuccess ||
      hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess) {
    delete p;
    if (g->st) (void)hipStreamDestroy(g->st);
    sv->arena.give(off, bytes);
    delete g;
    return srv_fail(CNLOS_EHIP, "stream or event creation failed");
  }
  uint8_t* ws = sv->arena.base + g->slots_off;
  layout_problem(p, cfg, ws, stride, g->st, g->hq, false);
  g->layout = p;
  // from here on a failure gives back the arena range, the stream and the
  // host objects (srv_group_free on a group that is not yet listed)
  if (sv->fail_next_groups > 0) {
    --sv->fail_next_groups;
    srv_group_free(sv, g);
    return srv_fail(CNLOS_EHIP, "slot-group creation failed (injected by the test hook)");
  }
  // the group's H^ (built once; the tables this writes into slot 0 are
  // rebuilt by each admission), then every slot parked
  {
    std::vector<uint8_t> all((size_t)cfg.nx * cfg.ny, 1);
    p->hq_shared = false;
    const cnlos_status bs = build_tables(p, &cfg, all.data());
    p->hq_shared = true;
    if (bs != CNLOS_OK) {
      srv_group_free(sv, g);
      return bs;
    }
  }
  DevCtl parked;
  memset(&parked, 0, sizeof(parked));
  parked.halt = 1;
  for (int i = 0; i < g->K; ++i)
    if (hipMemcpyAsync(ws + (size_t)i * stride, &parked, sizeof(DevCtl), hipMemcpyHostToDevice,
                       g->st) != hipSuccess) {
      srv_group_free(sv, g);
      return srv_fail(CNLOS_EHIP, "controller initialization failed");
    }
  if (hipStreamSynchronize(g->st) != hipSuccess) {
    srv_group_free(sv, g);
    return srv_fail(CNLOS_EHIP, "stream failed");
  }
  sv->groups.push_back(g);
  *out = g;
  return CNLOS_OK;
}

void srv_group_free(cnlos_server* sv, SrvGroup* g) {
  for (cnlos_problem* m : g->slot)
    if (m) destroy_problem(m);
  if (g->st) {
    (void)hipStreamSynchronize(g->st);
    (void)hipStreamDestroy(g->st);
  }
  if (g->done) (void)hipEventDestroy(g->done);
  delete g->layout;
  sv->arena.give(g->off, g->bytes);
  delete g;
}

// a request that never reached a slot: its one completion carries the error
void srv_reject(cnlos_server* sv, const SrvReq& q, cnlos_status st) {
  cnlos_completion c{};
  c.id = q.r.id;
  c.status = st;
  c.energy = NAN;
  c.queued_steps = (double)(sv->step_no - q.submitted);
  sv->done.push_back(c);
}

void srv_complete(cnlos_server* sv, SrvGroup* g, int i, cnlos_status st) {
  cnlos_completion c{};
  c.id = g->req[i].r.id;
  c.status = st;
  cnlos_problem* m = g->slot[i];
  if (m && m->ctl_host) {
    c.iters = m->ctl_host->iter;
    c.energy = m->ctl_host->last_energy;
  }
  c.queued_steps = (double)(g->admitted[i] - g->req[i].submitted);
  c.served_steps = (double)(sv->step_no - g->admitted[i]);
  sv->done.push_back(c);
  if (m) destroy_problem(m);
  g->slot[i] = nullptr;
}

// place request q into free slot i of group g: tables, H^ and step constants
// for its geometry, its measurement, and a fresh run toward its budget
cnlos_status srv_admit(cnlos_server* sv, SrvGroup* g, int i, SrvReq& q) {
  cnlos_problem* m = nullptr;
  g->req[i] = q;
  g->admitted[i] = sv->step_no;
  cnlos_status st = create_into(&q.r.cfg, q.mask.data(),
                                sv->arena.base + g->slots_off + (size_t)i * g->stride, g->stride,
                                g->st, &m, g->hq, false, true);
  if (m) m->in_batch = true;
  g->slot[i] = m;
  if (st == CNLOS_OK) {
    // step constants; the unmasked estimate depends only on the group's
    // geometry, so one measurement serves every admission (the same
    // fixed-order computation each time, hence the same bits)
    const cnlos_config& c = q.r.cfg;
    double em = 0.0, eu = 0.0;
    if (c.L0 <= 0.0) st = power_estimate(m, true, &em);
    if (st == CNLOS_OK && c.model == CNLOS_MODEL_DUAL && c.L0_dual <= 0.0) {
      if (g->est_unmasked_iters == c.power_iters && g->est_unmasked > 0.0) {
        eu = g->est_unmasked;
      } else {
        st = power_estimate(m, false, &eu);
        if (st == CNLOS_OK) {
          g->est_unmasked = eu;
          g->est_unmasked_iters = c.power_iters;
        }
      }
    }
    if (st == CNLOS_OK) st = finish_create(m, em, eu);
  }
  if (st == CNLOS_OK) st = cnlos_set_measurement(m, q.r.tau0_dev);
  if (st == CNLOS_OK) {
    Group one;
    one.lead = m;
    one.mem.push_back(m);
    std::vector<SceneRun> runs;
    st = group_start(one, runs, 0);
    if (st == CNLOS_OK) g->run[i] = runs[0];
  }
  if (st != CNLOS_OK) {
    // park the slot again before giving it back
    if (m && !m->poisoned && m->ctl_host) {
      m->ctl_host->halt = 1;
      (void)hipMemcpyAsync(m->ctl, m->ctl_host, sizeof(DevCtl), hipMemcpyHostToDevice, g->st);
      (void)hipStreamSynchronize(g->st);
    }
    srv_complete(sv, g, i, st);
  }
  return st;
}

}  // namespace

extern "C" {

cnlos_status cnlos_server_create(void* arena_dev, uint64_t arena_bytes, int32_t slots,
                                 int32_t rounds, cnlos_server** out) {
  if (!out) return fail(CNLOS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!arena_dev || ((uintptr_t)arena_dev) % kAlign) return fail(CNLOS_EINVAL, "arena must be non-NULL and 256-byte aligned");
  if (slots < 1 || slots > 64) return fail(CNLOS_EINVAL, "slots must be in [1, 64]");
  if (rounds < 1) return fail(CNLOS_EINVAL, "rounds must be >= 1");
  cnlos_server* sv = new (std::nothrow) cnlos_server();
  if (!sv) return fail(CNLOS_ENOMEM, "host allocation failed");
  sv->arena.base = (uint8_t*)arena_dev;
  sv->arena.bytes = arena_bytes & ~(uint64_t)(kAlign - 1);
  sv->arena.holes.push_back({0, sv->arena.bytes});
  sv->K = slots;
  sv->rounds = rounds;
  *out = sv;
  return CNLOS_OK;
}

cnlos_status cnlos_server_submit(cnlos_server* sv, const cnlos_request* r) {
  if (!sv || !r) return fail(CNLOS_EINVAL, "NULL argument");
  cnlos_status st = cnlos_validate(&r->cfg, r->mask_host);
  if (st != CNLOS_OK) return st;
  if (!r->mask_host || !r->tau0_dev || !r->out_dev) return fail(CNLOS_EINVAL, "mask, measurement and output are required");
  if (r->cfg.model == CNLOS_MODEL_OPERATOR) return fail(CNLOS_EINVAL, "a request needs a solver model");
  if ((uint64_t)carve(nullptr, r->cfg, nullptr, false) * sv->K + hq_bytes(r->cfg) > sv->arena.bytes)
    return fail(CNLOS_ENOMEM, "a slot group of this shape does not fit the arena");
  SrvReq q;
  q.r = *r;
  q.mask.assign(r->mask_host, r->mask_host + (size_t)r->cfg.nx * r->cfg.ny);
  q.r.mask_host = nullptr;
  q.submitted = sv->step_no;
  sv->queue.push_back(std::move(q));
  return CNLOS_OK;
}

cnlos_status cnlos_server_step(cnlos_server* sv, int32_t* active, int32_t* queued) {
  if (!sv) return fail(CNLOS_EINVAL, "server is NULL");
  // Groups advance independently: a group whose rounds have finished is
  // absorbed, its finished requests retired, its free slots refilled and its
  // next rounds enqueued, while the other groups' rounds keep running.
  auto absorb = [&](SrvGroup* g) -> cnlos_status {
    g->busy = false;
    cnlos_status st = group_absorb(g->view, g->vruns);
    if (st != CNLOS_OK) return st;
    for (size_t j = 0; j < g->vidx.size(); ++j) g->run[g->vidx[j]] = g->vruns[j];
    return CNLOS_OK;
  };
  bool progressed = false;
  for (SrvGroup* g : sv->groups) {
    if (!g->busy) continue;
    const hipError_t q = hipEventQuery(g->done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(CNLOS_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    cnlos_status st = absorb(g);
    if (st != CNLOS_OK) return st;
    progressed = true;
  }
  // retire finished requests of idle groups: copy the volume out, free the slot
  auto retire = [&]() {
    for (SrvGroup* g : sv->groups) {
      if (g->busy) continue;
      for (int i = 0; i < g->K; ++i) {
        cnlos_problem* m = g->slot[i];
        if (!m || g->run[i].active) continue;
        cnlos_status st = g->run[i].status;
        if (st == CNLOS_OK) st = cnlos_get_volume(m, g->req[i].r.out_dev);
        if (hipStreamSynchronize(g->st) != hipSuccess && st == CNLOS_OK) st = fail(CNLOS_EHIP, "stream failed");
        srv_complete(sv, g, i, st);
      }
    }
  };
  retire();
  // admission, first come first served within each shape, into idle groups
  // (a request whose group is busy waits for its next step).  The queue is
  // rebuilt from the requests that keep waiting, so no exit path leaves an
  // admitted or moved-from request in it, and every request gets exactly one
  // completion.
  std::vector<SrvReq> pending;
  pending.swap(sv->queue);
  for (SrvReq& q : pending) {
    SrvGroup* g = nullptr;
    int free_slot = -1;
    bool shape_busy = false;
    for (SrvGroup* c : sv->groups) {
      if (!same_shared(c->proto, q.r.cfg) || !same_geometry(c->proto, q.r.cfg)) continue;
      if (c->busy) {
        shape_busy = true;
        continue;
      }
      for (int i = 0; i < c->K && free_slot < 0; ++i)
        if (!c->slot[i]) free_slot = i;
      if (free_slot >= 0) {
        g = c;
        break;
      }
    }
    if (!g && shape_busy) {
      sv->queue.push_back(std::move(q));
      continue;
    }
    if (!g) {
      cnlos_status st = srv_group_new(sv, q.r.cfg, &g);
      if (st == CNLOS_ENOMEM && !g) {
        // give back the arena of idle empty groups and try once more
        for (size_t k = 0; k < sv->groups.size();) {
          if (!sv->groups[k]->busy && sv->groups[k]->occupied() == 0) {
            srv_group_free(sv, sv->groups[k]);
            sv->groups.erase(sv->groups.begin() + k);
          } else {
            ++k;
          }
        }
        st = srv_group_new(sv, q.r.cfg, &g);
      }
      if (st == CNLOS_ENOMEM && !g) {
        sv->queue.push_back(std::move(q));
        continue;
      }
      if (st != CNLOS_OK) {
        // this request fails (its group could not be made); the others go on
        srv_reject(sv, q, st);
        continue;
      }
      free_slot = 0;
    }
    srv_admit(sv, g, free_slot, q);
  }
  // enqueue the next rounds of every idle group with occupants
  for (SrvGroup* g : sv->groups) {
    if (g->busy) continue;
    Group& v = g->view;
    v.lead = g->layout;
    v.bt = Batch{g->K, g->stride, G_NONE, true};
    v.mem.clear();
    g->vruns.clear();
    g->vidx.clear();
    for (int i = 0; i < g->K; ++i)
      if (g->slot[i] && g->run[i].active) {
        v.mem.push_back(g->slot[i]);
        g->vruns.push_back(g->run[i]);
        g->vidx.push_back(i);
      }
    if (v.mem.empty()) continue;
    bool e = false;
    cnlos_status st = group_enqueue(v, g->vruns, sv->rounds, &e);
    if (st != CNLOS_OK) return st;
    if (hipEventRecord(g->done, g->st) != hipSuccess) return fail(CNLOS_EHIP, "hipEventRecord failed");
    g->busy = true;
    g->busy_since = ++sv->enqueues;
    progressed = true;
  }
  // nothing finished and nothing could start: wait for the oldest rounds
  if (!progressed) {
    SrvGroup* oldest = nullptr;
    for (SrvGroup* g : sv->groups)
      if (g->busy && (!oldest || g->busy_since < oldest->busy_since)) oldest = g;
    if (oldest) {
      if (hipEventSynchronize(oldest->done) != hipSuccess) return fail(CNLOS_EHIP, "hipEventSynchronize failed");
      cnlos_status st = absorb(oldest);
      if (st != CNLOS_OK) return st;
      retire();
    }
  }
  ++sv->step_no;
  int act = 0;
  for (SrvGroup* g : sv->groups) act += g->occupied();
  if (active) *active = act;
  if (queued) *queued = (int32_t)sv->queue.size();
  return CNLOS_OK;
}

cnlos_status cnlos_server_fail_next_groups(cnlos_server* sv, int32_t count) {
  if (!sv || count < 0) return fail(CNLOS_EINVAL, "NULL server or negative count");
  sv->fail_next_groups = count;
  return CNLOS_OK;
}

cnlos_status cnlos_server_poll(cnlos_server* sv, cnlos_completion* out, int32_t cap, int32_t* n) {
  if (!sv || !n || (cap > 0 && !out)) return fail(CNLOS_EINVAL, "NULL argument");
  const int k = std::min<int>(cap, (int)sv->done.size());
  for (int i = 0; i < k; ++i) out[i] = sv->done[i];
  sv->done.erase(sv->done.begin(), sv->done.begin() + k);
  *n = k;
  return CNLOS_OK;
}

cnlos_status cnlos_server_usage(cnlos_server* sv, uint64_t* bytes_used, int32_t* groups) {
  if (!sv) return fail(CNLOS_EINVAL, "server is NULL");
  if (bytes_used) *bytes_used = sv->arena.used;
  if (groups) *groups = (int32_t)sv->groups.size();
  return CNLOS_OK;
}

cnlos_status cnlos_server_destroy(cnlos_server* sv) {
  if (!sv) return CNLOS_OK;
  for (SrvGroup* g : sv->groups) srv_group_free(sv, g);
  delete sv;
  return CNLOS_OK;
}

}  // extern "C"

namespace {

cnlos_status destroy_problem(cnlos_problem* p) {
  if (p->ctl_host) {
    if (!p->poisoned) (void)hipStreamSynchronize(p->st);
    (void)hipHostFree(p->ctl_host);
  }
  p->prof.release();
  delete p;
  return CNLOS_OK;
}

}  // namespace
