// ADMM stencil and control kernels (Sections 3.1-3.2 and 4.1).
//
// Volumes are [n][n][m] float32 with t fastest; every difference operator is
// periodic with unit spacing (the periodicity is what makes the FFT solve of
// eq. (11) exact).  nabla is the forward difference, nabla^* its adjoint
// (minus the backward-difference divergence).  Reductions accumulate in FP64
// and are combined in a fixed order, so results are bitwise reproducible.
#include <math.h>

#include "cnlos_internal.h"
#include "fft_device.h"
#include "stencil_device.h"

namespace cnlos {

constexpr int kStencilThreads = 256;
constexpr int kCtlThreads = 1024;

// Blocks of the stencil kernels: one thread per voxel (bin pair) up to a cap
// that the volume sets.  Each block walks a contiguous range of bin pairs, and
// all blocks of an XCD read the neighbour rows of each other's ranges at
// about the same time, so how many run at once decides whether those reads
// still find the data in L2.  Measured for the post kernels: 2048 blocks at
// 2^21 voxels (64x64x512: 42.4 against 45.4 us per launch with 1024), 512 at
// 2^24 (128x128x1024: 442 against 463 us); 1024 between.  The count is fixed
// by the shape, so results do not depend on timing.
int stencil_blocks(int logn, int logm) {
  const int logv = 2 * logn + logm;
  const size_t V = (size_t)1 << logv;
  const size_t cap = logv <= 21 ? 2048 : (logv >= 24 ? 512 : 1024);
  size_t nb = (V + kStencilThreads - 1) / kStencilThreads;
  if (nb > cap) nb = cap;
  return (int)nb;
}

// Common head of the iteration kernels: shift the controller to this launch's
// scene, apply the phase gate, and (first kernel of an iteration slot) clear
// the previous slot's rejection.
__device__ __forceinline__ bool iter_gate(DevCtl* ctl, const CtlHead& hd, int gate) {
  if (gated_off(hd, gate)) return false;
  if ((gate & G_FIRST) && blockIdx.x == 0 && threadIdx.x == 0) ctl->reject = 0;
  return true;
}
__device__ __forceinline__ bool iter_head(DevCtl*& ctl, size_t zo, int gate) {
  ctl = zsh(ctl, zo);
  return iter_gate(ctl, ctl_head(ctl), gate);
}
// Backtracking decision (Beck-Teboulle).  For the quadratic data term f the
// sufficient-decrease test f(u+) <= f(ubar) + <u+ - ubar, grad f(ubar)> +
// L/2 |u+ - ubar|^2 is exactly |B (u+ - ubar)|^2 <= L |u+ - ubar|^2, B = A_D
// (object) or A (dual); the left side comes from the difference of A u+ and
// the cached A ubar, free of the cancellation of the literal form.  Every
// block of the post kernel takes the decision from the same fixed-order FP64
// sums of the check and step partials, so all blocks agree; L changes only in
// k_finalize, after the post kernel.
enum Decision : int { D_ACCEPT = 0, D_REJECT = 1, D_NONFINITE = 2 };
__device__ __forceinline__ int check_decision(const double* __restrict__ partials,
                                              const CheckArgs& ck, double L) {
  constexpr int NW = kStencilThreads / 64;
  __shared__ double red[2][NW];
  __shared__ int dec;
  // both slots' loads of four steps of kStencilThreads partials issue
  // together: index clamped, value masked (a load under a per-lane condition
  // compiles to a branch with a wait after it; the masked zeros leave the
  // sums unchanged)
  constexpr int kSteps = 4;
  const double* pc = partials + (size_t)SL_CHECK * kMaxBlocks;
  const double* ps = partials + (size_t)SL_STEP * kMaxBlocks;
  const int nmax = ck.nb_conv > ck.nb_step ? ck.nb_conv : ck.nb_step;
  double a = 0.0, b = 0.0;
  for (int base = 0; base < nmax; base += kSteps * kStencilThreads) {
    double va[kSteps], vb[kSteps];
#pragma unroll
    for (int j = 0; j < kSteps; ++j) {
      const int i = base + j * kStencilThreads + threadIdx.x;
      va[j] = pc[i < ck.nb_conv ? i : 0];
      vb[j] = ps[i < ck.nb_step ? i : 0];
    }
#pragma unroll
    for (int j = 0; j < kSteps; ++j) {
      const int i = base + j * kStencilThreads + threadIdx.x;
      a += i < ck.nb_conv ? va[j] : 0.0;
      b += i < ck.nb_step ? vb[j] : 0.0;
    }
  }
  double ab[2] = {a, b};
  wave_sum_n<2>(ab);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = ab[0];
    red[1][wid] = ab[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      sa += red[0][w];
      sb += red[1][w];
    }
    dec = (!isfinite(sa) || !isfinite(sb)) ? D_NONFINITE
          : (ck.bt_on && !(sa <= L * sb)) ? D_REJECT
                                          : D_ACCEPT;
  }
  __syncthreads();
  return dec;
}

// The post kernel's blocks stop at a rejected or non-finite trial; block 0
// records the outcome (the rest of the slot is then a no-op, and k_finalize
// does the bookkeeping of a rejection).
__device__ __forceinline__ bool trial_accepted(DevCtl* ctl, const double* partials,
                                               const CheckArgs& ck, double L) {
  const int dec = check_decision(partials, ck, L);
  if (dec == D_ACCEPT) return true;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (dec == D_NONFINITE) {
      ctl->halt = 1;
      ctl->reason = HR_NONFINITE;
    } else {
      ctl->reject = 1;
    }
  }
  return false;
}

__device__ __forceinline__ float* vol_at(const Vol& v, const DevCtl* c, size_t zo) {
  return vol_resolve(v, c, zo);
}

// derived fields on request: v (or w) and f from the current state
__global__ void __launch_bounds__(kStencilThreads)
k_vstep(const float* __restrict__ xb, const float* __restrict__ lam, const float* __restrict__ phi,
        float* __restrict__ v, float inv_mu, int logn, int logm) {
  const size_t V = (size_t)1 << (2 * logn + logm);
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < V;
       g += (size_t)gridDim.x * blockDim.x) {
    float vx, vy, vt;
    v_at(xb, lam, phi, inv_mu, g, V, logn, logm, vx, vy, vt);
    v[g] = vx;
    v[V + g] = vy;
    v[2 * V + g] = vt;
  }
}

__global__ void __launch_bounds__(kStencilThreads)
k_fstep(const float* __restrict__ taubar, const float* __restrict__ lam3,
        const float* __restrict__ tau0, const uint8_t* __restrict__ mask, float* __restrict__ f,
        float lambda, float mu3, int logn, int logm) {
  const size_t V = (size_t)1 << (2 * logn + logm);
  const float inv_kept = 1.f / (lambda + mu3), inv_mu3 = 1.f / mu3;
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < V;
       g += (size_t)gridDim.x * blockDim.x)
    f[g] = f_at(taubar[g], lam3[g], tau0[g], mask[g >> logm] != 0, lambda, mu3, inv_kept, inv_mu3);
}

// Contiguous range of bin pairs of this block: XCD-aware order, so that the
// blocks of one XCD cover one contiguous part of the volume and the x / y
// neighbour columns a pair reads are mostly in that XCD's L2.
struct PairRange {
  uint32_t q0, q1;
};
__device__ __forceinline__ PairRange pair_range(uint32_t P) {
  const uint32_t nb = gridDim.x, L = xcd_block(blockIdx.x, nb);
  const uint32_t chunk = ((P + nb - 1) / nb + blockDim.x - 1) / blockDim.x * blockDim.x;
  PairRange r;
  r.q0 = min(P, L * chunk);
  r.q1 = min(P, r.q0 + chunk);
  return r;
}

// After the accepted step: multiplier ascent (eq. (12)), FISTA extrapolation,
// curvature weight refresh, and the FP64 energy/residual partials, on the bin
// pair (k, k + 1) of one scan column.
// u mode : Lambda += mu (v - grad x+), xbar', phi_u; partials TV_U, PRIMAL, DUAL.
// tau mode: Lambda2 += mu2 (w - grad tau+), Lambda3 += mu3 (f - tau+), taubar',
//           phi_tau; partials TV_TAU, FIT (|A u+ - tau+|^2), FID (|D(tau+ - tau0)|^2).
// v (w) and f are those of this iteration: recomputed from the xbar, Lambda and
// phi the iteration started from, read here before they are overwritten.
// The curvature kappa = div^-( grad x+ / sqrt(|grad x+|^2 + eta^2) ) needs the
// gradient at the voxel and at its x - 1, y - 1 and t - 1 neighbours; for bin
// k + 1 the t - 1 neighbour is bin k.
template <bool TAU>
__device__ __forceinline__ void post_pair(const float* __restrict__ xn,
                                          const float* __restrict__ xo,
                                          const float* __restrict__ xb, float* __restrict__ lam,
                                          float* __restrict__ xbn, float* __restrict__ phi,
                                          float mu, const PhiArgs& pa, float eta2, float beta,
                                          float* __restrict__ lam3, float mu3, float lambda,
                                          const float* __restrict__ au,
                                          const float* __restrict__ tau0,
                                          const uint8_t* __restrict__ mask, uint32_t V,
                                          const PairOff& o, double& s_tv, double& s_a,
                                          double& s_b) {
  const uint32_t ck = o.c + o.k;
  // v = shrink(grad xbar - Lambda/mu, phi/mu) at both bins (eq. (7))
  const float inv_mu = 1.f / mu;
  const float2 b0 = ld2(xb, ck), bx = ld2(xb, o.cxp + o.k), by = ld2(xb, o.cyp + o.k);
  const float bn = ld1(xb, o.c + o.kn);
  const float2 l0 = ld2(lam, ck), l1 = ld2(lam, V + ck), l2 = ld2(lam, 2 * V + ck);
  const float2 p0 = ld2(phi, ck);
  const float gb[2][3] = {{bx.x - b0.x, by.x - b0.x, b0.y - b0.x},
                          {bx.y - b0.y, by.y - b0.y, bn - b0.y}};
  const float lm[2][3] = {{l0.x, l1.x, l2.x}, {l0.y, l1.y, l2.y}};
  const float pold[2] = {p0.x, p0.y};
  float v[2][3];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float ax = gb[h][0] - lm[h][0] * inv_mu;
    const float ay = gb[h][1] - lm[h][1] * inv_mu;
    const float at = gb[h][2] - lm[h][2] * inv_mu;
    const float sh = shrink_factor(ax * ax + ay * ay + at * at, pold[h] * inv_mu);
    v[h][0] = ax * sh;
    v[h][1] = ay * sh;
    v[h][2] = at * sh;
  }
  // gradients of x+ at the pair and at the neighbours the curvature reaches
  const float2 a = ld2(xn, ck), ax = ld2(xn, o.cxp + o.k), ay = ld2(xn, o.cyp + o.k);
  const float an = ld1(xn, o.c + o.kn);
  const float2 mx = ld2(xn, o.cxm + o.k), mxy = ld2(xn, o.cxmyp + o.k);
  const float mxn = ld1(xn, o.cxm + o.kn);
  const float2 my = ld2(xn, o.cym + o.k), myx = ld2(xn, o.cymxp + o.k);
  const float myn = ld1(xn, o.cym + o.kn);
  const float tm = ld1(xn, o.c + o.km), tmx = ld1(xn, o.cxp + o.km), tmy = ld1(xn, o.cyp + o.km);
  const float x0[2] = {a.x, a.y};
  const float g[2][3] = {{ax.x - a.x, ay.x - a.x, a.y - a.x}, {ax.y - a.y, ay.y - a.y, an - a.y}};
  const float gxm[2][3] = {{a.x - mx.x, mxy.x - mx.x, mx.y - mx.x},
                           {a.y - mx.y, mxy.y - mx.y, mxn - mx.y}};
  const float gym[2][3] = {{myx.x - my.x, a.x - my.x, my.y - my.x},
                           {myx.y - my.y, a.y - my.y, myn - my.y}};
  const float gtm[3] = {tmx - tm, tmy - tm, a.x - tm};
  auto n2 = [](const float (&q)[3]) { return q[0] * q[0] + q[1] * q[1] + q[2] * q[2]; };
  float i0[2], ph[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) i0[h] = rsq(n2(g[h]) + eta2);
  const float ntm[2] = {gtm[2] * rsq(n2(gtm) + eta2), g[0][2] * i0[0]};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float nxm = gxm[h][0] * rsq(n2(gxm[h]) + eta2);
    const float nym = gym[h][1] * rsq(n2(gym[h]) + eta2);
    const float kappa = (g[h][0] * i0[h] - nxm) + (g[h][1] * i0[h] - nym) + (g[h][2] * i0[h] - ntm[h]);
    ph[h] = phi_eval(kappa, pa);
  }
  st2(phi, ck, make_float2(ph[0], ph[1]));
  st2(lam, ck, make_float2(l0.x + mu * (v[0][0] - g[0][0]), l0.y + mu * (v[1][0] - g[1][0])));
  st2(lam, V + ck, make_float2(l1.x + mu * (v[0][1] - g[0][1]), l1.y + mu * (v[1][1] - g[1][1])));
  st2(lam, 2 * V + ck,
      make_float2(l2.x + mu * (v[0][2] - g[0][2]), l2.y + mu * (v[1][2] - g[1][2])));
  const float2 q0 = ld2(xo, ck);
  const float d[2] = {a.x - q0.x, a.y - q0.y};
  st2(xbn, ck, make_float2(a.x + beta * d[0], a.y + beta * d[1]));
#pragma unroll
  for (int h = 0; h < 2; ++h) s_tv += (double)ph[h] * (double)__builtin_amdgcn_sqrtf(n2(g[h]));
  if (!TAU) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float rx = v[h][0] - g[h][0], ry = v[h][1] - g[h][1], rt = v[h][2] - g[h][2];
      s_a += (double)rx * rx + (double)ry * ry + (double)rt * rt;
    }
    const float2 qx = ld2(xo, o.cxp + o.k), qy = ld2(xo, o.cyp + o.k);
    const float qn = ld1(xo, o.c + o.kn);
    const float dn[2][3] = {{(ax.x - qx.x) - d[0], (ay.x - qy.x) - d[0], d[1] - d[0]},
                            {(ax.y - qx.y) - d[1], (ay.y - qy.y) - d[1], (an - qn) - d[1]}};
#pragma unroll
    for (int h = 0; h < 2; ++h)
      s_b += (double)dn[h][0] * dn[h][0] + (double)dn[h][1] * dn[h][1] +
             (double)dn[h][2] * dn[h][2];
  } else {
    const bool kept = mask[o.col] != 0;
    const float2 l3 = ld2(lam3, ck), t0 = ld2(tau0, ck), av = ld2(au, ck);
    const float ik = 1.f / (lambda + mu3), im = 1.f / mu3;
    const float f0 = f_at(b0.x, l3.x, t0.x, kept, lambda, mu3, ik, im);
    const float f1 = f_at(b0.y, l3.y, t0.y, kept, lambda, mu3, ik, im);
    st2(lam3, ck, make_float2(l3.x + mu3 * (f0 - x0[0]), l3.y + mu3 * (f1 - x0[1])));
    const float r0 = av.x - x0[0], r1 = av.y - x0[1];
    s_a += (double)r0 * r0;
    s_a += (double)r1 * r1;
    if (kept) {
      const float e0 = x0[0] - t0.x, e1 = x0[1] - t0.y;
      s_b += (double)e0 * e0;
      s_b += (double)e1 * e1;
    }
  }
}

// Algorithm 1's updates after the accepted step (u side).
__global__ void __launch_bounds__(kStencilThreads)
k_post(PostArgs pu, double* __restrict__ partials, CheckArgs ck, int logn, int logm, DevCtl* ctl,
       size_t zs, int gate) {
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  const double L = ctl->L, t = ctl->t;
  const float* xn = vol_resolve(pu.xn, hd, zo);
  const float* xo = vol_resolve(pu.xo, hd, zo);
  const float* xb = vol_resolve(pu.xb, hd, zo);
  float* xbn = vol_resolve(pu.xbn, hd, zo);
  if (!iter_gate(ctl, hd, gate)) return;
  partials = zsh(partials, zo);
  if (!trial_accepted(ctl, partials, ck, L)) return;
  pu.lam = zsh(pu.lam, zo);
  pu.phi = zsh(pu.phi, zo);
  const uint32_t V = 1u << (2 * logn + logm), P = V / 2;
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  const float beta = (float)((t - 1.0) / tn);
  const float eta2 = pu.pa.eta * pu.pa.eta;
  double s_tv = 0.0, s_a = 0.0, s_b = 0.0;
  const PairRange pr = pair_range(P);
  for (uint32_t q = pr.q0 + threadIdx.x; q < pr.q1; q += blockDim.x)
    post_pair<false>(xn, xo, xb, pu.lam, xbn, pu.phi, pu.mu, pu.pa, eta2, beta, nullptr, 0.f,
                     0.f, nullptr, nullptr, nullptr, V, pair_offsets(q, logn, logm), s_tv, s_a,
                     s_b);
  double vals[3] = {s_tv, s_a, s_b};
  const int slots[3] = {SL_TV_U, SL_PRIMAL, SL_DUAL};
  block_sum_store<3>(vals, partials, slots, kMaxBlocks);
}

// Algorithm 2's updates after the accepted step, u side and tau side in one pass.
__global__ void __launch_bounds__(kStencilThreads)
k_post_dual(PostArgs pu, PostArgs pt, float* __restrict__ lam3, float mu3, float lambda,
            Vol au_v, const float* __restrict__ tau0, const uint8_t* __restrict__ mask,
            double* __restrict__ partials, CheckArgs ck, int logn, int logm, DevCtl* ctl,
            size_t zs, int gate) {
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  const double L = ctl->L, t = ctl->t;
  const float* uxn = vol_resolve(pu.xn, hd, zo);
  const float* uxo = vol_resolve(pu.xo, hd, zo);
  const float* uxb = vol_resolve(pu.xb, hd, zo);
  float* uxbn = vol_resolve(pu.xbn, hd, zo);
  const float* txn = vol_resolve(pt.xn, hd, zo);
  const float* txo = vol_resolve(pt.xo, hd, zo);
  const float* txb = vol_resolve(pt.xb, hd, zo);
  float* txbn = vol_resolve(pt.xbn, hd, zo);
  const float* au = vol_resolve(au_v, hd, zo);
  if (!iter_gate(ctl, hd, gate)) return;
  partials = zsh(partials, zo);
  if (!trial_accepted(ctl, partials, ck, L)) return;
  pu.lam = zsh(pu.lam, zo);
  pu.phi = zsh(pu.phi, zo);
  pt.lam = zsh(pt.lam, zo);
  pt.phi = zsh(pt.phi, zo);
  lam3 = zsh(lam3, zo);
  tau0 = zsh(tau0, zo);
  mask = zsh(mask, zo);
  const uint32_t V = 1u << (2 * logn + logm), P = V / 2;
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  const float beta = (float)((t - 1.0) / tn);
  const float eu = pu.pa.eta * pu.pa.eta, et = pt.pa.eta * pt.pa.eta;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const PairRange pr = pair_range(P);
  for (uint32_t q = pr.q0 + threadIdx.x; q < pr.q1; q += blockDim.x) {
    const PairOff o = pair_offsets(q, logn, logm);
    post_pair<false>(uxn, uxo, uxb, pu.lam, uxbn, pu.phi, pu.mu, pu.pa, eu, beta, nullptr, 0.f,
                     0.f, nullptr, nullptr, nullptr, V, o, s[0], s[1], s[2]);
    post_pair<true>(txn, txo, txb, pt.lam, txbn, pt.phi, pt.mu, pt.pa, et, beta, lam3, mu3,
                    lambda, au, tau0, mask, V, o, s[3], s[4], s[5]);
  }
  const int slots[6] = {SL_TV_U, SL_PRIMAL, SL_DUAL, SL_TV_TAU, SL_FIT, SL_FID};
  block_sum_store<6>(s, partials, slots, kMaxBlocks);
}

// phi = phi(kappa(x)) (warm-start hand-over and resets)
__global__ void __launch_bounds__(kStencilThreads)
k_phi_of(const float* __restrict__ x, float* __restrict__ phi, PhiArgs pa, int logn, int logm) {
  const size_t V = (size_t)1 << (2 * logn + logm);
  const float eta2 = pa.eta * pa.eta;
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < V;
       g += (size_t)gridDim.x * blockDim.x) {
    const Nbr nb = neighbours(g, logn, logm);
  float gx, gy, gt;
    phi[g] = phi_eval(curvature_at(x, g, nb, logn, logm, eta2, gx, gy, gt), pa);
  }
}

// After a rejected trial: one more trial for this iteration with L doubled,
// or a halt when the trials are exhausted.  After an accepted one: energy,
// residuals, log row, FISTA t update, stopping rule.
__global__ void __launch_bounds__(kCtlThreads)
k_finalize(DevCtl* ctl, double* __restrict__ logbuf, const double* __restrict__ partials,
           int nb_conv, int nb_sten, int dual, double lambda, double mu_res, size_t zs, int gate) {
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  logbuf = zsh(logbuf, zo);
  partials = zsh(partials, zo);
  // every controller field thread 0 needs is read up front, with the gate
  // fields (not after the reduction's barriers)
  const CtlHead hd = ctl_head(ctl);
  const double Ep = ctl->energy_prev, L = ctl->L, t = ctl->t, eps_stop = ctl->eps_stop;
  const double bt_factor = ctl->bt_factor;
  const int log_count = ctl->log_count, bt_rejects = ctl->bt_rejects, bt_max = ctl->bt_max_trials;
  if (!iter_gate(ctl, hd, gate)) return;
  if (hd.reject) {
    if (threadIdx.x == 0) {
      const int trials = hd.trials + 1;
      ctl->trials = trials;
      ctl->bt_rejects = bt_rejects + 1;
      if (trials > bt_max) {
        ctl->halt = 1;
        ctl->reason = HR_BACKTRACK;
      } else {
        // the next slot repeats the iteration
        ctl->L = L * bt_factor;
      }
    }
    return;
  }
  double E, prim, dres;
  if (!dual) {
    const int slots[4] = {SL_TV_U, SL_PRIMAL, SL_DUAL, SL_DATA};
    const int nbs[4] = {nb_sten, nb_sten, nb_sten, nb_conv};
    double v[4];
    block_sum_partials_k<4>(partials, slots, nbs, kMaxBlocks, v);
    prim = v[1];
    dres = v[2];
    E = 0.5 * v[3] + v[0];
  } else {
    const int slots[6] = {SL_TV_U, SL_PRIMAL, SL_DUAL, SL_FIT, SL_FID, SL_TV_TAU};
    const int nbs[6] = {nb_sten, nb_sten, nb_sten, nb_sten, nb_sten, nb_sten};
    double v[6];
    block_sum_partials_k<6>(partials, slots, nbs, kMaxBlocks, v);
    prim = v[1];
    dres = v[2];
    E = 0.5 * v[3] + 0.5 * lambda * v[4] + v[0] + v[5];
  }
  if (threadIdx.x == 0) {
    if (!isfinite(E)) {
      ctl->halt = 1;
      ctl->reason = HR_NONFINITE;
      return;
    }
    const double rel = (isfinite(Ep) && E != 0.0) ? fabs(Ep - E) / fabs(E) : INFINITY;
    const double primal = sqrt(prim), dualr = mu_res * sqrt(dres);
    double* row = logbuf + (size_t)(log_count % kLogRows) * kLogCols;
    row[0] = E;
    row[1] = primal;
    row[2] = dualr;
    row[3] = L;
    row[4] = (double)hd.trials;
    row[5] = rel;
    ctl->log_count = log_count + 1;
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    ctl->beta = (t - 1.0) / tn;
    // optional momentum restart after an energy rise: the next extrapolation
    // weight is 0 (off: the printed extrapolation)
    const double rtol = ctl->restart_tol;
    const bool restart = rtol > 0.0 && isfinite(Ep) && E > Ep * (1.0 + rtol);
    ctl->t = restart ? 1.0 : tn;
    ctl->iter = hd.iter + 1;
    ctl->trials = 0;
    // the trial becomes the current iterate (buffer roles rotate)
    ctl->slot[R_U_CUR] = hd.slot[R_U_TR];
    ctl->slot[R_U_TR] = hd.slot[R_U_CUR];
    ctl->slot[R_AU_PREV] = hd.slot[R_AU_CUR];
    ctl->slot[R_AU_CUR] = hd.slot[R_AU_TR];
    ctl->slot[R_AU_TR] = hd.slot[R_AU_PREV];
    ctl->slot[R_T_CUR] = hd.slot[R_T_TR];
    ctl->slot[R_T_TR] = hd.slot[R_T_CUR];
    ctl->slot[R_UB_CUR] = hd.slot[R_UB_NEW];
    ctl->slot[R_UB_NEW] = hd.slot[R_UB_CUR];
    ctl->slot[R_TB_CUR] = hd.slot[R_TB_NEW];
    ctl->slot[R_TB_NEW] = hd.slot[R_TB_CUR];
    ctl->energy_prev = E;
    ctl->last_energy = E;
    ctl->last_primal = primal;
    ctl->last_dual = dualr;
    if (eps_stop > 0.0 && rel <= eps_stop) {
      ctl->halt = 1;
      ctl->reason = HR_STOP;
    }
  }
}

// Hand-over from the Algorithm-1 warm start to Algorithm 2, due once the warm
// start's iterations are done and before the first Algorithm-2 iteration
// (idempotent: the last of its kernels leaves stage 1).
__device__ __forceinline__ bool transition_due(const DevCtl* c) {
  return !c->halt && c->stage == 1 && c->iter == c->stage1_end && c->iter < c->target;
}

// ubar = u, phi_u = phi(kappa(u)), phi_tau = phi(0); tau, taubar, w, f and the
// multipliers are zeroed by k_zero_if_stage1.
__global__ void __launch_bounds__(kStencilThreads)
k_transition_fields(const DevCtl* ctl, Vol u_v, Vol ubar_v,
                    float* __restrict__ phi_u, PhiArgs pa, float* __restrict__ phi_tau,
                    float phi_tau0, int logn, int logm, size_t zs) {
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  if (!transition_due(ctl)) return;
  const float* __restrict__ u = vol_resolve(u_v, ctl, zo);
  float* __restrict__ ubar = vol_resolve(ubar_v, ctl, zo);
  phi_u = zsh(phi_u, zo);
  phi_tau = zsh(phi_tau, zo);
  const size_t V = (size_t)1 << (2 * logn + logm);
  const float eta2 = pa.eta * pa.eta;
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < V;
       g += (size_t)gridDim.x * blockDim.x) {
    const Nbr nb = neighbours(g, logn, logm);
  float gx, gy, gt;
    phi_u[g] = phi_eval(curvature_at(u, g, nb, logn, logm, eta2, gx, gy, gt), pa);
    ubar[g] = u[g];
    phi_tau[g] = phi_tau0;
  }
}

__global__ void __launch_bounds__(kStencilThreads)
k_zero_if_stage1(const DevCtl* ctl, float* __restrict__ x, size_t n, size_t zs) {
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  if (!transition_due(ctl)) return;
  x = zsh(x, zo);
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x)
    x[g] = 0.f;
}

__global__ void k_transition_scalars(DevCtl* ctl, size_t zs) {
  ctl = zsh(ctl, (size_t)blockIdx.z * zs);
  if (!transition_due(ctl)) return;
  ctl->stage = 2;
  ctl->t = 1.0;
  ctl->beta = 0.0;
  ctl->L = ctl->L0_dual;
  ctl->trials = 0;
  ctl->energy_prev = NAN;
}

__global__ void __launch_bounds__(kStencilThreads) k_fill(float* __restrict__ x, size_t n, float val) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x)
    x[g] = val;
}

__global__ void __launch_bounds__(kStencilThreads)
k_copy(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x)
    dst[g] = src[g];
}

// measurement: out = mask * r3[k] * raw; partial max and non-finite count
__global__ void __launch_bounds__(kStencilThreads)
k_meas_prep(const float* __restrict__ raw, const uint8_t* __restrict__ mask,
            const float* __restrict__ r3, float* __restrict__ out, double* __restrict__ partials,
            int logn, int logm) {
  const size_t V = (size_t)1 << (2 * logn + logm);
  const size_t M = (size_t)1 << logm;
  float mx = 0.f;
  double bad = 0.0;
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < V;
       g += (size_t)gridDim.x * blockDim.x) {
    const float x = raw[g];
    if (!isfinite(x)) bad += 1.0;
    float y = mask[g >> logm] ? x : 0.f;
    if (r3) y *= r3[g & (M - 1)];
    out[g] = y;
    mx = fmaxf(mx, y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  __shared__ float redm[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) redm[wid] = mx;
  double vals[1] = {bad};
  const int slots[1] = {SL_BAD};
  block_sum_store<1>(vals, partials, slots, kMaxBlocks);   // contains a barrier
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) m = fmaxf(m, redm[k]);
    partials[(size_t)SL_MAX * kMaxBlocks + blockIdx.x] = (double)m;
  }
}

__global__ void __launch_bounds__(256)
k_meas_reduce(DevCtl* ctl, const double* __restrict__ partials, int nb) {
  const double bad = block_sum_partials(partials, SL_BAD, nb, kMaxBlocks);
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    m = fmax(m, partials[(size_t)SL_MAX * kMaxBlocks + i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  __shared__ double redm[4];
  if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, redm[k]);
    m = fmax(m, redm[0]);
    ctl->meas_scale = m;
    ctl->reason = bad > 0.0 ? HR_NONFINITE : HR_NONE;
  }
}

__global__ void __launch_bounds__(kStencilThreads)
k_meas_scale(float* __restrict__ out, const DevCtl* ctl, int logn, int logm) {
  const double s = ctl->meas_scale;
  if (!(s > 0.0) || ctl->reason != HR_NONE) return;
  const float inv = (float)(1.0 / s);
  const size_t V = (size_t)1 << (2 * logn + logm);
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < V;
       g += (size_t)gridDim.x * blockDim.x)
    out[g] *= inv;
}

__global__ void __launch_bounds__(256) k_pow_finalize(DevCtl* ctl, const double* __restrict__ partials,
                                                      int nb, size_t zs) {
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  partials = zsh(partials, zo);
  const double s = block_sum_partials(partials, SL_NORM, nb, kMaxBlocks);
  if (threadIdx.x == 0) ctl->pow_est = sqrt(s);
}

__global__ void k_clear_halt(DevCtl* ctl) {
  ctl->halt = 0;
  ctl->reason = HR_NONE;
}

// ---------------------------------------------------------------- launchers
static dim3 sgrid(int logn, int logm) { return dim3(stencil_blocks(logn, logm)); }

static dim3 sgrid_z(int logn, int logm, const Batch& bt) {
  return dim3(stencil_blocks(logn, logm), 1, bt.nz);
}

hipError_t launch_vstep(int logn, int logm, const float* xbar, const float* lam, const float* phi,
                        float* v, double mu, hipStream_t st) {
  hipLaunchKernelGGL(k_vstep, sgrid(logn, logm), dim3(kStencilThreads), 0, st, xbar, lam, phi, v,
                     (float)(1.0 / mu), logn, logm);
  return hipGetLastError();
}

hipError_t launch_fstep(int logn, int logm, const float* taubar, const float* lam3,
                        const float* tau0, const uint8_t* mask, float* f, double lambda,
                        double mu3, hipStream_t st) {
  hipLaunchKernelGGL(k_fstep, sgrid(logn, logm), dim3(kStencilThreads), 0, st, taubar, lam3, tau0,
                     mask, f, (float)lambda, (float)mu3, logn, logm);
  return hipGetLastError();
}

hipError_t launch_post_dual(int logn, int logm, const PostArgs& pu, const PostArgs& pt,
                            float* lam3, double mu3, double lambda, Vol au, const float* tau0,
                            const uint8_t* mask, double* partials, const CheckArgs& ck,
                            const DevCtl* ctl, const Batch& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_post_dual, sgrid_z(logn, logm, bt), dim3(kStencilThreads), 0, st, pu, pt,
                     lam3, (float)mu3, (float)lambda, au, tau0, mask, partials, ck, logn, logm,
                     const_cast<DevCtl*>(ctl), bt.zs, bt.gate);
  return hipGetLastError();
}


hipError_t launch_post(int logn, int logm, const PostArgs& pa, double* partials,
                       const CheckArgs& ck, const DevCtl* ctl, const Batch& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_post, sgrid_z(logn, logm, bt), dim3(kStencilThreads), 0, st, pa, partials,
                     ck, logn, logm, const_cast<DevCtl*>(ctl), bt.zs, bt.gate);
  return hipGetLastError();
}

hipError_t launch_finalize(DevCtl* ctl, double* log, const double* partials, int nb_conv,
                           int nb_sten, int dual, double lambda, double mu_res, const Batch& bt,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1, 1, bt.nz), dim3(kCtlThreads), 0, st, ctl, log, partials,
                     nb_conv, nb_sten, dual, lambda, mu_res, bt.zs, bt.gate);
  return hipGetLastError();
}

hipError_t launch_transition(int logn, int logm, DevCtl* ctl, Vol u, Vol ubar,
                             float* phi_u, const PhiArgs& pa_u, float* phi_tau, double phi_tau0,
                             float* const* zero_fields, const size_t* zero_counts, int nzero,
                             const Batch& bt, hipStream_t st) {
  hipLaunchKernelGGL(k_transition_fields, sgrid_z(logn, logm, bt), dim3(kStencilThreads), 0, st,
                     ctl, u, ubar, phi_u, pa_u, phi_tau, (float)phi_tau0, logn, logm, bt.zs);
  for (int i = 0; i < nzero; ++i) {
    size_t nb = (zero_counts[i] + kStencilThreads - 1) / kStencilThreads;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_zero_if_stage1, dim3((unsigned)nb, 1, bt.nz), dim3(kStencilThreads), 0,
                       st, ctl, zero_fields[i], zero_counts[i], bt.zs);
  }
  hipLaunchKernelGGL(k_transition_scalars, dim3(1, 1, bt.nz), dim3(1), 0, st, ctl, bt.zs);
  return hipGetLastError();
}

hipError_t launch_fill(float* x, size_t n, float val, hipStream_t st) {
  size_t nb = (n + kStencilThreads - 1) / kStencilThreads;
  if (nb > 4096) nb = 4096;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(kStencilThreads), 0, st, x, n, val);
  return hipGetLastError();
}

hipError_t launch_copy(float* dst, const float* src, size_t n, hipStream_t st) {
  size_t nb = (n + kStencilThreads - 1) / kStencilThreads;
  if (nb > 4096) nb = 4096;
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(kStencilThreads), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_phi_of_u(int logn, int logm, const float* u, float* phi, const PhiArgs& pa,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_phi_of, sgrid(logn, logm), dim3(kStencilThreads), 0, st, u, phi, pa, logn,
                     logm);
  return hipGetLastError();
}

hipError_t launch_meas_prep(int logn, int logm, const float* raw, const uint8_t* mask,
                            const float* r3, float* out, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(k_meas_prep, sgrid(logn, logm), dim3(kStencilThreads), 0, st, raw, mask, r3,
                     out, partials, logn, logm);
  return hipGetLastError();
}

hipError_t launch_meas_finish(int logn, int logm, float* out, DevCtl* ctl, double* partials,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_meas_reduce, dim3(1), dim3(256), 0, st, ctl, partials,
                     stencil_blocks(logn, logm));
  hipLaunchKernelGGL(k_meas_scale, sgrid(logn, logm), dim3(kStencilThreads), 0, st, out, ctl, logn,
                     logm);
  return hipGetLastError();
}

hipError_t launch_pow_finalize(DevCtl* ctl, const double* partials, int nb, const Batch& bt,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_pow_finalize, dim3(1, 1, bt.nz), dim3(256), 0, st, ctl, partials, nb, bt.zs);
  return hipGetLastError();
}

hipError_t launch_ctl_clear_halt(DevCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_halt, dim3(1), dim3(1), 0, st, ctl);
  return hipGetLastError();
}

}  // namespace cnlos
