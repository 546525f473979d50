// Device helpers of the difference operators and the splitting steps
// (Sections 3.1 and 4.1), shared by the stencil kernels and the kernels that
// fold a right-hand side into a transform.  Volumes are [n][n][m], t fastest,
// periodic, unit spacing.
#pragma once
#include <math.h>

#include "cnlos_internal.h"

namespace cnlos {

// element o of q for a 32-bit element offset o (a 32-bit byte offset from
// the uniform base, so the access takes the scalar-base addressing form);
// offsets are per scene, below 2^30 elements
__device__ __forceinline__ float2 ld2(const float* __restrict__ q, uint32_t o) {
  return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(q) + (o << 2));
}
__device__ __forceinline__ float ld1(const float* __restrict__ q, uint32_t o) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(q) + (o << 2));
}
__device__ __forceinline__ void st2(float* __restrict__ q, uint32_t o, float2 v) {
  *reinterpret_cast<float2*>(reinterpret_cast<char*>(q) + (o << 2)) = v;
}

// reciprocal square root of an argument that is never zero or denormal
// (|g|^2 + eta^2 with eta > 0)
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Offsets of a bin pair (k, k + 1), k even, of one scan column and of the
// neighbour columns the difference operators reach (periodic in x, y, t).
struct PairOff {
  uint32_t col;                            // scan column i n + j
  uint32_t c, cxp, cyp, cxm, cym;          // column offsets (times m): own, x+1, y+1, x-1, y-1
  uint32_t cxmyp, cymxp;                   // (x-1, y+1), (x+1, y-1)
  uint32_t k, kn, km;                      // k, (k + 2) mod m, (k - 1) mod m
};

__device__ __forceinline__ PairOff pair_offsets(uint32_t q, int logn, int logm) {
  const uint32_t N = 1u << logn, M = 1u << logm;
  const uint32_t col = q >> (logm - 1), k = 2 * (q & (M / 2 - 1));
  const uint32_t i = col >> logn, j = col & (N - 1);
  auto cof = [&](uint32_t a, uint32_t b) {
    return (((a & (N - 1)) << logn) | (b & (N - 1))) << logm;
  };
  PairOff o;
  o.col = col;
  o.c = col << logm;
  o.cxp = cof(i + 1, j);
  o.cyp = cof(i, j + 1);
  o.cxm = cof(i - 1, j);
  o.cym = cof(i, j - 1);
  o.cxmyp = cof(i - 1, j + 1);
  o.cymxp = cof(i + 1, j - 1);
  o.k = k;
  o.kn = (k + 2) & (M - 1);
  o.km = (k - 1) & (M - 1);
  return o;
}

// periodic neighbour offsets of voxel g
struct Nbr {
  size_t xp, xm, yp, ym, tp, tm;
};

__device__ __forceinline__ Nbr neighbours(size_t g, int logn, int logm) {
  const size_t M = (size_t)1 << logm, N = (size_t)1 << logn;
  const size_t sx = N * M, sy = M;
  const size_t k = g & (M - 1);
  const size_t j = (g >> logm) & (N - 1);
  const size_t i = g >> (logm + logn);
  Nbr r;
  r.xp = (i == N - 1) ? g - (N - 1) * sx : g + sx;
  r.xm = (i == 0) ? g + (N - 1) * sx : g - sx;
  r.yp = (j == N - 1) ? g - (N - 1) * sy : g + sy;
  r.ym = (j == 0) ? g + (N - 1) * sy : g - sy;
  r.tp = (k == M - 1) ? g - (M - 1) : g + 1;
  r.tm = (k == 0) ? g + (M - 1) : g - 1;
  return r;
}

__device__ __forceinline__ float phi_eval(float kappa, const PhiArgs& pa) {
  const float a = (float)pa.a, b = (float)pa.b;
  if (pa.kind == 1) return a + b * fabsf(kappa);
  if (pa.kind == 2) return sqrtf(a + b * kappa * kappa);
  return a + b * kappa * kappa;
}

// forward-difference gradient of x at voxel g (neighbours given)
__device__ __forceinline__ void grad_at(const float* __restrict__ x, size_t g, size_t xp, size_t yp,
                                        size_t tp, float& gx, float& gy, float& gt) {
  const float x0 = x[g];
  gx = x[xp] - x0;
  gy = x[yp] - x0;
  gt = x[tp] - x0;
}

// kappa = div^-( grad x / sqrt(|grad x|^2 + eta^2) ) at voxel g, plus grad x(g)
__device__ __forceinline__ float curvature_at(const float* __restrict__ x, size_t g, const Nbr& nb,
                                              int logn, int logm, float eta2, float& gx0,
                                              float& gy0, float& gt0) {
  grad_at(x, g, nb.xp, nb.yp, nb.tp, gx0, gy0, gt0);
  const float i0 = rsq(gx0 * gx0 + gy0 * gy0 + gt0 * gt0 + eta2);
  float ax, ay, at;
  const Nbr bx = neighbours(nb.xm, logn, logm);
  grad_at(x, nb.xm, bx.xp, bx.yp, bx.tp, ax, ay, at);
  const float nxm = ax * rsq(ax * ax + ay * ay + at * at + eta2);
  const Nbr by = neighbours(nb.ym, logn, logm);
  grad_at(x, nb.ym, by.xp, by.yp, by.tp, ax, ay, at);
  const float nym = ay * rsq(ax * ax + ay * ay + at * at + eta2);
  const Nbr bt = neighbours(nb.tm, logn, logm);
  grad_at(x, nb.tm, bt.xp, bt.yp, bt.tp, ax, ay, at);
  const float ntm = at * rsq(ax * ax + ay * ay + at * at + eta2);
  return (gx0 * i0 - nxm) + (gy0 * i0 - nym) + (gt0 * i0 - ntm);
}

// factor s of the isotropic shrinkage shrink(a, thr) = s a for |a|^2 = n2:
// max(1 - thr / |a|, 0), branch-free through the hardware reciprocal square
// root; |a| <= 1e-15 is taken as a = 0 (the shrunk vector is then below
// 1e-15 in every case).
__device__ __forceinline__ float shrink_factor(float n2, float thr) {
  const float inv = n2 > 1e-30f ? __builtin_amdgcn_rsqf(n2) : 0.f;
  return fmaxf(1.f - thr * inv, 0.f);
}

// v = shrink(grad xbar - Lambda/mu, phi/mu) at voxel q, isotropic over the
// three components (eq. (7); the w-step of Algorithm 2 is the same on taubar).
// The splitting variables are never stored: every kernel that needs v (or w)
// recomputes it from xbar, Lambda and phi, which are unchanged between the
// v-step and its last use in the same iteration.
__device__ __forceinline__ void v_at(const float* __restrict__ xb, const float* __restrict__ lam,
                                     const float* __restrict__ phi, float inv_mu, size_t q,
                                     size_t V, int logn, int logm, float& vx, float& vy,
                                     float& vt) {
  const Nbr nb = neighbours(q, logn, logm);
  float gx, gy, gt;
  grad_at(xb, q, nb.xp, nb.yp, nb.tp, gx, gy, gt);
  const float ax = gx - lam[q] * inv_mu;
  const float ay = gy - lam[V + q] * inv_mu;
  const float at = gt - lam[2 * V + q] * inv_mu;
  const float s = shrink_factor(ax * ax + ay * ay + at * at, phi[q] * inv_mu);
  vx = ax * s;
  vy = ay * s;
  vt = at * s;
}

// f: pointwise minimizer of lambda/2 |f - tau0|^2 on kept points
//    + <Lambda3, f - taubar> + mu3/2 |f - taubar|^2 (never stored, as v)
// (inv_kept = 1 / (lambda + mu3), inv_mu3 = 1 / mu3)
__device__ __forceinline__ float f_at(float tb, float l3, float t0, bool kept, float lambda,
                                      float mu3, float inv_kept, float inv_mu3) {
  return kept ? (lambda * t0 + mu3 * tb - l3) * inv_kept : tb - l3 * inv_mu3;
}

}  // namespace cnlos
