// Spectral kernels: the zero-padded 3-D FFT convolution of the light-cone
// transform (the H of eq. (3)) and the FFT-diagonal solve of eq. (11).
//
// Both are split the same way over the [n][n][m] volume (t fastest):
//   t pass   : per scan column, resample (R_z, convolution only), real-to-
//              complex FFT along t, written as spectrum planes [kt][n*n];
//   plane    : per kt plane, 2-D FFT over (x, y), pointwise spectral operation
//              (multiply by H^ / its conjugate, or divide by c + mu*sigma),
//              inverse 2-D FFT, in place;
//   t pass   : per scan column, complex-to-real inverse FFT along t, crop,
//              R_t^{-1} (S^T and the falloff weight), fused epilogue.
// The t axis of the convolution is padded to 2m and the real input makes only
// kt = 0..m necessary; the (x, y) padding to 2n x 2n is done inside the plane
// kernel by splitting the padded grid into its four parity quadrants, each an
// n x n transform with a twist, so an n x n plane never leaves registers/LDS.
#include "cnlos_internal.h"
#include "fft_device.h"

namespace cnlos {

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
template <int LOGM>
struct TCfg {
  static constexpr int J = LOGM <= 8 ? 16 : (LOGM <= 10 ? 8 : 4);   // columns per block
  static constexpr int ES = J + 1;                                  // padded LDS stride
  static constexpr int NT = 256;
};

template <int LOGN>
struct PlaneCfg {
  static constexpr int NN = 1 << (2 * LOGN);
  static constexpr int NT = (NN / 16) > 256 ? (NN / 16) : 256;
  static constexpr int PER = (NN / NT) > 0 ? (NN / NT) : 1;
};

// ---------------------------------------------------------------------------
// t pass, forward, convolution: x -> S x -> zero-pad to 2m -> R2C -> planes
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ void __launch_bounds__(256)
k_tfwd_conv(ConvSrc src, ResampleTables S, const float2* __restrict__ tw, float2* __restrict__ spec,
            int nn, const DevCtl* ctl) {
  constexpr int M = 1 << LOGM, H = M / 2;
  constexpr int J = TCfg<LOGM>::J, ES = TCfg<LOGM>::ES;
  __shared__ float2 z[M * ES];
  __shared__ float2 tws[M];
  if (ctl != nullptr && ctl->halt) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col0 = blockIdx.x * J;
  for (int i = tid; i < M; i += nthr) tws[i] = tw[i];

  float ca = 1.f, cb = 0.f;
  if (src.lincache) {
    const double beta = ctl->beta;
    ca = (float)(1.0 + beta);
    cb = (float)(-beta);
  }
  const float sc = src.scale_div ? (float)(1.0 / *src.scale_div) : 1.f;

  // real input of each column, staged in the (still unused) upper half
  float* xf = reinterpret_cast<float*>(z + H * ES);
  for (int it = tid; it < J * M; it += nthr) {
    const int k = it & (M - 1), b = it >> LOGM;
    const int col = col0 + b;
    const size_t g = (size_t)col * M + k;
    float x = ca * src.a[g];
    if (src.b) x += cb * src.b[g];
    if (src.c) x -= src.c[g];
    if (src.w) x *= src.w[k];
    if (src.mask) x *= (float)src.mask[col];
    xf[k * ES + b] = x * sc;
  }
  __syncthreads();
  // R_z: squared-distance bins q = 2p, 2p+1 packed as one complex value
  for (int it = tid; it < J * H; it += nthr) {
    const int b = it % J, p = it / J;
    float r[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int4 ri = S.rows[2 * p + s];
      float acc = 0.f;
      for (int t = 0; t < ri.y; ++t) acc += S.rvals[ri.z + t] * xf[(ri.x + t) * ES + b];
      r[s] = acc;
    }
    z[p * ES + b] = make_float2(r[0], r[1]);
  }
  __syncthreads();
  // first DIF stage against the zero upper half
  for (int it = tid; it < J * H; it += nthr) {
    const int b = it % J, p = it / J;
    z[(p + H) * ES + b] = cmul(z[p * ES + b], tws[2 * p]);
  }
  __syncthreads();
  FftRun<LOGM, 1, LOGM, 3, false>::go(z, J, 1, ES, tws, LOGM + 1, tid, nthr);
  // untangle the packed real transform: X[k], k = 0..m
  for (int it = tid; it < J * (M + 1); it += nthr) {
    const int b = it % J, k = it / J;
    const float2 zk = z[brev(k & (M - 1), LOGM) * ES + b];
    const float2 zm = z[brev((M - k) & (M - 1), LOGM) * ES + b];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 o = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
    const float2 wk = k < M ? tws[k] : make_float2(-1.f, 0.f);
    const float2 wo = cmul(wk, o);
    spec[(size_t)k * nn + col0 + b] = make_float2(e.x + wo.y, e.y - wo.x);
  }
}

// ---------------------------------------------------------------------------
// t pass, inverse, convolution: planes -> C2R (length 2m) -> crop -> S^T -> epilogue
// ---------------------------------------------------------------------------
template <int LOGM, int EPI>
__global__ void __launch_bounds__(256)
k_tinv_conv(const float2* __restrict__ spec, int nn, ResampleTables S,
            const float2* __restrict__ tw, ConvEpi ep, float scale, const DevCtl* ctl) {
  constexpr int M = 1 << LOGM, H = M / 2;
  constexpr int J = TCfg<LOGM>::J, ES = TCfg<LOGM>::ES;
  __shared__ float2 z[M * ES];
  __shared__ float2 tws[M];
  if (ctl != nullptr && ctl->halt) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col0 = blockIdx.x * J;
  for (int i = tid; i < M; i += nthr) tws[i] = tw[i];
  __syncthreads();

  // Hermitian pair (k, m-k) -> packed even/odd spectrum Z, bit-reversed
  for (int it = tid; it < J * (H + 1); it += nthr) {
    const int b = it % J, k = it / J;
    const int col = col0 + b;
    const float2 Xk = spec[(size_t)k * nn + col];
    const float2 Xm = spec[(size_t)(M - k) * nn + col];
    const float2 wk = tws[k];
    {
      const float2 e = make_float2(0.5f * (Xk.x + Xm.x), 0.5f * (Xk.y - Xm.y));
      const float2 o = make_float2(0.5f * (Xk.x - Xm.x), 0.5f * (Xk.y + Xm.y));
      const float2 wo = cmulc(o, wk);
      z[brev(k, LOGM) * ES + b] = make_float2(e.x - wo.y, e.y + wo.x);
    }
    if (k != 0 && k != H) {
      const float2 e = make_float2(0.5f * (Xm.x + Xk.x), 0.5f * (Xm.y - Xk.y));
      const float2 o = make_float2(0.5f * (Xm.x - Xk.x), 0.5f * (Xm.y + Xk.y));
      float2 wo = cmul(o, wk);
      wo = make_float2(-wo.x, -wo.y);
      z[brev(M - k, LOGM) * ES + b] = make_float2(e.x - wo.y, e.y + wo.x);
    }
  }
  __syncthreads();
  FftRun<LOGM, 0, LOGM - 1, 3, true>::go(z, J, 1, ES, tws, LOGM + 1, tid, nthr);
  // last DIT stage, lower half only (the crop to the first m real samples)
  for (int it = tid; it < J * H; it += nthr) {
    const int b = it % J, p = it / J;
    z[p * ES + b] = cadd(z[p * ES + b], cmulc(z[(p + H) * ES + b], tws[2 * p]));
  }
  __syncthreads();

  const float* zf = reinterpret_cast<const float*>(z);
  double acc0 = 0.0, acc1 = 0.0;
  float ca = 1.f, cb = 0.f;
  if (EPI == EPI_FWD_OBJ || EPI == EPI_FWD_DUAL) {
    const double beta = ctl->beta;
    ca = (float)(1.0 + beta);
    cb = (float)(-beta);
  }
  for (int it = tid; it < J * M; it += nthr) {
    const int k = it & (M - 1), b = it >> LOGM;
    const int col = col0 + b;
    const int4 ci = S.cols[k];
    float tk = 0.f;
    for (int t = 0; t < ci.y; ++t) {
      const int q = ci.x + t;
      tk += S.cvals[ci.z + t] * zf[((q >> 1) * ES + b) * 2 + (q & 1)];
    }
    tk *= scale;
    if (ep.w) tk *= ep.w[k];
    const size_t g = (size_t)col * M + k;
    if (EPI == EPI_PLAIN || EPI == EPI_NORM) {
      if (ep.mask) tk *= (float)ep.mask[col];
      ep.out[g] = tk;
      if (EPI == EPI_NORM) acc0 += (double)tk * (double)tk;
    } else {
      ep.out[g] = tk;
      const float aub = ca * ep.au[g] + cb * ep.au_prev[g];
      const float d = tk - aub;
      if (EPI == EPI_FWD_OBJ) {
        if (ep.mask[col]) {
          acc0 += (double)d * (double)d;
          const float r = tk - ep.tau0[g];
          acc1 += (double)r * (double)r;
        }
      } else {
        acc0 += (double)d * (double)d;
      }
    }
  }
  if (EPI == EPI_NORM) {
    double v[1] = {acc0};
    const int slots[1] = {SL_NORM};
    block_sum_store<1>(v, ep.partials, slots, kMaxBlocks);
  } else if (EPI == EPI_FWD_OBJ) {
    double v[2] = {acc0, acc1};
    const int slots[2] = {SL_CHECK, SL_DATA};
    block_sum_store<2>(v, ep.partials, slots, kMaxBlocks);
  } else if (EPI == EPI_FWD_DUAL) {
    double v[1] = {acc0};
    const int slots[1] = {SL_CHECK};
    block_sum_store<1>(v, ep.partials, slots, kMaxBlocks);
  }
}

// ---------------------------------------------------------------------------
// plane kernel of the convolution: padded 2n x 2n transform of an n x n plane
// via its four parity quadrants, times H^ (or conj H^), cropped back to n x n.
// The output is unnormalized; the inverse t pass applies the scale.
// ---------------------------------------------------------------------------
template <int LOGN, bool ADJ>
__global__ void __launch_bounds__(PlaneCfg<LOGN>::NT)
k_plane_conv(float2* __restrict__ spec, const float2* __restrict__ hq,
             const float2* __restrict__ tw, const DevCtl* ctl) {
  constexpr int N = 1 << LOGN, NP = N + 1, NN = N * N, N1 = N + 1;
  constexpr int NT = PlaneCfg<LOGN>::NT, PER = PlaneCfg<LOGN>::PER;
  __shared__ float2 A[N * NP];
  __shared__ float2 tws[N];
  if (ctl != nullptr && ctl->halt) return;
  const int tid = threadIdx.x;
  const int plane = blockIdx.x;
  float2* P = spec + (size_t)plane * NN;
  const float2* Hp = hq + (size_t)plane * N1 * N1;
  for (int i = tid; i < N; i += NT) tws[i] = tw[i];
  float2 X[PER], OUT[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int e = tid + s * NT;
    X[s] = e < NN ? P[e] : make_float2(0.f, 0.f);
    OUT[s] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int px = q & 1, py = q >> 1;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int e = tid + s * NT;
      if (e < NN) {
        const int i = e >> LOGN, j = e & (N - 1);
        const int n = px * i + py * j;
        const float2 w = n < N ? tws[n] : make_float2(-tws[n - N].x, -tws[n - N].y);
        A[i * NP + j] = cmul(X[s], w);
      }
    }
    __syncthreads();
    FftRun<LOGN, 0, LOGN, 3, false>::go(A, N, NP, 1, tws, LOGN + 1, tid, NT);
    FftRun<LOGN, 0, LOGN, 3, false>::go(A, N, 1, NP, tws, LOGN + 1, tid, NT);
    for (int e = tid; e < NN; e += NT) {
      const int pi = e >> LOGN, pj = e & (N - 1);
      int kx = 2 * brev(pi, LOGN) + px, ky = 2 * brev(pj, LOGN) + py;
      kx = kx <= N ? kx : 2 * N - kx;
      ky = ky <= N ? ky : 2 * N - ky;
      const float2 h = Hp[kx * N1 + ky];
      const float2 a = A[pi * NP + pj];
      A[pi * NP + pj] = ADJ ? cmulc(a, h) : cmul(a, h);
    }
    __syncthreads();
    FftRun<LOGN, 0, LOGN, 3, true>::go(A, N, 1, NP, tws, LOGN + 1, tid, NT);
    FftRun<LOGN, 0, LOGN, 3, true>::go(A, N, NP, 1, tws, LOGN + 1, tid, NT);
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int e = tid + s * NT;
      if (e < NN) {
        const int i = e >> LOGN, j = e & (N - 1);
        const int n = px * i + py * j;
        const float2 w = n < N ? tws[n] : make_float2(-tws[n - N].x, -tws[n - N].y);
        OUT[s] = cadd(OUT[s], cmulc(A[i * NP + j], w));
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int e = tid + s * NT;
    if (e < NN) P[e] = OUT[s];
  }
}

// ---------------------------------------------------------------------------
// FFT-diagonal solve, eq. (11):  (c I + mu nabla^* nabla) x = rhs, periodic.
// t pass forward (R2C, length m), plane (2-D FFT, divide, inverse), t pass inverse.
// ---------------------------------------------------------------------------
template <int LOGM>
__global__ void __launch_bounds__(256)
k_tfwd_solve(const float* __restrict__ src, const float2* __restrict__ tw,
             float2* __restrict__ spec, int nn, const DevCtl* ctl) {
  constexpr int M = 1 << LOGM, H = M / 2, LOGH = LOGM - 1;
  constexpr int J = TCfg<LOGM>::J, ES = TCfg<LOGM>::ES;
  __shared__ float2 z[H * ES];
  __shared__ float2 tws[M];
  if (ctl != nullptr && ctl->halt) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col0 = blockIdx.x * J;
  for (int i = tid; i < M; i += nthr) tws[i] = tw[i];
  const float2* src2 = reinterpret_cast<const float2*>(src);
  for (int it = tid; it < J * H; it += nthr) {
    const int p = it & (H - 1), b = it >> LOGH;
    z[p * ES + b] = src2[(size_t)(col0 + b) * H + p];
  }
  __syncthreads();
  FftRun<LOGH, 0, LOGH, 3, false>::go(z, J, 1, ES, tws, LOGM + 1, tid, nthr);
  for (int it = tid; it < J * (H + 1); it += nthr) {
    const int b = it % J, k = it / J;
    const float2 zk = z[brev(k & (H - 1), LOGH) * ES + b];
    const float2 zm = z[brev((H - k) & (H - 1), LOGH) * ES + b];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 o = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
    const float2 wk = k < H ? tws[2 * k] : make_float2(-1.f, 0.f);
    const float2 wo = cmul(wk, o);
    spec[(size_t)k * nn + col0 + b] = make_float2(e.x + wo.y, e.y - wo.x);
  }
}

template <int LOGN>
__global__ void __launch_bounds__(PlaneCfg<LOGN>::NT)
k_plane_solve(float2* __restrict__ spec, const float2* __restrict__ tw,
              const float* __restrict__ sig_xy, const float* __restrict__ sig_t,
              const double* c_dev, float c_val, float mu, const DevCtl* ctl) {
  constexpr int N = 1 << LOGN, NP = N + 1, NN = N * N;
  constexpr int NT = PlaneCfg<LOGN>::NT;
  __shared__ float2 A[N * NP];
  __shared__ float2 tws[N];
  __shared__ float sg[N];
  if (ctl != nullptr && ctl->halt) return;
  const int tid = threadIdx.x;
  const int plane = blockIdx.x;
  float2* P = spec + (size_t)plane * NN;
  for (int i = tid; i < N; i += NT) {
    tws[i] = tw[i];
    sg[i] = sig_xy[i];
  }
  for (int e = tid; e < NN; e += NT) A[(e >> LOGN) * NP + (e & (N - 1))] = P[e];
  __syncthreads();
  FftRun<LOGN, 0, LOGN, 3, false>::go(A, N, NP, 1, tws, LOGN + 1, tid, NT);
  FftRun<LOGN, 0, LOGN, 3, false>::go(A, N, 1, NP, tws, LOGN + 1, tid, NT);
  const float c = c_dev ? (float)(*c_dev) : c_val;
  const float base = c + mu * sig_t[plane];
  for (int e = tid; e < NN; e += NT) {
    const int pi = e >> LOGN, pj = e & (N - 1);
    const float den = base + mu * (sg[brev(pi, LOGN)] + sg[brev(pj, LOGN)]);
    A[pi * NP + pj] = cscale(A[pi * NP + pj], 1.f / den);
  }
  __syncthreads();
  FftRun<LOGN, 0, LOGN, 3, true>::go(A, N, 1, NP, tws, LOGN + 1, tid, NT);
  FftRun<LOGN, 0, LOGN, 3, true>::go(A, N, NP, 1, tws, LOGN + 1, tid, NT);
  for (int e = tid; e < NN; e += NT) P[e] = A[(e >> LOGN) * NP + (e & (N - 1))];
}

template <int LOGM>
__global__ void __launch_bounds__(256)
k_tinv_solve(const float2* __restrict__ spec, int nn, const float2* __restrict__ tw,
             SolveEpi ep, float scale, const DevCtl* ctl) {
  constexpr int M = 1 << LOGM, H = M / 2, LOGH = LOGM - 1, Q = H / 2;
  constexpr int J = TCfg<LOGM>::J, ES = TCfg<LOGM>::ES;
  __shared__ float2 z[H * ES];
  __shared__ float2 tws[M];
  if (ctl != nullptr && ctl->halt) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col0 = blockIdx.x * J;
  for (int i = tid; i < M; i += nthr) tws[i] = tw[i];
  __syncthreads();
  for (int it = tid; it < J * (Q + 1); it += nthr) {
    const int b = it % J, k = it / J;
    const int col = col0 + b;
    const float2 Xk = spec[(size_t)k * nn + col];
    const float2 Xm = spec[(size_t)(H - k) * nn + col];
    const float2 wk = tws[2 * k];   // W_m^k
    {
      const float2 e = make_float2(0.5f * (Xk.x + Xm.x), 0.5f * (Xk.y - Xm.y));
      const float2 o = make_float2(0.5f * (Xk.x - Xm.x), 0.5f * (Xk.y + Xm.y));
      const float2 wo = cmulc(o, wk);
      z[brev(k & (H - 1), LOGH) * ES + b] = make_float2(e.x - wo.y, e.y + wo.x);
    }
    if (k != 0 && k != Q) {
      const float2 e = make_float2(0.5f * (Xm.x + Xk.x), 0.5f * (Xm.y - Xk.y));
      const float2 o = make_float2(0.5f * (Xm.x - Xk.x), 0.5f * (Xm.y + Xk.y));
      float2 wo = cmul(o, wk);
      wo = make_float2(-wo.x, -wo.y);
      z[brev(H - k, LOGH) * ES + b] = make_float2(e.x - wo.y, e.y + wo.x);
    }
  }
  __syncthreads();
  FftRun<LOGH, 0, LOGH, 3, true>::go(z, J, 1, ES, tws, LOGM + 1, tid, nthr);
  double acc = 0.0;
  float2* out2 = reinterpret_cast<float2*>(ep.out);
  const float2* ref2 = reinterpret_cast<const float2*>(ep.ref);
  for (int it = tid; it < J * H; it += nthr) {
    const int p = it & (H - 1), b = it >> LOGH;
    const size_t g = (size_t)(col0 + b) * H + p;
    const float2 y = cscale(z[p * ES + b], scale);
    out2[g] = y;
    if (ep.ref) {
      const float2 r = ref2[g];
      const float d0 = y.x - r.x, d1 = y.y - r.y;
      acc += (double)d0 * (double)d0 + (double)d1 * (double)d1;
    }
  }
  if (ep.ref) {
    double v[1] = {acc};
    const int slots[1] = {SL_STEP};
    block_sum_store<1>(v, ep.partials, slots, kMaxBlocks);
  }
}

// ---------------------------------------------------------------------------
// H^ setup: the kernel h of eq. (3) is even in dx and dy, so its padded
// spectrum is a real cosine sum in (kx, ky) and a complex exponential in kt:
//   H^[kt][kx][ky] = (1/Z) sum_{dx,dy >= 0} c_dx c_dy cos(pi kx dx / n)
//                    cos(pi ky dy / n) exp(-pi i kt dq(dx,dy) / m),
// c_0 = 1, c_d = 2.  One block per (kt, chunk of ky); FP64 accumulation; the
// inner dy sum is staged in LDS.  Stored for kx, ky in [0, n] (the quarter).
// ---------------------------------------------------------------------------
template <int LOGN>
__global__ void __launch_bounds__(256)
k_build_hq(float2* __restrict__ hq, int m, const int* __restrict__ dq,
           const double2* __restrict__ etab, const double* __restrict__ cosn, double invZ) {
  constexpr int N = 1 << LOGN, N1 = N + 1, KYC = N1 < 32 ? N1 : 32;
  __shared__ double2 G[KYC * N];
  __shared__ double cs[2 * N];
  const int kt = blockIdx.x, ky0 = blockIdx.y * KYC, tid = threadIdx.x;
  const int nky = (N1 - ky0) < KYC ? (N1 - ky0) : KYC;
  const int two_m = 2 * m;
  for (int i = tid; i < 2 * N; i += blockDim.x) cs[i] = cosn[i];
  __syncthreads();
  // inner sum over dy for this block's ky range
  for (int it = tid; it < nky * N; it += blockDim.x) {
    const int kyl = it / N, dx = it % N, ky = ky0 + kyl;
    double sr = 0.0, si = 0.0;
    for (int dy = 0; dy < N; ++dy) {
      const int q = dq[dx * N + dy];
      if (q < 0) continue;
      const double w = (dy ? 2.0 : 1.0) * cs[(ky * dy) % (2 * N)];
      const double2 e = etab[(int)(((long long)kt * q) % two_m)];
      sr += w * e.x;
      si += w * e.y;
    }
    G[kyl * N + dx] = make_double2(sr, si);
  }
  __syncthreads();
  // outer sum over dx
  for (int it = tid; it < N1 * nky; it += blockDim.x) {
    const int kx = it / nky, kyl = it % nky;
    double ar = 0.0, ai = 0.0;
    for (int dx = 0; dx < N; ++dx) {
      const double w = (dx ? 2.0 : 1.0) * cs[(kx * dx) % (2 * N)];
      const double2 gv = G[kyl * N + dx];
      ar += w * gv.x;
      ai += w * gv.y;
    }
    hq[(size_t)kt * N1 * N1 + (size_t)kx * N1 + ky0 + kyl] =
        make_float2((float)(ar * invZ), (float)(ai * invZ));
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int LOGM>
static int cols_per_block() { return TCfg<LOGM>::J; }

static int cols_per_block_rt(int logm) {
  return logm <= 8 ? 16 : (logm <= 10 ? 8 : 4);
}

int conv_blocks(int logn, int logm) { return (1 << (2 * logn)) / cols_per_block_rt(logm); }

template <int LOGN, int LOGM>
static hipError_t conv_impl(const Tables& tb, const ConvSrc& src, float2* spec, bool adjoint,
                            int epi, const ConvEpi& ep, const DevCtl* ctl, hipStream_t st) {
  constexpr int N = 1 << LOGN, M = 1 << LOGM, NN = N * N;
  const int nb = NN / TCfg<LOGM>::J;
  hipLaunchKernelGGL(k_tfwd_conv<LOGM>, dim3(nb), dim3(256), 0, st, src, tb.S, tb.tw_t, spec, NN,
                     ctl);
  if (adjoint)
    hipLaunchKernelGGL((k_plane_conv<LOGN, true>), dim3(M + 1), dim3(PlaneCfg<LOGN>::NT), 0, st,
                       spec, tb.hq, tb.tw_xy, ctl);
  else
    hipLaunchKernelGGL((k_plane_conv<LOGN, false>), dim3(M + 1), dim3(PlaneCfg<LOGN>::NT), 0, st,
                       spec, tb.hq, tb.tw_xy, ctl);
  const float scale = (float)(1.0 / (4.0 * (double)NN * (double)M));
  switch (epi) {
    case EPI_PLAIN:
      hipLaunchKernelGGL((k_tinv_conv<LOGM, EPI_PLAIN>), dim3(nb), dim3(256), 0, st, spec, NN,
                         tb.S, tb.tw_t, ep, scale, ctl);
      break;
    case EPI_FWD_OBJ:
      hipLaunchKernelGGL((k_tinv_conv<LOGM, EPI_FWD_OBJ>), dim3(nb), dim3(256), 0, st, spec, NN,
                         tb.S, tb.tw_t, ep, scale, ctl);
      break;
    case EPI_FWD_DUAL:
      hipLaunchKernelGGL((k_tinv_conv<LOGM, EPI_FWD_DUAL>), dim3(nb), dim3(256), 0, st, spec, NN,
                         tb.S, tb.tw_t, ep, scale, ctl);
      break;
    default:
      hipLaunchKernelGGL((k_tinv_conv<LOGM, EPI_NORM>), dim3(nb), dim3(256), 0, st, spec, NN,
                         tb.S, tb.tw_t, ep, scale, ctl);
      break;
  }
  return hipGetLastError();
}

template <int LOGN, int LOGM>
static hipError_t solve_impl(const Tables& tb, const float* rhs, float2* spec, const double* c_dev,
                             double c_val, double mu, const SolveEpi& ep, const DevCtl* ctl,
                             hipStream_t st) {
  constexpr int N = 1 << LOGN, M = 1 << LOGM, NN = N * N;
  const int nb = NN / TCfg<LOGM>::J;
  hipLaunchKernelGGL(k_tfwd_solve<LOGM>, dim3(nb), dim3(256), 0, st, rhs, tb.tw_t, spec, NN, ctl);
  hipLaunchKernelGGL(k_plane_solve<LOGN>, dim3(M / 2 + 1), dim3(PlaneCfg<LOGN>::NT), 0, st, spec,
                     tb.tw_xy, tb.sig_xy, tb.sig_t, c_dev, (float)c_val, (float)mu, ctl);
  const float scale = (float)(2.0 / ((double)NN * (double)M));
  hipLaunchKernelGGL(k_tinv_solve<LOGM>, dim3(nb), dim3(256), 0, st, spec, NN, tb.tw_t, ep, scale,
                     ctl);
  return hipGetLastError();
}

#define CNLOS_DISPATCH_M(LOGN, FN, ...)                                  \
  switch (logm) {                                                        \
    case 4: return FN<LOGN, 4>(__VA_ARGS__);                             \
    case 5: return FN<LOGN, 5>(__VA_ARGS__);                             \
    case 6: return FN<LOGN, 6>(__VA_ARGS__);                             \
    case 7: return FN<LOGN, 7>(__VA_ARGS__);                             \
    case 8: return FN<LOGN, 8>(__VA_ARGS__);                             \
    case 9: return FN<LOGN, 9>(__VA_ARGS__);                             \
    case 10: return FN<LOGN, 10>(__VA_ARGS__);                           \
    case 11: return FN<LOGN, 11>(__VA_ARGS__);                           \
    default: return hipErrorInvalidValue;                                \
  }

#define CNLOS_DISPATCH_NM(FN, ...)                                       \
  switch (logn) {                                                        \
    case 3: CNLOS_DISPATCH_M(3, FN, __VA_ARGS__)                         \
    case 4: CNLOS_DISPATCH_M(4, FN, __VA_ARGS__)                         \
    case 5: CNLOS_DISPATCH_M(5, FN, __VA_ARGS__)                         \
    case 6: CNLOS_DISPATCH_M(6, FN, __VA_ARGS__)                         \
    case 7: CNLOS_DISPATCH_M(7, FN, __VA_ARGS__)                         \
    default: return hipErrorInvalidValue;                                \
  }

hipError_t launch_conv(int logn, int logm, const Tables& tb, const ConvSrc& src, float2* spec,
                       bool adjoint, int epi, const ConvEpi& ep, const DevCtl* ctl,
                       hipStream_t st) {
  CNLOS_DISPATCH_NM(conv_impl, tb, src, spec, adjoint, epi, ep, ctl, st)
}

hipError_t launch_solve(int logn, int logm, const Tables& tb, const float* rhs, float2* spec,
                        const double* c_dev, double c_val, double mu, const SolveEpi& ep,
                        const DevCtl* ctl, hipStream_t st) {
  CNLOS_DISPATCH_NM(solve_impl, tb, rhs, spec, c_dev, c_val, mu, ep, ctl, st)
}

hipError_t launch_build_hq(int logn, int logm, float2* hq, const int* dq, const double2* etab,
                           const double* cosn, double invZ, hipStream_t st) {
  const int m = 1 << logm, n1 = (1 << logn) + 1;
  const int kyc = n1 < 32 ? n1 : 32;
  const dim3 grid(m + 1, (n1 + kyc - 1) / kyc);
  switch (logn) {
    case 3: hipLaunchKernelGGL(k_build_hq<3>, grid, dim3(256), 0, st, hq, m, dq, etab, cosn, invZ); break;
    case 4: hipLaunchKernelGGL(k_build_hq<4>, grid, dim3(256), 0, st, hq, m, dq, etab, cosn, invZ); break;
    case 5: hipLaunchKernelGGL(k_build_hq<5>, grid, dim3(256), 0, st, hq, m, dq, etab, cosn, invZ); break;
    case 6: hipLaunchKernelGGL(k_build_hq<6>, grid, dim3(256), 0, st, hq, m, dq, etab, cosn, invZ); break;
    case 7: hipLaunchKernelGGL(k_build_hq<7>, grid, dim3(256), 0, st, hq, m, dq, etab, cosn, invZ); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cnlos
