// Device building blocks shared by the spectral kernels: complex arithmetic,
// register-resident lane-split FFT stages, and deterministic FP64 block
// reductions.
//
// FFT convention.  The forward transform is decimation in frequency (DIF): it
// takes natural-order input and leaves the spectrum in bit-reversed order.
// The inverse is decimation in time (DIT) with conjugate twiddles: it takes a
// bit-reversed spectrum and returns natural order, unnormalized.  A forward
// transform, a pointwise spectral operation that knows each position's
// frequency, and an inverse transform therefore need no reordering pass.
//
// Butterfly twiddles come from a per-span table twc[d + k] = exp(-pi i k / d)
// (d = 1, 2, 4, ..., k < d), computed in FP64 on the host; one table of size
// 2^b serves every transform of length up to 2^b.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cnlos {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

__device__ __forceinline__ int brev(int x, int bits) {
  return bits == 0 ? 0 : (int)(__brev((unsigned)x) >> (32 - bits));
}

// ---------------------------------------------------------------------------
// Lane-split register FFT.  A group of LANES consecutive lanes holds one
// sequence; lane s keeps the elements at positions p = LANES * r + s,
// r < E, in registers.  Stages whose span is a multiple of LANES are done in
// registers ("in-lane"); spans LANES/2 .. 1 pair lanes s and s ^ span
// ("cross-lane") through DPP / swizzle lane exchanges.  Stage twiddles come
// from the per-span table twc[d + k] = W_{2d}^k (d = 1, 2, 4, ...), which
// neighbouring lanes read at neighbouring addresses (no LDS bank conflicts).
// ---------------------------------------------------------------------------
// Value of lane (lane ^ D).  D = 1, 2: DPP quad permutation; D < 32:
// ds_swizzle in bit-mask mode (lane' = lane ^ D within 32-lane halves);
// D = 32: ds_bpermute.
template <int D>
__device__ __forceinline__ int lane_xor_bits(int i) {
  if constexpr (D == 1) {
    return __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false);   // [1,0,3,2]
  } else if constexpr (D == 2) {
    return __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false);   // [2,3,0,1]
  } else if constexpr (D < 32) {
    return __builtin_amdgcn_ds_swizzle(i, 0x1F | (D << 10));
  } else {
    return __shfl_xor(i, D, 64);
  }
}

template <int D>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor_bits<D>(__float_as_int(v)));
}

template <int D>
__device__ __forceinline__ double lane_xor_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)lane_xor_bits<D>((int)(unsigned)b);
  const unsigned hi = (unsigned)lane_xor_bits<D>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int D>
__device__ __forceinline__ float2 lane_xor2(float2 v) {
  return make_float2(lane_xor<D>(v.x), lane_xor<D>(v.y));
}

// One cross-lane DIF stage of span D.  Lower lane: a + b; upper lane:
// (a - b) w, written branch-free as (o + sgn x) w' with sgn = -1, w' = w on
// the upper lane and sgn = 1, w' = 1 on the lower one.
template <int D, int E>
__device__ __forceinline__ void dif_xstage(float2 (&x)[E], int s, const float2* __restrict__ twc) {
  const bool upper = (s & D) != 0;
  const float sg = upper ? -1.f : 1.f;
  if constexpr (D == 1) {
    // span 1: the twiddle is 1
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 o = lane_xor2<D>(x[r]);
      x[r] = make_float2(o.x + sg * x[r].x, o.y + sg * x[r].y);
    }
  } else if constexpr (D == 2) {
    // span 2: the twiddles are 1 and -i
    const bool rot = upper && (s & 1);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 o = lane_xor2<D>(x[r]);
      const float2 y = make_float2(o.x + sg * x[r].x, o.y + sg * x[r].y);
      x[r] = rot ? make_float2(y.y, -y.x) : y;
    }
  } else {
    const float2 tw_ = twc[D + (s & (D - 1))];
    const float2 w = upper ? tw_ : make_float2(1.f, 0.f);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 o = lane_xor2<D>(x[r]);
      x[r] = cmul(make_float2(o.x + sg * x[r].x, o.y + sg * x[r].y), w);
    }
  }
}

// One cross-lane DIT stage of span D.  Lower lane: a + b conj(w); upper
// lane: a - b conj(w).  The upper lane scales its own value by conj(w) before
// the exchange (the lower lane by 1), so both results are o + sgn t with t
// the lane's scaled value and o the partner's: no selects per element.
// Spans 1 and 2 have the twiddles 1 and (1, i after conjugation).
template <int D, int E>
__device__ __forceinline__ void dit_xstage(float2 (&x)[E], int s, const float2* __restrict__ twc) {
  const bool upper = (s & D) != 0;
  const float sg = upper ? -1.f : 1.f;
  if constexpr (D == 1) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 o = lane_xor2<D>(x[r]);
      x[r] = make_float2(o.x + sg * x[r].x, o.y + sg * x[r].y);
    }
  } else if constexpr (D == 2) {
    const bool rot = upper && (s & 1);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 t = rot ? make_float2(-x[r].y, x[r].x) : x[r];   // times conj(-i) = i
      const float2 o = lane_xor2<D>(t);
      x[r] = make_float2(o.x + sg * t.x, o.y + sg * t.y);
    }
  } else {
    const float2 tw_ = twc[D + (s & (D - 1))];
    const float2 w = upper ? tw_ : make_float2(1.f, 0.f);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 t = cmulc(x[r], w);
      const float2 o = lane_xor2<D>(t);
      x[r] = make_float2(o.x + sg * t.x, o.y + sg * t.y);
    }
  }
}

// DIF stages with spans LANES*DR0, ..., LANES (r distances DR0 .. 1).
template <int LANES, int E, int DR0>
__device__ __forceinline__ void dif_inlane(float2 (&x)[E], int s, const float2* __restrict__ twc) {
#pragma unroll
  for (int dr = DR0; dr >= 1; dr >>= 1) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if (r & dr) continue;
      const float2 a = x[r], b = x[r + dr];
      const int pos = LANES * (r & (dr - 1)) + s;
      x[r] = cadd(a, b);
      x[r + dr] = cmul(csub(a, b), twc[LANES * dr + pos]);
    }
  }
}

// DIF stages with spans LANES/2 .. 1 across the lanes of a group.
template <int LANES, int E>
__device__ __forceinline__ void dif_xlane(float2 (&x)[E], int s, const float2* __restrict__ twc) {
  if constexpr (LANES >= 64) dif_xstage<32, E>(x, s, twc);
  if constexpr (LANES >= 32) dif_xstage<16, E>(x, s, twc);
  if constexpr (LANES >= 16) dif_xstage<8, E>(x, s, twc);
  if constexpr (LANES >= 8) dif_xstage<4, E>(x, s, twc);
  if constexpr (LANES >= 4) dif_xstage<2, E>(x, s, twc);
  if constexpr (LANES >= 2) dif_xstage<1, E>(x, s, twc);
}

// DIT stages with spans 1 .. LANES/2 across the lanes (conjugate twiddles).
template <int LANES, int E>
__device__ __forceinline__ void dit_xlane(float2 (&x)[E], int s, const float2* __restrict__ twc) {
  if constexpr (LANES >= 2) dit_xstage<1, E>(x, s, twc);
  if constexpr (LANES >= 4) dit_xstage<2, E>(x, s, twc);
  if constexpr (LANES >= 8) dit_xstage<4, E>(x, s, twc);
  if constexpr (LANES >= 16) dit_xstage<8, E>(x, s, twc);
  if constexpr (LANES >= 32) dit_xstage<16, E>(x, s, twc);
  if constexpr (LANES >= 64) dit_xstage<32, E>(x, s, twc);
}

// DIT stages with spans LANES, ..., LANES*DRMAX (r distances 1 .. DRMAX).
template <int LANES, int E, int DRMAX>
__device__ __forceinline__ void dit_inlane(float2 (&x)[E], int s, const float2* __restrict__ twc) {
#pragma unroll
  for (int dr = 1; dr <= DRMAX; dr <<= 1) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if (r & dr) continue;
      const int pos = LANES * (r & (dr - 1)) + s;
      const float2 a = x[r], b = cmulc(x[r + dr], twc[LANES * dr + pos]);
      x[r] = cadd(a, b);
      x[r + dr] = csub(a, b);
    }
  }
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: wave shuffle, then LDS in lane order, then a
// per-block partial written to partials[slot * max_blocks + blockIdx.x].
// ---------------------------------------------------------------------------
// Butterfly sums over the 64 lanes, offsets 32, 16, ..., 1 in that order, so
// every lane ends with the same value and the order of the additions is
// fixed.  The exchanges of all NV values at one offset issue together (one
// wait per offset); offsets 1 and 2 are DPP moves, 4 .. 16 swizzles.
template <int D, int NV>
__device__ __forceinline__ void wave_xor_add(double (&v)[NV]) {
  double o[NV];
#pragma unroll
  for (int s = 0; s < NV; ++s) o[s] = lane_xor_d<D>(v[s]);
#pragma unroll
  for (int s = 0; s < NV; ++s) v[s] += o[s];
}

template <int NV>
__device__ __forceinline__ void wave_sum_n(double (&v)[NV]) {
  wave_xor_add<32>(v);
  wave_xor_add<16>(v);
  wave_xor_add<8>(v);
  wave_xor_add<4>(v);
  wave_xor_add<2>(v);
  wave_xor_add<1>(v);
}

__device__ __forceinline__ double wave_sum(double v) {
  double a[1] = {v};
  wave_sum_n<1>(a);
  return a[0];
}

template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* __restrict__ partials,
                                                const int* slots, int max_blocks) {
  __shared__ double red[NV][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  wave_sum_n<NV>(v);
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < NV; ++s) red[s][wid] = v[s];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      double acc = 0.0;
      for (int k = 0; k < nw; ++k) acc += red[s][k];
      partials[(size_t)slots[s] * max_blocks + blockIdx.x] = acc;
    }
  }
}

// Sums of K partial arrays partials[slot[k]][0..nb[k]) by one block of 1024
// threads (nb[k] <= 4096), all K loaded and reduced together, each in a fixed
// order; results valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum_partials_k(const double* __restrict__ partials,
                                                     const int (&slot)[K], const int (&nb)[K],
                                                     int max_blocks, double (&out)[K]) {
  __shared__ double red[K][16];
  double acc[K];
  // every load is issued before the first add (fixed trip counts, unrolled):
  // one memory round trip for all K arrays and every chunk of blockDim
  // partials that the longest array reaches (the chunk test is the same for
  // the whole block; within a chunk a load under a per-lane condition would
  // compile to a branch with a wait after it, so the index is clamped and the
  // value masked instead; the masked zeros leave each sum unchanged)
  constexpr int kPer = 4;   // covers 4 x blockDim >= max_blocks partials (1024 threads)
  int nbmax = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) nbmax = nb[k] > nbmax ? nb[k] : nbmax;
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  double vals[kPer][K];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = threadIdx.x + j * (int)blockDim.x;
    if (j * (int)blockDim.x < nbmax) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        vals[j][k] = partials[(size_t)slot[k] * max_blocks + (i < nb[k] ? i : 0)];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) vals[j][k] = 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = threadIdx.x + j * (int)blockDim.x;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += i < nb[k] ? vals[j][k] : 0.0;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  wave_sum_n<K>(acc);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][wid] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double tot = 0.0;
      for (int j = 0; j < nw; ++j) tot += red[k][j];
      out[k] = tot;
    }
  }
  __syncthreads();
}

// Sum of partials[slot][0..nb) by one block, in a fixed order; result valid in
// thread 0.
__device__ __forceinline__ double block_sum_partials(const double* __restrict__ partials, int slot,
                                                     int nb, int max_blocks) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[(size_t)slot * max_blocks + i];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) tot += red[k];
  }
  __syncthreads();
  return tot;
}

}  // namespace cnlos
