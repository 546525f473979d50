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
// kt = 0..m necessary (the two real bins kt = 0, m share one plane);
// the (x, y) padding to 2n x 2n lives only inside the plane kernel: rows and
// columns are transformed with their zero halves folded into twists, and the
// n x n crop is taken before anything leaves the CU (n = 128 splits the plane
// by ky parity to fit LDS).
#include "cnlos_internal.h"
#include "fft_device.h"
#include "stencil_device.h"

namespace cnlos {

// the volume behind v for this launch's scene (zo: the scene's byte offset)
__device__ __forceinline__ const float* vol_in(const Vol& v, const CtlHead& h, size_t zo) {
  return vol_resolve(v, h, zo);
}
__device__ __forceinline__ float* vol_out(const Vol& v, const CtlHead& h, size_t zo) {
  return vol_resolve(v, h, zo);
}
__device__ __forceinline__ void zsh_tables(ResampleTables& S, size_t zo) {
  S.rows = zsh(S.rows, zo);
  S.rvals = zsh(S.rvals, zo);
  S.cols = zsh(S.cols, zo);
  S.cvals = zsh(S.cvals, zo);
}

// ---------------------------------------------------------------------------
// t passes.  A block handles J scan columns (t_columns); each column's FFT
// lives in the registers of a group of G <= 64 lanes, so within one wave
// (lane s keeps positions G*r + s).  Spectrum planes are exchanged with global
// memory through an LDS staging tile [kt][J], so every plane access is a
// J * 8-byte segment (64 bytes from m = 256 on).  Fewer lanes per column (more
// elements per lane, fewer cross-lane stages) measured slower: the passes are
// bound by the latency of their phases, and fewer waves hide less of it.
// ---------------------------------------------------------------------------
// Columns per block of a t pass of length 2^logf: 8 for lengths 256 to 1024,
// where a block's 512 threads, about 60 KB of LDS (at 512) and its registers
// leave room for two blocks per CU, so one block's loads overlap the other's
// transform (measured faster than 16-column blocks of 1024 threads with
// 128-byte segments, one per CU: 61.7 against 62.6 ms per 64x64x512
// reconstruction, 408 against 442 ms for a batch of eight); 16 for shorter
// transforms (the solve phase of a fused pass needs whole waves), 4 at 2048
// (LDS).
constexpr int t_columns(int logf) { return logf <= 7 ? 16 : (logf <= 10 ? 8 : 4); }

template <int LOGF>
struct TGeo {                                 // transform of length F = 2^LOGF
  static constexpr int F = 1 << LOGF;
  static constexpr int G = (F / 2) < 64 ? (F / 2) : 64;   // lanes per column
  static constexpr int E = F / G;                         // elements per lane (>= 2)
  static constexpr int J = t_columns(LOGF);               // columns per block
  static constexpr int NT = J * G;
};

// Block-strided copies with compile-time extents.  A loop whose trip count
// depends on the thread index is not unrolled, and each of its iterations
// then waits for its own load before its store; here a thread issues up to 8
// loads (indices clamped into range) before its first store.
template <int NT, int COUNT, typename Ld, typename St>
__device__ __forceinline__ void block_copy(int tid, Ld ld, St st) {
  constexpr int NS = (COUNT + NT - 1) / NT, CH = NS < 8 ? NS : 8;
#pragma unroll
  for (int c0 = 0; c0 < NS; c0 += CH) {
    decltype(ld(0)) v[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int it = tid + (c0 + j) * NT;
      v[j] = ld(it < COUNT ? it : COUNT - 1);
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int it = tid + (c0 + j) * NT;
      if (c0 + j < NS && it < COUNT) st(it, v[j]);
    }
  }
}

// A block-strided copy split into its loads (into registers, indices clamped
// into range) and its stores.  Copies whose loads are all issued before the
// first store (copy_together) cost one memory round trip together, where
// copies done one after the other wait for each in turn.
template <int NT, int COUNT, typename T, typename Ld, typename St>
struct SplitCopy {
  static constexpr int NS = (COUNT + NT - 1) / NT;
  Ld ld;
  St st;
  T v[NS];
  __device__ __forceinline__ void load(int tid) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int it = tid + j * NT;
      v[j] = ld(it < COUNT ? it : COUNT - 1);
    }
  }
  // unconditional: a lane past the end stores the last element's value to
  // the last element, as its owner does (a store under a per-lane condition
  // lets the compiler sink its load into the branch, behind a wait for every
  // load before it)
  __device__ __forceinline__ void store(int tid) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int it = tid + j * NT;
      st(it < COUNT ? it : COUNT - 1, v[j]);
    }
  }
};
template <int NT, int COUNT, typename Ld, typename St>
__device__ __forceinline__ auto split_copy(Ld ld, St st) {
  using T = decltype(ld(0));
  return SplitCopy<NT, COUNT, T, Ld, St>{ld, st, {}};
}
template <typename... C>
__device__ __forceinline__ void copy_together(int tid, C&&... c) {
  (c.load(tid), ...);
  (c.store(tid), ...);
}
template <int NT, int COUNT, typename T>
__device__ __forceinline__ auto table_copy(T* dst, const T* __restrict__ src) {
  return split_copy<NT, COUNT>([=](int i) { return src[i]; }, [=](int i, T v) { dst[i] = v; });
}

// LDS index of staging element (kt, column b): rows of J + 1 plus one extra
// slot every 8 rows, so that rows kt and kt + 8 (bit-reversed neighbours) and
// consecutive rows fall into different banks.
template <int J>
__device__ __forceinline__ int stg(int k, int b) { return k * (J + 1) + (k >> 3) + b; }
template <int J>
constexpr int stg_size(int rows) { return rows * (J + 1) + rows / 8 + J; }
// planes k < NP of the block's J columns <-> the LDS staging tile
template <int J, int NT, int NP>
__device__ __forceinline__ auto planes_copy(float2* lds, const float2* __restrict__ spec, int nn,
                                            int col0) {
  return split_copy<NT, NP * J>(
      [=](int it) { return spec[(size_t)(it / J) * nn + col0 + it % J]; },
      [=](int it, float2 v) { lds[stg<J>(it / J, it % J)] = v; });
}
template <int J, int NT, int NP>
__device__ __forceinline__ void lds_to_planes(const float2* lds, float2* __restrict__ spec, int nn,
                                              int col0, int tid) {
  block_copy<NT, NP * J>(
      tid, [&](int it) { return lds[stg<J>(it / J, it % J)]; },
      [&](int it, float2 v) { spec[(size_t)(it / J) * nn + col0 + it % J] = v; });
}
// LDS index of a column's transform element p, padded every 8 elements so
// that bit-reversed access patterns spread over the banks.
__device__ __forceinline__ int zix(int p) { return p + (p >> 3); }

// The resampling sums below are branch-free: a load under a per-lane
// condition compiles to a branch with a wait after it, so the indices of
// absent taps are clamped into the row (or to 0 for an empty row) and their
// terms masked by selects; all of a lane's table and sample loads can then
// issue together.  The sums keep the order of the tap-by-tap form.
//
// R_z of one z bin from its row (first sample k0, cnt taps, weights at off):
// rows of more than 3 taps (interior weights exactly 1) from the exclusive
// prefix sums pf, shorter rows tap by tap.
__device__ __forceinline__ float rz_row(const int4 ri, const float* sval, const float* xf,
                                        const float* pf) {
  const int cnt = ri.y;
  const bool any = cnt > 0;
  const int k0 = any ? ri.x : 0, off = any ? ri.z : 0;
  const int t1 = any ? cnt - 1 : 0, i1 = cnt > 1 ? 1 : 0;
  const float wa = sval[off], wb = sval[off + t1], wm = sval[off + i1];
  const float xa = xf[k0], xb = xf[k0 + t1], xm = xf[k0 + i1];
  const float pa = pf[k0 + t1], pb = pf[k0 + i1];
  const float acc_l = wa * xa + (pa - pb) + wb * xb;
  float acc_s = wa * xa;
  acc_s = cnt == 3 ? fmaf(wm, xm, acc_s) : acc_s;
  acc_s = cnt >= 2 ? fmaf(wb, xb, acc_s) : acc_s;
  return cnt > 3 ? acc_l : (any ? acc_s : 0.f);
}

// S^T of one t bin from its column of at most 3 taps (first sample x, weights
// at z; checked on the host).
__device__ __forceinline__ float st_taps(const int4 ci, const float* sval, const float* g) {
  const int cnt = ci.y;
  const int x = cnt > 0 ? ci.x : 0, z = cnt > 0 ? ci.z : 0;
  const int i1 = cnt > 1 ? 1 : 0, i2 = cnt > 2 ? 2 : i1;
  const float w0 = sval[z], w1 = sval[z + i1], w2 = sval[z + i2];
  const float g0 = g[x], g1 = g[x + i1], g2 = g[x + i2];
  float tk = cnt > 0 ? w0 * g0 : 0.f;
  tk = cnt > 1 ? fmaf(w1, g1, tk) : tk;
  tk = cnt > 2 ? fmaf(w2, g2, tk) : tk;
  return tk;
}

// t pass, forward, convolution: x -> R_z x -> zero-pad to 2m -> R2C -> planes.
// The real length-2m transform is a complex length-m transform of the packed
// pairs (x[2p], x[2p+1]); its upper half is zero, so the first DIF stage is a
// twist.  With PK the two real bins kt = 0 and kt = m share plane 0 as
// X_0 + i X_m, so the transform fills exactly m planes.
// Forward t pass of the convolution from a column whose real input is in
// LDS (xf, with xv[r] = xf[G r + s] in registers): R_z, packed real-to-complex
// transform of length 2m, untangle, staged coalesced plane writes.
template <int LOGM, bool PK>
__device__ __forceinline__ void tfwd_conv_from_lds(float2* lds, const float2* tws,
                                                   const float2* twc, const int4* srow,
                                                   const float* sval, float (&xv)[TGeo<LOGM>::E],
                                                   int tid, int col0, float2* __restrict__ spec,
                                                   int nn) {
  using T = TGeo<LOGM>;
  constexpr int M = 1 << LOGM, G = T::G, E = T::E, J = T::J, NT = T::NT;
  constexpr int ZS = M + M / 8 + 4;
  const int b = tid / G, s = tid % G;
  float* xf = reinterpret_cast<float*>(lds + b * ZS);
  float* pf = xf + M;
  // R_z rows of more than 3 taps (small q, where a z bin spans many t bins)
  // have interior weights exactly 1, so they are computed as w x[k0] +
  // (P[k1] - P[k0 + 1]) + w' x[k1] from exclusive prefix sums P of the first
  // RS G inputs (those rows end below m/4 + 8, checked when the tables are
  // built); rows of at most 3 taps are summed directly.  No row loops, so no
  // lane waits for the longest row of its wave.
  constexpr int RS = resample_scan_rows(M, G);
  float carry = 0.f;
#pragma unroll
  for (int r = 0; r < RS; ++r) {
    float inc = xv[r];
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const float y = __shfl_up(inc, d, G);
      if (s >= d) inc += y;
    }
    pf[G * r + s] = carry + (inc - xv[r]);
    carry += __shfl(inc, G - 1, G);
  }
  __syncthreads();
  // R_z rows 2p, 2p+1 packed as one complex value, lower half of the transform
  float2 x[E];
#pragma unroll
  for (int r = 0; r < E / 2; ++r) {
    const int p = G * r + s;
    float v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) v[h] = rz_row(srow[2 * p + h], sval, xf, pf);
    x[r] = make_float2(v[0], v[1]);
  }
#pragma unroll
  for (int r = 0; r < E / 2; ++r) x[r + E / 2] = cmul(x[r], tws[2 * (G * r + s)]);
  dif_inlane<G, E, E / 4>(x, s, twc);
  dif_xlane<G, E>(x, s, twc);
  __syncthreads();                                 // every column's input consumed
  float2* z = lds + b * ZS;
#pragma unroll
  for (int r = 0; r < E; ++r) z[zix(G * r + s)] = x[r];
  __syncthreads();
  // untangle the packed real transform: X[k] = 1/2 (Z_k + conj Z_{m-k}) - i/2 W^k (Z_k - conj Z_{m-k})
  float2 X[E];
  float2 XM = make_float2(0.f, 0.f);
#pragma unroll
  for (int r = 0; r <= E; ++r) {
    const int k = r < E ? G * r + s : M;
    if (r == E && s != 0) break;
    const float2 zk = z[zix(brev(k & (M - 1), LOGM))];
    const float2 zm = z[zix(brev((M - k) & (M - 1), LOGM))];
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 o = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
    const float2 wk = k < M ? tws[k] : make_float2(-1.f, 0.f);
    const float2 wo = cmul(wk, o);
    const float2 v = make_float2(e.x + wo.y, e.y - wo.x);
    if (r < E) X[r] = v; else XM = v;
  }
  // X_0 and X_m are real (their imaginary parts vanish identically)
  if (PK && s == 0) X[0].y = XM.x;
  __syncthreads();                                 // staging overwrites the columns
#pragma unroll
  for (int r = 0; r < E; ++r) lds[stg<J>(G * r + s, b)] = X[r];
  if (!PK && s == 0) lds[stg<J>(M, b)] = XM;
  __syncthreads();
  lds_to_planes<J, NT, PK ? M : M + 1>(lds, spec, nn, col0, tid);
}

template <int LOGM, bool PK>
__global__ void __launch_bounds__(TGeo<LOGM>::NT)
k_tfwd_conv(ConvSrc src, ResampleTables S, const float2* __restrict__ tw,
            const float2* __restrict__ twcg, float2* __restrict__ spec, int nn, const DevCtl* ctl,
            size_t zs, int gate) {
  using T = TGeo<LOGM>;
  constexpr int M = 1 << LOGM, G = T::G, E = T::E, J = T::J, NT = T::NT;
  constexpr int ZS = M + M / 8 + 4;               // per-column LDS stride (float2)
  constexpr int LDS2 = (J * ZS > stg_size<J>(M + 1)) ? J * ZS : stg_size<J>(M + 1);
  // the resampling table (<= 3m + 64 values) is staged in LDS up to m = 1024
  constexpr bool STAGE = M <= 1024;
  constexpr int NNZ = STAGE ? 3 * M + 64 : 1;
  __shared__ float2 lds[LDS2];
  __shared__ float2 tws[M];
  __shared__ float2 twc[M];
  __shared__ int4 srow_l[STAGE ? M : 1];
  __shared__ float sval_l[NNZ];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  const float* sa = vol_in(src.a, hd, zo);
  const float* sb = vol_in(src.b, hd, zo);
  const float* sc_ = vol_in(src.c, hd, zo);
  if (gated_off(hd, gate)) return;
  zsh_tables(S, zo);
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  spec = zsh(spec, zo);
  src.w = zsh(src.w, zo);
  src.mask = zsh(src.mask, zo);
  src.scale_div = zsh(src.scale_div, zo);
  const int tid = threadIdx.x, b = tid / G, s = tid % G;
  const int col0 = xcd_block(blockIdx.x, gridDim.x) * J, col = col0 + b;
  // the tables' loads issue with the operands' (one round trip for both);
  // they reach LDS after the operands are loaded
  auto t_tws = table_copy<NT, M>(tws, tw);
  auto t_twc = table_copy<NT, M>(twc, twcg);
  auto t_row = table_copy<NT, STAGE ? M : 1>(srow_l, S.rows);
  auto t_val = table_copy<NT, NNZ>(sval_l, S.rvals);
  t_tws.load(tid);
  t_twc.load(tid);
  if constexpr (STAGE) {
    t_row.load(tid);
    t_val.load(tid);
  }
  const int4* srow = STAGE ? srow_l : S.rows;
  const float* sval = STAGE ? sval_l : S.rvals;

  float ca = 1.f, cb = 0.f;
  if (src.lincache) {
    const double beta = ctl->beta;
    ca = (float)(1.0 + beta);
    cb = (float)(-beta);
  }
  const float sc = src.scale_div ? (float)(1.0 / *src.scale_div) : 1.f;
  const float mk = src.mask ? (float)src.mask[col] : 1.f;
  float* xf = reinterpret_cast<float*>(lds + b * ZS);     // this column's real input
  // every operand is loaded unconditionally (an absent one from a stand-in,
  // a, and replaced by the identity), so all of a lane's loads issue at once:
  // a load under a condition compiles to a branch with a wait after it
  const bool hb = sb != nullptr, hc = sc_ != nullptr, hw = src.w != nullptr;
  const float* pb = hb ? sb : sa;
  const float* pc = hc ? sc_ : sa;
  const float* pw = hw ? src.w : sa;
  float va[E], vb[E], vc[E], vw[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = G * r + s;
    const size_t g = (size_t)col * M + k;
    va[r] = sa[g];
    vb[r] = pb[g];
    vc[r] = pc[g];
    vw[r] = pw[k];
  }
  t_tws.store(tid);
  t_twc.store(tid);
  if constexpr (STAGE) {
    t_row.store(tid);
    t_val.store(tid);
  }
  float xv[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = G * r + s;
    float x = ca * va[r];
    x += cb * (hb ? vb[r] : 0.f);
    x -= hc ? vc[r] : 0.f;
    x *= hw ? vw[r] : 1.f;
    xv[r] = x * sc * mk;
    xf[k] = xv[r];
  }
  tfwd_conv_from_lds<LOGM, PK>(lds, tws, twc, srow, sval, xv, tid, col0, spec, nn);
}

// t pass, inverse, convolution: planes -> C2R (length 2m) -> crop -> S^T -> epilogue
// (PK: plane 0 holds X_0 + i X_m, as written by the forward pass)
template <int LOGM, int EPI, bool PK>
__global__ void __launch_bounds__(TGeo<LOGM>::NT)
k_tinv_conv(const float2* __restrict__ spec, int nn, ResampleTables S,
            const float2* __restrict__ tw, const float2* __restrict__ twcg, ConvEpi ep, float scale,
            const DevCtl* ctl, size_t zs, int gate) {
  using T = TGeo<LOGM>;
  constexpr int M = 1 << LOGM, H = M / 2, G = T::G, E = T::E, J = T::J, NT = T::NT;
  constexpr bool STAGE = M <= 1024;
  constexpr int NNZ = STAGE ? 3 * M + 64 : 1;
  __shared__ float2 lds[stg_size<J>(M + 1)];
  __shared__ float2 tws[M];
  __shared__ float2 twc[M];
  __shared__ int4 scol_l[STAGE ? M : 1];
  __shared__ float sval_l[NNZ];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  float* eout = vol_out(ep.out, hd, zo);
  const float* eau = (EPI == EPI_FWD_OBJ || EPI == EPI_FWD_DUAL) ? vol_in(ep.au, hd, zo) : nullptr;
  const float* eaup =
      (EPI == EPI_FWD_OBJ || EPI == EPI_FWD_DUAL) ? vol_in(ep.au_prev, hd, zo) : nullptr;
  if (gated_off(hd, gate)) return;
  zsh_tables(S, zo);
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  spec = zsh(spec, zo);
  ep.w = zsh(ep.w, zo);
  ep.mask = zsh(ep.mask, zo);
  ep.tau0 = zsh(ep.tau0, zo);
  ep.partials = zsh(ep.partials, zo);
  const int tid = threadIdx.x, b = tid / G, s = tid % G;
  const int col0 = xcd_block(blockIdx.x, gridDim.x) * J, col = col0 + b;
  // tables and the block's planes: one round trip
  if constexpr (STAGE)
    copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, M>(twc, twcg),
                  table_copy<NT, M>(scol_l, S.cols), table_copy<NT, NNZ>(sval_l, S.cvals),
                  planes_copy<J, NT, PK ? M : M + 1>(lds, spec, nn, col0));
  else
    copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, M>(twc, twcg),
                  planes_copy<J, NT, PK ? M : M + 1>(lds, spec, nn, col0));
  const int4* scol = STAGE ? scol_l : S.cols;
  const float* sval = STAGE ? sval_l : S.cvals;
  __syncthreads();
  // packed even/odd spectrum at this lane's bit-reversed positions:
  // Z[k] = 1/2 (X_k + conj X_{m-k}) + i/2 conj(W^k) (X_k - conj X_{m-k})
  float2 x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = brev(G * r + s, LOGM);
    float2 Xk = lds[stg<J>(k, b)];
    float2 Xm = lds[stg<J>(PK ? (M - k) & (M - 1) : M - k, b)];
    if (PK && k == 0) {
      Xm = make_float2(Xk.y, 0.f);
      Xk.y = 0.f;
    }
    const float2 e = make_float2(0.5f * (Xk.x + Xm.x), 0.5f * (Xk.y - Xm.y));
    const float2 o = make_float2(0.5f * (Xk.x - Xm.x), 0.5f * (Xk.y + Xm.y));
    const float2 wo = cmulc(o, tws[k]);
    x[r] = make_float2(e.x - wo.y, e.y + wo.x);
  }
  dit_xlane<G, E>(x, s, twc);
  dit_inlane<G, E, E / 4>(x, s, twc);
  // last stage (span m/2), lower half only: the crop to the first m samples
#pragma unroll
  for (int r = 0; r < E / 2; ++r) x[r] = cadd(x[r], cmulc(x[r + E / 2], tws[2 * (G * r + s)]));
  __syncthreads();                                 // staging consumed
  float2* g2 = lds + b * (H + 2);                  // this column's real samples, packed
#pragma unroll
  for (int r = 0; r < E / 2; ++r) g2[G * r + s] = cscale(x[r], scale);
  __syncthreads();
  const float* g = reinterpret_cast<const float*>(g2);
  double acc0 = 0.0, acc1 = 0.0;
  float ca = 1.f, cb = 0.f;
  if (EPI == EPI_FWD_OBJ || EPI == EPI_FWD_DUAL) {
    const double beta = ctl->beta;
    ca = (float)(1.0 + beta);
    cb = (float)(-beta);
  }
  const float mk = ep.mask ? (float)ep.mask[col] : 1.f;
  // global operands loaded unconditionally, absent ones from a stand-in (the
  // output column) and replaced by the identity, so the loads issue at once
  const bool hw = ep.w != nullptr;
  const float* pw = hw ? ep.w : eout + (size_t)col * M;
  float vw[E], vau[E], vaup[E], vt0[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = G * r + s;
    const size_t gi = (size_t)col * M + k;
    vw[r] = pw[k];
    if constexpr (EPI == EPI_FWD_OBJ || EPI == EPI_FWD_DUAL) {
      vau[r] = eau[gi];
      vaup[r] = eaup[gi];
    }
    if constexpr (EPI == EPI_FWD_OBJ) vt0[r] = ep.tau0[gi];
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = G * r + s;
    float tk = st_taps(scol[k], sval, g);
    tk *= hw ? vw[r] : 1.f;
    const size_t gi = (size_t)col * M + k;
    if (EPI == EPI_PLAIN || EPI == EPI_NORM) {
      tk *= mk;
      eout[gi] = tk;
      if (EPI == EPI_NORM) acc0 += (double)tk * (double)tk;
    } else {
      eout[gi] = tk;
      const float d = tk - (ca * vau[r] + cb * vaup[r]);
      if (EPI == EPI_FWD_OBJ) {
        const float rr = tk - vt0[r];
        const bool kept = mk != 0.f;
        acc0 += kept ? (double)d * (double)d : 0.0;
        acc1 += kept ? (double)rr * (double)rr : 0.0;
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
// Register-resident plane kernel of the convolution (n <= 64).  Rows: 8 lanes
// per row transform the zero-padded row (length 2n) with the upper half of
// the first stage folded into a twist; the 2n spectrum positions go to LDS.
// Columns: 8 lanes per spectrum column transform the zero-padded column,
// multiply by H^ (or its conjugate) at the position's frequency, transform
// back and keep the first n rows.  Rows again: inverse, keep the first n.
// LDS is touched three times per element; every butterfly runs in registers.
//
// Block 0 holds the two real planes kt = 0 and kt = m packed as
// Z = P_0 + i P_m.  H^ is real on both (h is even in x and y, and the t phase
// is +-1), and the spectra of the real planes are Hermitian, so the product
// separates with the partner frequency -k (see plane_conv_cols_packed); the
// result is conv(P_0) + i conv(P_m).
// ---------------------------------------------------------------------------
// YS: LDS row stride of the transposes, L + PAD.  The pad changes only where
// values sit in LDS (bank conflicts of the column accesses), never a result;
// the plan picks it per shape (1, 2 or 4; 2 when untuned).
template <int LOGN>
struct PlaneRegCfg {
  static constexpr int N = 1 << LOGN, L = 2 * N, NT = 8 * N;
  static constexpr int RE = L / 8;
};

// forward column transform of a zero-padded column whose first n entries are
// in c[0 .. RE/2): twist (folded first stage), then the remaining DIF stages
template <int LOGN>
__device__ __forceinline__ void col_fwd(float2 (&c)[PlaneRegCfg<LOGN>::RE], int s,
                                        const float2* tws, const float2* twc) {
  constexpr int RE = PlaneRegCfg<LOGN>::RE;
#pragma unroll
  for (int r = 0; r < RE / 2; ++r) c[r + RE / 2] = cmul(c[r], tws[8 * r + s]);
  dif_inlane<8, RE, RE / 4>(c, s, twc);
  dif_xlane<8, RE>(c, s, twc);
}

// inverse column transform, keeping the first n outputs in c[0 .. RE/2)
template <int LOGN>
__device__ __forceinline__ void col_inv(float2 (&c)[PlaneRegCfg<LOGN>::RE], int s,
                                        const float2* tws, const float2* twc) {
  constexpr int RE = PlaneRegCfg<LOGN>::RE;
  dit_xlane<8, RE>(c, s, twc);
  dit_inlane<8, RE, RE / 4>(c, s, twc);
#pragma unroll
  for (int r = 0; r < RE / 2; ++r) c[r] = cadd(c[r], cmulc(c[r + RE / 2], tws[8 * r + s]));
}

// column pass of block 0 (the packed real planes kt = 0 and kt = m).  The
// forward column spectra Z^ of all 2n columns go to LDS (2n rows), then each
// position combines its own value with the partner at (-kx, -ky):
//   Y(k) = Z^(k) (H_0 + H_m)/2 + conj(Z^(-k)) (H_0 - H_m)/2,
// the spectrum of conv(P_0) + i conv(P_m) (H_0, H_m real and even).  Plane 0
// of H^ holds the two factors as one pair (k_hq_pack_real).
// h0: plane 0 of H^ at this lane's positions of its first column, loaded by
// the caller before the column transforms.
template <int LOGN, int PAD>
__device__ __forceinline__ void plane_conv_cols_packed(float2* Y, const float2* Hab,
                                                       const float2 (&h0)[PlaneRegCfg<LOGN>::RE],
                                                       const float2* tws, const float2* twc,
                                                       int tid) {
  using PC = PlaneRegCfg<LOGN>;
  constexpr int N = PC::N, L = PC::L, LOGL = LOGN + 1, RE = PC::RE, YS = L + PAD;
  const int s = tid & 7;
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    const int col = (tid >> 3) + half * N;
    float2 c[RE];
#pragma unroll
    for (int r = 0; r < RE / 2; ++r) c[r] = Y[(8 * r + s) * YS + col];
    col_fwd<LOGN>(c, s, tws, twc);
#pragma unroll
    for (int r = 0; r < RE; ++r) Y[(8 * r + s) * YS + col] = c[r];
  }
  __syncthreads();
  float2 w[2][RE];
  // the partner of position 8r + s: frequency brev(8r + s) = 16 brev3(s) +
  // brev4(r) (the register part is a constant), negated; the column's once
  const int kxs = brev(s, 3) << (LOGL - 3);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int col = (tid >> 3) + half * N;
    const int colp = brev((L - brev(col, LOGL)) & (L - 1), LOGL);
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const int p = 8 * r + s;
      const int fx = kxs + brev(r, LOGL - 3);
      const int pp = brev((L - fx) & (L - 1), LOGL);
      const float2 own = Y[p * YS + col], par = Y[pp * YS + colp];
      const float2 ab = half == 0 ? h0[r] : Hab[(r * L + col) * 8 + s];   // lane-ordered H^ plane 0
      w[half][r] = make_float2(ab.x * own.x + ab.y * par.x, ab.x * own.y - ab.y * par.y);
    }
  }
  __syncthreads();                                 // every partner read before write-back
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int col = (tid >> 3) + half * N;
    col_inv<LOGN>(w[half], s, tws, twc);
#pragma unroll
    for (int r = 0; r < RE / 2; ++r) Y[(8 * r + s) * YS + col] = w[half][r];
  }
}

template <int LOGN, bool ADJ, int PAD>
__global__ void __launch_bounds__(PlaneRegCfg<LOGN>::NT)
k_plane_conv_reg(float2* __restrict__ spec, const float2* __restrict__ hq,
                 const float2* __restrict__ tw, const float2* __restrict__ twcg, const DevCtl* ctl,
                 size_t zs, size_t hzs, int gate) {
  using PC = PlaneRegCfg<LOGN>;
  constexpr int N = PC::N, L = PC::L, LOGL = LOGN + 1, NT = PC::NT;
  constexpr int RE = PC::RE, YS = L + PAD;
  // n rows of row spectra; block 0 uses all 2n rows for its column spectra
  __shared__ float2 Y[2 * N * YS];
  __shared__ float2 tws[N];
  __shared__ float2 twc[L];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  if (gated_off(ctl, gate)) return;
  spec = zsh(spec, zo);
  hq = zsh(hq, (size_t)blockIdx.z * hzs);   // 0: one H^ for every scene
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  const int tid = threadIdx.x, row = tid >> 3, s = tid & 7;
  float2* P = spec + (size_t)blockIdx.x * N * N;
  const float2* Hp = hq + (size_t)blockIdx.x * L * L;     // lane-ordered H^ of this plane
  // the block's rows and both twiddle tables in one round trip (NT >= L >=
  // N: every thread copies the entry of its index modulo the table size, so
  // entries are written more than once, always with their own value)
  float2 x[RE], h0[RE];
#pragma unroll
  for (int r = 0; r < RE / 2; ++r) x[r] = P[row * N + 8 * r + s];
  const float2 tv_s = tw[tid % N];
  const float2 tv_c = twcg[tid % L];
  tws[tid % N] = tv_s;
  twc[tid % L] = tv_c;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RE / 2; ++r) x[r + RE / 2] = cmul(x[r], tws[8 * r + s]);
  dif_inlane<8, RE, RE / 4>(x, s, twc);
  dif_xlane<8, RE>(x, s, twc);
#pragma unroll
  for (int r = 0; r < RE; ++r) Y[row * YS + 8 * r + s] = x[r];
  __syncthreads();
  // H^ at this lane's positions of a spectrum column (a wave's load of
  // register r reads 64 consecutive entries) is loaded before the column's
  // transforms, whose work hides its latency
#pragma unroll
  for (int r = 0; r < RE; ++r) h0[r] = Hp[(r * L + row) * 8 + s];
  if (blockIdx.x == 0) {
    plane_conv_cols_packed<LOGN, PAD>(Y, hq, h0, tws, twc, tid);
  } else {
    // 2n spectrum columns, 8 lanes each, two columns per lane group
    auto column = [&](int col, const float2 (&h)[RE]) {
      float2 c[RE];
#pragma unroll
      for (int r = 0; r < RE / 2; ++r) c[r] = Y[(8 * r + s) * YS + col];
      col_fwd<LOGN>(c, s, tws, twc);
#pragma unroll
      for (int r = 0; r < RE; ++r) c[r] = ADJ ? cmulc(c[r], h[r]) : cmul(c[r], h[r]);
      col_inv<LOGN>(c, s, tws, twc);
#pragma unroll
      for (int r = 0; r < RE / 2; ++r) Y[(8 * r + s) * YS + col] = c[r];
    };
    column(row, h0);
    float2 h1[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) h1[r] = Hp[(r * L + row + N) * 8 + s];
    column(row + N, h1);
  }
  __syncthreads();
  {
    const int row = tid >> 3, s = tid & 7;
    float2 x[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) x[r] = Y[row * YS + 8 * r + s];
    dit_xlane<8, RE>(x, s, twc);
    dit_inlane<8, RE, RE / 4>(x, s, twc);
#pragma unroll
    for (int r = 0; r < RE / 2; ++r) x[r] = cadd(x[r], cmulc(x[r + RE / 2], tws[8 * r + s]));
#pragma unroll
    for (int r = 0; r < RE / 2; ++r) P[row * N + 8 * r + s] = x[r];
  }
}

// Plane kernel of the convolution for n = 128, where one padded 2n x 2n
// plane does not fit in LDS.  The padded transform is split by the parity h
// of ky: the even and odd ky rows of the spectrum are n-point transforms of
// each row (the odd ones after the twist W_2n^y), so each half is
//   rows:    n-point DIF per row (twisted for h = 1) -> LDS [x][ky_h]
//   columns: zero-padded 2n-point transform per ky_h column, times H^ (or its
//            conjugate), inverse, keep the first n rows
//   rows:    n-point DIT back (untwisted for h = 1), accumulated in registers
// and the sum over both halves is the cropped padded convolution.  A lane
// group of 8 handles two rows / columns in turn.  Block 0 holds the packed
// real planes kt = 0 and kt = m (half_cols_packed), so the launch has m
// blocks, whole rounds of one block per CU.
template <int LOGN, int PAD = 2>
struct PlaneHalfCfg {
  static constexpr int N = 1 << LOGN, L = 2 * N, NT = 4 * N, G = NT / 8;
  static constexpr int RN = N / 8, YS = N + PAD;   // row stride (pad as in PlaneRegCfg)
};

// rows of the half-split plane kernel: forward n-point DIF of the two rows
// of a lane group (twisted by W_2n^y for the odd half) into LDS
template <int LOGN, int PAD>
__device__ __forceinline__ void half_rows_fwd(float2 (&v)[2][PlaneHalfCfg<LOGN>::RN], int h,
                                              float2* Y, const float2* tws, const float2* twc,
                                              int g, int s) {
  using PC = PlaneHalfCfg<LOGN, PAD>;
  constexpr int RN = PC::RN, YS = PC::YS, G = PC::G;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (h) {
#pragma unroll
      for (int r = 0; r < RN; ++r) v[i][r] = cmul(v[i][r], tws[8 * r + s]);
    }
    dif_inlane<8, RN, RN / 2>(v[i], s, twc);
    dif_xlane<8, RN>(v[i], s, twc);
#pragma unroll
    for (int r = 0; r < RN; ++r) Y[(g + G * i) * YS + 8 * r + s] = v[i][r];
  }
}

// columns of the half-split plane kernel: padded 2n-point transform of each
// ky_h column, H^ product, inverse, first n rows back to LDS
template <int LOGN, bool ADJ, int PAD>
__device__ __forceinline__ void half_cols(int h, float2* Y, const float2* Hp, const float2* tws,
                                          const float2* twc, int g, int s) {
  using PC = PlaneHalfCfg<LOGN, PAD>;
  constexpr int N = PC::N, YS = PC::YS, G = PC::G;
  constexpr int RE = PlaneRegCfg<LOGN>::RE;
#pragma unroll 1
  for (int i = 0; i < 2; ++i) {
    const int col = g + G * i;
    // H^ (lane-ordered: a wave's load reads 64 consecutive entries) in chunks
    // of 8, so that its loads do not all stay live at once; the first chunk
    // is loaded before the forward transform and each next one before the
    // products of the current one, so that their latency is hidden
    const float2* Hh = Hp + ((size_t)h * RE * N + col) * 8 + s;
    float2 hc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) hc[r] = Hh[r * N * 8];
    float2 c[RE];
#pragma unroll
    for (int r = 0; r < RE / 2; ++r) c[r] = Y[(8 * r + s) * YS + col];
    col_fwd<LOGN>(c, s, tws, twc);
#pragma unroll
    for (int r0 = 0; r0 < RE; r0 += 8) {
      float2 hn[8];
      if (r0 + 8 < RE) {
#pragma unroll
        for (int r = 0; r < 8; ++r) hn[r] = Hh[(r0 + 8 + r) * N * 8];
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) c[r0 + r] = ADJ ? cmulc(c[r0 + r], hc[r]) : cmul(c[r0 + r], hc[r]);
      __builtin_amdgcn_sched_barrier(0);
      if (r0 + 8 < RE) {
#pragma unroll
        for (int r = 0; r < 8; ++r) hc[r] = hn[r];
      }
    }
    col_inv<LOGN>(c, s, tws, twc);
#pragma unroll
    for (int r = 0; r < RE / 2; ++r) Y[(8 * r + s) * YS + col] = c[r];
  }
}

// bits of x reversed within `bits` (a constant after unrolling)
__device__ __forceinline__ constexpr int rev_bits(int x, int bits) {
  int y = 0;
  for (int i = 0; i < bits; ++i) y |= ((x >> i) & 1) << (bits - 1 - i);
  return y;
}

// Columns of block 0 of the half-split plane kernel, which holds the two real
// planes kt = 0 and kt = m packed as Z = P_0 + i P_m.  As in
// plane_conv_cols_packed, each spectrum position combines its own value with
// the partner at (-kx, -ky):
//   Y(k) = Z^(k) (H_0 + H_m)/2 + conj(Z^(-k)) (H_0 - H_m)/2
// (the two factors as one pair in plane 0 of H^).  Negating ky keeps its
// parity, so the partner column lies in the same half; a lane group takes a
// column A and its partner B (ky_h and n - ky_h for h = 0, n - 1 - ky_h for
// h = 1; group 0 of the even half the two self-partnered columns 0 and n/2).
// In a column, position 8r + s holds kx = brev(8r + s); -kx sits at register
// r' = brev(2^b - brev(r)) (b bits of r; r' = 0 for r = 0) and lane 7 - s, or
// for r = 0 at the lane whose reversed index is -brev3(s) mod 8.  r and r'
// share their highest set bit, so the lower and the upper half of the
// registers pair only within themselves.
// Registers hold one column spectrum per transform: A's spectrum (2n
// entries) waits in the n LDS slots of A and the n of B while B is
// transformed, and A's combined spectrum again while B is transformed back.
template <int LOGN, int PAD>
__device__ __forceinline__ void half_cols_packed(int h, float2* Y, const float2* Hab,
                                                 const float2* tws, const float2* twc, int g,
                                                 int s) {
  using PC = PlaneHalfCfg<LOGN, PAD>;
  constexpr int N = PC::N, YS = PC::YS;
  constexpr int RE = PlaneRegCfg<LOGN>::RE, RH = RE / 2, LR = LOGN + 1 - 3;
  const bool self = h == 0 && g == 0;
  const int ka = g, kb = self ? N / 2 : (h == 0 ? N - g : N - 1 - g);
  const int colA = brev(ka, LOGN), colB = brev(kb, LOGN);
  auto slot = [&](int r, int col) -> float2& { return Y[(8 * r + s) * YS + col]; };
  // A forward: upper half to A's slots; lower half to B's once B is loaded
  float2 c[RE];
  {
    float2 a[RE];
#pragma unroll
    for (int r = 0; r < RH; ++r) a[r] = slot(r, colA);
    col_fwd<LOGN>(a, s, tws, twc);
#pragma unroll
    for (int r = 0; r < RH; ++r) slot(r, colA) = a[r + RH];
#pragma unroll
    for (int r = 0; r < RH; ++r) c[r] = slot(r, colB);
#pragma unroll
    for (int r = 0; r < RH; ++r) slot(r, colB) = a[r];
  }
  col_fwd<LOGN>(c, s, tws, twc);                   // B's spectrum in registers
  const float2* HA = Hab + ((size_t)h * RE * N + colA) * 8 + s;
  const float2* HB = Hab + ((size_t)h * RE * N + colB) * 8 + s;
  const int lane = threadIdx.x & 63, base = lane & ~7;
  const int s0 = brev((8 - brev(s, 3)) & 7, 3);            // partner lane of register 0
  // value of the partner position of register r: lane s ^ 7, or s0 for r = 0
  auto par = [&](float2 v, int r) {
    const int src = base | (r == 0 ? s0 : (s ^ 7));
    return make_float2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
  };
  auto comb = [&](float2 own, float2 pv, float2 ab) {
    return make_float2(ab.x * own.x + ab.y * pv.x, ab.x * own.y - ab.y * pv.y);
  };
  // combine the registers r0 .. r0 + RH - 1 of A (aa) and B (c) in place,
  // pair by pair; the partner column of A is B, of B is A (each itself in
  // group 0 of the even half)
  float2 ua[RH], la[RH];
  auto combine = [&](float2 (&aa)[RH], int r0) {
#pragma unroll
    for (int i = 0; i < RH; ++i) {
      const int r = r0 + i;
      const int rp = r == 0 ? 0 : rev_bits((RE - rev_bits(r, LR)) & (RE - 1), LR);
      const int ip = rp - r0;
      if (ip < i) continue;                        // the pair was done at r' (static)
      const float2 pA_r = par(self ? aa[ip] : c[rp], r), pA_rp = par(self ? aa[i] : c[r], rp);
      const float2 pB_r = par(self ? c[rp] : aa[ip], r), pB_rp = par(self ? c[r] : aa[i], rp);
      const float2 nA_r = comb(aa[i], pA_r, HA[r * N * 8]);
      const float2 nB_r = comb(c[r], pB_r, HB[r * N * 8]);
      if (ip != i) {
        const float2 nA_rp = comb(aa[ip], pA_rp, HA[rp * N * 8]);
        const float2 nB_rp = comb(c[rp], pB_rp, HB[rp * N * 8]);
        aa[ip] = nA_rp;
        c[rp] = nB_rp;
      }
      aa[i] = nA_r;
      c[r] = nB_r;
      // one pair's H^ loads and shuffles at a time (no hoisting of all of them)
      __builtin_amdgcn_sched_barrier(0);
    }
  };
#pragma unroll
  for (int r = 0; r < RH; ++r) ua[r] = slot(r, colA);
  combine(ua, RH);
#pragma unroll
  for (int r = 0; r < RH; ++r) la[r] = slot(r, colB);
  combine(la, 0);
  // A's combined spectrum to the slots, B back, then A back
#pragma unroll
  for (int r = 0; r < RH; ++r) {
    slot(r, colA) = la[r];
    slot(r, colB) = ua[r];
  }
  col_inv<LOGN>(c, s, tws, twc);
  float2 ob[RH];
#pragma unroll
  for (int r = 0; r < RH; ++r) ob[r] = c[r];
  {
    float2 a[RE];
#pragma unroll
    for (int r = 0; r < RH; ++r) {
      a[r] = slot(r, colA);
      a[r + RH] = slot(r, colB);
    }
#pragma unroll
    for (int r = 0; r < RH; ++r) slot(r, colB) = ob[r];
    col_inv<LOGN>(a, s, tws, twc);
#pragma unroll
    for (int r = 0; r < RH; ++r) slot(r, colA) = a[r];
  }
}

// inverse rows: n-point DIT of a row from LDS (untwisted for the odd half)
template <int LOGN, int PAD>
__device__ __forceinline__ void half_row_inv(float2 (&v)[PlaneHalfCfg<LOGN>::RN], int h, int x,
                                             const float2* Y, const float2* tws, const float2* twc,
                                             int s) {
  using PC = PlaneHalfCfg<LOGN, PAD>;
  constexpr int RN = PC::RN, YS = PC::YS;
#pragma unroll
  for (int r = 0; r < RN; ++r) v[r] = Y[x * YS + 8 * r + s];
  dit_xlane<8, RN>(v, s, twc);
  dit_inlane<8, RN, RN / 2>(v, s, twc);
  if (h) {
#pragma unroll
    for (int r = 0; r < RN; ++r) v[r] = cmulc(v[r], tws[8 * r + s]);
  }
}

// One plane through the half-split transform: per ky half, rows forward,
// columns (PACKED: block 0's pairs of partner columns, else the H^ product),
// rows back, the odd half accumulated onto the even one.
template <int LOGN, bool ADJ, bool PACKED, int PAD>
__device__ __forceinline__ void plane_half_body(float2* __restrict__ P, const float2* Hp,
                                                float2* Y, float2* tws, float2* twc, float2 tv_s,
                                                float2 tv_c, int g, int s) {
  using PC = PlaneHalfCfg<LOGN>;
  constexpr int N = PC::N, L = PC::L, G = PC::G, RN = PC::RN;
  // even ky half; each thread owns plane elements (g + G i, 8 r + s) throughout
  float2 v[2][RN];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < RN; ++r) v[i][r] = P[(g + G * i) * N + 8 * r + s];
  {
    const int tid = threadIdx.x;
    tws[tid % N] = tv_s;
    twc[tid % L] = tv_c;
  }
  __syncthreads();
  half_rows_fwd<LOGN, PAD>(v, 0, Y, tws, twc, g, s);
  __syncthreads();
  if constexpr (PACKED) half_cols_packed<LOGN, PAD>(0, Y, Hp, tws, twc, g, s);
  else half_cols<LOGN, ADJ, PAD>(0, Y, Hp, tws, twc, g, s);
  __syncthreads();
  // the odd half's input, then the even half's output in its place
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < RN; ++r) v[i][r] = P[(g + G * i) * N + 8 * r + s];
#pragma unroll 1
  for (int i = 0; i < 2; ++i) {
    float2 o[RN];
    half_row_inv<LOGN, PAD>(o, 0, g + G * i, Y, tws, twc, s);
#pragma unroll
    for (int r = 0; r < RN; ++r) P[(g + G * i) * N + 8 * r + s] = o[r];
  }
  __syncthreads();                                 // Y is rewritten by the odd half
  half_rows_fwd<LOGN, PAD>(v, 1, Y, tws, twc, g, s);
  __syncthreads();
  if constexpr (PACKED) half_cols_packed<LOGN, PAD>(1, Y, Hp, tws, twc, g, s);
  else half_cols<LOGN, ADJ, PAD>(1, Y, Hp, tws, twc, g, s);
  __syncthreads();
#pragma unroll 1
  for (int i = 0; i < 2; ++i) {
    float2 o[RN];
    half_row_inv<LOGN, PAD>(o, 1, g + G * i, Y, tws, twc, s);
#pragma unroll
    for (int r = 0; r < RN; ++r) {
      float2* q = P + (g + G * i) * N + 8 * r + s;
      *q = cadd(*q, o[r]);
    }
  }
}

template <int LOGN, bool ADJ, int PAD>
__global__ void __launch_bounds__(PlaneHalfCfg<LOGN>::NT)
k_plane_conv_half(float2* __restrict__ spec, const float2* __restrict__ hq,
                  const float2* __restrict__ tw, const float2* __restrict__ twcg, const DevCtl* ctl,
                  size_t zs, size_t hzs, int gate) {
  using PC = PlaneHalfCfg<LOGN, PAD>;
  constexpr int N = PC::N, L = PC::L, NT = PC::NT, G = PC::G, YS = PC::YS;
  static_assert(2 * G == N, "two rows per lane group");
  __shared__ float2 Y[N * YS];
  __shared__ float2 tws[N];
  __shared__ float2 twc[L];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  if (gated_off(ctl, gate)) return;
  spec = zsh(spec, zo);
  hq = zsh(hq, (size_t)blockIdx.z * hzs);   // 0: one H^ for every scene
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  const int tid = threadIdx.x, g = tid >> 3, s = tid & 7;
  float2* P = spec + (size_t)blockIdx.x * N * N;
  const float2* Hp = hq + (size_t)blockIdx.x * L * L;     // lane-ordered H^ of this plane
  // twiddle tables: every thread copies the entry of its index modulo the
  // table size (NT >= L >= N), in the same round trip as the first rows
  const float2 tv_s = tw[tid % N], tv_c = twcg[tid % L];
  // block 0: the packed real planes kt = 0 and kt = m, a separate path so that
  // its register demand does not weigh on the other blocks' code
  if (blockIdx.x == 0) plane_half_body<LOGN, ADJ, true, PAD>(P, Hp, Y, tws, twc, tv_s, tv_c, g, s);
  else plane_half_body<LOGN, ADJ, false, PAD>(P, Hp, Y, tws, twc, tv_s, tv_c, g, s);
}

// Register-resident plane kernel of the diagonal solve (n <= 128): rows and
// columns of length n by LN lanes each (16 at n = 64, so that a block has 16
// waves to hide its phases' latencies; 8 otherwise), divide at the column step.
// YS is the LDS row stride of the transpose, N + PAD (a layout choice only;
// the plan picks 2, 4 or 8 per shape; untuned: 2 at n = 64, 4 at n = 128 and
// 8 otherwise, the fastest of the pads measured by hand).
template <int LOGN, int PAD = (LOGN == 6 ? 2 : LOGN == 7 ? 4 : 8)>
struct PlaneSolveCfg {
  static constexpr int N = 1 << LOGN, LN = LOGN == 6 ? 16 : 8, NT = LN * N, E = N / LN,
                       YS = N + PAD;
};

template <int LOGN, int PAD>
__global__ void __launch_bounds__(PlaneSolveCfg<LOGN>::NT)
k_plane_solve_reg(float2* __restrict__ spec, const float2* __restrict__ twcg,
                  const float* __restrict__ sig_xy, const float* __restrict__ sig_t,
                  const double* c_dev, float c_val, float mu, const DevCtl* ctl, size_t zs,
                  int gate) {
  using PC = PlaneSolveCfg<LOGN, PAD>;
  constexpr int N = PC::N, LN = PC::LN, NT = PC::NT, E = PC::E, YS = PC::YS;
  __shared__ float2 Y[N * YS];
  __shared__ float2 twc[N];
  __shared__ float sg[N];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  if (gated_off(ctl, gate)) return;
  spec = zsh(spec, zo);
  twcg = zsh(twcg, zo);
  sig_xy = zsh(sig_xy, zo);
  sig_t = zsh(sig_t, zo);
  c_dev = zsh(c_dev, zo);
  const int tid = threadIdx.x;
  const int plane = blockIdx.x;
  float2* P = spec + (size_t)plane * N * N;
  const int g = tid / LN, s = tid % LN;
  // the plane's loads issue before the tables' copy waits for its own
  float2 x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) x[r] = P[g * N + LN * r + s];
  for (int i = tid; i < N; i += NT) {
    twc[i] = twcg[i];
    sg[i] = sig_xy[i];
  }
  __syncthreads();
  dif_inlane<LN, E, E / 2>(x, s, twc);
  dif_xlane<LN, E>(x, s, twc);
#pragma unroll
  for (int r = 0; r < E; ++r) Y[g * YS + LN * r + s] = x[r];
  __syncthreads();
  const float c = c_dev ? (float)(*c_dev) : c_val;
  if (plane == 0) {
    // the real planes kt = 0 and kt = m/2, packed as P_0 + i P_{m/2}: separate
    // their row spectra with the partner column -ky, divide each by its own
    // eigenvalue, recombine as Y_0 + i Y_{m/2}
    const int gp = brev((N - brev(g, LOGN)) & (N - 1), LOGN);
    float2 xh[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float2 a = Y[(LN * r + s) * YS + g];
      const float2 d = Y[(LN * r + s) * YS + gp];
      x[r] = make_float2(0.5f * (a.x + d.x), 0.5f * (a.y - d.y));
      xh[r] = make_float2(0.5f * (a.y + d.y), 0.5f * (d.x - a.x));
    }
    __syncthreads();                               // partners read before any write-back
    dif_inlane<LN, E, E / 2>(x, s, twc);
    dif_xlane<LN, E>(x, s, twc);
    dif_inlane<LN, E, E / 2>(xh, s, twc);
    dif_xlane<LN, E>(xh, s, twc);
    const float base0 = c + mu * (sig_t[0] + sg[brev(g, LOGN)]);
    const float baseh = c + mu * (sig_t[gridDim.x] + sg[brev(g, LOGN)]);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const float sk = mu * sg[brev(LN * r + s, LOGN)];
      const float2 y0 = cscale(x[r], 1.f / (base0 + sk)), yh = cscale(xh[r], 1.f / (baseh + sk));
      x[r] = make_float2(y0.x - yh.y, y0.y + yh.x);
    }
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) x[r] = Y[(LN * r + s) * YS + g];
    dif_inlane<LN, E, E / 2>(x, s, twc);
    dif_xlane<LN, E>(x, s, twc);
    const float base = c + mu * (sig_t[plane] + sg[brev(g, LOGN)]);
#pragma unroll
    for (int r = 0; r < E; ++r) x[r] = cscale(x[r], 1.f / (base + mu * sg[brev(LN * r + s, LOGN)]));
  }
  dit_xlane<LN, E>(x, s, twc);
  dit_inlane<LN, E, E / 2>(x, s, twc);
#pragma unroll
  for (int r = 0; r < E; ++r) Y[(LN * r + s) * YS + g] = x[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < E; ++r) x[r] = Y[g * YS + LN * r + s];
  dit_xlane<LN, E>(x, s, twc);
  dit_inlane<LN, E, E / 2>(x, s, twc);
#pragma unroll
  for (int r = 0; r < E; ++r) P[g * N + LN * r + s] = x[r];
}

// ---------------------------------------------------------------------------
// FFT-diagonal solve, eq. (11):  (c I + mu nabla^* nabla) x = rhs, periodic.
// t pass forward (R2C, length m), plane (2-D FFT, divide, inverse), t pass inverse.
// ---------------------------------------------------------------------------
// t pass, forward, diagonal solve: real length m -> complex length m/2 of the
// packed pairs -> untangle -> planes kt = 0 .. m/2 - 1, the two real bins
// kt = 0 and kt = m/2 sharing plane 0 as X_0 + i X_{m/2}.
//
// With SRC != RHS_LOAD the source is the solve's right-hand side, computed
// here per bin (RhsSrc) instead of being read from a stored volume; the u
// solve's instance is the first kernel of an iteration slot
// and clears the previous slot's rejection (G_FIRST).
// p = mu v + Lambda at the two bins k, k + 1 (k even) of one scan column,
// v = shrink(grad xbar - Lambda/mu, phi/mu) as in the v-step (eq. (7)).
// c, cxp, cyp: offsets of the column and of its x + 1 and y + 1 neighbours;
// kn = (k + 2) mod m.  Offsets are per scene and below 2^31.
struct PPair {
  float2 xb;                 // xbar at the two bins
  float px[2], py[2], pt[2];
};

__device__ __forceinline__ PPair p_pair(const float* __restrict__ xb, const float* __restrict__ lam,
                                        const float* __restrict__ phi, float mu, float inv_mu,
                                        uint32_t V, uint32_t c, uint32_t cxp, uint32_t cyp,
                                        uint32_t k, uint32_t kn) {
  PPair r;
  const float2 a = ld2(xb, c + k), ax = ld2(xb, cxp + k), ay = ld2(xb, cyp + k);
  const float an = ld1(xb, c + kn);
  const float2 l0 = ld2(lam, c + k), l1 = ld2(lam, V + c + k), l2 = ld2(lam, 2 * V + c + k);
  const float2 ph = ld2(phi, c + k);
  r.xb = a;
  const float gx[2] = {ax.x - a.x, ax.y - a.y};
  const float gy[2] = {ay.x - a.x, ay.y - a.y};
  const float gt[2] = {a.y - a.x, an - a.y};
  const float lx[2] = {l0.x, l0.y}, ly[2] = {l1.x, l1.y}, lt[2] = {l2.x, l2.y};
  const float pv[2] = {ph.x, ph.y};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float bx = gx[h] - lx[h] * inv_mu;
    const float by = gy[h] - ly[h] * inv_mu;
    const float bt = gt[h] - lt[h] * inv_mu;
    const float sh = shrink_factor(bx * bx + by * by + bt * bt, pv[h] * inv_mu);
    r.px[h] = mu * (bx * sh) + lx[h];
    r.py[h] = mu * (by * sh) + ly[h];
    r.pt[h] = mu * (bt * sh) + lt[h];
  }
  return r;
}

// Right-hand side of a diagonal solve at the bin pairs (2p, 2p + 1),
// p = G r + s, of the block's J scan columns, into x[r] as (rhs_2p, rhs_2p+1):
//   u side:   rhs = L ubar - grad f + nabla^*(mu v + Lambda)             (eqs. (10), (11))
//   tau side: rhs = A u+ + mu3 f + Lambda3 + nabla^*(mu2 w + Lambda2)   (tau-subproblem)
// with nabla^* q = -(backward-difference divergence of q).  Each p = mu v +
// Lambda is formed at the lane's own voxels and at their x - 1 neighbours; the
// y - 1 neighbour's p_y comes from the neighbouring column through LDS (a
// halo column when that column is in another block) and the t - 1
// neighbour's p_t from the previous lane.
// (PL: the pointwise operand of the block's columns is in LDS, gfl [J][m]:
// grad f (RHS_U) instead of rs.gf, A u+ (RHS_TAU) instead of au;
// active: this thread's wave takes part, the others only meet the barrier)
template <int SRC, int G, int E, int J, int M, int NT, bool PL = false>
__device__ __forceinline__ void rhs_pairs(float2 (&x)[E], const RhsSrc& rs, const DevCtl* ctl,
                                          const float* __restrict__ xb,
                                          const float* __restrict__ au, int col0, int b, int s,
                                          int tid, int nn, float* pyl,
                                          const float* gfl = nullptr, bool active = true) {
  const int logn = rs.logn;
  const uint32_t N = 1u << logn, V = (uint32_t)nn * M;
  const float mu = rs.mu, inv_mu = 1.f / mu;
  auto cof = [&](uint32_t i, uint32_t j) { return (((i & (N - 1)) << logn) | (j & (N - 1))) * (uint32_t)M; };
  const uint32_t col = col0 + b, i = col >> logn, j = col & (N - 1);
  const uint32_t c = cof(i, j), cxp = cof(i + 1, j), cyp = cof(i, j + 1);
  const uint32_t cxm = cof(i - 1, j), cxmyp = cof(i - 1, j + 1);
  // p_y of the column before the block's first one (y - 1 of column col0)
  if (J < (int)N) {
    const uint32_t i0 = (uint32_t)col0 >> logn, j0 = col0 & (N - 1);
    const uint32_t ch = cof(i0, j0 - 1), chxp = cof(i0 + 1, j0 - 1), chyp = cof(i0, j0);
    for (int h = tid; h < M / 2; h += NT) {
      const PPair q = p_pair(xb, rs.lam, rs.phi, mu, inv_mu, V, ch, chxp, chyp, 2 * h,
                             (2 * h + 2) & (M - 1));
      pyl[2 * h] = q.py[0];
      pyl[2 * h + 1] = q.py[1];
    }
  }
  // x gets everything but the two neighbour terms that other lanes supply
  float t1[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (!active) break;
    const uint32_t k = 2 * (G * r + s), kn = (k + 2) & (M - 1);
    const PPair q = p_pair(xb, rs.lam, rs.phi, mu, inv_mu, V, c, cxp, cyp, k, kn);
    const PPair qm = p_pair(xb, rs.lam, rs.phi, mu, inv_mu, V, cxm, c, cxmyp, k, kn);
    pyl[(b + 1) * M + k] = q.py[0];
    pyl[(b + 1) * M + k + 1] = q.py[1];
    float b0, b1;
    if constexpr (SRC == RHS_U) {
      const float L = (float)ctl->L;
      float2 g;
      if constexpr (PL) g = *reinterpret_cast<const float2*>(gfl + b * M + k);
      else g = ld2(rs.gf, c + k);
      b0 = L * q.xb.x - g.x;
      b1 = L * q.xb.y - g.y;
    } else {
      float2 a;
      if constexpr (PL) a = *reinterpret_cast<const float2*>(gfl + b * M + k);
      else a = ld2(au, c + k);
      const float2 l3 = ld2(rs.lam3, c + k), t0 = ld2(rs.tau0, c + k);
      const bool kept = rs.mask[col] != 0;
      const float ik = 1.f / (rs.lambda + rs.mu3), im = 1.f / rs.mu3;
      const float f0 = f_at(q.xb.x, l3.x, t0.x, kept, rs.lambda, rs.mu3, ik, im);
      const float f1 = f_at(q.xb.y, l3.y, t0.y, kept, rs.lambda, rs.mu3, ik, im);
      b0 = a.x + rs.mu3 * f0 + l3.x;
      b1 = a.y + rs.mu3 * f1 + l3.y;
    }
    x[r].x = b0 - ((q.px[0] - qm.px[0]) + q.py[0] + q.pt[0]);
    x[r].y = b1 - ((q.px[1] - qm.px[1]) + q.py[1] + (q.pt[1] - q.pt[0]));
    t1[r] = q.pt[1];
    // finish every second pair here (no sinking of its arithmetic past the
    // loop): two pairs' loads in flight at a time, without spills
    if ((r & 1) == 1 || r == E - 1) {
      if (r & 1) asm volatile("" : "+v"(x[r - 1].x), "+v"(x[r - 1].y), "+v"(t1[r - 1]));
      asm volatile("" : "+v"(x[r].x), "+v"(x[r].y), "+v"(t1[r]));
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // p_t at bin k - 1: the second bin of the previous lane's pair (lane G - 1
  // of the previous r for s = 0; bin m - 1 for k = 0)
  float up[E];
#pragma unroll
  for (int r = 0; r < E; ++r) up[r] = active ? __shfl(t1[r], (s + G - 1) & (G - 1), G) : 0.f;
  __syncthreads();
  if (!active) return;
  // slot of the y - 1 neighbour column: previous column, the same row's last
  // column when the block holds whole rows, else the halo
  const int ym = j > 0 ? b : (J >= (int)N ? b + (int)N : 0);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = 2 * (G * r + s);
    x[r].x += pyl[ym * M + k] + (s > 0 ? up[r] : up[(r + E - 1) % E]);
    x[r].y += pyl[ym * M + k + 1];
  }
}

// Forward t pass of a diagonal solve from the right-hand side in registers
// (x[r] = bins 2p, 2p + 1, p = G r + s): complex transform of length m/2,
// untangle, planes kt = 0 .. m/2 - 1 (bins 0 and m/2 packed in plane 0),
// staged coalesced writes.  J columns per block; waves with !act only meet
// the barriers.
template <int LOGM, int J, int NT>
__device__ __forceinline__ void tfwd_solve_from_regs(float2 (&x)[TGeo<LOGM - 1>::E], bool act,
                                                     float2* lds, const float2* tws,
                                                     const float2* twc, int tid, int col0,
                                                     float2* __restrict__ spec, int nn) {
  using T = TGeo<LOGM - 1>;
  constexpr int M = 1 << LOGM, H = M / 2, LOGH = LOGM - 1;
  constexpr int G = T::G, E = T::E, ZS = H + H / 8 + 4;
  const int b = tid / G, s = tid % G;
  __syncthreads();
  float2* z = lds + b * ZS;
  if (act) {
    dif_inlane<G, E, E / 2>(x, s, twc);
    dif_xlane<G, E>(x, s, twc);
#pragma unroll
    for (int r = 0; r < E; ++r) z[zix(G * r + s)] = x[r];
  }
  __syncthreads();
  float2 X[E];
  if (act) {
    float2 XH = make_float2(0.f, 0.f);
#pragma unroll
    for (int r = 0; r <= E; ++r) {
      const int k = r < E ? G * r + s : H;
      if (r == E && s != 0) break;
      const float2 zk = z[zix(brev(k & (H - 1), LOGH))];
      const float2 zm = z[zix(brev((H - k) & (H - 1), LOGH))];
      const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      const float2 o = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
      const float2 wk = k < H ? tws[2 * k] : make_float2(-1.f, 0.f);
      const float2 wo = cmul(wk, o);
      const float2 v = make_float2(e.x + wo.y, e.y - wo.x);
      if (r < E) X[r] = v; else XH = v;
    }
    if (s == 0) X[0].y = XH.x;
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < E; ++r) lds[stg<J>(G * r + s, b)] = X[r];
  }
  __syncthreads();
  lds_to_planes<J, NT, H>(lds, spec, nn, col0, tid);
}

template <int LOGM, int SRC>
__global__ void __launch_bounds__(TGeo<LOGM - 1>::NT)
k_tfwd_solve(const float* __restrict__ src, RhsSrc rs, const float2* __restrict__ tw,
             const float2* __restrict__ twcg, float2* __restrict__ spec, int nn, DevCtl* ctl,
             size_t zs, int gate) {
  using T = TGeo<LOGM - 1>;
  constexpr int M = 1 << LOGM, H = M / 2, LOGH = LOGM - 1;
  constexpr int G = T::G, E = T::E, J = T::J, NT = T::NT, ZS = H + H / 8 + 4;
  constexpr int LDS2 = (J * ZS > stg_size<J>(H + 1)) ? J * ZS : stg_size<J>(H + 1);
  __shared__ float2 lds[LDS2];
  __shared__ float2 tws[M];
  __shared__ float2 twc[H];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  const float* xb = SRC != RHS_LOAD ? vol_resolve(rs.xb, hd, zo) : nullptr;
  const float* au = SRC == RHS_TAU ? vol_resolve(rs.au, hd, zo) : nullptr;
  if (gated_off(hd, gate)) return;
  if ((gate & G_FIRST) && blockIdx.x == 0 && threadIdx.x == 0) ctl->reject = 0;
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  spec = zsh(spec, zo);
  const int tid = threadIdx.x, b = tid / G, s = tid % G;
  const int col0 = xcd_block(blockIdx.x, gridDim.x) * J, col = col0 + b;
  // the tables' loads issue with the operands' (one round trip for both)
  auto t_tws = table_copy<NT, M>(tws, tw);
  auto t_twc = table_copy<NT, H>(twc, twcg);
  t_tws.load(tid);
  t_twc.load(tid);
  float2 x[E];
  if constexpr (SRC == RHS_LOAD) {
    src = zsh(src, zo);
    const float2* src2 = reinterpret_cast<const float2*>(src) + (size_t)col * H;
#pragma unroll
    for (int r = 0; r < E; ++r) x[r] = src2[G * r + s];
  } else {
    rs.gf = zsh(rs.gf, zo);
    rs.lam = zsh(rs.lam, zo);
    rs.phi = zsh(rs.phi, zo);
    rs.lam3 = zsh(rs.lam3, zo);
    rs.tau0 = zsh(rs.tau0, zo);
    rs.mask = zsh(rs.mask, zo);
    // p_y of the halo column and of the block's columns: [J + 1][m] floats
    static_assert((J + 1) * M <= 2 * LDS2, "p_y staging does not fit the transform's LDS");
    rhs_pairs<SRC, G, E, J, M, NT>(x, rs, ctl, xb, au, col0, b, s, tid, nn,
                                   reinterpret_cast<float*>(lds));
  }
  t_tws.store(tid);
  t_twc.store(tid);
  tfwd_solve_from_regs<LOGM, J, NT>(x, true, lds, tws, twc, tid, col0, spec, nn);
}

// t pass, inverse, diagonal solve: planes kt = 0 .. m/2 - 1 (plane 0 packed
// as above) -> C2R (length m).
template <int LOGM>
__global__ void __launch_bounds__(TGeo<LOGM - 1>::NT)
k_tinv_solve(const float2* __restrict__ spec, int nn, const float2* __restrict__ tw,
             const float2* __restrict__ twcg, SolveEpi ep, float scale, const DevCtl* ctl,
             size_t zs, int gate) {
  using T = TGeo<LOGM - 1>;
  constexpr int M = 1 << LOGM, H = M / 2, LOGH = LOGM - 1;
  constexpr int G = T::G, E = T::E, J = T::J, NT = T::NT;
  __shared__ float2 lds[stg_size<J>(H + 1)];
  __shared__ float2 tws[M];
  __shared__ float2 twc[H];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  float* eout = vol_out(ep.out, hd, zo);
  const float* eref = vol_in(ep.ref, hd, zo);
  if (gated_off(hd, gate)) return;
  spec = zsh(spec, zo);
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  ep.partials = zsh(ep.partials, zo);
  const int tid = threadIdx.x, b = tid / G, s = tid % G;
  const int col0 = xcd_block(blockIdx.x, gridDim.x) * J, col = col0 + b;
  copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, H>(twc, twcg),
                planes_copy<J, NT, H>(lds, spec, nn, col0));
  __syncthreads();
  float2 x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = brev(G * r + s, LOGH);
    float2 Xk = lds[stg<J>(k, b)];
    float2 Xm = lds[stg<J>((H - k) & (H - 1), b)];
    if (k == 0) {
      Xm = make_float2(Xk.y, 0.f);
      Xk.y = 0.f;
    }
    const float2 e = make_float2(0.5f * (Xk.x + Xm.x), 0.5f * (Xk.y - Xm.y));
    const float2 o = make_float2(0.5f * (Xk.x - Xm.x), 0.5f * (Xk.y + Xm.y));
    const float2 wo = cmulc(o, tws[2 * k]);
    x[r] = make_float2(e.x - wo.y, e.y + wo.x);
  }
  dit_xlane<G, E>(x, s, twc);
  dit_inlane<G, E, E / 2>(x, s, twc);
  float2* out2 = reinterpret_cast<float2*>(eout) + (size_t)col * H;
  if (!eref) {
#pragma unroll
    for (int r = 0; r < E; ++r) out2[G * r + s] = cscale(x[r], scale);
    return;
  }
  // with a reference (the same for the whole launch): its loads issue
  // together, ahead of the stores and the step partial
  const float2* ref2 = reinterpret_cast<const float2*>(eref) + (size_t)col * H;
  float2 rv[E];
#pragma unroll
  for (int r = 0; r < E; ++r) rv[r] = ref2[G * r + s];
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int p = G * r + s;
    const float2 y = cscale(x[r], scale);
    out2[p] = y;
    const float d0 = y.x - rv[r].x, d1 = y.y - rv[r].y;
    acc += (double)d0 * (double)d0 + (double)d1 * (double)d1;
  }
  double v[1] = {acc};
  const int slots[1] = {SL_STEP};
  block_sum_store<1>(v, ep.partials, slots, kMaxBlocks);
}

// Inverse t pass of a convolution fused with the forward t pass of the
// diagonal solve that consumes its output pointwise:
//   EPI_PLAIN:    the adjoint, grad f = A^T (A ubar - tau0) (eq. (10)), into
//                 the u solve's right-hand side (eq. (11)); grad f is not
//                 written to HBM;
//   EPI_FWD_DUAL: the forward operator, A u+ (written, with the backtracking
//                 partial), into the tau solve's right-hand side (Algorithm 2).
// The output of the block's columns stays in LDS, where the right-hand side
// reads it; the right-hand side's neighbour terms come from volumes this
// launch does not change.  Block geometry of the convolution pass; the solve
// phase runs on J x G_s threads (whole waves).  The spectrum buffer is
// reused in place.
template <int LOGM, bool PK, int EPI>
__global__ void __launch_bounds__(TGeo<LOGM>::NT)
k_tinv_conv_rhs(float2* __restrict__ spec, int nn, ResampleTables S,
                const float2* __restrict__ tw, const float2* __restrict__ twcg, ConvEpi ep,
                float scale, RhsSrc rs, DevCtl* ctl, size_t zs, int gate) {
  static_assert(EPI == EPI_PLAIN || EPI == EPI_FWD_DUAL, "fused epilogues");
  constexpr int SRC = EPI == EPI_PLAIN ? RHS_U : RHS_TAU;
  using T = TGeo<LOGM>;
  using TS = TGeo<LOGM - 1>;
  constexpr int M = 1 << LOGM, H = M / 2, G = T::G, E = T::E, J = T::J, NT = T::NT;
  constexpr int GS = TS::G, ES = TS::E;
  static_assert(J * GS <= NT && (J * GS) % 64 == 0, "solve phase on whole waves");
  constexpr int ZS = M + M / 8 + 4;
  constexpr int LDS2 = (J * ZS > stg_size<J>(M + 1)) ? J * ZS : stg_size<J>(M + 1);
  // LDS as floats: the C2R samples [0, J (m + 4)), the p_y rows of the
  // right-hand side [0, (J + 1) m), grad f at the top [2 LDS2 - J m, 2 LDS2)
  static_assert(2 * LDS2 >= J * (2 * M + 4) && 2 * LDS2 >= (2 * J + 1) * M, "LDS regions");
  constexpr int GFL = 2 * LDS2 - J * M;
  constexpr bool STAGE = M <= 1024;
  constexpr int NNZ = STAGE ? 3 * M + 64 : 1;
  __shared__ float2 lds[LDS2];
  __shared__ float2 tws[M];
  __shared__ float2 twc[M];
  __shared__ int4 scol_l[STAGE ? M : 1];
  __shared__ float sval_l[NNZ];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  const float* xb = vol_resolve(rs.xb, hd, zo);
  float* eout = EPI == EPI_FWD_DUAL ? vol_out(ep.out, hd, zo) : nullptr;
  const float* eau = EPI == EPI_FWD_DUAL ? vol_in(ep.au, hd, zo) : nullptr;
  const float* eaup = EPI == EPI_FWD_DUAL ? vol_in(ep.au_prev, hd, zo) : nullptr;
  if (gated_off(hd, gate)) return;
  if ((gate & G_FIRST) && blockIdx.x == 0 && threadIdx.x == 0) ctl->reject = 0;
  zsh_tables(S, zo);
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  spec = zsh(spec, zo);
  ep.w = zsh(ep.w, zo);
  ep.mask = zsh(ep.mask, zo);
  ep.partials = zsh(ep.partials, zo);
  rs.lam = zsh(rs.lam, zo);
  rs.phi = zsh(rs.phi, zo);
  rs.lam3 = zsh(rs.lam3, zo);
  rs.tau0 = zsh(rs.tau0, zo);
  rs.mask = zsh(rs.mask, zo);
  const int tid = threadIdx.x, b = tid / G, s = tid % G;
  const int col0 = xcd_block(blockIdx.x, gridDim.x) * J, col = col0 + b;
  // tables and the block's planes: one round trip
  if constexpr (STAGE)
    copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, M>(twc, twcg),
                  table_copy<NT, M>(scol_l, S.cols), table_copy<NT, NNZ>(sval_l, S.cvals),
                  planes_copy<J, NT, PK ? M : M + 1>(lds, spec, nn, col0));
  else
    copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, M>(twc, twcg),
                  planes_copy<J, NT, PK ? M : M + 1>(lds, spec, nn, col0));
  const int4* scol = STAGE ? scol_l : S.cols;
  const float* sval = STAGE ? sval_l : S.cvals;
  __syncthreads();
  // adjoint inverse t pass (as k_tinv_conv, plain epilogue)
  float2 x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = brev(G * r + s, LOGM);
    float2 Xk = lds[stg<J>(k, b)];
    float2 Xm = lds[stg<J>(PK ? (M - k) & (M - 1) : M - k, b)];
    if (PK && k == 0) {
      Xm = make_float2(Xk.y, 0.f);
      Xk.y = 0.f;
    }
    const float2 e = make_float2(0.5f * (Xk.x + Xm.x), 0.5f * (Xk.y - Xm.y));
    const float2 o = make_float2(0.5f * (Xk.x - Xm.x), 0.5f * (Xk.y + Xm.y));
    const float2 wo = cmulc(o, tws[k]);
    x[r] = make_float2(e.x - wo.y, e.y + wo.x);
  }
  dit_xlane<G, E>(x, s, twc);
  dit_inlane<G, E, E / 4>(x, s, twc);
#pragma unroll
  for (int r = 0; r < E / 2; ++r) x[r] = cadd(x[r], cmulc(x[r + E / 2], tws[2 * (G * r + s)]));
  __syncthreads();                                 // staging consumed
  float2* g2 = lds + b * (H + 2);
#pragma unroll
  for (int r = 0; r < E / 2; ++r) g2[G * r + s] = cscale(x[r], scale);
  __syncthreads();
  float* gfl = reinterpret_cast<float*>(lds) + GFL;
  {
    const float* g = reinterpret_cast<const float*>(g2);
    const float mk = ep.mask ? (float)ep.mask[col] : 1.f;
    float ca = 1.f, cb = 0.f;
    if constexpr (EPI == EPI_FWD_DUAL) {
      const double beta = ctl->beta;
      ca = (float)(1.0 + beta);
      cb = (float)(-beta);
    }
    double acc0 = 0.0;
    // global operands loaded up front, unconditionally (see k_tinv_conv)
    const bool hw = ep.w != nullptr;
    const float* pw = hw ? ep.w : xb + (size_t)col * M;
    float vw[E], vau[E], vaup[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int k = G * r + s;
      vw[r] = pw[k];
      if constexpr (EPI == EPI_FWD_DUAL) {
        const size_t gi = (size_t)col * M + k;
        vau[r] = eau[gi];
        vaup[r] = eaup[gi];
      }
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int k = G * r + s;
      float tk = st_taps(scol[k], sval, g);
      tk *= hw ? vw[r] : 1.f;
      if constexpr (EPI == EPI_PLAIN) {
        gfl[b * M + k] = tk * mk;
      } else {
        const size_t gi = (size_t)col * M + k;
        eout[gi] = tk;
        gfl[b * M + k] = tk;
        const float d = tk - (ca * vau[r] + cb * vaup[r]);
        acc0 += (double)d * (double)d;
      }
    }
    if constexpr (EPI == EPI_FWD_DUAL) {
      double v[1] = {acc0};
      const int slots[1] = {SL_CHECK};
      block_sum_store<1>(v, ep.partials, slots, kMaxBlocks);
    }
  }
  __syncthreads();                                 // the output in LDS; the samples are free
  // forward t pass of the u solve with its right-hand side
  const bool sact = tid < J * GS;
  const int bs = tid / GS, ss = tid % GS;
  float2 y[ES];
  rhs_pairs<SRC, GS, ES, J, M, NT, true>(y, rs, ctl, xb, nullptr, col0, bs, ss, tid, nn,
                                         reinterpret_cast<float*>(lds), gfl, sact);
  tfwd_solve_from_regs<LOGM, J, NT>(y, sact, lds, tws, twc, tid, col0, spec, nn);
}

// Inverse t pass of the u solve fused with the forward t pass of the
// convolution that follows it (A u+, Algorithms 1 and 2): the solve's real
// output column stays in LDS as the convolution's input, so u+ is not read
// back and one launch and one table staging are saved.  Both passes work on
// the same scan columns, so the spectrum buffer is reused in place (a block
// reads its columns' solve planes before it writes their convolution
// planes).  The block has the convolution pass's geometry (J columns, NT
// threads); the solve phase runs on J x G_s of them (whole waves).
template <int LOGM, bool PK>
__global__ void __launch_bounds__(TGeo<LOGM>::NT)
k_tinv_solve_fwd(float2* __restrict__ spec, int nn, ResampleTables S,
                 const float2* __restrict__ tw, const float2* __restrict__ twcg, SolveEpi ep,
                 float scale, const DevCtl* ctl, size_t zs, int gate) {
  using T = TGeo<LOGM>;
  using TS = TGeo<LOGM - 1>;
  constexpr int M = 1 << LOGM, H = M / 2, LOGH = LOGM - 1;
  constexpr int G = T::G, E = T::E, J = T::J, NT = T::NT;
  constexpr int GS = TS::G, ES = TS::E;
  static_assert(J * GS <= NT && (J * GS) % 64 == 0, "solve phase on whole waves");
  constexpr int ZS = M + M / 8 + 4;
  constexpr int LDS2 = (J * ZS > stg_size<J>(M + 1)) ? J * ZS : stg_size<J>(M + 1);
  static_assert(stg_size<J>(H + 1) <= LDS2, "solve staging fits");
  constexpr bool STAGE = M <= 1024;
  constexpr int NNZ = STAGE ? 3 * M + 64 : 1;
  __shared__ float2 lds[LDS2];
  __shared__ float2 tws[M];
  __shared__ float2 twc[M];
  __shared__ int4 srow_l[STAGE ? M : 1];
  __shared__ float sval_l[NNZ];
  const size_t zo = (size_t)blockIdx.z * zs;
  ctl = zsh(ctl, zo);
  const CtlHead hd = ctl_head(ctl);
  float* eout = vol_out(ep.out, hd, zo);
  const float* eref = vol_in(ep.ref, hd, zo);
  if (gated_off(hd, gate)) return;
  zsh_tables(S, zo);
  spec = zsh(spec, zo);
  tw = zsh(tw, zo);
  twcg = zsh(twcg, zo);
  ep.partials = zsh(ep.partials, zo);
  const int tid = threadIdx.x;
  const int col0 = xcd_block(blockIdx.x, gridDim.x) * J;
  // tables and the block's planes: one round trip
  if constexpr (STAGE)
    copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, M>(twc, twcg),
                  table_copy<NT, M>(srow_l, S.rows), table_copy<NT, NNZ>(sval_l, S.rvals),
                  planes_copy<J, NT, H>(lds, spec, nn, col0));
  else
    copy_together(tid, table_copy<NT, M>(tws, tw), table_copy<NT, M>(twc, twcg),
                  planes_copy<J, NT, H>(lds, spec, nn, col0));
  const int4* srow = STAGE ? srow_l : S.rows;
  const float* sval = STAGE ? sval_l : S.rvals;
  __syncthreads();
  // solve phase: packed real inverse of length m (as k_tinv_solve)
  const bool sact = tid < J * GS;
  const int bs = tid / GS, ss = tid % GS;
  float2 y[ES];
  if (sact) {
#pragma unroll
    for (int r = 0; r < ES; ++r) {
      const int k = brev(GS * r + ss, LOGH);
      float2 Xk = lds[stg<J>(k, bs)];
      float2 Xm = lds[stg<J>((H - k) & (H - 1), bs)];
      if (k == 0) {
        Xm = make_float2(Xk.y, 0.f);
        Xk.y = 0.f;
      }
      const float2 e = make_float2(0.5f * (Xk.x + Xm.x), 0.5f * (Xk.y - Xm.y));
      const float2 o = make_float2(0.5f * (Xk.x - Xm.x), 0.5f * (Xk.y + Xm.y));
      const float2 wo = cmulc(o, tws[2 * k]);
      y[r] = make_float2(e.x - wo.y, e.y + wo.x);
    }
  }
  __syncthreads();                                 // staging consumed: the columns' LDS is reused
  double acc = 0.0;
  if (sact) {
    dit_xlane<GS, ES>(y, ss, twc);
    dit_inlane<GS, ES, ES / 2>(y, ss, twc);
    const int col = col0 + bs;
    float2* out2 = reinterpret_cast<float2*>(eout) + (size_t)col * H;
    // the reference is read unconditionally (the output column stands in
    // when there is none), so its loads are not each behind a branch and a wait
    const bool hr = eref != nullptr;
    const float2* ref2 = reinterpret_cast<const float2*>(hr ? eref : eout) + (size_t)col * H;
    float2* xf2 = lds + bs * ZS;                   // the column's real samples, as pairs
    float2 rv[ES];
#pragma unroll
    for (int r = 0; r < ES; ++r) rv[r] = ref2[GS * r + ss];
#pragma unroll
    for (int r = 0; r < ES; ++r) {
      const int p = GS * r + ss;
      const float2 v = cscale(y[r], scale);
      out2[p] = v;
      xf2[p] = v;
      const float d0 = v.x - rv[r].x, d1 = v.y - rv[r].y;
      acc += hr ? (double)d0 * (double)d0 + (double)d1 * (double)d1 : 0.0;
    }
  }
  if (eref) {
    double v[1] = {acc};
    const int slots[1] = {SL_STEP};
    block_sum_store<1>(v, ep.partials, slots, kMaxBlocks);
  }
  __syncthreads();                                 // every column's u+ in LDS
  // convolution phase: R_z, packed transform of length 2m, planes
  const int b = tid / G, s = tid % G;
  const float* xf = reinterpret_cast<const float*>(lds + b * ZS);
  float xv[E];
#pragma unroll
  for (int r = 0; r < E; ++r) xv[r] = xf[G * r + s];
  tfwd_conv_from_lds<LOGM, PK>(lds, tws, twc, srow, sval, xv, tid, col0, spec, nn);
}

// exponentials staged in LDS by the H^ setup (2m <= this; 32 KB at most)
constexpr int kHqStagedExp = 2048;
// Layout of H^: lane-ordered, the full 2n x 2n spectrum of each kt plane in
// the order the plane kernel's lanes multiply it, so that a wave's load of
// one register reads 64 consecutive entries.  Frequency (fx, fy) in [0, 2n)^2
// sits at position p = brev(fx) (register p / 8, lane p % 8) of a column:
//   n <= 64 (register kernel):  [r][col][s], col = brev(fy) < 2n;
//   n = 128 (half-plane kernel): [h][r][col][s], h = fy % 2 (the ky half),
//                                col = brev(fy / 2) < n.
template <int LOGN>
__device__ __forceinline__ int hq_lane_index(int fx, int fy) {
  constexpr int N = 1 << LOGN, L = 2 * N, LOGL = LOGN + 1, RE = L / 8;
  const int p = brev(fx, LOGL);
  if constexpr (LOGN <= 6) {
    return ((p >> 3) * L + brev(fy, LOGL)) * 8 + (p & 7);
  } else {
    return (((fy & 1) * RE + (p >> 3)) * N + brev(fy >> 1, LOGN)) * 8 + (p & 7);
  }
}

// ---------------------------------------------------------------------------
// H^ setup: the kernel h of eq. (3) is even in dx and dy, so its padded
// spectrum is a real cosine sum in (kx, ky) and a complex exponential in kt:
//   H^[kt][kx][ky] = (1/Z) sum_{dx,dy >= 0} c_dx c_dy cos(pi kx dx / n)
//                    cos(pi ky dy / n) exp(-pi i kt dq(dx,dy) / m),
// c_0 = 1, c_d = 2.  One block per (kt, chunk of ky); FP64 accumulation; the
// inner dy sum is staged in LDS.  Computed for kx, ky in [0, n] (the
// quarter) and stored lane-ordered (hq_lane_index).
// The kernel offsets dq (n <= 64) and, with ET, the exponential table
// exp(-pi i j / m), j < 2m (dynamic LDS, 2m entries), are staged in LDS; 2m is
// a power of two, so the phase index kt q mod 2m is a mask (kt q < 2^31 for
// m <= 2^15).  Offsets outside the cone (dq < 0) enter with weight 0, so the
// sums run branch-free and unrolled (their loads issue together).  Both LDS
// tables a wave sweeps are laid out with the lane index fastest (dq
// transposed to [dy][dx], the inner sums as [dx][ky]): no bank conflicts.
// ---------------------------------------------------------------------------
template <int LOGN, bool ET>
__global__ void __launch_bounds__(256)
k_build_hq(float2* __restrict__ hq, int m, const int* __restrict__ dq,
           const double2* __restrict__ etab, const double* __restrict__ cosn, double invZ) {
  constexpr int N = 1 << LOGN, N1 = N + 1, KYC = N1 < 32 ? N1 : 32;
  constexpr bool DQ = N <= 64;
  __shared__ double2 G[N * KYC];                   // [dx][ky - ky0]
  __shared__ double cs[2 * N];
  __shared__ int dq_l[DQ ? N * N : 1];
  extern __shared__ double2 et_l[];
  const int kt = blockIdx.x, ky0 = blockIdx.y * KYC, tid = threadIdx.x;
  const int nky = (N1 - ky0) < KYC ? (N1 - ky0) : KYC;
  const int pmask = 2 * m - 1;
  for (int i = tid; i < 2 * N; i += blockDim.x) cs[i] = cosn[i];
  if constexpr (DQ) {
    for (int i = tid; i < N * N; i += blockDim.x) dq_l[(i % N) * N + i / N] = dq[i];
  }
  if constexpr (ET) {
    for (int i = tid; i < 2 * m; i += blockDim.x) et_l[i] = etab[i];
  }
  const double2* ets = ET ? et_l : etab;
  __syncthreads();
  // inner sum over dy for this block's ky range
  for (int it = tid; it < nky * N; it += blockDim.x) {
    const int kyl = it / N, dx = it % N, ky = ky0 + kyl;
    double sr = 0.0, si = 0.0;
#pragma unroll 8
    for (int dy = 0; dy < N; ++dy) {
      const int q = DQ ? dq_l[dy * N + dx] : dq[dx * N + dy];
      const bool in = q >= 0;
      const double2 e = ets[(kt * (in ? q : 0)) & pmask];
      const double w = in ? (dy ? 2.0 : 1.0) * cs[(ky * dy) & (2 * N - 1)] : 0.0;
      sr += w * e.x;
      si += w * e.y;
    }
    G[dx * KYC + kyl] = make_double2(sr, si);
  }
  __syncthreads();
  // outer sum over dx
  for (int it = tid; it < N1 * nky; it += blockDim.x) {
    const int kyl = it / N1, kx = it % N1, ky = ky0 + kyl;
    double ar = 0.0, ai = 0.0;
#pragma unroll 8
    for (int dx = 0; dx < N; ++dx) {
      const double w = (dx ? 2.0 : 1.0) * cs[(kx * dx) & (2 * N - 1)];
      const double2 gv = G[dx * KYC + kyl];
      ar += w * gv.x;
      ai += w * gv.y;
    }
    const float2 v = make_float2((float)(ar * invZ), (float)(ai * invZ));
    // every image (+-kx, +-ky) of the quarter entry, where the plane kernel
    // multiplies by it (H^ is even in kx and ky)
    constexpr int L = 2 * N;
    float2* Hk = hq + (size_t)kt * L * L;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int fx = (e & 1) ? (L - kx) & (L - 1) : kx;
      const int fy = (e & 2) ? (L - ky) & (L - 1) : ky;
      if (((e & 1) && (kx == 0 || kx == N)) || ((e & 2) && (ky == 0 || ky == N))) continue;
      Hk[hq_lane_index<LOGN>(fx, fy)] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// blocks of the t passes (their partial sums are indexed by block)
int conv_blocks(int logn, int logm) { return (1 << (2 * logn)) / t_columns(logm); }
int solve_blocks(int logn, int logm) { return (1 << (2 * logn)) / t_columns(logm - 1); }
int fused_solve_blocks(int logn, int logm) { return conv_blocks(logn, logm); }

#define CNLOS_TIMED(prof, kind, st, launch)                 \
  do {                                                     \
    const bool t_ = (prof) != nullptr && (prof)->on(kind); \
    if (t_) (void)(prof)->begin(kind, st);                 \
    launch;                                                \
    if (t_) (void)(prof)->end(kind, st);                   \
  } while (0)

// plane pass of a convolution with row pad PAD
template <int LOGN, int PAD>
static void plane_conv_pad(bool adjoint, int M, const Tables& tb, float2* spec, const DevCtl* ctl,
                           size_t zs, size_t hzs, int g, int nz, hipStream_t st) {
  if constexpr (LOGN <= 6) {
    if (adjoint)
      hipLaunchKernelGGL((k_plane_conv_reg<LOGN, true, PAD>), dim3(M, 1, nz),
                         dim3(PlaneRegCfg<LOGN>::NT), 0, st, spec, tb.hq, tb.tw_xy, tb.twc_xy, ctl,
                         zs, hzs, g);
    else
      hipLaunchKernelGGL((k_plane_conv_reg<LOGN, false, PAD>), dim3(M, 1, nz),
                         dim3(PlaneRegCfg<LOGN>::NT), 0, st, spec, tb.hq, tb.tw_xy, tb.twc_xy, ctl,
                         zs, hzs, g);
  } else {
    if (adjoint)
      hipLaunchKernelGGL((k_plane_conv_half<LOGN, true, PAD>), dim3(M, 1, nz),
                         dim3(PlaneHalfCfg<LOGN>::NT), 0, st, spec, tb.hq, tb.tw_xy, tb.twc_xy,
                         ctl, zs, hzs, g);
    else
      hipLaunchKernelGGL((k_plane_conv_half<LOGN, false, PAD>), dim3(M, 1, nz),
                         dim3(PlaneHalfCfg<LOGN>::NT), 0, st, spec, tb.hq, tb.tw_xy, tb.twc_xy,
                         ctl, zs, hzs, g);
  }
}

template <int LOGN>
static void plane_conv(bool adjoint, int M, const Tables& tb, float2* spec, const DevCtl* ctl,
                       size_t zs, size_t hzs, int g, int nz, hipStream_t st) {
  switch (tb.plan.conv_pad) {
    case 1: plane_conv_pad<LOGN, 1>(adjoint, M, tb, spec, ctl, zs, hzs, g, nz, st); break;
    case 4: plane_conv_pad<LOGN, 4>(adjoint, M, tb, spec, ctl, zs, hzs, g, nz, st); break;
    default: plane_conv_pad<LOGN, 2>(adjoint, M, tb, spec, ctl, zs, hzs, g, nz, st); break;
  }
}

// plane pass of a diagonal solve with the plan's row pad
template <int LOGN>
static void plane_solve(int M, const Tables& tb, float2* spec, const double* c_dev, float c_val,
                        float mu, const DevCtl* ctl, size_t zs, int g, int nz, hipStream_t st) {
  const int pad = tb.plan.solve_pad > 0 ? tb.plan.solve_pad : default_solve_pad(LOGN);
#define CNLOS_PSOLVE(P)                                                                         \
  hipLaunchKernelGGL((k_plane_solve_reg<LOGN, P>), dim3(M / 2, 1, nz),                          \
                     dim3(PlaneSolveCfg<LOGN, P>::NT), 0, st, spec, tb.twc_xy, tb.sig_xy, tb.sig_t, \
                     c_dev, c_val, mu, ctl, zs, g)
  switch (pad) {
    case 2: CNLOS_PSOLVE(2); break;
    case 4: CNLOS_PSOLVE(4); break;
    default: CNLOS_PSOLVE(8); break;
  }
#undef CNLOS_PSOLVE
}

template <int LOGN, int LOGM>
static hipError_t conv_impl(const Tables& tb, const ConvSrc& src, float2* spec, bool adjoint,
                            int epi, const ConvEpi& ep, const DevCtl* ctl, const Batch& bt,
                            hipStream_t st, Prof* prof, bool tfwd_done, const RhsSrc* rhs_next) {
  constexpr int N = 1 << LOGN, M = 1 << LOGM, NN = N * N;
  // the plane kernels take the real planes kt = 0, m packed in one (block 0)
  constexpr bool PK = true;
  using TG = TGeo<LOGM>;
  const int nb = NN / TG::J;
  const int nz = bt.nz, g = bt.gate;
  const size_t zs = bt.zs, hzs = bt.hq_shared ? 0 : zs;
  if (!tfwd_done)
    CNLOS_TIMED(prof, KK_T_FWD_CONV, st,
                hipLaunchKernelGGL((k_tfwd_conv<LOGM, PK>), dim3(nb, 1, nz), dim3(TG::NT), 0, st,
                                   src, tb.S, tb.tw_t, tb.twc_t, spec, NN, ctl, zs, g));
  CNLOS_TIMED(prof, KK_PLANE_CONV, st, plane_conv<LOGN>(adjoint, M, tb, spec, ctl, zs, hzs, g, nz, st));
  const float scale = (float)(1.0 / (4.0 * (double)NN * (double)M));
  if (rhs_next) {
    if (epi == EPI_FWD_DUAL)
      CNLOS_TIMED(prof, KK_T_INV_CONV, st,
                  hipLaunchKernelGGL((k_tinv_conv_rhs<LOGM, PK, EPI_FWD_DUAL>), dim3(nb, 1, nz),
                                     dim3(TG::NT), 0, st, spec, NN, tb.S, tb.tw_t, tb.twc_t, ep,
                                     scale, *rhs_next, const_cast<DevCtl*>(ctl), zs, g));
    else if (epi == EPI_PLAIN)
      CNLOS_TIMED(prof, KK_T_INV_CONV, st,
                  hipLaunchKernelGGL((k_tinv_conv_rhs<LOGM, PK, EPI_PLAIN>), dim3(nb, 1, nz),
                                     dim3(TG::NT), 0, st, spec, NN, tb.S, tb.tw_t, tb.twc_t, ep,
                                     scale, *rhs_next, const_cast<DevCtl*>(ctl), zs, g));
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
#define CNLOS_TINV(E)                                                                         \
  CNLOS_TIMED(prof, KK_T_INV_CONV, st,                                                        \
              hipLaunchKernelGGL((k_tinv_conv<LOGM, E, PK>), dim3(nb, 1, nz), dim3(TG::NT), 0, \
                                 st, spec, NN, tb.S, tb.tw_t, tb.twc_t, ep, scale, ctl, zs, g))
  switch (epi) {
    case EPI_PLAIN: CNLOS_TINV(EPI_PLAIN); break;
    case EPI_FWD_OBJ: CNLOS_TINV(EPI_FWD_OBJ); break;
    case EPI_FWD_DUAL: CNLOS_TINV(EPI_FWD_DUAL); break;
    default: CNLOS_TINV(EPI_NORM); break;
  }
#undef CNLOS_TINV
  return hipGetLastError();
}

template <int LOGN, int LOGM>
static hipError_t solve_impl(const Tables& tb, const float* rhs, const RhsSrc& rs, float2* spec,
                             const double* c_dev, double c_val, double mu, const SolveEpi& ep,
                             const DevCtl* ctl, const Batch& bt, hipStream_t st, Prof* prof,
                             bool fwd_next, bool tfwd_done) {
  constexpr int N = 1 << LOGN, M = 1 << LOGM, NN = N * N;
  using TG = TGeo<LOGM - 1>;
  const int nb = NN / TG::J;
  const int nz = bt.nz, g = bt.gate;
  const size_t zs = bt.zs;
  DevCtl* c = const_cast<DevCtl*>(ctl);
  if (!tfwd_done) {
    switch (rs.mode) {
      case RHS_U:
        CNLOS_TIMED(prof, KK_T_FWD_SOLVE, st,
                    hipLaunchKernelGGL((k_tfwd_solve<LOGM, RHS_U>), dim3(nb, 1, nz), dim3(TG::NT), 0,
                                       st, rhs, rs, tb.tw_t, tb.twc_t, spec, NN, c, zs, g));
        break;
      case RHS_TAU:
        CNLOS_TIMED(prof, KK_T_FWD_SOLVE, st,
                    hipLaunchKernelGGL((k_tfwd_solve<LOGM, RHS_TAU>), dim3(nb, 1, nz), dim3(TG::NT), 0,
                                       st, rhs, rs, tb.tw_t, tb.twc_t, spec, NN, c, zs, g));
        break;
      default:
        CNLOS_TIMED(prof, KK_T_FWD_SOLVE, st,
                    hipLaunchKernelGGL((k_tfwd_solve<LOGM, RHS_LOAD>), dim3(nb, 1, nz), dim3(TG::NT),
                                       0, st, rhs, rs, tb.tw_t, tb.twc_t, spec, NN, c, zs, g));
        break;
    }
  }
  CNLOS_TIMED(prof, KK_PLANE_SOLVE, st,
              plane_solve<LOGN>(M, tb, spec, c_dev, (float)c_val, (float)mu, ctl, zs, g, nz, st));
  const float scale = (float)(2.0 / ((double)NN * (double)M));
  if (fwd_next) {
    // with the forward t pass of the convolution of the result
    using TC = TGeo<LOGM>;
    constexpr bool PK = true;
    CNLOS_TIMED(prof, KK_T_INV_SOLVE, st,
                hipLaunchKernelGGL((k_tinv_solve_fwd<LOGM, PK>), dim3(NN / TC::J, 1, nz),
                                   dim3(TC::NT), 0, st, spec, NN, tb.S, tb.tw_t, tb.twc_t, ep,
                                   scale, ctl, zs, g));
  } else {
    CNLOS_TIMED(prof, KK_T_INV_SOLVE, st,
                hipLaunchKernelGGL(k_tinv_solve<LOGM>, dim3(nb, 1, nz), dim3(TG::NT), 0, st, spec,
                                   NN, tb.tw_t, tb.twc_t, ep, scale, ctl, zs, g));
  }
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
                       const Batch& bt, hipStream_t st, Prof* prof, bool tfwd_done,
                       const RhsSrc* rhs_next) {
  CNLOS_DISPATCH_NM(conv_impl, tb, src, spec, adjoint, epi, ep, ctl, bt, st, prof, tfwd_done,
                    rhs_next)
}

hipError_t launch_solve(int logn, int logm, const Tables& tb, const float* rhs, const RhsSrc& rs,
                        float2* spec, const double* c_dev, double c_val, double mu,
                        const SolveEpi& ep, const DevCtl* ctl, const Batch& bt, hipStream_t st,
                        Prof* prof, bool fwd_next, bool tfwd_done) {
  CNLOS_DISPATCH_NM(solve_impl, tb, rhs, rs, spec, c_dev, c_val, mu, ep, ctl, bt, st, prof,
                    fwd_next, tfwd_done)
}

// The real planes kt = 0 and kt = m are transformed together (packed as
// P_0 + i P_m), and the product with H^ separates into (H_0 + H_m)/2 times the
// value plus (H_0 - H_m)/2 times the partner's conjugate (both H^ planes are
// real).  Plane 0 of H^ therefore holds that pair of real factors,
// ((H_0 + H_m)/2, (H_0 - H_m)/2), one load per position; plane m is not read.
__global__ void __launch_bounds__(256) k_hq_pack_real(float2* __restrict__ hq, int m, int plane) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= plane) return;
  const float h0 = hq[q].x, hm = hq[(size_t)m * plane + q].x;
  hq[q] = make_float2(0.5f * (h0 + hm), 0.5f * (h0 - hm));
}

hipError_t launch_build_hq(int logn, int logm, float2* hq, const int* dq, const double2* etab,
                           const double* cosn, double invZ, hipStream_t st) {
  const int m = 1 << logm, n1 = (1 << logn) + 1;
  const int kyc = n1 < 32 ? n1 : 32;
  const dim3 grid(m + 1, (n1 + kyc - 1) / kyc);
  const bool et = 2 * m <= kHqStagedExp;
#define CNLOS_HQ(LN)                                                                           \
  case LN:                                                                                     \
    if (et)                                                                                    \
      hipLaunchKernelGGL((k_build_hq<LN, true>), grid, dim3(256), 2 * m * sizeof(double2), st,  \
                         hq, m, dq, etab, cosn, invZ);                                         \
    else                                                                                       \
      hipLaunchKernelGGL((k_build_hq<LN, false>), grid, dim3(256), 0, st, hq, m, dq, etab,      \
                         cosn, invZ);                                                          \
    break;
  switch (logn) {
    CNLOS_HQ(3)
    CNLOS_HQ(4)
    CNLOS_HQ(5)
    CNLOS_HQ(6)
    CNLOS_HQ(7)
    default: return hipErrorInvalidValue;
  }
#undef CNLOS_HQ
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int plane = 4 << (2 * logn);
  hipLaunchKernelGGL(k_hq_pack_real, dim3((plane + 255) / 256), dim3(256), 0, st, hq, m, plane);
  return hipGetLastError();
}

}  // namespace cnlos
