// Non-confocal forward model (Section 2's general model, one illumination
// point and a scanned detector grid) applied by direct summation, and its
// transpose.
//
// With the wall normals along z the direction terms reduce, as in the
// confocal case, to the volumetric albedo weight 1 / (d_i^2 d_d^2), where d_i
// is the distance from the illuminated wall point to the voxel and d_d from
// the voxel to the detector; the path d_i + d_d selects the time bin.  The
// model is not shift-invariant (every detector sees every voxel along its own
// ellipsoids), so it has no FFT form: one application evaluates n^4 m paths.
//
// Grid conventions (the confocal ones): detector and voxel column (i, j) at
// x_i = (i + 1/2) W / n - W / 2, depth bin k at z_k = (k + 1/2) R / m with
// R = m c dt / 2, and time bin b holding path lengths in [b, b + 1) c dt.
//
// The time bin is an integer that floating point decides, so it is computed
// in FP64 with every operation in the order written here and no contraction
// into fused multiply-adds; the weight and the sums are FP64 as well, and only
// the stored results are FP32.  Both kernels are deterministic: the forward
// sums each detector's bins in a fixed order (a wave's lanes take consecutive
// depths of one column, whose bins never decrease with depth, and a segmented
// scan over equal bins leaves one writer per bin; each wave owns a histogram),
// and the transpose gathers over the detectors in index order.
#include "cnlos_internal.h"

namespace cnlos {

namespace {

constexpr int kNcWaves = 4;          // waves per block of the forward kernel
constexpr int kNcThreads = 64 * kNcWaves;
constexpr int kNcMaxGridDev = 256;   // detectors per side (the host checks it)

struct NcPath {
  int bin;      // time bin, m when the path leaves the window
  double w;     // albedo weight (1 when not literal)
};

__device__ __forceinline__ double nc_lateral(const NcGeo& g, int i) {
#pragma clang fp contract(off)
  return ((i + 0.5) * g.wall) / g.n - g.wall / 2.0;
}
__device__ __forceinline__ double nc_depth(const NcGeo& g, int k) {
#pragma clang fp contract(off)
  return ((k + 0.5) * g.range) / g.m;
}

// path of the detector at (xd, yd) through voxel (xv, yv, z), where the
// illumination distance di of the voxel is already known
__device__ __forceinline__ NcPath nc_path(const NcGeo& g, double xd, double yd, double xv,
                                          double yv, double z, double di) {
#pragma clang fp contract(off)
  const double ex = xv - xd, ey = yv - yd;
  const double dd = sqrt((ex * ex + ey * ey) + z * z);
  const double len = di + dd;
  const double fb = floor(len / g.cdt);
  NcPath r;
  r.bin = fb < (double)g.m ? (int)fb : g.m;
  r.w = g.literal ? 1.0 / (((di * di) * dd) * dd) : 1.0;
  return r;
}

__device__ __forceinline__ double nc_illum_dist(const NcGeo& g, double xv, double yv, double z) {
#pragma clang fp contract(off)
  const double ex = xv - g.ix, ey = yv - g.iy;
  return sqrt((ex * ex + ey * ey) + z * z);
}

// Lateral positions of the n columns and depths of the m bins, once per block
// (FP64, the same operations as nc_lateral / nc_depth).
__device__ __forceinline__ void nc_positions(const NcGeo& g, double* xs, double* zs, int nt) {
  for (int i = threadIdx.x; i < g.n; i += nt) xs[i] = nc_lateral(g, i);
  if (zs)
    for (int k = threadIdx.x; k < g.m; k += nt) zs[k] = nc_depth(g, k);
  __syncthreads();
}

// tau[det][b] = sum over voxels with path bin b of w u.  One block per
// detector; wave w takes the (column, 64-depth chunk) items w, w + 4, ... in
// order, lane l the depth 64 c + l of the chunk.
__global__ void __launch_bounds__(kNcThreads)
k_nc_forward(NcGeo g, const float* __restrict__ u, float* __restrict__ tau) {
  extern __shared__ double nc_lds[];           // histograms [kNcWaves][m], then depths [m]
  __shared__ double xs[kNcMaxGridDev];
  const int m = g.m, n = g.n;
  double* zs = nc_lds + kNcWaves * m;
  const int det = blockIdx.x, i = det / n, j = det - i * n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < kNcWaves * m; b += kNcThreads) nc_lds[b] = 0.0;
  nc_positions(g, xs, zs, kNcThreads);
  const double xd = xs[i], yd = xs[j];
  const int nchunk = (m + 63) >> 6;
  const int items = n * n * nchunk;
  double* h = nc_lds + wv * m;
  for (int it = wv; it < items; it += kNcWaves) {
    const int col = it / nchunk, k = (it - col * nchunk) * 64 + lane;
    const int p = col / n, q = col - p * n;
    double val = 0.0;
    int bin = m;
    if (k < m) {
      const double xv = xs[p], yv = xs[q], z = zs[k];
      const NcPath r = nc_path(g, xd, yd, xv, yv, z, nc_illum_dist(g, xv, yv, z));
      bin = r.bin;
      val = r.bin < m ? r.w * (double)u[(size_t)col * m + k] : 0.0;
    }
    // segmented inclusive scan over runs of equal bins (bins never decrease
    // with the lane: the path grows with the depth)
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double v2 = __shfl_up(val, d, 64);
      const int b2 = __shfl_up(bin, d, 64);
      val += (lane >= d && b2 == bin) ? v2 : 0.0;
    }
    const int bn = __shfl_down(bin, 1, 64);
    if ((lane == 63 || bn != bin) && bin < m) h[bin] += val;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < m; b += kNcThreads) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kNcWaves; ++w) s += nc_lds[w * m + b];
    tau[(size_t)det * m + b] = (float)s;
  }
}

// u[p][q][k] = sum over detectors (in index order) of w tau[det][bin].
__global__ void __launch_bounds__(256)
k_nc_transpose(NcGeo g, const float* __restrict__ tau, float* __restrict__ u) {
  __shared__ double xs[kNcMaxGridDev];
  const int m = g.m, n = g.n;
  nc_positions(g, xs, nullptr, 256);
  const size_t V = (size_t)n * n * m;
  const size_t vox = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (vox >= V) return;
  const int col = (int)(vox / m), k = (int)(vox - (size_t)col * m);
  const int p = col / n, q = col - p * n;
  const double xv = xs[p], yv = xs[q], z = nc_depth(g, k);
  const double di = nc_illum_dist(g, xv, yv, z);
  double acc = 0.0;
  for (int i = 0; i < n; ++i) {
    const double xd = xs[i];
    // loads are unconditional (bin clamped into the column, term masked), so
    // the unrolled iterations' loads issue together
#pragma unroll 4
    for (int j = 0; j < n; ++j) {
      const NcPath r = nc_path(g, xd, xs[j], xv, yv, z, di);
      const int b = r.bin < m ? r.bin : m - 1;
      const float t = tau[(size_t)(i * n + j) * m + b];
      acc += r.bin < m ? r.w * (double)t : 0.0;
    }
  }
  u[vox] = (float)acc;
}

}  // namespace

size_t nc_forward_lds_bytes(int m) { return (size_t)(kNcWaves + 1) * m * sizeof(double); }

hipError_t launch_nc_forward(const NcGeo& g, const float* u, float* tau, hipStream_t st) {
  // at most (4 + 1) 1024 doubles = 40 KiB of dynamic LDS (the host limits m)
  hipLaunchKernelGGL(k_nc_forward, dim3(g.n * g.n), dim3(kNcThreads), nc_forward_lds_bytes(g.m), st,
                     g, u, tau);
  return hipGetLastError();
}

hipError_t launch_nc_transpose(const NcGeo& g, const float* tau, float* u, hipStream_t st) {
  const size_t V = (size_t)g.n * g.n * g.m;
  hipLaunchKernelGGL(k_nc_transpose, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, g, tau, u);
  return hipGetLastError();
}

}  // namespace cnlos
