// Grid-side terms of the training loss and the surfel grid itself:
//   * elevation smoothness over the four grid neighbours (Eq. 10; the
//     neighbours come from the pixel index of the meshgrid, supp. Sec. 3.3)
//     and the LiDAR elevation loss (Eq. 11), both per surfel;
//   * the LiDAR targets: height of the point nearest to each surfel in the
//     xy-plane (Eq. 11);
//   * the meshgrid layout (Sec. 3.1): vehicle positions on a raster, a disk
//     dilation into the road mask, surfels at its pixels indexed by a running
//     count, neighbour indices from adjacent pixels, and the pose-based
//     initial height and rotation (Eq. 4; supp. Sec. 1).
#include <math.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "rogs_internal.h"

namespace rogs {


namespace {

constexpr int kRegBlock = 256;

// Block partial sums of rogs_elev_loss_static: one float per block of the
// largest accepted surfel count (ROGS_ELEV_STATIC_MAX_N).  Each GPU the
// library runs on holds its own copy until the process ends.  Host code uses
// only the per-device address from hipGetSymbolAddress, never this name.
constexpr int64_t kElevStaticFloats = ((int64_t)ROGS_ELEV_STATIC_MAX_N + kRegBlock - 1) / kRegBlock + 1;
static __device__ __align__(256) float scratch[kElevStaticFloats];

// Per surfel i, with r_d = z_i - z_{nbr[d][i]} and a symmetric table (a
// neighbour's opposite neighbour is the surfel itself):
//   loss_i = lambda_s / 4 * sum_d r_d^2 + lambda_z * (z_i - zbar_i)^2
//   dL/dz_i = lambda_s * sum_d r_d + 2 lambda_z (z_i - zbar_i)
// (each edge enters the loss from both ends, hence 2 * 2 / K = 1 for K = 4).
// The gradient goes to out_dz (overwritten) or is added to acc_dz; block sums
// of the loss go to part[blockIdx.x] in a fixed order.
__global__ __launch_bounds__(kRegBlock) void k_elev_reg(int n, const float* __restrict__ z,
                                                        const int32_t* __restrict__ nbr,
                                                        float lam_s, const float* __restrict__ zbar,
                                                        float lam_z, float* __restrict__ out_dz,
                                                        float* __restrict__ acc_dz,
                                                        float* __restrict__ part) {
  __shared__ float s_w[kRegBlock / 64];
  const int i = blockIdx.x * kRegBlock + threadIdx.x;
  float l = 0.0f;
  if (i < n) {
    const float zi = z[i];
    float g = 0.0f;
    if (nbr) {
      float s = 0.0f, t = 0.0f;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const float r = zi - z[nbr[(size_t)d * n + i]];
        s += r * r;
        t += r;
      }
      l = (lam_s * 0.25f) * s;
      g = lam_s * t;
    }
    if (zbar) {
      const float r = zi - zbar[i];
      l += lam_z * (r * r);
      g += (2.0f * lam_z) * r;
    }
    if (out_dz) out_dz[i] = g;
    if (acc_dz) acc_dz[i] += g;
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < kRegBlock / 64; ++w) t += s_w[w];
    part[blockIdx.x] = t;
  }
}

// Sums the block partials in order (one wave, lane-strided then a fixed tree).
__global__ __launch_bounds__(64) void k_reg_total(const float* __restrict__ part, int nb,
                                                  float* __restrict__ total, int accumulate) {
  float t = 0.0f;
  for (int k = threadIdx.x; k < nb; k += 64) t += part[k];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (threadIdx.x == 0) *total = accumulate ? (*total + t) : t;
}

// Nearest point in the xy-plane: squared distance in binary64 of the binary32
// inputs, ties to the lower point index.  The points are bucketed into a
// uniform grid over the bounding box of surfels and points (about 2 m cells,
// m = point count; the cell size is chosen on the device), sorted into cell
// order by counting, and each surfel searches rings of cells around its own
// cell outward.  After ring r every point not yet visited lies at least
// r h - (rounding) from the surfel, so the search stops once the best
// distance is below r h - 1e-6 m: the result is the brute-force one.
constexpr int kNNBlock = 256;

struct NNGrid {
  double x0, y0, h, inv_h;
  int32_t W, H;
  int32_t pad[2];
};
static_assert(sizeof(NNGrid) == 48, "grid header");

__device__ __forceinline__ void nn_cell(const NNGrid& g, float x, float y, int& cx, int& cy) {
#pragma clang fp contract(off)
  const double fx = floor(((double)x - g.x0) * g.inv_h);
  const double fy = floor(((double)y - g.y0) * g.inv_h);
  cx = fx < 0.0 ? 0 : (fx > (double)(g.W - 1) ? g.W - 1 : (int)fx);
  cy = fy < 0.0 ? 0 : (fy > (double)(g.H - 1) ? g.H - 1 : (int)fy);
}

// Per-block minimum and maximum of x and y over the surfels and the points.
__global__ __launch_bounds__(kNNBlock) void k_nn_bbox(int n, const float* __restrict__ x,
                                                      const float* __restrict__ y, int m,
                                                      const float* __restrict__ px,
                                                      const float* __restrict__ py,
                                                      float4* __restrict__ part) {
  __shared__ float4 s[kNNBlock / 64];
  float4 b = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
  const int64_t tot = (int64_t)n + m;
  for (int64_t k = (int64_t)blockIdx.x * kNNBlock + threadIdx.x; k < tot;
       k += (int64_t)gridDim.x * kNNBlock) {
    const float u = k < n ? x[k] : px[k - n];
    const float v = k < n ? y[k] : py[k - n];
    b.x = fminf(b.x, u); b.y = fminf(b.y, v); b.z = fmaxf(b.z, u); b.w = fmaxf(b.w, v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    b.x = fminf(b.x, __shfl_xor(b.x, o, 64)); b.y = fminf(b.y, __shfl_xor(b.y, o, 64));
    b.z = fmaxf(b.z, __shfl_xor(b.z, o, 64)); b.w = fmaxf(b.w, __shfl_xor(b.w, o, 64));
  }
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kNNBlock / 64; ++w) {
      b.x = fminf(b.x, s[w].x); b.y = fminf(b.y, s[w].y);
      b.z = fmaxf(b.z, s[w].z); b.w = fmaxf(b.w, s[w].w);
    }
    part[blockIdx.x] = b;
  }
}

// The grid over the bounding box (block 0): cell size h with about 2m cells,
// enlarged until W * H <= max_cells.  Every block clears its share of the
// max_cells + 1 cell counters.
__global__ __launch_bounds__(256) void k_nn_grid(const float4* __restrict__ part, int nparts,
                                                 int m, int64_t max_cells,
                                                 NNGrid* __restrict__ g,
                                                 uint32_t* __restrict__ cnt) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k <= max_cells;
       k += (int64_t)gridDim.x * 256)
    cnt[k] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float4 b = part[0];
    for (int k = 1; k < nparts; ++k) {
      b.x = fminf(b.x, part[k].x); b.y = fminf(b.y, part[k].y);
      b.z = fmaxf(b.z, part[k].z); b.w = fmaxf(b.w, part[k].w);
    }
    const double ex = (double)b.z - (double)b.x, ey = (double)b.w - (double)b.y;
    double h = sqrt((ex * ey) / (2.0 * (double)m));
    if (!(h > 0.0)) h = fmax(fmax(ex, ey) / (2.0 * (double)m), 1e-3);
    for (int it = 0; it < 200; ++it) {
      const double w = floor(ex / h) + 1.0, hh = floor(ey / h) + 1.0;
      if (w * hh <= (double)max_cells) break;
      h *= 1.25;
    }
    NNGrid gg;
    gg.x0 = (double)b.x;
    gg.y0 = (double)b.y;
    gg.h = h;
    gg.inv_h = 1.0 / h;
    gg.W = (int32_t)(floor(ex / h) + 1.0);
    gg.H = (int32_t)(floor(ey / h) + 1.0);
    gg.pad[0] = gg.pad[1] = 0;
    *g = gg;
  }
}

// Cell of every point and its rank among the points of its cell.
__global__ __launch_bounds__(kNNBlock) void k_nn_count(int m, const float* __restrict__ px,
                                                       const float* __restrict__ py,
                                                       const NNGrid* __restrict__ g,
                                                       uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ rank) {
  const int k = blockIdx.x * kNNBlock + threadIdx.x;
  if (k >= m) return;
  const NNGrid gg = *g;
  int cx, cy;
  nn_cell(gg, px[k], py[k], cx, cy);
  rank[k] = atomicAdd(&cnt[(int64_t)cy * gg.W + cx], 1u);
}

// Points in cell order: index, x, y at their cell's start plus their rank.
__global__ __launch_bounds__(kNNBlock) void k_nn_scatter(int m, const float* __restrict__ px,
                                                         const float* __restrict__ py,
                                                         const NNGrid* __restrict__ g,
                                                         const uint32_t* __restrict__ start,
                                                         const uint32_t* __restrict__ rank,
                                                         int32_t* __restrict__ sidx,
                                                         float2* __restrict__ sxy) {
  const int k = blockIdx.x * kNNBlock + threadIdx.x;
  if (k >= m) return;
  const NNGrid gg = *g;
  int cx, cy;
  const float u = px[k], v = py[k];
  nn_cell(gg, u, v, cx, cy);
  const uint32_t p = start[(int64_t)cy * gg.W + cx] + rank[k];
  sidx[p] = k;
  sxy[p] = make_float2(u, v);
}

__device__ __forceinline__ void nn_visit(const uint32_t* __restrict__ start,
                                         const int32_t* __restrict__ sidx,
                                         const float2* __restrict__ sxy, int64_t cell, double xi,
                                         double yi, double& best, int& bi) {
#pragma clang fp contract(off)
  const uint32_t a = start[cell], b = start[cell + 1];
  for (uint32_t s = a; s < b; ++s) {
    const float2 p = sxy[s];
    const double dx = xi - (double)p.x;
    const double dy = yi - (double)p.y;
    const double d2 = dx * dx + dy * dy;
    const int k = sidx[s];
    if (d2 < best || (d2 == best && k < bi)) {
      best = d2;
      bi = k;
    }
  }
}

__global__ __launch_bounds__(kNNBlock) void k_nn_search(int n, const float* __restrict__ x,
                                                        const float* __restrict__ y,
                                                        const NNGrid* __restrict__ g,
                                                        const uint32_t* __restrict__ start,
                                                        const int32_t* __restrict__ sidx,
                                                        const float2* __restrict__ sxy,
                                                        const float* __restrict__ pz,
                                                        float* __restrict__ zbar,
                                                        int32_t* __restrict__ idx) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * kNNBlock + threadIdx.x;
  if (i >= n) return;
  const NNGrid gg = *g;
  const float xf = x[i], yf = y[i];
  const double xi = (double)xf, yi = (double)yf;
  int cx, cy;
  nn_cell(gg, xf, yf, cx, cy);
  double best = __longlong_as_double(0x7ff0000000000000ll);
  int bi = -1;
  const int rmax = max(gg.W, gg.H);
  for (int r = 0; r <= rmax; ++r) {
    if (r == 0) {
      nn_visit(start, sidx, sxy, (int64_t)cy * gg.W + cx, xi, yi, best, bi);
    } else {
      // the ring at Chebyshev distance r: its rows cy - r and cy + r, then
      // the columns cx - r and cx + r between them
      for (int dy = -r; dy <= r; dy += 2 * r) {
        const int j = cy + dy;
        if (j < 0 || j >= gg.H) continue;
        for (int ii = max(cx - r, 0); ii <= min(cx + r, gg.W - 1); ++ii)
          nn_visit(start, sidx, sxy, (int64_t)j * gg.W + ii, xi, yi, best, bi);
      }
      for (int dx = -r; dx <= r; dx += 2 * r) {
        const int ii = cx + dx;
        if (ii < 0 || ii >= gg.W) continue;
        for (int j = max(cy - r + 1, 0); j <= min(cy + r - 1, gg.H - 1); ++j)
          nn_visit(start, sidx, sxy, (int64_t)j * gg.W + ii, xi, yi, best, bi);
      }
    }
    // points outside rings 0..r are at least r h from the surfel
    const double bound = (double)r * gg.h - 1e-6;
    if (bi >= 0 && bound > 0.0 && best < bound * bound) break;
  }
  zbar[i] = bi >= 0 ? pz[bi] : 0.0f;
  if (idx) idx[i] = bi;
}

// ------------------------------------------------------------ meshgrid layout

__global__ void k_pose_pixels(int np, const rogs_pose* __restrict__ poses, double x0, double y0,
                              float h, int2* __restrict__ pix) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  pix[k] = make_int2((int)floor(((double)poses[k].x - x0) / (double)h + 0.5),
                     (int)floor(((double)poses[k].y - y0) / (double)h + 0.5));
}

// Disk dilation by stamping: every pose marks the pixels within radius r of
// its cell (all writers store the same value 1).
__global__ void k_stamp(int np, const int2* __restrict__ pix, int r, int W, int H,
                        uint32_t* __restrict__ mask) {
  const int k = blockIdx.x;
  if (k >= np) return;
  const int2 c = pix[k];
  const int side = 2 * r + 1;
  for (int t = threadIdx.x; t < side * side; t += blockDim.x) {
    const int dy = t / side - r, dx = t % side - r;
    if ((int64_t)dx * dx + (int64_t)dy * dy > (int64_t)r * r) continue;
    const int col = c.x + dx, row = c.y + dy;
    if (col < 0 || col >= W || row < 0 || row >= H) continue;
    mask[(size_t)row * W + col] = 1u;
  }
}

__device__ __forceinline__ void quat_of(const float* R, float q[4]) {
#pragma clang fp contract(off)
  const double m00 = R[0], m01 = R[1], m02 = R[2], m10 = R[3], m11 = R[4], m12 = R[5],
               m20 = R[6], m21 = R[7], m22 = R[8];
  double w, a, b, d;
  const double tr = m00 + m11 + m22;
  if (tr > 0.0) {
    const double s = sqrt(tr + 1.0) * 2.0;
    w = 0.25 * s; a = (m21 - m12) / s; b = (m02 - m20) / s; d = (m10 - m01) / s;
  } else if (m00 > m11 && m00 > m22) {
    const double s = sqrt(1.0 + m00 - m11 - m22) * 2.0;
    w = (m21 - m12) / s; a = 0.25 * s; b = (m01 + m10) / s; d = (m02 + m20) / s;
  } else if (m11 > m22) {
    const double s = sqrt(1.0 + m11 - m00 - m22) * 2.0;
    w = (m02 - m20) / s; a = (m01 + m10) / s; b = 0.25 * s; d = (m12 + m21) / s;
  } else {
    const double s = sqrt(1.0 + m22 - m00 - m11) * 2.0;
    w = (m10 - m01) / s; a = (m02 + m20) / s; b = (m12 + m21) / s; d = 0.25 * s;
  }
  if (w < 0.0) { w = -w; a = -a; b = -b; d = -d; }
  q[0] = (float)w; q[1] = (float)a; q[2] = (float)b; q[3] = (float)d;
}

// One thread per raster pixel: road pixels get their surfel (position,
// neighbours, Eq. 4 height, rotation of the nearest pose); idx = -1 off the
// road.  mask holds 0/1, sidx the running count (exclusive scan of mask).
__global__ void k_layout_fill(int W, int H, const uint32_t* __restrict__ mask,
                              const uint32_t* __restrict__ sidx, double x0, double y0, float h,
                              int np, const rogs_pose* __restrict__ poses, int64_t n,
                              int32_t* __restrict__ idx, float* __restrict__ x,
                              float* __restrict__ y, float* __restrict__ z, float* __restrict__ q,
                              int32_t* __restrict__ nbr) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)W * H) return;
  if (!mask[p]) {
    idx[p] = -1;
    return;
  }
  const int row = (int)(p / W), col = (int)(p - (int64_t)row * W);
  const int32_t i = (int32_t)sidx[p];
  idx[p] = i;
  const float xi = (float)(x0 + (double)col * (double)h);
  const float yi = (float)(y0 + (double)row * (double)h);
  x[i] = xi;
  y[i] = yi;
  auto at = [&](int rr, int cc) -> int32_t {
    if (rr < 0 || rr >= H || cc < 0 || cc >= W) return i;
    const int64_t o = (int64_t)rr * W + cc;
    return mask[o] ? (int32_t)sidx[o] : i;
  };
  nbr[0 * n + i] = at(row - 1, col);
  nbr[1 * n + i] = at(row + 1, col);
  nbr[2 * n + i] = at(row, col - 1);
  nbr[3 * n + i] = at(row, col + 1);
  double best = __longlong_as_double(0x7ff0000000000000ll);
  int bk = 0;
  for (int k = 0; k < np; ++k) {
    const double dx = (double)xi - (double)poses[k].x;
    const double dy = (double)yi - (double)poses[k].y;
    const double d2 = dx * dx + dy * dy;
    if (d2 < best) {
      best = d2;
      bk = k;
    }
  }
  const rogs_pose& P = poses[bk];
  const double n31 = P.R[2], n32 = P.R[5], n33 = P.R[8];
  const double t = (n31 * ((double)xi - (double)P.x) + n32 * ((double)yi - (double)P.y)) / n33;
  z[i] = (float)((double)P.z - t);
  float qq[4];
  quat_of(P.R, qq);
  for (int c = 0; c < 4; ++c) q[(size_t)c * n + i] = qq[c];
}

}  // namespace

int64_t elev_reg_blocks(int n) { return (n + kRegBlock - 1) / kRegBlock; }

void launch_elev_reg(int n, const float* z, const int32_t* nbr, float lam_s, const float* zbar,
                     float lam_z, float* out_dz, float* acc_dz, float* part, float* total,
                     bool accumulate_total, hipStream_t st) {
  const int nb = (int)elev_reg_blocks(n);
  hipLaunchKernelGGL(k_elev_reg, dim3((unsigned)nb), dim3(kRegBlock), 0, st, n, z, nbr, lam_s,
                     zbar, lam_z, out_dz, acc_dz, part);
  hipLaunchKernelGGL(k_reg_total, dim3(1), dim3(64), 0, st, part, nb, total,
                     accumulate_total ? 1 : 0);
}

size_t lidar_scratch_bytes(int n, int m) {
  const int64_t cells = 2 * (int64_t)m + 64;
  const int64_t nparts = std::min<int64_t>(((int64_t)n + m + kNNBlock - 1) / kNNBlock, 1024);
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = (o + b + 255) / 256 * 256; return r; };
  take(sizeof(NNGrid));
  take(16 * (size_t)nparts);
  take(4 * (size_t)(cells + 2));
  take(4 * scan_tmp_words(cells + 1));
  take(4 * (size_t)m);       // rank
  take(4 * (size_t)m);       // sorted index
  take(8 * (size_t)m);       // sorted x, y
  return o;
}

void launch_lidar_nn(int n, const float* x, const float* y, int m, const float* px,
                     const float* py, const float* pz, float* zbar, int32_t* idx, void* scratch,
                     hipStream_t st) {
  const int64_t cells = 2 * (int64_t)m + 64;
  const int64_t nparts = std::min<int64_t>(((int64_t)n + m + kNNBlock - 1) / kNNBlock, 1024);
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = (o + b + 255) / 256 * 256; return r; };
  char* base = static_cast<char*>(scratch);
  NNGrid* g = reinterpret_cast<NNGrid*>(base + take(sizeof(NNGrid)));
  float4* part = reinterpret_cast<float4*>(base + take(16 * (size_t)nparts));
  uint32_t* cnt = reinterpret_cast<uint32_t*>(base + take(4 * (size_t)(cells + 2)));
  uint32_t* tmp = reinterpret_cast<uint32_t*>(base + take(4 * scan_tmp_words(cells + 1)));
  uint32_t* rank = reinterpret_cast<uint32_t*>(base + take(4 * (size_t)m));
  int32_t* sidx = reinterpret_cast<int32_t*>(base + take(4 * (size_t)m));
  float2* sxy = reinterpret_cast<float2*>(base + take(8 * (size_t)m));
  hipLaunchKernelGGL(k_nn_bbox, dim3((unsigned)nparts), dim3(kNNBlock), 0, st, n, x, y, m, px, py,
                     part);
  const unsigned cb = (unsigned)std::min<int64_t>((cells + 1 + 2047) / 2048, 4096);
  hipLaunchKernelGGL(k_nn_grid, dim3(cb), dim3(256), 0, st, part, (int)nparts, m, cells, g, cnt);
  const unsigned pb = (unsigned)((m + kNNBlock - 1) / kNNBlock);
  hipLaunchKernelGGL(k_nn_count, dim3(pb), dim3(kNNBlock), 0, st, m, px, py, g, cnt, rank);
  // cells beyond the grid's W * H hold zeros: the scan runs over the bound
  scan_u32(cnt, cnt, cells + 1, nullptr, tmp, st);
  hipLaunchKernelGGL(k_nn_scatter, dim3(pb), dim3(kNNBlock), 0, st, m, px, py, g, cnt, rank, sidx,
                     sxy);
  hipLaunchKernelGGL(k_nn_search, dim3((unsigned)((n + kNNBlock - 1) / kNNBlock)), dim3(kNNBlock),
                     0, st, n, x, y, g, cnt, sidx, sxy, pz, zbar, idx);
}

size_t layout_scratch_bytes(int W, int H, int np) {
  const int64_t cells = (int64_t)W * H;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up(8 * (size_t)np) + 2 * up(4 * (size_t)cells) + up(4 * scan_tmp_words(cells)) + 256;
}

void launch_layout_mask(const rogs_pose* poses, int np, double x0, double y0, float h, int W,
                        int H, int r, void* scratch, uint32_t* n_dev, hipStream_t st) {
  const int64_t cells = (int64_t)W * H;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  uint8_t* s = static_cast<uint8_t*>(scratch);
  int2* pix = reinterpret_cast<int2*>(s);
  uint32_t* mask = reinterpret_cast<uint32_t*>(s + up(8 * (size_t)np));
  uint32_t* sidx = mask + up(4 * (size_t)cells) / 4;
  uint32_t* tmp = sidx + up(4 * (size_t)cells) / 4;
  hipLaunchKernelGGL(k_pose_pixels, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, poses,
                     x0, y0, h, pix);
  fill_u32(mask, 0u, cells, st);
  hipLaunchKernelGGL(k_stamp, dim3((unsigned)np), dim3(256), 0, st, np, pix, r, W, H, mask);
  scan_u32(mask, sidx, cells, n_dev, tmp, st);
}

void launch_layout_fill(const rogs_pose* poses, int np, double x0, double y0, float h, int W,
                        int H, void* scratch, int64_t n, int32_t* idx, float* x, float* y,
                        float* z, float* q, int32_t* nbr, hipStream_t st) {
  const int64_t cells = (int64_t)W * H;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  uint8_t* s = static_cast<uint8_t*>(scratch);
  const uint32_t* mask = reinterpret_cast<const uint32_t*>(s + up(8 * (size_t)np));
  const uint32_t* sidx = mask + up(4 * (size_t)cells) / 4;
  hipLaunchKernelGGL(k_layout_fill, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, W, H,
                     mask, sidx, x0, y0, h, np, poses, n, idx, x, y, z, q, nbr);
}

}  // namespace rogs

extern "C" {

size_t rogs_elev_scratch_bytes(int32_t n) {
  return n < 1 ? 0 : (size_t)(rogs::elev_reg_blocks(n) + 1) * 4;
}

int rogs_elev_loss(rogs_ctx* c, int32_t n, const float* z, const int32_t* nbr, float lambda_smooth,
                   const float* zbar, float lambda_z, float* dz, float* loss_out, void* scratch,
                   size_t scratch_bytes, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (n < 1 || !z || !dz || !loss_out || !scratch)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_elev_loss: null argument or n < 1");
  if (scratch_bytes < rogs_elev_scratch_bytes(n))
    return rogs::ctx_fail(c, ROGS_ENOMEM, "rogs_elev_loss: scratch too small");
  if ((nbr && !std::isfinite(lambda_smooth)) || (zbar && !std::isfinite(lambda_z)))
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_elev_loss: weights must be finite");
  if (!nbr && !zbar) return ROGS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* part = static_cast<float*>(scratch);
  rogs::launch_elev_reg(n, z, nbr, lambda_smooth, zbar, lambda_z, nullptr, dz, part, loss_out,
                        true, st);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROGS_OK
                         : rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_elev_loss: ") +
                                                            hipGetErrorString(e));
}

int rogs_elev_loss_static(rogs_ctx* c, int32_t n, const float* z, const int32_t* nbr,
                          float lambda_smooth, const float* zbar, float lambda_z, float* dz,
                          float* loss_out, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (n < 1 || !z || !dz || !loss_out)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_elev_loss_static: null argument or n < 1");
  if (n > ROGS_ELEV_STATIC_MAX_N)
    return rogs::ctx_fail(c, ROGS_EINVAL,
                          "rogs_elev_loss_static: n exceeds ROGS_ELEV_STATIC_MAX_N (" +
                              std::to_string(ROGS_ELEV_STATIC_MAX_N) + ")");
  if ((nbr && !std::isfinite(lambda_smooth)) || (zbar && !std::isfinite(lambda_z)))
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_elev_loss_static: weights must be finite");
  // the array's device address, looked up once per device with that device current
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_elev_loss_static: hipGetDevice: ") +
                                            hipGetErrorString(e));
  if (dev < 0 || dev >= 64)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_elev_loss_static: device ordinal above 63");
  void* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(rogs::scratch));
      if (e != hipSuccess || !p)
        return rogs::ctx_fail(c, ROGS_EHIP,
                              std::string("rogs_elev_loss_static: hipGetSymbolAddress: ") +
                                  hipGetErrorString(e));
      addr[dev] = p;
    }
    part = addr[dev];
  }
  if (!nbr && !zbar) return ROGS_OK;
  // every block overwrites its own partial before the total reads it: nothing
  // in the array needs clearing between calls
  rogs::launch_elev_reg(n, z, nbr, lambda_smooth, zbar, lambda_z, nullptr, dz,
                        static_cast<float*>(part), loss_out, true,
                        static_cast<hipStream_t>(stream));
  e = hipGetLastError();
  return e == hipSuccess ? ROGS_OK
                         : rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_elev_loss_static: ") +
                                                            hipGetErrorString(e));
}

size_t rogs_lidar_scratch_bytes(int32_t n, int32_t m) {
  if (n < 1 || m < 1) return 0;
  return rogs::lidar_scratch_bytes(n, m);
}

int rogs_lidar_targets(rogs_ctx* c, int32_t n, const float* x, const float* y, int32_t m,
                       const float* px, const float* py, const float* pz, float* zbar,
                       int32_t* idx, void* scratch, size_t scratch_bytes, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (n < 1 || m < 1 || !x || !y || !px || !py || !pz || !zbar || !scratch)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_lidar_targets: null argument or empty set");
  if (m > (1 << 29))
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_lidar_targets: at most 2^29 points");
  if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_lidar_targets: scratch must be 256-byte aligned");
  if (scratch_bytes < rogs_lidar_scratch_bytes(n, m))
    return rogs::ctx_fail(c, ROGS_ENOMEM, "rogs_lidar_targets: scratch too small");
  rogs::launch_lidar_nn(n, x, y, m, px, py, pz, zbar, idx, scratch,
                        static_cast<hipStream_t>(stream));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ROGS_OK
                         : rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_lidar_targets: ") +
                                                            hipGetErrorString(e));
}

size_t rogs_meshgrid_scratch_bytes(int32_t W, int32_t H, int32_t n_poses) {
  if (W < 1 || H < 1 || n_poses < 1) return 0;
  return rogs::layout_scratch_bytes(W, H, n_poses);
}

int rogs_meshgrid_layout(rogs_ctx* c, const rogs_pose* poses, int32_t n_poses, double x0,
                         double y0, float spacing, int32_t W, int32_t H, int32_t radius_px,
                         int32_t* idx, int64_t capacity, float* x, float* y, float* z, float* q,
                         int32_t* nbr, int64_t* n_out, void* scratch, size_t scratch_bytes,
                         void* stream) {
  if (!c) return ROGS_EINVAL;
  if (!poses || n_poses < 1 || W < 1 || H < 1 || (int64_t)W * H >= (int64_t(1) << 31) ||
      radius_px < 0 || radius_px > 4096 || !(spacing > 0.0f) || !std::isfinite(x0) ||
      !std::isfinite(y0) || !n_out || !scratch || capacity < 0)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_meshgrid_layout: invalid argument");
  const size_t need = rogs::layout_scratch_bytes(W, H, n_poses);
  if (scratch_bytes < need) return rogs::ctx_fail(c, ROGS_ENOMEM, "rogs_meshgrid_layout: scratch too small");
  const bool query = capacity == 0 && !idx && !x && !y && !z && !q && !nbr;
  if (!query && (!idx || !x || !y || !z || !q || !nbr))
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_meshgrid_layout: null output array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t* n_dev = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(scratch) + need - 256);
  rogs::launch_layout_mask(poses, n_poses, x0, y0, spacing, W, H, radius_px, scratch, n_dev, st);
  uint32_t n_host = 0;
  hipError_t e = hipMemcpyAsync(&n_host, n_dev, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    return rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_meshgrid_layout: ") + hipGetErrorString(e));
  *n_out = (int64_t)n_host;
  if (query) return ROGS_OK;
  if ((int64_t)n_host > capacity)
    return rogs::ctx_fail(c, ROGS_ECAPACITY, "rogs_meshgrid_layout: " + std::to_string(n_host) +
                                                 " road cells exceed the capacity");
  rogs::launch_layout_fill(poses, n_poses, x0, y0, spacing, W, H, scratch, capacity, idx, x, y, z,
                           q, nbr, st);
  e = hipGetLastError();
  return e == hipSuccess ? ROGS_OK
                         : rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_meshgrid_layout: ") +
                                                            hipGetErrorString(e));
}

}  // extern "C"
