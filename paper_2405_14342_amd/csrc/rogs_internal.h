// Internal declarations of librogs: workspace layout, the device view table,
// the FP32 key contract as device code, and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rogs.h"

namespace rogs {

constexpr int kProjBlock = 256;     // threads per block of the per-surfel kernels
constexpr int kSortBlock = 256;     // threads per radix-sort block
constexpr int kSortIPT = 16;        // keys per thread per radix-sort block
constexpr int kSortTile = kSortBlock * kSortIPT;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kScanChunk = 4096;    // elements per block of the generic scan
constexpr int kMaxViews = 4096;

// Device view table entry (one per camera of a batch).
struct ViewDev {
  int64_t pix_off;      // first pixel of the view in the batch's image layout
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float znear;
  float o[2], ex[2], ez[2];
  float lat, fwd;
  int32_t w, h, model;
  int32_t tiles_x, tiles_y;
  int32_t tile_off;     // first global tile index of the view
  int32_t pad[2];
};

// Number of semantic classes with a compiled kernel set.
inline bool sem_supported(int C) { return (C >= 1 && C <= 8) || C == 16; }
inline int feat_stride(int C) { return ((3 + C) + 3) & ~3; }      // rgb + sem, padded to float4
inline int grad_stride(int C) { return ((10 + C) + 3) & ~3; }     // per-pair gradient record

// Layout of one batch inside the caller's workspace (byte offsets).
struct Layout {
  int32_t N = 0, C = 0, V = 0;
  int32_t tw = 16, th = 16, ppl = 4;
  int32_t FS = 0, GS = 0;
  int32_t nb = 0;              // blocks of kProjBlock surfels
  int32_t tile_bits = 1;
  int64_t total_pix = 0, total_tiles = 0, max_view_pix = 0, cap = 0;
  int64_t slots = 0;           // V * N
  int64_t sort_blocks = 0;     // ceil(cap / kSortTile)
  float eps2d = 0.3f, q_cut = 9.0f, alpha_max = 0.99f, t_eps = 1e-6f;
  size_t o_views, o_cnt, o_off, o_rec, o_rect, o_feat, o_part, o_parttmp;
  size_t o_keys, o_vals, o_keys2, o_vals2, o_pslot, o_ranges, o_tfin, o_nlast, o_gpair;
  size_t o_hist, o_histtmp, o_misc, o_lpart, o_mcount;
  size_t total = 0;
};

// misc counters (uint32 slots at o_misc)
enum MiscSlot { kMiscPairs = 0, kMiscOverflow = 1, kMiscCount = 16 };

int make_layout(const rogs_surfels* s, const rogs_camera* cams, int n_views,
                const rogs_render_opts* opts, int64_t cap, Layout* L, const char** why);

template <typename T>
__host__ __device__ inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ------------------------------------------------------------------ contract

struct Proj {
  bool vis;
  float u, v, A, B, C, tz;
  int x0, x1, y0, y1;
};

__device__ __forceinline__ int clamp_tile(float f, int hi) {
  if (!(f > 0.0f)) return 0;
  if (f > (float)hi) return hi;
  return (int)f;
}

// FP32 key contract (see rogs.h).  Compiled without FMA contraction; every
// line is one rounded binary32 operation in the documented order.
__device__ inline Proj project_contract(const ViewDev& c, float eps, float qcut, int tw, int th,
                                        float x, float y, float z, float qw, float qx, float qy,
                                        float qz, float sx, float sy) {
#pragma clang fp contract(off)
  Proj r;
  r.vis = false;
  r.u = r.v = r.A = r.B = r.C = 0.0f;
  r.x0 = r.x1 = r.y0 = r.y1 = 0;
  const float* R = c.R;
  float tx = ((R[0] * x + R[1] * y) + R[2] * z) + c.t[0];
  float ty = ((R[3] * x + R[4] * y) + R[5] * z) + c.t[1];
  float tz = ((R[6] * x + R[7] * y) + R[8] * z) + c.t[2];
  r.tz = tz;
  if (!(tz >= c.znear)) return r;
  if (c.lat > 0.0f) {
    float dx = x - c.o[0];
    float dy = y - c.o[1];
    float a = dx * c.ex[0] + dy * c.ex[1];
    float b = dx * c.ez[0] + dy * c.ez[1];
    if (!(fabsf(a) <= c.lat)) return r;
    if (!(b >= 0.0f && b <= c.fwd)) return r;
  }
  float nn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(nn > 0.0f) || !isfinite(nn)) return r;
  float nq = sqrtf(nn);
  float w = qw / nq, a = qx / nq, b = qy / nq, cc = qz / nq;
  float r1x = 1.0f - 2.0f * (b * b + cc * cc);
  float r1y = 2.0f * (a * b + w * cc);
  float r1z = 2.0f * (a * cc - w * b);
  float r2x = 2.0f * (a * b - w * cc);
  float r2y = 1.0f - 2.0f * (a * a + cc * cc);
  float r2z = 2.0f * (b * cc + w * a);
  float T10 = sx * r1x, T11 = sx * r1y, T12 = sx * r1z;
  float T20 = sy * r2x, T21 = sy * r2y, T22 = sy * r2z;
  float c10 = (R[0] * T10 + R[1] * T11) + R[2] * T12;
  float c11 = (R[3] * T10 + R[4] * T11) + R[5] * T12;
  float c12 = (R[6] * T10 + R[7] * T11) + R[8] * T12;
  float c20 = (R[0] * T20 + R[1] * T21) + R[2] * T22;
  float c21 = (R[3] * T20 + R[4] * T21) + R[5] * T22;
  float c22 = (R[6] * T20 + R[7] * T21) + R[8] * T22;
  float j00, j11, j02, j12, u, v;
  if (c.model == ROGS_PINHOLE) {
    float limx = (0.65f * (float)c.w) / c.fx;
    float limy = (0.65f * (float)c.h) / c.fy;
    float xr = tx / tz, yr = ty / tz;
    float xc = (xr < -limx) ? -limx : xr;
    xc = (limx < xc) ? limx : xc;
    float yc = (yr < -limy) ? -limy : yr;
    yc = (limy < yc) ? limy : yc;
    j00 = c.fx / tz;
    j11 = c.fy / tz;
    j02 = -(j00 * xc);
    j12 = -(j11 * yc);
    u = c.fx * xr + c.cx;
    v = c.fy * yr + c.cy;
  } else {
    j00 = c.fx; j11 = c.fy; j02 = 0.0f; j12 = 0.0f;
    u = c.fx * tx + c.cx;
    v = c.fy * ty + c.cy;
  }
  float m00 = j00 * c10 + j02 * c12;
  float m01 = j00 * c20 + j02 * c22;
  float m10 = j11 * c11 + j12 * c12;
  float m11 = j11 * c21 + j12 * c22;
  float g0 = m00 * m00 + m01 * m01;
  float g1 = m10 * m10 + m11 * m11;
  float s00 = g0 + eps, s11 = g1 + eps;
  float s01 = m00 * m10 + m01 * m11;
  float dm = m00 * m11 - m01 * m10;
  float det = (dm * dm + eps * (g0 + g1)) + eps * eps;
  if (!(det > 0.0f) || !isfinite(det)) return r;
  float A = s11 / det;
  float B = -(s01 / det);
  float C = s00 / det;
  float hx = sqrtf(qcut * s00) + 1.0f;
  float hy = sqrtf(qcut * s11) + 1.0f;
  if (!isfinite(u) || !isfinite(v) || !isfinite(hx) || !isfinite(hy) || !isfinite(A) ||
      !isfinite(B) || !isfinite(C))
    return r;
  int x0 = clamp_tile(floorf((u - hx) / (float)tw), c.tiles_x);
  int x1 = clamp_tile(floorf((u + hx) / (float)tw) + 1.0f, c.tiles_x);
  int y0 = clamp_tile(floorf((v - hy) / (float)th), c.tiles_y);
  int y1 = clamp_tile(floorf((v + hy) / (float)th) + 1.0f, c.tiles_y);
  if (x0 >= x1 || y0 >= y1) return r;
  r.vis = true;
  r.u = u; r.v = v; r.A = A; r.B = B; r.C = C;
  r.x0 = x0; r.x1 = x1; r.y0 = y0; r.y1 = y1;
  return r;
}

__device__ __forceinline__ float pixel_q32(float A, float B, float C, float dx, float dy) {
#pragma clang fp contract(off)
  float t0 = dx * dx;
  float t1 = dy * dy;
  float t2 = dx * dy;
  float a = A * t0;
  float c = C * t1;
  float b = B * t2;
  return (a + c) + 2.0f * b;
}

// ------------------------------------------------------------------ launchers

void launch_project(const Layout& L, void* ws, const rogs_surfels* s, bool pack_feat,
                    hipStream_t st);
void launch_scan_part(const Layout& L, void* ws, hipStream_t st);
void launch_emit(const Layout& L, void* ws, hipStream_t st);
int launch_sort(const Layout& L, void* ws, int64_t n_host, hipStream_t st);
void launch_ranges(const Layout& L, void* ws, int64_t n_host, hipStream_t st);
int launch_render_fwd(const Layout& L, void* ws, const rogs_surfels* s, float* out, hipStream_t st);
void launch_loss(const Layout& L, void* ws, const float* out, const rogs_targets* t, float* G,
                 float* loss_out, float* d_exp, hipStream_t st);
int launch_render_bwd(const Layout& L, void* ws, const rogs_surfels* s, const float* out,
                      const float* G, hipStream_t st);
void launch_proj_bwd(const Layout& L, void* ws, const rogs_surfels* s, float* grads,
                     bool accumulate, hipStream_t st);
void launch_adam(int n, int C, float* params, const float* grads, float* m, float* v,
                 float* s_act, float* a_act, const rogs_lr* lr, int64_t step, float b1, float b2,
                 float eps, float* expo, const float* dexpo, float* me, float* ve, int nv,
                 hipStream_t st);
// Exclusive scan of n uint32 values; total written to *total (device) if non-null.
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
              hipStream_t st);
size_t scan_tmp_words(int64_t n);
void fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st);

}  // namespace rogs
