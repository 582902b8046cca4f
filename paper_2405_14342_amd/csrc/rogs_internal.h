// Internal declarations of librogs: workspace layout, the device view table,
// the key contract as device code, and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/rogs.h"

namespace rogs {

constexpr int kProjBlock = 256;     // threads per block of the per-surfel kernels
constexpr int kMaskChunk = 8192;   // mask bytes per side block of the projection launch
constexpr int kScanChunk = 4096;    // elements per block of the generic scan
constexpr int kMaxViews = 4096;
// A tile's work item (tile, list begin, list end, view | tile row << kViewBits):
// the view index takes the low bits, the tile's row in its view the rest.
constexpr int kViewBits = 12;
static_assert(kMaxViews <= (1 << kViewBits), "view index field");
// Binning block sizes, shared with the workspace layout that sizes their
// tables: pairs per emission block (one first-slot entry per block) and
// tiles per block of the tile layout (kTPart partial words per block).
constexpr int kEmitPairs = 512;    // timed faster than 1024 (more waves per SIMD)
constexpr int kTileBlk = 1024;
constexpr int kTPart = 17;          // per block: pairs, then the 16 bucket sizes

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
  uint32_t ch;          // ROGS_CH_* planes to composite (rogs_render_fwd ANDs its mask)
  int16_t tw, th;       // the view's tile shape (tw divides 64; tw * th is the batch's tile area)
  // binary64 constants of the key contract, formed on the host with the
  // contract's own operations: the pinhole clamp limits 0.65 W / f_x and
  // 0.65 H / f_y, and 1 / tw, 1 / th (exact: the tile sides are powers of
  // two, so multiplying by them rounds exactly as dividing by the sides)
  double limx, limy, itw, ith;
};

// Number of semantic classes with a compiled kernel set.
inline bool sem_supported(int C) { return (C >= 1 && C <= 8) || C == 16; }
inline int feat_stride(int C) { return ((4 + C) + 3) & ~3; }      // rgb, sem, alpha; float4-padded
// floats per per-pair gradient record: 10 + C values padded to whole float4
__host__ __device__ constexpr uint32_t grad_stride_c(int C) { return ((10 + C) + 3) & ~3; }
inline int grad_stride(int C) { return (int)grad_stride_c(C); }

// Layout of one batch inside the caller's workspace (byte offsets).
struct Layout {
  int32_t N = 0, C = 0, V = 0;
  int32_t tw = 16, th = 16, ppl = 4;   // the options' tile shape (views may differ, same area)
  int32_t stage = 32;                   // list entries staged in LDS per batch
  int32_t FS = 0, GS = 0;
  int32_t nb = 0;              // blocks of kProjBlock surfels
  int64_t total_pix = 0, total_tiles = 0, max_view_pix = 0, max_view_tiles = 0, cap = 0;
  int64_t scap = 0;            // visible-slot capacity (<= cap)
  int64_t slots = 0;           // V * N
  float eps2d = 0.3f, q_cut = 9.0f, alpha_max = 0.99f, t_eps = 1e-6f;
  size_t o_views, o_dzr, o_regpart, o_regtot, o_cnt, o_rec, o_rect, o_rspan, o_bstart, o_feat, o_part, o_partv, o_parttmp;
  size_t o_keys, o_vals, o_keys2, o_vals2, o_pslot, o_ranges, o_tfin, o_nlast, o_gpair;
  size_t o_drel = 0;           // per pixel: relative depth sum w (t_z - t0) and t0 (float2)
  size_t o_spair;              // slot of each tile-sorted pair
  size_t o_pdep;               // t_z bits of each emitted pair (the tile sort's key)
  size_t o_tcnt, o_tstart, o_tscan;   // pairs per tile, first list position, scan partials
  size_t o_tinfo;              // per launch position: tile, list begin, list end, view
  size_t o_mpart = 0;          // fused path: per-view mask counts of the projection's side blocks
  size_t o_sval, o_scnt, o_soff;               // visible slots in (view, surfel id) order
  size_t o_ssum, o_pos, o_long;                 // per-slot gradient sums, slot -> sorted position
  size_t o_histtmp, o_misc, o_lpart, o_mcount;
  size_t o_tpart = 0, o_status = 0;   // fused path only (0 = absent)
  size_t total = 0;
};

// Side blocks per view of the fused projection launch that count mask bytes.
inline int mask_chunks(const Layout& L) {
  return (int)((L.max_view_pix + kMaskChunk - 1) / kMaskChunk);
}

// misc counters (uint32 slots at o_misc)
// misc words: pair count, overflow flag, visible-slot count, long-slot count,
// pairs actually emitted (min of the pair count, the capacity and the pairs of
// the slots that fit the slot capacity)
enum MiscSlot {
  kMiscPairs = 0, kMiscOverflow = 1, kMiscVisible = 2, kMiscLong = 3, kMiscEmit = 4,
  kMiscTicketScan = 5,   // last-block ticket of the count-table scan
  kMiscWork = 8,   // two 64-bit work counters (words 8-11)
  kMiscCount = 16
};

// Last-block election for a grid-wide tail: each block calls it once, after
// writing its partial results, from every thread; it returns true in exactly
// one block, the last to arrive, which then sees every block's writes.  The
// ticket word must be zero before the launch and is zero again afterwards.
__device__ __forceinline__ bool last_block(uint32_t* ticket) {
  __shared__ uint32_t s_last;
  __threadfence();                     // this block's results, visible device-wide
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const uint32_t n = gridDim.x * gridDim.y;
    const uint32_t t = atomicAdd(ticket, 1u);
    s_last = (t == n - 1u) ? 1u : 0u;
    if (t == n - 1u) atomicExch(ticket, 0u);
  }
  __syncthreads();
  const bool last = s_last != 0u;
  if (last) __threadfence();           // acquire the other blocks' results
  return last;
}

int make_layout(const rogs_surfels* s, const rogs_camera* cams, int n_views,
                const rogs_render_opts* opts, int64_t cap, int64_t scap, Layout* L,
                const char** why, bool fused = false);

template <typename T>
__host__ __device__ inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ------------------------------------------------------------------ contract

struct Proj {
  bool vis;
  float uh, vh, ul, vl;   // centre as a binary32 pair (u = uh + ul)
  float A, B, C, tz;
  int x0, x1, y0, y1;
};

__device__ __forceinline__ int clamp_tile(double f, int hi) {
  if (!(f > 0.0)) return 0;
  if (f > (double)hi) return hi;
  return (int)f;
}

// The ground-rectangle part of the cull (supp. Sec. 2.1) in the contract's
// binary64 arithmetic: |d.ex| <= lat and 0 <= d.ez <= fwd, d = (x, y) - o.
// True when the rectangle is disabled (lat <= 0).
__device__ inline bool ground_inside(const ViewDev& c, float xf, float yf) {
#pragma clang fp contract(off)
  if (!(c.lat > 0.0f)) return true;
  const double dx = (double)xf - (double)c.o[0];
  const double dy = (double)yf - (double)c.o[1];
  const double a = dx * (double)c.ex[0] + dy * (double)c.ex[1];
  const double b = dx * (double)c.ez[0] + dy * (double)c.ez[1];
  return fabs(a) <= (double)c.lat && b >= 0.0 && b <= (double)c.fwd;
}

// Key contract (see rogs.h): the projection in binary64 from the binary32
// inputs, without FMA contraction, one rounded operation per step in the
// documented order, rounded once into the binary32 record.
__device__ inline Proj project_contract(const ViewDev& c, float eps_f, float qcut_f, float xf,
                                        float yf, float zf, float qwf, float qxf, float qyf, float qzf, float sxf, float syf) {
#pragma clang fp contract(off)
  Proj r;
  r.vis = false;
  r.uh = r.vh = r.ul = r.vl = r.A = r.B = r.C = 0.0f;
  r.x0 = r.x1 = r.y0 = r.y1 = 0;
  const double x = xf, y = yf, z = zf, qw = qwf, qx = qxf, qy = qyf, qz = qzf;
  const double sx = sxf, sy = syf;
  const double R0 = c.R[0], R1 = c.R[1], R2 = c.R[2], R3 = c.R[3], R4 = c.R[4], R5 = c.R[5];
  const double R6 = c.R[6], R7 = c.R[7], R8 = c.R[8];
  const double tx = ((R0 * x + R1 * y) + R2 * z) + (double)c.t[0];
  const double ty = ((R3 * x + R4 * y) + R5 * z) + (double)c.t[1];
  const double tz = ((R6 * x + R7 * y) + R8 * z) + (double)c.t[2];
  r.tz = (float)tz;
  if (!(tz >= (double)c.znear)) return r;
  if (!ground_inside(c, xf, yf)) return r;
  const double nn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(nn > 0.0) || !isfinite(nn)) return r;
  const double nq = sqrt(nn);
  const double w = qw / nq, a = qx / nq, b = qy / nq, cc = qz / nq;
  const double r1x = 1.0 - 2.0 * (b * b + cc * cc);
  const double r1y = 2.0 * (a * b + w * cc);
  const double r1z = 2.0 * (a * cc - w * b);
  const double r2x = 2.0 * (a * b - w * cc);
  const double r2y = 1.0 - 2.0 * (a * a + cc * cc);
  const double r2z = 2.0 * (b * cc + w * a);
  const double T10 = sx * r1x, T11 = sx * r1y, T12 = sx * r1z;
  const double T20 = sy * r2x, T21 = sy * r2y, T22 = sy * r2z;
  const double c10 = (R0 * T10 + R1 * T11) + R2 * T12;
  const double c11 = (R3 * T10 + R4 * T11) + R5 * T12;
  const double c12 = (R6 * T10 + R7 * T11) + R8 * T12;
  const double c20 = (R0 * T20 + R1 * T21) + R2 * T22;
  const double c21 = (R3 * T20 + R4 * T21) + R5 * T22;
  const double c22 = (R6 * T20 + R7 * T21) + R8 * T22;
  const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
  double j00, j11, j02, j12, u, v;
  if (c.model == ROGS_PINHOLE) {
    const double limx = c.limx;
    const double limy = c.limy;
    const double xr = tx / tz, yr = ty / tz;
    double xc = (xr < -limx) ? -limx : xr;
    xc = (limx < xc) ? limx : xc;
    double yc = (yr < -limy) ? -limy : yr;
    yc = (limy < yc) ? limy : yc;
    j00 = fx / tz;
    j11 = fy / tz;
    j02 = -(j00 * xc);
    j12 = -(j11 * yc);
    u = fx * xr + cx;
    v = fy * yr + cy;
  } else {
    j00 = fx; j11 = fy; j02 = 0.0; j12 = 0.0;
    u = fx * tx + cx;
    v = fy * ty + cy;
  }
  const double eps = eps_f, qcut = qcut_f;
  const double m00 = j00 * c10 + j02 * c12;
  const double m01 = j00 * c20 + j02 * c22;
  const double m10 = j11 * c11 + j12 * c12;
  const double m11 = j11 * c21 + j12 * c22;
  const double g0 = m00 * m00 + m01 * m01;
  const double g1 = m10 * m10 + m11 * m11;
  const double s00 = g0 + eps, s11 = g1 + eps;
  const double s01 = m00 * m10 + m01 * m11;
  const double dm = m00 * m11 - m01 * m10;
  const double det = (dm * dm + eps * (g0 + g1)) + eps * eps;
  if (!(det > 0.0) || !isfinite(det)) return r;
  const double A = s11 / det;
  const double B = -(s01 / det);
  const double C = s00 / det;
  const double hx = sqrt(qcut * s00) + 1.0;
  const double hy = sqrt(qcut * s11) + 1.0;
  if (!isfinite(u) || !isfinite(v) || !isfinite(hx) || !isfinite(hy) || !isfinite(A) ||
      !isfinite(B) || !isfinite(C))
    return r;
  const int x0 = clamp_tile(floor((u - hx) * c.itw), c.tiles_x);
  const int x1 = clamp_tile(floor((u + hx) * c.itw) + 1.0, c.tiles_x);
  const int y0 = clamp_tile(floor((v - hy) * c.ith), c.tiles_y);
  const int y1 = clamp_tile(floor((v + hy) * c.ith) + 1.0, c.tiles_y);
  if (x0 >= x1 || y0 >= y1) return r;
  r.vis = true;
  r.uh = (float)u;
  r.ul = (float)(u - (double)r.uh);
  r.vh = (float)v;
  r.vl = (float)(v - (double)r.vh);
  r.A = (float)A; r.B = (float)B; r.C = (float)C;
  r.x0 = x0; r.x1 = x1; r.y0 = y0; r.y1 = y1;
  return r;
}

// Tight tile culling of the key contract: the tiles of one rectangle row that
// the record's 3-sigma ellipse can reach.  The per-pixel binary32 test below
// rounds q by less than 2^-19.8 q / (1 - rho), rho = |B| / sqrt(AC), so the
// ellipse is inflated to q <= q_cut (1 + 2^-18 / (1 - rho)); its x-extent over
// the tile row's pixel-centre rows bounds the reached pixel columns.  A conic
// with 1 - rho < 2^-16 or without a positive determinant keeps the whole
// rectangle row.  Binary64 from the binary32 record, one rounding per step,
// no contraction; span_setup holds the per-record part, span_row one row.
// Row-span descriptor of a slot, written by the projection for the emission:
// up to kSpanRows rectangle rows of at most 255 tiles, one 16-bit word per row
// (lo - x0 | (hi - x0) << 8).  Slots beyond those limits are recomputed.
constexpr int kSpanRows = 8;
__host__ __device__ inline bool span_desc_ok(int x0, int x1, int y0, int y1) {
  return y1 - y0 <= kSpanRows && x1 - x0 <= 255;
}

struct Span {
  double A, B, det, qe, u, v, dym, dys;
  int x0, x1;
  bool full;
};

__device__ inline Span span_setup(float uh, float vh, float ul, float vl, float Af, float Bf,
                                  float Cf, float qcut_f, int x0, int x1) {
#pragma clang fp contract(off)
  Span s;
  s.x0 = x0;
  s.x1 = x1;
  s.full = true;
  s.A = s.B = s.det = s.qe = s.u = s.v = s.dym = s.dys = 0.0;
  const double A = Af, B = Bf, C = Cf;
  if (!(A > 0.0) || !(C > 0.0)) return s;
  const double det = A * C - B * B;
  const double gap = 1.0 - fabs(B) / sqrt(A * C);
  if (!(det > 0.0) || !(gap >= 0x1p-16)) return s;
  s.full = false;
  s.A = A;
  s.B = B;
  s.det = det;
  s.qe = (double)qcut_f * (1.0 + 0x1p-18 / gap);
  s.u = (double)uh + (double)ul;
  s.v = (double)vh + (double)vl;
  s.dym = sqrt((A * s.qe) / det);
  s.dys = B * sqrt(s.qe / (C * det));
  return s;
}

// Tiles [lo, hi) of tile row ty (inside the rectangle) for an image W x H.
__device__ inline void span_row(const Span& s, int tw, int th, int W, int H, int ty, int& lo,
                                int& hi) {
#pragma clang fp contract(off)
  lo = s.x0;
  hi = s.x1;
  if (s.full) return;
  hi = s.x0;
  const int r0 = ty * th;
  const int r1 = min(r0 + th, H);
  double a = ((double)r0 + 0.5) - s.v;
  double b = ((double)r1 - 0.5) - s.v;
  if (b < -s.dym || a > s.dym) return;
  if (a < -s.dym) a = -s.dym;
  if (b > s.dym) b = s.dym;
  // left boundary convex in dy, minimum at dys; right boundary its mirror
  const double tl = s.dys < a ? a : (s.dys > b ? b : s.dys);
  const double tr = -s.dys < a ? a : (-s.dys > b ? b : -s.dys);
  double dl = s.A * s.qe - s.det * (tl * tl);
  double dr = s.A * s.qe - s.det * (tr * tr);
  if (dl < 0.0) dl = 0.0;
  if (dr < 0.0) dr = 0.0;
  const double xl = s.u + (-(s.B * tl) - sqrt(dl)) / s.A;
  const double xr = s.u + (-(s.B * tr) + sqrt(dr)) / s.A;
  const double pl = ceil(xl - 0.5);
  const double pr = floor(xr - 0.5);
  if (!(pl <= pr) || pl > (double)(W - 1) || pr < 0.0) return;
  const int cl = pl < 0.0 ? 0 : (int)pl;
  const int cr = pr > (double)(W - 1) ? W - 1 : (int)pr;
  const int sh = __builtin_ctz((unsigned)tw);      // tw is a power of two; cl, cr >= 0
  const int l = max(cl >> sh, s.x0);
  const int h = min((cr >> sh) + 1, s.x1);
  if (l < h) {
    lo = l;
    hi = h;
  }
}

// Per-pixel contribution test of the contract (binary32):
// q = fma(dx, fma(A, dx, B2 dy), (C dy) dy) with B2 = 2B (exact), each
// product and fma rounded once, nothing else contracted.  dx = ((px + 0.5) -
// u_hi) - u_lo and dy likewise are formed by the caller.
__device__ __forceinline__ float pixel_q32(float A, float B2, float C, float dx, float dy) {
#pragma clang fp contract(off)
  const float t = __builtin_fmaf(A, dx, B2 * dy);
  const float c = (C * dy) * dy;
  return __builtin_fmaf(dx, t, c);
}

// Footprint weight g = exp(-q/2) = 2^(q * (-log2(e)/2)): one multiply and the
// hardware base-2 exponential.  The forward and the backward both use this
// function, so the backward recomputes the forward's transmittance exactly.
__device__ __forceinline__ float gauss_weight(float q) {
  return __builtin_amdgcn_exp2f(q * -0.72134752044448170f);
}

// Opacity clamp alpha' = min(alpha g, alpha_max) (neither operand is NaN).
__device__ __forceinline__ float clamp_alpha(float ag, float amax) { return fminf(ag, amax); }

__device__ __forceinline__ float pixel_offset(float pc, float hi, float lo) {
#pragma clang fp contract(off)
  return (pc - hi) - lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block-wide exclusive scan of one value per thread (kProjBlock threads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_w, uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x, lane);
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kProjBlock / 64; ++w) {
    uint32_t t = s_w[w];
    pre += (w < wv) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - x;
}

// Last index j in [0, n) with off[j] <= k, for non-decreasing off with off[0] <= k.
__device__ __forceinline__ int last_le(const uint32_t* off, int n, uint32_t k) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Wave reduce-scatter of N per-lane values (gfx950).  Six exchange stages pair
// every lane with its partner across lane bit 32, 16, 8, 4, 2, 1.  While a lane
// still holds more than one value, each stage halves the list: the lane with
// the bit clear keeps the first half and the partner the second half, and each
// adds what the other sends (so the lane sends the half it gives away).  The
// stages use v_permlane32_swap, v_permlane16_swap (both swap whole half-waves
// between two registers, so one swap serves both directions) and DPP
// row_mirror (bit 8), row_half_mirror (bit 4) and quad_perm (bits 2, 1).  After
// the six stages lane l holds the wave total of component rs_comp(l, N); lanes
// that differ only in bits where a single value was left hold identical bits.

__host__ __device__ constexpr int rs_half(int n) { return (n + 1) / 2; }

// Component held by lane l after reducing N values (-1: padding).
__host__ __device__ constexpr int rs_comp(int lane, int N) {
  int arr = N, valid = N, off = 0;
  for (int s = 0; s < 6; ++s) {
    const int bit = 32 >> s;
    if (arr > 1) {
      const int h = rs_half(arr);
      if (lane & bit) {
        off += h;
        valid = valid - h > 0 ? valid - h : 0;
      } else {
        valid = valid < h ? valid : h;
      }
      arr = h;
    }
  }
  return valid >= 1 ? off : -1;
}

// Lane bits of the stages where only one value was left (its holders agree).
__host__ __device__ constexpr int rs_dup_bits(int N) {
  int arr = N, m = 0;
  for (int s = 0; s < 6; ++s) {
    if (arr > 1) arr = rs_half(arr); else m |= 32 >> s;
  }
  return m;
}

template <int STAGE>
__device__ __forceinline__ float rs_dpp(float x) {
  constexpr int ctrl = STAGE == 2 ? 0x140 : STAGE == 3 ? 0x141 : STAGE == 4 ? 0x4E : 0xB1;
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, false));
}

template <int N, int STAGE>
__device__ __forceinline__ void rs_stage(const float* in, float* out, int lane) {
  constexpr int H = N > 1 ? rs_half(N) : 1;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float a = in[k];
    const float b = (N == 1) ? in[0] : ((k + H < N) ? in[k + H] : 0.0f);
    if constexpr (STAGE == 0) {
      const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
      out[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else if constexpr (STAGE == 1) {
      const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
      out[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
      const bool hi = (lane & (32 >> STAGE)) != 0;
      const float mine = hi ? b : a;
      const float other = hi ? a : b;
      out[k] = mine + rs_dpp<STAGE>(other);
    }
  }
}

// x of lane (lane ^ j) for j = 1, 2, 4, 8, 16 or 32, a constant once the
// caller's loop is unrolled: DPP quad swaps for 1 and 2, a swizzle inside
// each half-wave for 4, a row rotation by 8 (which is lane ^ 8 inside each
// row of 16) for 8, and for 16 and 32 the half-wave swaps, whose two results
// hold x and x[lane ^ j] in some order, so their sum minus x is the latter
// (exact in 32-bit wrap-around).
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, uint32_t j) {
  if (j == 1u) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xf, 0xf, false);
  if (j == 2u) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xf, 0xf, false);
  if (j == 4u) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x101F);
  if (j == 8u) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xf, 0xf, false);
  if (j == 16u) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (uint32_t)r[0] + (uint32_t)r[1] - x;
  }
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return (uint32_t)r[0] + (uint32_t)r[1] - x;
}

// Maximum over the wave, in every lane: the exchanges of the reduce-scatter
// (lane bits 32 and 16 by half-wave swaps, then the row mirrors and quad
// swaps, which together reach all 16 lanes of a row) with max in place of
// the sum.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  const auto r32 = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  x = max((uint32_t)r32[0], (uint32_t)r32[1]);
  const auto r16 = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  x = max((uint32_t)r16[0], (uint32_t)r16[1]);
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xf, 0xf, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xf, 0xf, false));
  return x;
}

template <int N>
__device__ __forceinline__ float wave_reduce_scatter(const float* v, int lane) {
  constexpr int N1 = N > 1 ? rs_half(N) : 1;
  constexpr int N2 = N1 > 1 ? rs_half(N1) : 1;
  constexpr int N3 = N2 > 1 ? rs_half(N2) : 1;
  constexpr int N4 = N3 > 1 ? rs_half(N3) : 1;
  constexpr int N5 = N4 > 1 ? rs_half(N4) : 1;
  float t1[N1], t2[N2], t3[N3], t4[N4], t5[N5], t6[1];
  rs_stage<N, 0>(v, t1, lane);
  rs_stage<N1, 1>(t1, t2, lane);
  rs_stage<N2, 2>(t2, t3, lane);
  rs_stage<N3, 3>(t3, t4, lane);
  rs_stage<N4, 4>(t4, t5, lane);
  rs_stage<N5, 5>(t5, t6, lane);
  return t6[0];
}
static_assert(rs_comp(0, 18) == 0 && rs_comp(63, 18) == -1, "reduce-scatter map");

// ------------------------------------------------------------------ loss seed

// Per-pixel loss of Eq. 7-9 and 12 for one masked pixel.  o: the composited
// R, G, B and C semantic logits; t: the target colour.  wc, ws: lambda_c and
// lambda_s times the view scale over |M_v|; ea = e^a, b: the view's exposure.
// Writes dL/d(o) into g (3 + C values) and adds the pixel's loss and its
// dL/da, dL/db to l, da, db.  Shared by the stand-alone loss kernel and the
// fused forward epilogue so that both produce identical bits.
template <int C>
__device__ __forceinline__ void pixel_loss(const float* o, const float* t, int label, float wc,
                                           float ws, float ea, float b, float* g, float& l,
                                           float& da, float& db) {
  // no multiply-add contraction: each inlined copy rounds every step the
  // same way, whatever the surrounding code lets the compiler fuse
#pragma clang fp contract(off)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float cc = o[c];
    const float r = (ea * cc + b) - t[c];
    const float sg = (r > 0.0f) ? 1.0f : ((r < 0.0f) ? -1.0f : 0.0f);
    l += wc * fabsf(r);
    g[c] = wc * sg * ea;
    da += wc * sg * ea * cc;
    db += wc * sg;
  }
  float sv[C];
  float mx = -INFINITY;
#pragma unroll
  for (int c = 0; c < C; ++c) mx = fmaxf(mx, o[3 + c]);
  // softmax with the hardware base-2 exponential and logarithm and the
  // hardware reciprocal: every exponent is <= 0 and 1 <= se <= C, where each
  // is within a few ulp (relative 1e-6 at the worst exponent that matters)
  constexpr float kLog2e = 1.44269504088896341f, kLn2 = 0.69314718055994531f;
  float se = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    sv[c] = __builtin_amdgcn_exp2f((o[3 + c] - mx) * kLog2e);
    se += sv[c];
  }
  float olb = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) olb = (c == label) ? o[3 + c] : olb;
  l += ws * ((mx + __builtin_amdgcn_logf(se) * kLn2) - olb);
  const float inv = __builtin_amdgcn_rcpf(se);
#pragma unroll
  for (int c = 0; c < C; ++c) g[3 + c] = ws * (sv[c] * inv - ((c == label) ? 1.0f : 0.0f));
}

// pixel_loss for a pixel whose outputs are all 0 (a tile without entries):
// the loss and its dL/db term with every step rounded as pixel_loss rounds
// it at o = 0 (dL/da is +-0 there and dL/dO is not formed).
template <int C>
__device__ __forceinline__ void pixel_loss_empty(const float* t, float wc, float ws, float ea,
                                                 float b, float& l, float& db) {
#pragma clang fp contract(off)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float r = (ea * 0.0f + b) - t[c];
    const float sg = (r > 0.0f) ? 1.0f : ((r < 0.0f) ? -1.0f : 0.0f);
    l += wc * fabsf(r);
    db += wc * sg;
  }
  // softmax of C zeros: the exponentials are exactly 1 and their sum C
  constexpr float kLn2 = 0.69314718055994531f;
  l += ws * (__builtin_amdgcn_logf((float)C) * kLn2);
}

// Per-view loss constants (uniform over a view).
struct LossView {
  float wc, ws, ea, b;
  bool any;
};

__device__ __forceinline__ LossView loss_view(const float* expo, const uint32_t* mcount, int v,
                                              float lam_c, float lam_s, float scale) {
  LossView r;
  const uint32_t mc = mcount[v];
  r.any = mc > 0;
  // 1/|M_v| with the hardware reciprocal (within 1 ulp): evaluated once per
  // wave by every loss kernel
  const float inv = __builtin_amdgcn_rcpf((float)mc);
  r.wc = r.any ? (lam_c * scale) * inv : 0.0f;
  r.ws = r.any ? (lam_s * scale) * inv : 0.0f;
  r.ea = expf(expo[2 * v]);
  r.b = expo[2 * v + 1];
  return r;
}

// Inputs of the loss fused into the forward epilogue.
struct FusedLoss {
  const float* tgt;        // target colour, 3 planes per view
  const uint8_t* label;
  const uint8_t* mask;
  const float* expo;       // [V][2]
  const uint32_t* mcount;  // |M_v|
  float lam_c, lam_s, scale;
  float* part;             // per-tile (loss, dL/da, dL/db)
};

// Device-resident state of the fused step (caller-owned, 64 bytes, zeroed by
// the caller before the first step).
struct StepState {
  int64_t step;      // Adam steps applied
  int64_t skipped;   // steps skipped because the pair capacity overflowed
  float loss;        // loss of the last applied step
  float lr_z;        // z learning rate of the last applied step
  float pad[10];
};
static_assert(sizeof(StepState) == 64, "step state is 64 bytes");

struct AdamArgs {
  rogs_lr lr;                 // lr.z used as is unless a schedule is given
  float b1, b2, eps;
  float z_start, z_end;       // log-linear z schedule (fused path)
  int64_t total_steps;        // 0: no schedule, use lr.z
  int64_t step;               // step number of this update (>= 1); ignored with state
  const StepState* state;     // fused path: step = state->step + 1
  const uint32_t* misc;       // fused path: skip the update on overflow
};

// ------------------------------------------------------------------ launchers

void launch_project(const Layout& L, void* ws, const rogs_surfels* s, bool pack_feat,
                    hipStream_t st, const uint8_t* mask = nullptr);
void launch_scan_part(const Layout& L, void* ws, hipStream_t st, bool mask_parts = false);
// Compaction of the visible slots, emission with per-tile counting, the
// tiles' first list positions, ranges and compositing work items, and the
// pairs grouped by tile (o_vals).  Counts
// < 0 are read on the device.  counts_cleared: the per-tile counters were
// zeroed by the projection launch.
void launch_binning(const Layout& L, void* ws, int64_t n_pairs, int64_t n_vis, hipStream_t st,
                    bool counts_cleared = false);
// Each tile's list by depth.  With a side stream (and two events) the lists
// longer than 64 entries are sorted there, concurrently with the short ones,
// and st waits for them before returning; the events' record / wait results
// are returned.
hipError_t launch_ranges(const Layout& L, void* ws, hipStream_t st, hipStream_t side = nullptr,
                         hipEvent_t fork = nullptr, hipEvent_t join = nullptr);
void launch_count_work(const Layout& L, void* ws, unsigned long long* counts, hipStream_t st);
int64_t elev_reg_blocks(int n);
void launch_elev_reg(int n, const float* z, const int32_t* nbr, float lam_s, const float* zbar,
                     float lam_z, float* out_dz, float* acc_dz, float* part, float* total,
                     bool accumulate_total, hipStream_t st);
size_t lidar_scratch_bytes(int n, int m);
void launch_lidar_nn(int n, const float* x, const float* y, int m, const float* px,
                     const float* py, const float* pz, float* zbar, int32_t* idx, void* scratch,
                     hipStream_t st);
size_t layout_scratch_bytes(int W, int H, int np);
void launch_layout_mask(const rogs_pose* poses, int np, double x0, double y0, float h, int W,
                        int H, int r, void* scratch, uint32_t* n_dev, hipStream_t st);
void launch_layout_fill(const rogs_pose* poses, int np, double x0, double y0, float h, int W,
                        int H, void* scratch, int64_t n, int32_t* idx, float* x, float* y,
                        float* z, float* q, int32_t* nbr, hipStream_t st);
int launch_render_fwd(const Layout& L, void* ws, const rogs_surfels* s, float* out, uint32_t mask,
                      hipStream_t st);
// Channel sets (ROGS_CH_*) of the views of the next rogs_project call on this
// context (n entries, one per view; n = 0 clears: every view gets all
// planes).  Used by the render server for per-request channel sets.
// Waits for the fused steps in flight and forgets them and the captured
// graph: the next rogs_step_fused starts afresh and rogs_fused_status reports
// no step until then.
void ctx_fused_forget(rogs_ctx* c);
int ctx_set_view_channels(rogs_ctx* c, const uint32_t* ch, int n);
void launch_loss(const Layout& L, void* ws, const float* out, const rogs_targets* t, float* G,
                 float* loss_out, float* d_exp, hipStream_t st);
int launch_render_bwd(const Layout& L, void* ws, const rogs_surfels* s, const float* out,
                      const float* G, hipStream_t st);
int launch_render_step(const Layout& L, void* ws, const FusedLoss& fl, hipStream_t st);
// Per-slot sums of the per-pair gradient records (before the projection adjoint).
// Sums each visible slot's per-pair gradient records.  clear = reset the
// long-slot count first (false only where the projection's counter reset is
// known to be the last write to it).
void launch_slot_sums(const Layout& L, void* ws, hipStream_t st, bool clear = true);
void launch_proj_bwd(const Layout& L, void* ws, const rogs_surfels* s, float* grads,
                     bool accumulate, hipStream_t st);
void launch_adam(int n, int C, float* params, const float* grads, float* m, float* v,
                 float* s_act, float* a_act, const rogs_optim& o, int64_t step, float* expo,
                 const float* dexpo, float* me, float* ve, int nv, hipStream_t st);
// Fused: projection adjoint of every surfel followed by its Adam update (and
// the exposure update); optional gradient output.  Skipped on overflow.
// dzr (nullable): per-surfel dL/dz of the grid-side terms, added to the
// height gradient before the update.
void launch_proj_bwd_adam(const Layout& L, void* ws, const float* x, const float* y, float* params,
                          float* m, float* v, float* s_act, float* a_act, float* grads_out,
                          const AdamArgs& aa, float* expo, const float* dexpo, float* me,
                          float* ve, const float* dzr, hipStream_t st);
// Fused: per-view loss and dL/d(a, b) (overwritten) from the per-tile partials.
void launch_loss_tiles(const Layout& L, void* ws, float* d_exp, float* expo, float* m_exp,
                       float* v_exp, const AdamArgs& aa, hipStream_t st);
void launch_mask_count(const Layout& L, void* ws, const uint8_t* mask, hipStream_t st);
void launch_step_end(const Layout& L, void* ws, StepState* state, const AdamArgs& aa,
                     const float* reg_total, hipStream_t st);
// Exclusive scan of n uint32 values; total written to *total (device) if non-null.
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
              hipStream_t st);

size_t scan_tmp_words(int64_t n);
// Stores msg as the context's last error and returns code.
int ctx_fail(rogs_ctx* c, int code, const std::string& msg);
void fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st);

}  // namespace rogs
