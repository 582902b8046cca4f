// Front-to-back alpha compositing of the sorted tile lists (Eq. 6) and its
// adjoint.
//
// Mapping: one 64-lane wave per tile, tiles launched longest list first; a
// tile of tile_w x tile_h = 64 * PPL pixels gives every lane PPL pixels of one
// column, so the per-pair x offset is shared and each broadcast record read
// from LDS feeds PPL pixels.  A wave starts from one precomputed record
// (tile, list range, view) and reads each entry's slot directly, so the
// prologue is two dependent global loads before the records arrive.
// The wave stages KS list entries at a time in LDS (projection record +
// the surfel's colour/semantic features), then every lane walks them in
// order.  A pixel stops after the surfel that takes its transmittance below
// t_eps; the wave leaves the list once all of its pixels have stopped.
//
// Depth is composited relative to a reference depth t0 per pixel, the depth
// of the first (nearest) list entry that reaches the pixel: D' = sum w (t_z -
// t0), D = D' + t0 A.  The backward differentiates D' and A, so the FP32
// suffix term below cancels in proportion to the spread of the depths a pixel
// sees instead of the absolute depth (tens of metres).  The entries a pixel
// sees, and so t0, do not depend on the tile shape.
//
// The backward walks the list front to back again, recomputing T exactly as
// the forward did, and uses sum_{j>k} w_j f_j = O - prefix - w_k f_k for the
// suffix term of dO/d(alpha_k).  Per (tile, pair) it writes one record of
// 10 + C gradient values at the pair's emission index: the five moments of
// dL/dq over the pixel offsets and dalpha are summed across the wave with a
// reduce-scatter; the colour, semantic and depth gradients sum_p w_p G_p are
// a small matrix product per 16 entries on the matrix cores.  The projection
// adjoint later sums each surfel's records and applies the conic.  No
// atomics: the result does not depend on timing.
//
// The fused training step runs forward, loss and backward of a tile in one
// kernel (k_render_step): the per-pixel loss gradient, G.O, T_final and n_last
// stay in registers between the two passes instead of going through HBM, and
// a list the forward staged whole is not staged again.
#include <cfloat>

#include "rogs_internal.h"

namespace rogs {

namespace {

__device__ __forceinline__ int find_view(const ViewDev* __restrict__ views, int V, int gt) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_off <= gt) lo = mid; else hi = mid - 1;
  }
  return lo;
}


// List entries staged in LDS at a time: the template parameter KS of the
// compositing kernels, 16, 32 or 64 (rogs_render_opts.stage).

// Per-tile constants of the compositing kernels.
struct TileGeom {
  int gt, v, W, H, px, py0, rows;
  float pxc;
  uint32_t rbeg, rend, sbase;
  const ViewDev* vw;
};

__device__ __forceinline__ TileGeom tile_geom(const ViewDev* __restrict__ views, int N,
                                              const uint4* __restrict__ tinfo) {
  TileGeom t;
  const int lane = threadIdx.x;
  // tile, list begin, list end, view | tile row << kViewBits
  const uint4 ti = tinfo[blockIdx.x];
  t.gt = (int)ti.x;
  t.v = (int)(ti.w & ((1u << kViewBits) - 1u));
  t.vw = &views[t.v];
  t.W = t.vw->w;
  t.H = t.vw->h;
  const int lt = t.gt - t.vw->tile_off;
  const int ty = (int)(ti.w >> kViewBits), tx = lt - ty * t.vw->tiles_x;
  const int tw = t.vw->tw, th = t.vw->th;
  const int sh = __builtin_ctz((unsigned)tw);      // tile_w divides 64: a power of two
  t.rows = 64 >> sh;
  t.px = tx * tw + (lane & (tw - 1));
  t.py0 = ty * th + (lane >> sh);
  t.pxc = (float)t.px + 0.5f;
  t.rbeg = ti.y;
  t.rend = ti.z;
  t.sbase = (uint32_t)t.v * (uint32_t)N;
  return t;
}

// Stages list entries [base, base + cnt) of the tile in LDS: the projection
// record (with 2B in place of B) and the surfel's feature record, entry j at
// s_r0[j (2 + FS4)], s_r1[j (2 + FS4)] and s_f[j (2 + FS4) + f] of one
// interleaved array (so one address serves all of an entry's reads).  With
// kE, returns this lane's emission index (lane < cnt).
template <int FS4, bool kE>
__device__ __forceinline__ uint32_t stage_entries(uint32_t base, int cnt, uint32_t sbase,
                                                  const uint32_t* __restrict__ vals,
                                                  const uint32_t* __restrict__ spair,
                                                  const float4* __restrict__ rec,
                                                  const float4* __restrict__ feat, float4* s_r0,
                                                  float4* s_r1, float4* s_f) {
  const int lane = threadIdx.x;
  uint32_t e = 0;
  if (lane < cnt) {
    if (kE) e = vals[base + lane];
    const uint32_t slot = spair[base + lane];
    s_r0[lane * (2 + FS4)] = rec[2 * (size_t)slot];
    const float4 r1 = rec[2 * (size_t)slot + 1];
    s_r1[lane * (2 + FS4)] = make_float4(r1.x, 2.0f * r1.y, r1.z, r1.w);   // A, 2B, C, t_z
    const uint32_t i = slot - sbase;
#pragma unroll
    for (int f = 0; f < FS4; ++f) s_f[lane * (2 + FS4) + f] = feat[(size_t)i * FS4 + f];
  }
  return e;
}

// Forward pass over the tile's list (Eq. 6): acc = sum w f (features, then
// with kD the relative depth sum w (t_z - t0)), T, and nl = entries up to the
// one that stopped the pixel.  With kD, t0 = the depth of the pixel's first
// contributing entry: the list is in ascending depth, so the running minimum
// of the contributing depths (FLT_MAX while none).  With kE, e_first = this
// lane's emission index in the first staged batch.  ch (ROGS_CH_* bits,
// uniform): the colour, semantic and depth sums are formed only when
// selected; T, n_last and the order of operations do not depend on it.
constexpr int kFwdUnroll = 4;       // forward entries per stop test

// With kG (16, one pixel per lane) the footprint weights g of the list's
// first kG entries are kept in gsave for the backward: gsave[j] is the
// weight of every entry the forward evaluates, which covers each pixel's
// entries before n_last, the only ones the backward reads it for, and 0 for
// the others (past the list's end or after the whole wave has stopped).
template <int C, int PPL, int KS, bool kE, bool kD, int kG = 0>
__device__ __forceinline__ void forward_tile(const TileGeom& tg, float qcut, float amax,
                                             float teps, const uint32_t* __restrict__ vals,
                                             const uint32_t* __restrict__ spair,
                                             const float4* __restrict__ rec,
                                             const float4* __restrict__ feat, float4* s_r0,
                                             float4* s_r1, float4* s_f, const float* pyc,
                                             float (*acc)[3 + C + 1], float* T, uint32_t* nl,
                                             uint32_t& e_first, float* t0, uint32_t ch,
                                             float* gsave = nullptr) {
  // every multiply-add is written out: the forward rounds the same in every
  // kernel it is inlined into
#pragma clang fp contract(off)
  static_assert(kG == 0 || (kG == 16 && PPL == 1 && KS >= kG), "kept weights");
  constexpr int F = 3 + C;            // composited features besides depth
  constexpr int FS4 = (F + 4) / 4;    // float4 per feature record (features, alpha)
  // a pixel is live while T >= t_eps (T only falls, and t_eps < 1); a pixel
  // outside the image starts at T = 0, which no update changes
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = tg.py0 + k * tg.rows;
    T[k] = (tg.px < tg.W && py < tg.H) ? 1.0f : 0.0f;
    nl[k] = 0;
    if (kD) t0[k] = FLT_MAX;
#pragma unroll
    for (int f = 0; f <= F; ++f) acc[k][f] = 0.0f;
  }
  bool stop_all = false;
  for (uint32_t base = tg.rbeg; base < tg.rend && !stop_all; base += KS) {
    const int cnt = (int)min((uint32_t)KS, tg.rend - base);
    const uint32_t e =
        stage_entries<FS4, kE>(base, cnt, tg.sbase, vals, spair, rec, feat, s_r0, s_r1, s_f);
    if (base == tg.rbeg) e_first = e;
    __syncthreads();
    // one list entry for every pixel of the lane (gout: its g, or nullptr)
    auto fentry = [&](const int j, float* gout) {
      const float4 r0 = s_r0[j * (2 + FS4)], r1 = s_r1[j * (2 + FS4)];   // u_hi v_hi u_lo v_lo | A 2B C tz
      float fv[FS4 * 4];
#pragma unroll
      for (int f = 0; f < FS4; ++f) {
        const float4 t4 = s_f[j * (2 + FS4) + f];
        fv[4 * f] = t4.x; fv[4 * f + 1] = t4.y; fv[4 * f + 2] = t4.z; fv[4 * f + 3] = t4.w;
      }
      const float al = fv[F];
      const float dx = pixel_offset(tg.pxc, r0.x, r0.z);
      // Lanes whose pixel the entry does not reach, or has stopped, run the
      // same arithmetic with g = 0: w = 0 leaves T and the sums as they are
      // (T >= 0 and every feature is finite), so the result is that of a
      // branch around the update without its exec-mask bookkeeping.
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const float dy = pixel_offset(pyc[k], r0.y, r0.w);
        const float q = pixel_q32(r1.x, r1.y, r1.z, dx, dy);
        const bool live = T[k] >= teps;
        const bool hit = live && q <= qcut;
        // the exponential of every lane, then a select (no branch around it)
        const float ge = gauss_weight(q);
        const float g = hit ? ge : 0.0f;
        if (gout) gout[k] = g;
        const float a = clamp_alpha(al * g, amax);
        const float w = a * T[k];
        if (ch & ROGS_CH_RGB)
#pragma unroll
          for (int f = 0; f < 3; ++f) acc[k][f] = __builtin_fmaf(w, fv[f], acc[k][f]);
        if (ch & ROGS_CH_SEM)
#pragma unroll
          for (int f = 3; f < F; ++f) acc[k][f] = __builtin_fmaf(w, fv[f], acc[k][f]);
        if (kD && (ch & ROGS_CH_D)) {
          t0[k] = hit ? fminf(t0[k], r1.w) : t0[k];
          acc[k][F] = __builtin_fmaf(w, r1.w - t0[k], acc[k][F]);
        }
        T[k] -= w;                     // T (1 - alpha)
        // entries seen while live: at the entry that stops the pixel, its
        // position in the list plus one
        nl[k] += live ? 1u : 0u;
      }
    };
    // every lane of the wave runs this loop: the ballot is the stop test
    auto all_stopped = [&]() {
      bool live = false;
#pragma unroll
      for (int k = 0; k < PPL; ++k) live = live || T[k] >= teps;
      return __builtin_amdgcn_ballot_w64(live) == 0;
    };
    // groups of kFwdUnroll entries, the stop test after each group: entries
    // past a pixel's stop change nothing for it, so the results are those
    // of a test after every entry.  The first kG entries of the list are
    // unrolled whole, so that their weights land in registers.
    // (a constant trip count without early exits: it unrolls fully)
    int jstart = 0;
    if (kG > 0 && base == tg.rbeg) {
#pragma unroll
      for (int j = 0; j < kG; ++j) {
        if (j < cnt && !stop_all) {
          fentry(j, gsave + j);
          if (j % kFwdUnroll == kFwdUnroll - 1 && all_stopped()) stop_all = true;
        } else {
          gsave[j] = 0.0f;
        }
      }
      jstart = kG;
    }
    for (int j0 = jstart; j0 < cnt && !stop_all; j0 += kFwdUnroll) {
#pragma unroll
      for (int u = 0; u < kFwdUnroll; ++u) {
        const int j = j0 + u;
        if (j >= cnt) break;
        fentry(j, nullptr);
      }
      if (all_stopped()) stop_all = true;
    }
    __syncthreads();
  }
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// Floats of the backward's LDS block for one block of 16 list entries: the
// per-pixel weights w of 16 entries (rows of 64 * PPL + 4 floats), also used
// once per tile to transpose the per-pixel gradient vectors.
template <int C, int PPL>
__host__ __device__ constexpr int bwd_lds_floats() {
  constexpr int NFB = (3 + C + 1 + 15) / 16;
  constexpr int a = 16 * (64 * PPL + 4), b = 64 * PPL * (16 * NFB + 1);
  return a > b ? a : b;
}

// Feature and depth gradients of up to 16 list entries as one matrix product
// on the matrix cores: D[m][n] = sum over the tile's pixels p of
// w[m][p] * gamma[p][n], where gamma[p] = (dL/dfeatures, dL/dD) of pixel p.
// v_mfma_f32_16x16x4_f32 takes A[m][k] from lane m + 16k, B[k][n] from lane
// n + 16k and returns D[4g + i][n] in lane n + 16g, element i.  The k-th
// step of 4 covers pixels kk * 64 + kgrp * 16 + c, so a lane reads its A
// operands as 16 contiguous floats of its entry's row.
template <int C, int PPL>
__device__ __forceinline__ void feature_gemm(const float* s_w, const uint32_t* s_e, int nrows,
                                             const float (&bG)[(3 + C + 1 + 15) / 16][PPL][16],
                                             float* __restrict__ gpair) {
  constexpr int F = 3 + C;
  constexpr uint32_t GS = grad_stride_c(C);
  constexpr int NG = F + 1;
  constexpr int NFB = (NG + 15) / 16;
  constexpr int WS = 64 * PPL + 4;
  const int lane = threadIdx.x;
  const int mrow = lane & 15, kgrp = lane >> 4;
  float a[PPL][16];
#pragma unroll
  for (int kk = 0; kk < PPL; ++kk) {
    const float4* ap = reinterpret_cast<const float4*>(s_w + mrow * WS + kk * 64 + kgrp * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = ap[q];
      a[kk][4 * q] = t.x; a[kk][4 * q + 1] = t.y; a[kk][4 * q + 2] = t.z; a[kk][4 * q + 3] = t.w;
    }
  }
  uint32_t e4[4];
  bool ok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = 4 * kgrp + i;
    ok[i] = m < nrows;
    e4[i] = s_e[m];
  }
#pragma unroll
  for (int nb = 0; nb < NFB; ++nb) {
    mfma_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < PPL; ++kk)
#pragma unroll
      for (int c = 0; c < 16; ++c)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk][c], bG[nb][kk][c], acc, 0, 0, 0);
    const int n = nb * 16 + mrow;
    if (n < NG) {
      const int col = n < F ? 7 + n : 6;       // record: ..., dt_z (6), features (7 ...)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (ok[i]) gpair[(size_t)e4[i] * GS + col] = acc[i];
    }
  }
}

// Backward pass over the tile's list, given per pixel the output gradient
// Gv (features, depth, alpha), G.O (with the relative depth D'), T_final,
// n_last and the reference depth t0 (used with kDA).  Writes one record of NV
// gradient values per pair at its emission index: the five moments and
// dalpha are summed across the wave with a reduce-scatter, the feature and
// depth gradients come from feature_gemm once per 16 entries.  With kG (16,
// one pixel per lane) gsave holds the forward's footprint weights of the
// list's first kG entries, valid for the entries before n_last.
template <int C, int PPL, int KS, bool kDA, int kG = 0>
__device__ __forceinline__ void backward_tile(const TileGeom& tg, float qcut, float amax,
                                              const uint32_t* __restrict__ vals,
                                              const uint32_t* __restrict__ spair,
                                              const float4* __restrict__ rec,
                                              const float4* __restrict__ feat, float4* s_r0,
                                              float4* s_r1, float4* s_f, float* s_w,
                                              uint32_t* s_e, const float* pyc,
                                              const float (*Gv)[3 + C + 2], const float* GO,
                                              const float* Tf, const uint32_t* nl,
                                              float* __restrict__ gpair, bool staged,
                                              uint32_t e_pre, const float* t0,
                                              const float* gsave = nullptr) {
  // every multiply-add is written out: the backward rounds the same in the
  // fused step and in the stand-alone backward
#pragma clang fp contract(off)
  static_assert(kG == 0 || (kG == 16 && PPL == 1 && KS >= kG), "kept weights");
  constexpr int F = 3 + C;
  constexpr int FS4 = (F + 4) / 4;
  // per pair: sum gda dx, sum gda dy, sum gda dx^2, sum gda dx dy,
  // sum gda dy^2 (gda = dL/d(alpha) per pixel; dL/dq = -(alpha / 2) gda),
  // dalpha = sum gda, dtz, drgb[3], dsem[C]
  constexpr int NV = 10 + C;
  constexpr uint32_t GS = grad_stride_c(C);   // floats per record
  constexpr int NR = 6;                       // reduced across the wave
  constexpr int NFB = (F + 1 + 15) / 16;
  constexpr int WS = 64 * PPL + 4;
  const int lane = threadIdx.x;
  const int my_comp = rs_comp(lane, NR);
  const bool writer = my_comp >= 0 && (lane & rs_dup_bits(NR)) == 0;
  float T[PPL], Spre[PPL], GAf[PPL];
  uint32_t maxn = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    T[k] = 1.0f;
    Spre[k] = 0.0f;
    maxn = max(maxn, nl[k]);
    // D = D' + t0 A: the alpha channel's gradient carries t0 dL/dD, times
    // T_final for dA/d(alpha_k) = T_final / (1 - alpha_k)
    GAf[k] = kDA ? __builtin_fmaf(t0[k], Gv[k][F], Gv[k][F + 1]) * Tf[k] : 0.0f;
  }
  // every lane holds the maximum: as a scalar the list loop is scalar control
  maxn = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_u32(maxn));
  const uint32_t stop = tg.rbeg + min(maxn, tg.rend - tg.rbeg);
  // B operand of feature_gemm: gamma[pixel][n] for pixel kk * 64 + kgrp * 16
  // + c, transposed through LDS (pixel-major rows of 16 * NFB + 1 floats);
  // not needed when no entry is visited
  float bG[NFB][PPL][16];
  if (stop > tg.rbeg) {
    constexpr int GR = 16 * NFB + 1;
    const int mrow = lane & 15, kgrp = lane >> 4;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      float* row = s_w + (k * 64 + lane) * GR;
#pragma unroll
      for (int n = 0; n < 16 * NFB; ++n) row[n] = n <= F ? Gv[k][n] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < NFB; ++nb)
#pragma unroll
      for (int kk = 0; kk < PPL; ++kk)
#pragma unroll
        for (int c = 0; c < 16; ++c)
          bG[nb][kk][c] = s_w[(kk * 64 + kgrp * 16 + c) * GR + nb * 16 + mrow];
    __syncthreads();
  }
  // this lane's column of the reduced values in every record: lanes that
  // hold a copy of a component write the same bits to the same address, and
  // where the record has padding, the lanes without a component write
  // theirs into its first padding column, so the store needs no lane mask
  constexpr bool kPadCol = GS > (uint32_t)NV;
  float* const gcol = gpair + (my_comp >= 0 ? my_comp : (kPadCol ? NV : 0));
  for (uint32_t base = tg.rbeg; base < stop; base += KS) {
    const int cnt = __builtin_amdgcn_readfirstlane((int)min((uint32_t)KS, stop - base));
    // a list the forward staged whole is still in LDS
    const uint32_t e_mine =
        staged ? e_pre
               : stage_entries<FS4, true>(base, cnt, tg.sbase, vals, spair, rec, feat, s_r0,
                                          s_r1, s_f);
    if (lane < KS) s_e[lane] = e_mine;
    __syncthreads();
    // blocks of 16 entries: the per-entry pass, then their feature gradients
    for (int j0 = 0; j0 < cnt; j0 += 16) {
      const int j1 = min(j0 + 16, cnt);
      // two entries per iteration (immediate LDS offsets, half the loop
      // bookkeeping); the second is skipped past the block's end
      // gk: the pixels' kept weights of entry j, or nullptr
      auto entry = [&](const int j, const float* gk) {
        const uint32_t idx = base - tg.rbeg + (uint32_t)j;
        const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)e_mine, j);
        const float4 r0 = s_r0[j * (2 + FS4)], r1 = s_r1[j * (2 + FS4)];
        const float A = r1.x, B2 = r1.y, Cc = r1.z, tz = r1.w;
        const float dx = pixel_offset(tg.pxc, r0.x, r0.z);
        float* wrow = s_w + (j - j0) * WS + lane;
        float dy[PPL], gw[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          dy[k] = pixel_offset(pyc[k], r0.y, r0.w);
          if (gk) {
            gw[k] = idx < nl[k] ? gk[k] : 0.0f;
          } else {
            const float q = pixel_q32(A, B2, Cc, dx, dy[k]);
            const float ge = gauss_weight(q);
            gw[k] = (idx < nl[k] && q <= qcut) ? ge : 0.0f;
          }
        }
        float fv[FS4 * 4];
#pragma unroll
        for (int f = 0; f < FS4; ++f) {
          const float4 t4 = s_f[j * (2 + FS4) + f];
          fv[4 * f] = t4.x; fv[4 * f + 1] = t4.y; fv[4 * f + 2] = t4.z; fv[4 * f + 3] = t4.w;
        }
        const float al = fv[F];
        // Lanes whose pixel the pair does not reach run the same arithmetic
        // with g = 0: alpha = w = 0, T and the prefix unchanged, terms +-0 (a
        // pair that reaches no pixel of the tile gets a zero record this way;
        // a branch around it would copy T and the prefix on every entry).
        float pv[NR];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          const float g = gw[k];
          const float araw = al * g;
          const float a = clamp_alpha(araw, amax);
          const float w = a * T[k];
          wrow[k * 64] = w;
          float gf = kDA ? Gv[k][F] * (tz - t0[k]) : 0.0f;
#pragma unroll
          for (int f = 0; f < F; ++f) gf = __builtin_fmaf(Gv[k][f], fv[f], gf);
          const float om = 1.0f - a;
          const float inv = __builtin_amdgcn_rcpf(om);
          // the suffix G.O - sum over entries up to this one of w gf
          Spre[k] = __builtin_fmaf(w, gf, Spre[k]);
          const float suffix = GO[k] - Spre[k];
          float da = __builtin_fmaf(T[k], gf, -(suffix * inv));
          if (kDA) da = __builtin_fmaf(GAf[k], inv, da);
          // the clamp cuts alpha's dependence on g: gda = g da is dL/d(alpha)
          // where it does not hold (0 where it does), and dL/dq = -(alpha / 2)
          // gda, the factor -alpha / 2 being applied to the slot's sums by
          // the projection adjoint
          const float gda = araw > amax ? 0.0f : g * da;
          // moments of gda over the pixel offsets; the projection adjoint
          // turns them into dL/d(u, v, A, B, C) with the pair's conic (the
          // first pixel of a lane sets the values, later ones add to them)
          const float dyk = dy[k];
          const float gx = gda * dx, gy = gda * dyk;
          if (k == 0) {
            pv[5] = gda;
            pv[0] = gx;
            pv[1] = gy;
            pv[2] = gx * dx;
            pv[3] = gx * dyk;
            pv[4] = gy * dyk;
          } else {
            pv[5] += gda;
            pv[0] += gx;
            pv[1] += gy;
            pv[2] = __builtin_fmaf(gx, dx, pv[2]);
            pv[3] = __builtin_fmaf(gx, dyk, pv[3]);
            pv[4] = __builtin_fmaf(gy, dyk, pv[4]);
          }
          T[k] -= w;                       // as in the forward
        }
        const float tot = wave_reduce_scatter<NR>(pv, lane);
        if (kPadCol || writer) gcol[(size_t)e * GS] = tot;
      };
      if (kG > 0 && base == tg.rbeg && j0 == 0) {
        // the list's first block, unrolled whole so that the kept weights
        // are read from registers
#pragma unroll
        for (int j = 0; j < kG; ++j)
          if (j < j1) entry(j, gsave + j);
      } else {
        for (int j = j0; j < j1; j += 2) {
          entry(j, nullptr);
          if (j + 1 < j1) entry(j + 1, nullptr);
        }
      }
      __syncthreads();
      feature_gemm<C, PPL>(s_w, s_e + j0, j1 - j0, bG, gpair);
      __syncthreads();
    }
    __syncthreads();
  }
  // pairs that no pixel of the tile reached contribute nothing
  for (uint32_t p = stop + lane; p < tg.rend; p += 64) {
    const uint32_t e = vals[p];
    for (int c = 0; c < NV; ++c) gpair[(size_t)e * GS + c] = 0.0f;
  }
}

// Forward compositing of the batch: of the 5 + C output planes per view the
// ones selected by mask and the view's own channel set, and, when all are
// selected, per pixel T_final, n_last, the relative depth D' and its
// reference t0 for the backward.
template <int C, int PPL, int KS>
__global__ __launch_bounds__(64) void k_render_fwd(
    const ViewDev* __restrict__ views, int V, int N, float qcut, float amax,
    float teps, const uint4* __restrict__ tinfo, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ spair,
    const float4* __restrict__ rec, const float4* __restrict__ feat, float* __restrict__ out,
    float* __restrict__ tfin, uint32_t* __restrict__ nlast, float2* __restrict__ drel,
    uint32_t mask) {
  constexpr int F = 3 + C;
  constexpr int FS4 = (F + 4) / 4;
  constexpr int NO = 5 + C;           // output channels
  // staged entries: projection record, conic, features, one record per entry
  __shared__ float4 s_st[KS * (2 + FS4)];
  float4* const s_r0 = s_st;
  float4* const s_r1 = s_st + 1;
  float4* const s_f = s_st + 2;
  const TileGeom tg = tile_geom(views, N, tinfo);
  float T[PPL], acc[PPL][F + 1], pyc[PPL];
  uint32_t nl[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) pyc[k] = (float)(tg.py0 + k * tg.rows) + 0.5f;
  uint32_t e_first;
  float t0[PPL];
  const uint32_t ch = (uint32_t)tg.vw->ch & mask;
  constexpr uint32_t kPlanes = ROGS_CH_RGB | ROGS_CH_SEM | ROGS_CH_D | ROGS_CH_A;
  forward_tile<C, PPL, KS, false, true>(tg, qcut, amax, teps, vals, spair, rec, feat, s_r0, s_r1,
                                        s_f, pyc, acc, T, nl, e_first, t0, ch);
  const uint32_t len = tg.rend - tg.rbeg;
  const size_t HW = (size_t)tg.W * tg.H;
  float* o = out + (size_t)NO * tg.vw->pix_off;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = tg.py0 + k * tg.rows;
    if (!(tg.px < tg.W && py < tg.H)) continue;
    const size_t p = (size_t)py * tg.W + tg.px;
    if (ch & ROGS_CH_RGB)
#pragma unroll
      for (int f = 0; f < 3; ++f) o[f * HW + p] = acc[k][f];
    if (ch & ROGS_CH_SEM)
#pragma unroll
      for (int f = 3; f < F; ++f) o[f * HW + p] = acc[k][f];
    const float al = 1.0f - T[k];
    const float t0k = t0[k] < FLT_MAX ? t0[k] : 0.0f;        // 0 where nothing contributed
    if (ch & ROGS_CH_D) o[F * HW + p] = __builtin_fmaf(t0k, al, acc[k][F]);   // D = D' + t0 A
    if (ch & ROGS_CH_A) o[(F + 1) * HW + p] = al;
    if ((ch & kPlanes) == kPlanes) {
      tfin[tg.vw->pix_off + p] = T[k];
      nlast[tg.vw->pix_off + p] = (T[k] < teps) ? nl[k] : len;
      drel[tg.vw->pix_off + p] = make_float2(acc[k][F], t0k);
    }
  }
}

// Backward compositing of the batch from the output gradient G (5 + C planes
// per view), the outputs, T_final and n_last.
// Register budgets of the backward kernels: with one pixel per lane and up
// to 8 classes, 7 waves per SIMD at 16-entry staging (what its LDS block
// allows) and 5 at 32 entries (timed slightly faster than 6, the most its
// LDS block allows); the compiler meets them without spilling in the entry
// loops.  Other instances keep the compiler's own budget (1).
template <int C, int PPL, int KS>
constexpr int kWavesPerEu() {
  return (PPL == 1 && C <= 8 && KS <= 32) ? (KS <= 16 ? 7 : 5) : 1;
}
template <int C, int PPL, int KS>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(kWavesPerEu<C, PPL, KS>()))) void k_render_bwd(
    const ViewDev* __restrict__ views, int V, int N, float qcut, float amax,
    const uint4* __restrict__ tinfo, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ spair,
    const float4* __restrict__ rec, const float4* __restrict__ feat, const float* __restrict__ out,
    const float* __restrict__ G, const float* __restrict__ tfin,
    const uint32_t* __restrict__ nlast, const float2* __restrict__ drel,
    float* __restrict__ gpair) {
  constexpr int F = 3 + C;
  constexpr int FS4 = (F + 4) / 4;
  constexpr int NO = 5 + C;
  // staged entries: projection record, conic, features, one record per entry
  __shared__ float4 s_st[KS * (2 + FS4)];
  float4* const s_r0 = s_st;
  float4* const s_r1 = s_st + 1;
  float4* const s_f = s_st + 2;
  __shared__ float4 s_w4[bwd_lds_floats<C, PPL>() / 4];
  __shared__ uint32_t s_e[KS];
  const TileGeom tg = tile_geom(views, N, tinfo);
  const size_t HW = (size_t)tg.W * tg.H;
  float Gv[PPL][F + 2], GO[PPL], Tf[PPL], pyc[PPL], t0[PPL];
  uint32_t nl[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = tg.py0 + k * tg.rows;
    pyc[k] = (float)py + 0.5f;
    GO[k] = 0.0f;
    Tf[k] = 1.0f;
    nl[k] = 0;
    t0[k] = 0.0f;
#pragma unroll
    for (int f = 0; f < F + 2; ++f) Gv[k][f] = 0.0f;
    if (tg.px < tg.W && py < tg.H) {
      const size_t p = (size_t)py * tg.W + tg.px;
      const float* g = G + (size_t)NO * tg.vw->pix_off + p;
      const float* o = out + (size_t)NO * tg.vw->pix_off + p;
      float go = 0.0f;
#pragma unroll
      for (int f = 0; f < F + 2; ++f) Gv[k][f] = g[f * HW];
#pragma unroll
      for (int f = 0; f < F; ++f) go = __builtin_fmaf(Gv[k][f], o[f * HW], go);
      const float2 dr = drel[tg.vw->pix_off + p];          // D' and t0 of the forward
      go = __builtin_fmaf(Gv[k][F], dr.x, go);
      GO[k] = go;
      t0[k] = dr.y;
      Tf[k] = tfin[tg.vw->pix_off + p];
      nl[k] = nlast[tg.vw->pix_off + p];
    }
  }
  backward_tile<C, PPL, KS, true>(tg, qcut, amax, vals, spair, rec, feat, s_r0, s_r1, s_f,
                              reinterpret_cast<float*>(s_w4), s_e, pyc, Gv, GO, Tf, nl, gpair,
                              false, 0u, t0);
}

// The fused step's compositing: forward, the loss of Eq. 7-9 and 12 per pixel
// (its gradient, G.O, and this tile's share of the loss and of dL/d(a, b)),
// then the backward, in one kernel per tile.
// Register budget as for k_render_bwd.
template <int C, int PPL, int KS>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(kWavesPerEu<C, PPL, KS>()))) void k_render_step(
    const ViewDev* __restrict__ views, int V, int N, float qcut, float amax,
    float teps, const uint4* __restrict__ tinfo, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ spair,
    const float4* __restrict__ rec, const float4* __restrict__ feat, float* __restrict__ gpair,
    FusedLoss fl) {
  constexpr int F = 3 + C;
  constexpr int FS4 = (F + 4) / 4;
  // staged entries: projection record, conic, features, one record per entry
  __shared__ float4 s_st[KS * (2 + FS4)];
  float4* const s_r0 = s_st;
  float4* const s_r1 = s_st + 1;
  float4* const s_f = s_st + 2;
  __shared__ float4 s_w4[bwd_lds_floats<C, PPL>() / 4];
  __shared__ uint32_t s_e[KS];
  const int lane = threadIdx.x;
  const TileGeom tg = tile_geom(views, N, tinfo);
  float pyc[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) pyc[k] = (float)(tg.py0 + k * tg.rows) + 0.5f;
  float Gv[PPL][F + 2], GO[PPL], Tf[PPL];
  uint32_t nl[PPL];
  // the loss inputs of this lane's pixels (mask, target colour and label, in
  // parallel), requested before the forward so that their latency overlaps it
  const LossView lv = loss_view(fl.expo, fl.mcount, tg.v, fl.lam_c, fl.lam_s, fl.scale);
  bool lmask[PPL];
  uint32_t lab[PPL];
  float tv[PPL][3];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = tg.py0 + k * tg.rows;
    uint32_t m = 0;
    lab[k] = 0;
    tv[k][0] = tv[k][1] = tv[k][2] = 0.0f;
    if (tg.px < tg.W && py < tg.H && lv.any) {
      const size_t p = (size_t)py * tg.W + tg.px;
      const size_t pix = tg.vw->pix_off + p;
      const float* t = fl.tgt + 3 * (size_t)tg.vw->pix_off + p;
      const size_t HW = (size_t)tg.W * tg.H;
      m = fl.mask[pix];
      lab[k] = fl.label[pix];
      tv[k][0] = t[0];
      tv[k][1] = t[HW];
      tv[k][2] = t[2 * HW];
    }
    lmask[k] = m != 0;
  }
  if (tg.rend == tg.rbeg) {
    // a tile without entries: its pixels' outputs are 0 and there is nothing
    // to differentiate, so only its shares of the loss and of dL/db are
    // formed (dL/da is 0 at a zero output)
    float l = 0.0f, dbl = 0.0f;
#pragma unroll
    for (int k = 0; k < PPL; ++k)
      pixel_loss_empty<C>(tv[k], lmask[k] ? lv.wc : 0.0f, lmask[k] ? lv.ws : 0.0f, lv.ea, lv.b,
                          l, dbl);
    const float lp[3] = {l, 0.0f, dbl};
    const float tot = wave_reduce_scatter<3>(lp, lane);
    const int c = rs_comp(lane, 3);
    if (c >= 0 && (lane & rs_dup_bits(3)) == 0) fl.part[3 * (size_t)tg.gt + c] = tot;
    return;
  }
  {
    float T[PPL], acc[PPL][F + 1];
    uint32_t nlf[PPL];
    uint32_t e_first = 0;
    float t0[PPL];          // not used: the fused loss has no depth term
#pragma unroll
    for (int k = 0; k < PPL; ++k) t0[k] = 0.0f;
    // the footprint weights of the list's first 16 entries, kept from the
    // forward for the backward where the register budget has room for them
    // (one pixel per lane; up to 8 classes only with 32-entry staging, since
    // at 16 they would spill; with 16 classes the kernel runs 3 waves per
    // SIMD with or without them)
    constexpr int kG = (PPL == 1 && (C > 8 || KS == 32)) ? 16 : 0;
    float gsv[16];
    forward_tile<C, PPL, KS, true, false, kG>(tg, qcut, amax, teps, vals, spair, rec, feat, s_r0,
                                              s_r1, s_f, pyc, acc, T, nlf, e_first, t0,
                                              ROGS_CH_RGB | ROGS_CH_SEM, gsv);
    // loss epilogue: dL/dO and G.O per pixel, this tile's loss partials
    const uint32_t len = tg.rend - tg.rbeg;
    float l = 0.0f, dal = 0.0f, dbl = 0.0f;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int py = tg.py0 + k * tg.rows;
      float g[F];
      // every lane evaluates the loss; a pixel outside the mask or the image
      // has zero weights, so its gradient and loss terms are +-0
      pixel_loss<C>(acc[k], tv[k], lab[k], lmask[k] ? lv.wc : 0.0f, lmask[k] ? lv.ws : 0.0f,
                    lv.ea, lv.b, g, l, dal, dbl);
#pragma unroll
      for (int f = 0; f < F; ++f) Gv[k][f] = g[f];
      Gv[k][F] = 0.0f;         // the fused loss has no depth or alpha term
      Gv[k][F + 1] = 0.0f;
      // G.O over the composited channels, in the same form as the stand-alone
      // backward so that both round alike (its depth term adds 0 * D' = +0)
      float go = 0.0f;
#pragma unroll
      for (int f = 0; f < F; ++f) go = __builtin_fmaf(Gv[k][f], acc[k][f], go);
      const bool in_img = tg.px < tg.W && py < tg.H;
      const float tf = in_img ? T[k] : 1.0f;
      const uint32_t nlk = in_img ? ((T[k] < teps) ? nlf[k] : len) : 0u;
      GO[k] = go;
      Tf[k] = tf;
      nl[k] = nlk;
    }
    {
      const float lp[3] = {l, dal, dbl};
      const float tot = wave_reduce_scatter<3>(lp, lane);
      const int c = rs_comp(lane, 3);
      if (c >= 0 && (lane & rs_dup_bits(3)) == 0) fl.part[3 * (size_t)tg.gt + c] = tot;
    }
    // the fused loss has no depth or alpha term: their gradient rows are zero
    backward_tile<C, PPL, KS, false, kG>(tg, qcut, amax, vals, spair, rec, feat, s_r0, s_r1,
                                         s_f, reinterpret_cast<float*>(s_w4), s_e, pyc, Gv, GO,
                                         Tf, nl, gpair, len <= (uint32_t)KS, e_first, t0, gsv);
  }
}

// Work counts of a rendered batch (diagnostics): per pixel, the list entries
// it visits in front-to-back order up to its termination (n_last) and, of
// those, the ones whose 3-sigma test passes.  Summed over the batch into
// counts[0] (evaluated) and counts[1] (contributing) with 64-bit atomics.
__global__ __launch_bounds__(64) void k_count_work(
    const ViewDev* __restrict__ views, int V, int ppl, float qcut,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ pslot, const float4* __restrict__ rec,
    const uint32_t* __restrict__ nlast, unsigned long long* __restrict__ counts) {
  const int lane = threadIdx.x;
  const int gt = blockIdx.x;
  const int v = find_view(views, V, gt);
  const ViewDev& vw = views[v];
  const int lt = gt - vw.tile_off;
  const int ty = lt / vw.tiles_x, tx = lt - ty * vw.tiles_x;
  const int tw = vw.tw, th = vw.th;
  const int rows = 64 / tw;
  const int px = tx * tw + (lane % tw);
  const float pxc = (float)px + 0.5f;
  uint32_t nl[4];
  float pyc[4];
  uint32_t maxn = 0;
  for (int k = 0; k < 4; ++k) {
    const int py = ty * th + lane / tw + k * rows;
    pyc[k] = (float)py + 0.5f;
    nl[k] = (k < ppl && px < vw.w && py < vw.h) ? nlast[vw.pix_off + (size_t)py * vw.w + px] : 0u;
    maxn = max(maxn, nl[k]);
  }
  for (int o = 32; o > 0; o >>= 1) maxn = max(maxn, (uint32_t)__shfl_xor((int)maxn, o, 64));
  const uint2 rg = ranges[gt];
  const uint32_t stop = rg.x + min(maxn, rg.y - rg.x);
  unsigned long long ev = 0, co = 0;
  for (uint32_t p = rg.x; p < stop; ++p) {
    const uint32_t slot = pslot[vals[p]];
    const float4 r0 = rec[2 * (size_t)slot], r1 = rec[2 * (size_t)slot + 1];
    const float dx = pixel_offset(pxc, r0.x, r0.z);
    const uint32_t idx = p - rg.x;
    for (int k = 0; k < 4; ++k) {
      if (idx >= nl[k]) continue;
      ev += 1;
      const float dy = pixel_offset(pyc[k], r0.y, r0.w);
      if (pixel_q32(r1.x, 2.0f * r1.y, r1.z, dx, dy) <= qcut) co += 1;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    ev += (unsigned long long)__shfl_xor((long long)ev, o, 64);
    co += (unsigned long long)__shfl_xor((long long)co, o, 64);
  }
  if (lane == 0) {
    atomicAdd(&counts[0], ev);
    atomicAdd(&counts[1], co);
  }
}

template <int C, int PPL, int KS>
void fwd_launch(const Layout& L, void* ws, float* out, uint32_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_render_fwd<C, PPL, KS>), dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.q_cut, L.alpha_max,
                     L.t_eps, at<const uint4>(ws, L.o_tinfo), at<const uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_spair),
                     at<const float4>(ws, L.o_rec), at<const float4>(ws, L.o_feat), out,
                     at<float>(ws, L.o_tfin), at<uint32_t>(ws, L.o_nlast),
                     at<float2>(ws, L.o_drel), mask);
}

template <int C, int PPL, int KS>
void bwd_launch(const Layout& L, void* ws, const float* out, const float* G, hipStream_t st) {
  hipLaunchKernelGGL((k_render_bwd<C, PPL, KS>), dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.q_cut, L.alpha_max,
                     at<const uint4>(ws, L.o_tinfo), at<const uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_spair),
                     at<const float4>(ws, L.o_rec), at<const float4>(ws, L.o_feat), out, G,
                     at<const float>(ws, L.o_tfin), at<const uint32_t>(ws, L.o_nlast),
                     at<const float2>(ws, L.o_drel), at<float>(ws, L.o_gpair));
}

template <int C, int PPL, int KS>
void step_launch(const Layout& L, void* ws, const FusedLoss& fl, hipStream_t st) {
  hipLaunchKernelGGL((k_render_step<C, PPL, KS>), dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.q_cut, L.alpha_max,
                     L.t_eps, at<const uint4>(ws, L.o_tinfo), at<const uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_spair),
                     at<const float4>(ws, L.o_rec), at<const float4>(ws, L.o_feat),
                     at<float>(ws, L.o_gpair), fl);
}

// which: 0 forward, 1 backward, 2 fused step
template <int C, int PPL, int KS>
void launch_one(const Layout& L, void* ws, const float* out, const float* G, float* outw,
                const FusedLoss* fl, int which, uint32_t mask, hipStream_t st) {
  if (which == 0) fwd_launch<C, PPL, KS>(L, ws, outw, mask, st);
  else if (which == 1) bwd_launch<C, PPL, KS>(L, ws, out, G, st);
  else step_launch<C, PPL, KS>(L, ws, *fl, st);
}

template <int C, int PPL>
int dispatch_stage(const Layout& L, void* ws, const float* out, const float* G, float* outw,
                   const FusedLoss* fl, int which, uint32_t mask, hipStream_t st) {
  switch (L.stage) {
    case 16: launch_one<C, PPL, 16>(L, ws, out, G, outw, fl, which, mask, st); return 0;
    case 32: launch_one<C, PPL, 32>(L, ws, out, G, outw, fl, which, mask, st); return 0;
    case 64: launch_one<C, PPL, 64>(L, ws, out, G, outw, fl, which, mask, st); return 0;
    default: return -1;
  }
}

template <int C>
int dispatch_ppl(const Layout& L, void* ws, const float* out, const float* G, float* outw,
                 const FusedLoss* fl, int which, uint32_t mask, hipStream_t st) {
  switch (L.ppl) {
    case 1: return dispatch_stage<C, 1>(L, ws, out, G, outw, fl, which, mask, st);
    case 2: return dispatch_stage<C, 2>(L, ws, out, G, outw, fl, which, mask, st);
    case 4: return dispatch_stage<C, 4>(L, ws, out, G, outw, fl, which, mask, st);
    default: return -1;
  }
}

int dispatch(const Layout& L, void* ws, const float* out, const float* G, float* outw,
             const FusedLoss* fl, int which, uint32_t mask, hipStream_t st) {
  switch (L.C) {
    case 1: return dispatch_ppl<1>(L, ws, out, G, outw, fl, which, mask, st);
    case 2: return dispatch_ppl<2>(L, ws, out, G, outw, fl, which, mask, st);
    case 3: return dispatch_ppl<3>(L, ws, out, G, outw, fl, which, mask, st);
    case 4: return dispatch_ppl<4>(L, ws, out, G, outw, fl, which, mask, st);
    case 5: return dispatch_ppl<5>(L, ws, out, G, outw, fl, which, mask, st);
    case 6: return dispatch_ppl<6>(L, ws, out, G, outw, fl, which, mask, st);
    case 7: return dispatch_ppl<7>(L, ws, out, G, outw, fl, which, mask, st);
    case 8: return dispatch_ppl<8>(L, ws, out, G, outw, fl, which, mask, st);
    case 16: return dispatch_ppl<16>(L, ws, out, G, outw, fl, which, mask, st);
    default: return -1;
  }
}

}  // namespace

int launch_render_fwd(const Layout& L, void* ws, const rogs_surfels*, float* out, uint32_t mask,
                      hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  return dispatch(L, ws, nullptr, nullptr, out, nullptr, 0, mask, st);
}

int launch_render_bwd(const Layout& L, void* ws, const rogs_surfels*, const float* out,
                      const float* G, hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  return dispatch(L, ws, out, G, nullptr, nullptr, 1, 0u, st);
}

void launch_count_work(const Layout& L, void* ws, unsigned long long* counts, hipStream_t st) {
  if (L.total_tiles <= 0) return;
  hipLaunchKernelGGL(k_count_work, dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.ppl, L.q_cut,
                     at<const uint2>(ws, L.o_ranges), at<const uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_pslot), at<const float4>(ws, L.o_rec),
                     at<const uint32_t>(ws, L.o_nlast), counts);
}

int launch_render_step(const Layout& L, void* ws, const FusedLoss& fl, hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  return dispatch(L, ws, nullptr, nullptr, nullptr, &fl, 2, 0u, st);
}

}  // namespace rogs
