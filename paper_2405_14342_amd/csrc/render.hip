// Front-to-back alpha compositing of the sorted tile lists (Eq. 6) and its
// adjoint.
//
// Mapping: one 64-lane wave per tile, tiles launched longest list first; a tile of tile_w x tile_h = 64 * PPL
// pixels gives every lane PPL pixels of one column, so the per-pair x
// offset is shared and each broadcast record read from LDS feeds PPL pixels.
// The wave stages 64 list entries at a time in LDS (projection record + the
// surfel's colour/semantic features), then every lane walks them in order.
// A pixel stops after the surfel that takes its transmittance below t_eps;
// the wave leaves the list once all of its pixels have stopped.
//
// The backward walks the list front to back again, recomputing T exactly as
// the forward did, and uses sum_{j>k} w_j f_j = O - prefix - w_k f_k for the
// suffix term of dO/d(alpha_k).  Per (tile, pair) the 10 + C gradient values
// are summed over the lane's pixels and then over the wave, and written as
// one record at the pair's emission index; the projection adjoint later sums
// each surfel's records.  No atomics: the result does not depend on timing.
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


// Tile-major per-pixel record of the fused path: channel ch of in-tile pixel
// p of global tile gt is at tm[(gt * NCH + ch) * (64 * PPL) + p], with NCH =
// 3 + C gradients, then G.O, T_final and n_last (as bits).
template <int C>
__host__ __device__ constexpr int fused_channels() { return 3 + C + 3; }

template <int C, int PPL, bool FUSED>
__global__ __launch_bounds__(64) void k_render_fwd(
    const ViewDev* __restrict__ views, int V, int N, int tw, int th, float qcut, float amax,
    float teps, const uint32_t* __restrict__ order, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ pslot, const float4* __restrict__ rec,
    const float4* __restrict__ feat, float* __restrict__ out, float* __restrict__ tfin,
    uint32_t* __restrict__ nlast, FusedLoss fl) {
  constexpr int F = 3 + C;            // composited features besides depth
  constexpr int FS4 = (F + 4) / 4;    // float4 per feature record (features, alpha)
  constexpr int NO = 5 + C;           // output channels
  __shared__ float4 s_r0[64], s_r1[64];
  __shared__ float4 s_f[64 * FS4];
  const int lane = threadIdx.x;
  const int gt = (int)order[blockIdx.x];
  const int v = find_view(views, V, gt);
  const ViewDev& vw = views[v];
  const int W = vw.w, H = vw.h;
  const int lt = gt - vw.tile_off;
  const int ty = lt / vw.tiles_x, tx = lt - ty * vw.tiles_x;
  const int rows = 64 / tw;
  const int px = tx * tw + (lane % tw);
  const int py0 = ty * th + lane / tw;
  const float pxc = (float)px + 0.5f;

  float T[PPL], acc[PPL][F + 1], pyc[PPL];
  bool done[PPL];
  uint32_t nl[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = py0 + k * rows;
    done[k] = !(px < W && py < H);
    T[k] = 1.0f;
    nl[k] = 0;
    pyc[k] = (float)py + 0.5f;
#pragma unroll
    for (int f = 0; f <= F; ++f) acc[k][f] = 0.0f;
  }
  const uint2 rg = ranges[gt];
  const uint32_t len = rg.y - rg.x;
  const uint32_t sbase = (uint32_t)v * (uint32_t)N;
  bool stop_all = false;
  for (uint32_t base = rg.x; base < rg.y && !stop_all; base += 64) {
    const int cnt = (int)min(64u, rg.y - base);
    if (lane < cnt) {
      const uint32_t e = vals[base + lane];
      const uint32_t slot = pslot[e];
      s_r0[lane] = rec[2 * (size_t)slot];
      s_r1[lane] = rec[2 * (size_t)slot + 1];
      const uint32_t i = slot - sbase;
#pragma unroll
      for (int f = 0; f < FS4; ++f) s_f[lane * FS4 + f] = feat[(size_t)i * FS4 + f];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const float4 r0 = s_r0[j], r1 = s_r1[j];   // u_hi v_hi u_lo v_lo | A B C tz
      float fv[FS4 * 4];
#pragma unroll
      for (int f = 0; f < FS4; ++f) {
        const float4 t4 = s_f[j * FS4 + f];
        fv[4 * f] = t4.x; fv[4 * f + 1] = t4.y; fv[4 * f + 2] = t4.z; fv[4 * f + 3] = t4.w;
      }
      const float al = fv[F];
      const float dx = pixel_offset(pxc, r0.x, r0.z);
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        if (done[k]) continue;
        const float dy = pixel_offset(pyc[k], r0.y, r0.w);
        const float q = pixel_q32(r1.x, r1.y, r1.z, dx, dy);
        if (q <= qcut) {
          const float g = gauss_weight(q);
          const float a = clamp_alpha(al * g, amax);
          const float w = a * T[k];
#pragma unroll
          for (int f = 0; f < F; ++f) acc[k][f] += w * fv[f];
          acc[k][F] += w * r1.w;
          T[k] *= (1.0f - a);
          if (T[k] < teps) {
            done[k] = true;
            nl[k] = base - rg.x + (uint32_t)j + 1u;
          }
        }
      }
      bool mine = true;
#pragma unroll
      for (int k = 0; k < PPL; ++k) mine = mine && done[k];
      if (__all(mine)) { stop_all = true; break; }
    }
    __syncthreads();
  }
  if constexpr (!FUSED) {
    const size_t HW = (size_t)W * H;
    float* o = out + (size_t)NO * vw.pix_off;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int py = py0 + k * rows;
      if (!(px < W && py < H)) continue;
      const size_t p = (size_t)py * W + px;
#pragma unroll
      for (int f = 0; f <= F; ++f) o[f * HW + p] = acc[k][f];
      o[(F + 1) * HW + p] = 1.0f - T[k];
      tfin[vw.pix_off + p] = T[k];
      nlast[vw.pix_off + p] = (T[k] < teps) ? nl[k] : len;
    }
  } else {
    // loss epilogue: dL/dO, G.O, T and n_last per pixel in the tile-major
    // record, and this tile's share of the loss and of dL/d(a, b)
    constexpr int NCH = fused_channels<C>();
    constexpr int TP = 64 * PPL;
    const LossView lv = loss_view(fl.expo, fl.mcount, v, fl.lam_c, fl.lam_s, fl.scale);
    float* tm = fl.tm + (size_t)gt * NCH * TP;
    float l = 0.0f, dal = 0.0f, dbl = 0.0f;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int py = py0 + k * rows;
      const int pt = lane + 64 * k;
      float g[F];
#pragma unroll
      for (int f = 0; f < F; ++f) g[f] = 0.0f;
      float go = 0.0f, tf = 1.0f;
      uint32_t nlk = 0;
      if (px < W && py < H) {
        const size_t p = (size_t)py * W + px;
        if (fl.mask[vw.pix_off + p] && lv.any) {
          const float* t = fl.tgt + 3 * (size_t)vw.pix_off + p;
          const size_t HW = (size_t)W * H;
          const float tv[3] = {t[0], t[HW], t[2 * HW]};
          pixel_loss<C>(acc[k], tv, fl.label[vw.pix_off + p], lv.wc, lv.ws, lv.ea, lv.b, g, l,
                        dal, dbl);
        }
        // G.O over the composited channels; the depth row of G is zero
        const float gd = 0.0f;
#pragma unroll
        for (int f = 0; f < F; ++f) go += g[f] * acc[k][f];
        go += gd * acc[k][F];
        tf = T[k];
        nlk = (T[k] < teps) ? nl[k] : len;
      }
#pragma unroll
      for (int f = 0; f < F; ++f) tm[f * TP + pt] = g[f];
      tm[F * TP + pt] = go;
      tm[(F + 1) * TP + pt] = tf;
      tm[(F + 2) * TP + pt] = __uint_as_float(nlk);
    }
    for (int o = 32; o > 0; o >>= 1) {
      l += __shfl_xor(l, o, 64);
      dal += __shfl_xor(dal, o, 64);
      dbl += __shfl_xor(dbl, o, 64);
    }
    if (lane == 0) {
      fl.part[3 * (size_t)gt] = l;
      fl.part[3 * (size_t)gt + 1] = dal;
      fl.part[3 * (size_t)gt + 2] = dbl;
    }
  }
}

template <int C, int PPL, bool FUSED>
__global__ __launch_bounds__(64) void k_render_bwd(
    const ViewDev* __restrict__ views, int V, int N, int tw, int th, float qcut, float amax,
    const uint32_t* __restrict__ order, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ pslot, const float4* __restrict__ rec,
    const float4* __restrict__ feat, const float* __restrict__ out, const float* __restrict__ G,
    const float* __restrict__ tfin, const uint32_t* __restrict__ nlast, float* __restrict__ gpair,
    int GS, const float* __restrict__ tm_in) {
  constexpr int F = 3 + C;
  constexpr int FS4 = (F + 4) / 4;
  constexpr int NO = 5 + C;
  constexpr int NV = 10 + C;          // du dv dA dB dC dalpha dtz drgb[3] dsem[C]
  // the fused loss has no depth or alpha term: their gradient rows are zero
  constexpr bool kDA = !FUSED;
  __shared__ float4 s_r0[64], s_r1[64];
  __shared__ float4 s_f[64 * FS4];
  const int lane = threadIdx.x;
  const int gt = (int)order[blockIdx.x];
  const int v = find_view(views, V, gt);
  const ViewDev& vw = views[v];
  const int W = vw.w, H = vw.h;
  const int lt = gt - vw.tile_off;
  const int ty = lt / vw.tiles_x, tx = lt - ty * vw.tiles_x;
  const int rows = 64 / tw;
  const int px = tx * tw + (lane % tw);
  const int py0 = ty * th + lane / tw;
  const float pxc = (float)px + 0.5f;
  const size_t HW = (size_t)W * H;
  const int my_comp = rs_comp(lane, NV);
  const bool writer = my_comp >= 0 && (lane & rs_dup_bits(NV)) == 0;

  float Gv[PPL][F + 2], GO[PPL], Tf[PPL], T[PPL], Spre[PPL], pyc[PPL];
  uint32_t nl[PPL];
  uint32_t maxn = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int py = py0 + k * rows;
    pyc[k] = (float)py + 0.5f;
    T[k] = 1.0f;
    Spre[k] = 0.0f;
    GO[k] = 0.0f;
    Tf[k] = 1.0f;
    nl[k] = 0;
#pragma unroll
    for (int f = 0; f < F + 2; ++f) Gv[k][f] = 0.0f;
    if constexpr (FUSED) {
      // tile-major record written by the fused forward (zeros off-image)
      constexpr int NCH = fused_channels<C>();
      constexpr int TP = 64 * PPL;
      const float* tm = tm_in + (size_t)gt * NCH * TP + lane + 64 * k;
#pragma unroll
      for (int f = 0; f < F; ++f) Gv[k][f] = tm[f * TP];
      GO[k] = tm[F * TP];
      Tf[k] = tm[(F + 1) * TP];
      nl[k] = __float_as_uint(tm[(F + 2) * TP]);
      maxn = max(maxn, nl[k]);
    } else if (px < W && py < H) {
      const size_t p = (size_t)py * W + px;
      const float* g = G + (size_t)NO * vw.pix_off + p;
      const float* o = out + (size_t)NO * vw.pix_off + p;
      float go = 0.0f;
#pragma unroll
      for (int f = 0; f < F + 2; ++f) Gv[k][f] = g[f * HW];
#pragma unroll
      for (int f = 0; f <= F; ++f) go += Gv[k][f] * o[f * HW];
      GO[k] = go;
      Tf[k] = tfin[vw.pix_off + p];
      nl[k] = nlast[vw.pix_off + p];
      maxn = max(maxn, nl[k]);
    }
  }
  for (int o = 32; o > 0; o >>= 1) maxn = max(maxn, (uint32_t)__shfl_xor((int)maxn, o, 64));
  const uint2 rg = ranges[gt];
  const uint32_t stop = rg.x + min(maxn, rg.y - rg.x);
  const uint32_t sbase = (uint32_t)v * (uint32_t)N;
  for (uint32_t base = rg.x; base < stop; base += 64) {
    const int cnt = (int)min(64u, stop - base);
    uint32_t e_mine = 0;
    if (lane < cnt) {
      e_mine = vals[base + lane];
      const uint32_t slot = pslot[e_mine];
      s_r0[lane] = rec[2 * (size_t)slot];
      s_r1[lane] = rec[2 * (size_t)slot + 1];
      const uint32_t i = slot - sbase;
#pragma unroll
      for (int f = 0; f < FS4; ++f) s_f[lane * FS4 + f] = feat[(size_t)i * FS4 + f];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const uint32_t idx = base - rg.x + (uint32_t)j;
      const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)e_mine, j);
      const float4 r0 = s_r0[j], r1 = s_r1[j];
      const float A = r1.x, B = r1.y, Cc = r1.z, tz = r1.w;
      const float dx = pixel_offset(pxc, r0.x, r0.z);
      float dy[PPL], q[PPL];
      bool hit[PPL];
      bool any = false;
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        dy[k] = pixel_offset(pyc[k], r0.y, r0.w);
        q[k] = pixel_q32(A, B, Cc, dx, dy[k]);
        hit[k] = idx < nl[k] && q[k] <= qcut;
        any = any || hit[k];
      }
      if (!__any(any)) {            // no pixel of the tile reached by this pair
        if (writer) gpair[(size_t)e * GS + my_comp] = 0.0f;
        continue;
      }
      float fv[FS4 * 4];
#pragma unroll
      for (int f = 0; f < FS4; ++f) {
        const float4 t4 = s_f[j * FS4 + f];
        fv[4 * f] = t4.x; fv[4 * f + 1] = t4.y; fv[4 * f + 2] = t4.z; fv[4 * f + 3] = t4.w;
      }
      const float al = fv[F];
      // Lanes whose pixel the pair does not reach run the same arithmetic with
      // g = 0: alpha = w = 0, T and the prefix unchanged, every term +-0.
      float pv[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) pv[c] = 0.0f;
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const float g = hit[k] ? gauss_weight(q[k]) : 0.0f;
        const float araw = al * g;
        const bool clamped = araw > amax;
        const float a = clamped ? amax : araw;
        const float w = a * T[k];
        float gf = kDA ? Gv[k][F] * tz : 0.0f;
#pragma unroll
        for (int f = 0; f < F; ++f) gf += Gv[k][f] * fv[f];
#pragma unroll
        for (int f = 0; f < F; ++f) pv[7 + f] += w * Gv[k][f];
        if (kDA) pv[6] += w * Gv[k][F];
        const float om = 1.0f - a;
        const float inv = __builtin_amdgcn_rcpf(om);
        const float suffix = (GO[k] - Spre[k]) - w * gf;
        float da = T[k] * gf - suffix * inv;
        if (kDA) da += Gv[k][F + 1] * Tf[k] * inv;
        Spre[k] += w * gf;
        const float gd = clamped ? 0.0f : g;      // the clamp cuts alpha's dependence on g
        pv[5] += gd * da;
        const float dq = -0.5f * gd * al * da;
        const float dyk = dy[k];
        pv[2] += dx * dx * dq;
        pv[3] += 2.0f * dx * dyk * dq;
        pv[4] += dyk * dyk * dq;
        pv[0] += -(2.0f * A * dx + 2.0f * B * dyk) * dq;
        pv[1] += -(2.0f * Cc * dyk + 2.0f * B * dx) * dq;
        T[k] *= om;
      }
      const float tot = wave_reduce_scatter<NV>(pv, lane);
      if (writer) gpair[(size_t)e * GS + my_comp] = tot;
    }
    __syncthreads();
  }
  // pairs that no pixel of the tile reached contribute nothing
  for (uint32_t p = stop + lane; p < rg.y; p += 64) {
    const uint32_t e = vals[p];
    for (int c = 0; c < NV; ++c) gpair[(size_t)e * GS + c] = 0.0f;
  }
}

// Work counts of a rendered batch (diagnostics): per pixel, the list entries
// it visits in front-to-back order up to its termination (n_last) and, of
// those, the ones whose 3-sigma test passes.  Summed over the batch into
// counts[0] (evaluated) and counts[1] (contributing) with 64-bit atomics.
__global__ __launch_bounds__(64) void k_count_work(
    const ViewDev* __restrict__ views, int V, int tw, int th, int ppl, float qcut,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ pslot, const float4* __restrict__ rec,
    const uint32_t* __restrict__ nlast, unsigned long long* __restrict__ counts) {
  const int lane = threadIdx.x;
  const int gt = blockIdx.x;
  const int v = find_view(views, V, gt);
  const ViewDev& vw = views[v];
  const int lt = gt - vw.tile_off;
  const int ty = lt / vw.tiles_x, tx = lt - ty * vw.tiles_x;
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
      if (pixel_q32(r1.x, r1.y, r1.z, dx, dy) <= qcut) co += 1;
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

template <int C, int PPL, bool FUSED>
void fwd_launch(const Layout& L, void* ws, float* out, const FusedLoss& fl, hipStream_t st) {
  hipLaunchKernelGGL((k_render_fwd<C, PPL, FUSED>), dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.tw, L.th, L.q_cut, L.alpha_max,
                     L.t_eps, at<const uint32_t>(ws, L.o_order), at<const uint2>(ws, L.o_ranges),
                     at<const uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_pslot), at<const float4>(ws, L.o_rec),
                     at<const float4>(ws, L.o_feat), out, at<float>(ws, L.o_tfin),
                     at<uint32_t>(ws, L.o_nlast), fl);
}

template <int C, int PPL, bool FUSED>
void bwd_launch(const Layout& L, void* ws, const float* out, const float* G, hipStream_t st) {
  hipLaunchKernelGGL((k_render_bwd<C, PPL, FUSED>), dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.tw, L.th, L.q_cut, L.alpha_max,
                     at<const uint32_t>(ws, L.o_order), at<const uint2>(ws, L.o_ranges),
                     at<const uint32_t>(ws, L.o_vals), at<const uint32_t>(ws, L.o_pslot),
                     at<const float4>(ws, L.o_rec), at<const float4>(ws, L.o_feat), out, G, at<const float>(ws, L.o_tfin),
                     at<const uint32_t>(ws, L.o_nlast), at<float>(ws, L.o_gpair), L.GS,
                     FUSED ? at<const float>(ws, L.o_tm) : nullptr);
}

template <int C, int PPL>
void launch_one(const Layout& L, void* ws, const float* out, const float* G, float* outw,
                const FusedLoss* fl, bool bwd, hipStream_t st) {
  if (bwd) {
    if (fl) bwd_launch<C, PPL, true>(L, ws, out, G, st);
    else bwd_launch<C, PPL, false>(L, ws, out, G, st);
  } else {
    if (fl) fwd_launch<C, PPL, true>(L, ws, outw, *fl, st);
    else fwd_launch<C, PPL, false>(L, ws, outw, FusedLoss{}, st);
  }
}

template <int C>
int dispatch_ppl(const Layout& L, void* ws, const float* out, const float* G, float* outw,
                 const FusedLoss* fl, bool bwd, hipStream_t st) {
  switch (L.ppl) {
    case 1: launch_one<C, 1>(L, ws, out, G, outw, fl, bwd, st); return 0;
    case 2: launch_one<C, 2>(L, ws, out, G, outw, fl, bwd, st); return 0;
    case 4: launch_one<C, 4>(L, ws, out, G, outw, fl, bwd, st); return 0;
    default: return -1;
  }
}

int dispatch(const Layout& L, void* ws, const float* out, const float* G, float* outw,
             const FusedLoss* fl, bool bwd, hipStream_t st) {
  switch (L.C) {
    case 1: return dispatch_ppl<1>(L, ws, out, G, outw, fl, bwd, st);
    case 2: return dispatch_ppl<2>(L, ws, out, G, outw, fl, bwd, st);
    case 3: return dispatch_ppl<3>(L, ws, out, G, outw, fl, bwd, st);
    case 4: return dispatch_ppl<4>(L, ws, out, G, outw, fl, bwd, st);
    case 5: return dispatch_ppl<5>(L, ws, out, G, outw, fl, bwd, st);
    case 6: return dispatch_ppl<6>(L, ws, out, G, outw, fl, bwd, st);
    case 7: return dispatch_ppl<7>(L, ws, out, G, outw, fl, bwd, st);
    case 8: return dispatch_ppl<8>(L, ws, out, G, outw, fl, bwd, st);
    case 16: return dispatch_ppl<16>(L, ws, out, G, outw, fl, bwd, st);
    default: return -1;
  }
}

}  // namespace

int launch_render_fwd(const Layout& L, void* ws, const rogs_surfels*, float* out, hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  return dispatch(L, ws, nullptr, nullptr, out, nullptr, false, st);
}

int launch_render_bwd(const Layout& L, void* ws, const rogs_surfels*, const float* out,
                      const float* G, hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  return dispatch(L, ws, out, G, nullptr, nullptr, true, st);
}

void launch_count_work(const Layout& L, void* ws, unsigned long long* counts, hipStream_t st) {
  if (L.total_tiles <= 0) return;
  hipLaunchKernelGGL(k_count_work, dim3((unsigned)L.total_tiles), dim3(64), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.tw, L.th, L.ppl, L.q_cut,
                     at<const uint2>(ws, L.o_ranges), at<const uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_pslot), at<const float4>(ws, L.o_rec),
                     at<const uint32_t>(ws, L.o_nlast), counts);
}

int launch_render_fwd_fused(const Layout& L, void* ws, const FusedLoss& fl, hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  return dispatch(L, ws, nullptr, nullptr, nullptr, &fl, false, st);
}

int launch_render_bwd_fused(const Layout& L, void* ws, hipStream_t st) {
  if (L.total_tiles <= 0) return 0;
  FusedLoss dummy{};
  return dispatch(L, ws, nullptr, nullptr, nullptr, &dummy, true, st);
}

}  // namespace rogs
