// Loss seed (Eq. 7-9, 12), projection adjoint (chain rule of Eq. 5 and the
// surfel covariance of Eq. 2 back to height, rotation and scale) and Adam.
#include "rogs_internal.h"

namespace rogs {

namespace {

constexpr int kLossBlock = 256;

__device__ __forceinline__ float wave_sum_f(float x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ int find_view_pix(const ViewDev* __restrict__ views, int V,
                                             int64_t p) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].pix_off <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// |M_v|: number of mask pixels per view.  grid.y = view; each block counts
// kMaskPerBlock bytes of the view's mask, 16 per thread and iteration (one
// 16-byte load where the group is aligned and whole), and adds its count with
// one integer atomic (exact, order-free).
constexpr int kMaskIters = 2;
constexpr int kMaskPerBlock = 16 * kLossBlock * kMaskIters;

__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t x) {
  // bit 7 of each byte of t is set iff that byte of x is nonzero
  const uint32_t t = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
  return (uint32_t)__popc(t & 0x80808080u);
}

__global__ __launch_bounds__(kLossBlock) void k_mask_count(const ViewDev* __restrict__ views,
                                                           const uint8_t* __restrict__ mask,
                                                           uint32_t* __restrict__ mcount) {
  __shared__ uint32_t s_w[kLossBlock / 64];
  const int v = blockIdx.y;
  const ViewDev& vw = views[v];
  const int64_t npix = (int64_t)vw.w * vw.h;
  const int64_t base = (int64_t)blockIdx.x * kMaskPerBlock;
  if (base >= npix) return;
  const uint8_t* m = mask + vw.pix_off;
  uint32_t c = 0;
#pragma unroll
  for (int it = 0; it < kMaskIters; ++it) {
    const int64_t p = base + 16 * ((int64_t)it * kLossBlock + threadIdx.x);
    if (p >= npix) continue;
    const uint8_t* g = m + p;
    if (p + 16 <= npix && (reinterpret_cast<uintptr_t>(g) & 15u) == 0) {
      const uint4 x = *reinterpret_cast<const uint4*>(g);
      c += nonzero_bytes(x.x) + nonzero_bytes(x.y) + nonzero_bytes(x.z) + nonzero_bytes(x.w);
    } else {
      const int n = (int)min<int64_t>(16, npix - p);
      for (int k = 0; k < n; ++k) c += g[k] ? 1u : 0u;
    }
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kLossBlock / 64; ++w) t += s_w[w];
    if (t) atomicAdd(&mcount[v], t);
  }
}

// Sums the per-block loss partials of each view: one block per view, a fixed
// assignment of partials to threads and a fixed tree, so the result does not
// depend on scheduling.  Then block 0 of a second launch adds the views.
__global__ __launch_bounds__(256) void k_loss_views(const int64_t* __restrict__ first_blk,
                                                    const float* __restrict__ part,
                                                    float* __restrict__ per_view,
                                                    float* __restrict__ d_exp) {
  __shared__ float s[3][256];
  const int v = blockIdx.x;
  float l = 0.0f, a = 0.0f, b = 0.0f;
  for (int64_t k = first_blk[v] + threadIdx.x; k < first_blk[v + 1]; k += 256) {
    l += part[3 * k];
    a += part[3 * k + 1];
    b += part[3 * k + 2];
  }
  s[0][threadIdx.x] = l;
  s[1][threadIdx.x] = a;
  s[2][threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
      s[2][threadIdx.x] += s[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    per_view[v] = s[0][0];
    if (d_exp) {
      d_exp[2 * v] += s[1][0];
      d_exp[2 * v + 1] += s[2][0];
    }
  }
}

__global__ void k_loss_total(int V, const float* __restrict__ per_view, float* __restrict__ loss_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && loss_out) {
    float t = 0.0f;
    for (int v = 0; v < V; ++v) t += per_view[v];
    loss_out[0] += t;
  }
}

}  // namespace

// ------------------------------------------------------------ projection adjoint

namespace {

// Reverse-mode chain of the projection (value path, FP32): given dL/d(u, v,
// A, B, C, t_z) of one (view, surfel) pair, accumulate dL/d(z, q, s).
__device__ __forceinline__ void proj_adjoint(const ViewDev& c, float eps, float x, float y,
                                             float z, const float q[4], float sx, float sy,
                                             float du, float dv, float dA, float dB, float dC,
                                             float dtz_direct, float& dz, float dq[4], float& dsx,
                                             float& dsy) {
  const float* R = c.R;
  const float tx = R[0] * x + R[1] * y + R[2] * z + c.t[0];
  const float ty = R[3] * x + R[4] * y + R[5] * z + c.t[1];
  const float tz = R[6] * x + R[7] * y + R[8] * z + c.t[2];
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float iq = 1.0f / qn;
  const float w = q[0] * iq, a = q[1] * iq, b = q[2] * iq, cc = q[3] * iq;
  const float r1[3] = {1.0f - 2.0f * (b * b + cc * cc), 2.0f * (a * b + w * cc),
                       2.0f * (a * cc - w * b)};
  const float r2[3] = {2.0f * (a * b - w * cc), 1.0f - 2.0f * (a * a + cc * cc),
                       2.0f * (b * cc + w * a)};
  float c1[3], c2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c1[k] = sx * (R[3 * k] * r1[0] + R[3 * k + 1] * r1[1] + R[3 * k + 2] * r1[2]);
    c2[k] = sy * (R[3 * k] * r2[0] + R[3 * k + 1] * r2[1] + R[3 * k + 2] * r2[2]);
  }
  float j00, j11, j02, j12, xr = 0.0f, yr = 0.0f, xc = 0.0f, yc = 0.0f;
  bool clx = false, cly = false;
  if (c.model == ROGS_PINHOLE) {
    const float limx = 0.65f * (float)c.w / c.fx, limy = 0.65f * (float)c.h / c.fy;
    xr = tx / tz;
    yr = ty / tz;
    clx = (xr < -limx) || (xr > limx);
    cly = (yr < -limy) || (yr > limy);
    xc = fminf(fmaxf(xr, -limx), limx);
    yc = fminf(fmaxf(yr, -limy), limy);
    j00 = c.fx / tz;
    j11 = c.fy / tz;
    j02 = -j00 * xc;
    j12 = -j11 * yc;
  } else {
    j00 = c.fx; j11 = c.fy; j02 = 0.0f; j12 = 0.0f;
  }
  const float m00 = j00 * c1[0] + j02 * c1[2];
  const float m01 = j00 * c2[0] + j02 * c2[2];
  const float m10 = j11 * c1[1] + j12 * c1[2];
  const float m11 = j11 * c2[1] + j12 * c2[2];
  const float g0 = m00 * m00 + m01 * m01, g1 = m10 * m10 + m11 * m11;
  const float s00 = g0 + eps, s11 = g1 + eps, s01 = m00 * m10 + m01 * m11;
  const float dm = m00 * m11 - m01 * m10;
  const float det = dm * dm + eps * (g0 + g1) + eps * eps;
  const float idet = 1.0f / det;
  const float A = s11 * idet, B = -s01 * idet, Cc = s00 * idet;
  // conic -> Sigma' -> M
  const float ds11 = dA * idet, ds01 = -dB * idet, ds00 = dC * idet;
  const float ddet = -(A * dA + B * dB + Cc * dC) * idet;
  const float ddm = 2.0f * dm * ddet;
  const float dg0 = eps * ddet + ds00, dg1 = eps * ddet + ds11;
  float dm00 = m11 * ddm + m10 * ds01 + 2.0f * m00 * dg0;
  float dm01 = -m10 * ddm + m11 * ds01 + 2.0f * m01 * dg0;
  float dm10 = -m01 * ddm + m00 * ds01 + 2.0f * m10 * dg1;
  float dm11 = m00 * ddm + m01 * ds01 + 2.0f * m11 * dg1;
  // M = J [c1 c2]
  float dj00 = c1[0] * dm00 + c2[0] * dm01;
  const float dj02 = c1[2] * dm00 + c2[2] * dm01;
  float dj11 = c1[1] * dm10 + c2[1] * dm11;
  const float dj12 = c1[2] * dm10 + c2[2] * dm11;
  const float dc1[3] = {j00 * dm00, j11 * dm10, j02 * dm00 + j12 * dm10};
  const float dc2[3] = {j00 * dm01, j11 * dm11, j02 * dm01 + j12 * dm11};
  float dt0 = 0.0f, dt1 = 0.0f, dt2 = dtz_direct;
  if (c.model == ROGS_PINHOLE) {
    dj00 += -xc * dj02;
    const float dxc = -j00 * dj02;
    dj11 += -yc * dj12;
    const float dyc = -j11 * dj12;
    dt2 += -(j00 / tz) * dj00 - (j11 / tz) * dj11;
    float dxr = clx ? 0.0f : dxc;
    float dyr = cly ? 0.0f : dyc;
    dxr += c.fx * du;
    dyr += c.fy * dv;
    dt0 += dxr / tz;
    dt1 += dyr / tz;
    dt2 += -(xr / tz) * dxr - (yr / tz) * dyr;
  } else {
    dt0 += c.fx * du;
    dt1 += c.fy * dv;
  }
  dz += R[2] * dt0 + R[5] * dt1 + R[8] * dt2;
  // c1 = R (sx r1), c2 = R (sy r2)
  float dT1[3], dT2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dT1[k] = R[k] * dc1[0] + R[3 + k] * dc1[1] + R[6 + k] * dc1[2];
    dT2[k] = R[k] * dc2[0] + R[3 + k] * dc2[1] + R[6 + k] * dc2[2];
  }
  dsx += r1[0] * dT1[0] + r1[1] * dT1[1] + r1[2] * dT1[2];
  dsy += r2[0] * dT2[0] + r2[1] * dT2[1] + r2[2] * dT2[2];
  const float dr1[3] = {sx * dT1[0], sx * dT1[1], sx * dT1[2]};
  const float dr2[3] = {sy * dT2[0], sy * dT2[1], sy * dT2[2]};
  float dw = 0.0f, da = 0.0f, db = 0.0f, dc = 0.0f;
  db += -4.0f * b * dr1[0]; dc += -4.0f * cc * dr1[0];
  da += 2.0f * b * dr1[1]; db += 2.0f * a * dr1[1]; dw += 2.0f * cc * dr1[1]; dc += 2.0f * w * dr1[1];
  da += 2.0f * cc * dr1[2]; dc += 2.0f * a * dr1[2]; dw += -2.0f * b * dr1[2]; db += -2.0f * w * dr1[2];
  da += 2.0f * b * dr2[0]; db += 2.0f * a * dr2[0]; dw += -2.0f * cc * dr2[0]; dc += -2.0f * w * dr2[0];
  da += -4.0f * a * dr2[1]; dc += -4.0f * cc * dr2[1];
  db += 2.0f * cc * dr2[2]; dc += 2.0f * b * dr2[2]; dw += 2.0f * a * dr2[2]; da += 2.0f * w * dr2[2];
  const float dot = w * dw + a * da + b * db + cc * dc;
  dq[0] += (dw - w * dot) * iq;
  dq[1] += (da - a * dot) * iq;
  dq[2] += (db - b * dot) * iq;
  dq[3] += (dc - cc * dot) * iq;
}

// Bias corrections of Adam for a step (same arithmetic on every path).
__device__ __forceinline__ void adam_bias(float b1, float b2, int64_t step, float& bc1,
                                          float& bc2s) {
  bc1 = (float)(1.0 - pow((double)b1, (double)step));
  bc2s = (float)sqrt(1.0 - pow((double)b2, (double)step));
}

// z learning rate of a step: z_start (z_end / z_start)^t, t = (step-1)/(total-1).
__device__ __forceinline__ float z_rate(const AdamArgs& aa, int64_t step) {
  if (aa.total_steps <= 1) return aa.total_steps == 1 ? aa.z_start : aa.lr.z;
  double t = (double)(step - 1) / (double)(aa.total_steps - 1);
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  return (float)((double)aa.z_start * pow((double)aa.z_end / (double)aa.z_start, t));
}

// Adam (torch semantics) on the 11 + C rows of surfel i, with the chain rule
// through s = exp(log s) and alpha = sigmoid(logit); refreshes s and alpha.
template <int C>
__device__ __forceinline__ void adam_surfel(int i, size_t N, float* __restrict__ P,
                                            float* __restrict__ M, float* __restrict__ Vv,
                                            float* __restrict__ s_act, float* __restrict__ a_act,
                                            const float* g, const rogs_lr& lr, float lr_z,
                                            float b1, float b2, float eps, float bc1,
                                            float bc2s) {
  const float sx = s_act[i], sy = s_act[N + i], al = a_act[i];
  // rows in groups of kRows: a group's loads are all issued before its
  // stores, so one memory round trip serves kRows rows (the rows of one
  // array are distinct addresses, which the compiler cannot prove itself)
  constexpr int NR = 11 + C, kRows = 8;
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += kRows) {
    float pm[kRows], pv[kRows], pp[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      if (r0 + u < NR) {
        const size_t j = (size_t)(r0 + u) * N + i;
        pm[u] = M[j];
        pv[u] = Vv[j];
        pp[u] = P[j];
      }
    }
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      const int r = r0 + u;
      if (r >= NR) break;
      const size_t j = (size_t)r * N + i;
      float gr = g[r];
      float lrr;
      if (r == 0) lrr = lr_z;
      else if (r <= 4) lrr = lr.q;
      else if (r <= 6) { lrr = lr.s; gr *= (r == 5) ? sx : sy; }      // d/d log s = s d/ds
      else if (r == 7) { lrr = lr.alpha; gr *= al * (1.0f - al); }   // d/d logit = a(1-a) d/da
      else if (r <= 10) lrr = lr.rgb;
      else lrr = lr.sem;
      const float m = b1 * pm[u] + (1.0f - b1) * gr;
      const float v = b2 * pv[u] + (1.0f - b2) * gr * gr;
      M[j] = m;
      Vv[j] = v;
      const float denom = sqrtf(v) / bc2s + eps;
      P[j] = pp[u] - (lrr / bc1) * (m / denom);
    }
  }
  s_act[i] = expf(P[5 * N + i]);
  s_act[N + i] = expf(P[6 * N + i]);
  a_act[i] = 1.0f / (1.0f + expf(-P[7 * N + i]));
}

// Per-slot sums of the per-pair gradient records.  The records of a visible
// slot are contiguous in emission order; a slot with at most kLongRows records
// is summed in record order by Q threads, one per float4 column of the record
// (so a wave's loads cover runs of whole records), a longer one by one wave
// (lane l takes records l, l + 64, ... in order, then the wave reduce-scatter).
// Each slot's sum depends only on its own records, not on how a batch is laid
// out.
constexpr uint32_t kLongRows = 32;

template <int C>
__global__ __launch_bounds__(256) void k_slot_sums(const uint32_t* __restrict__ misc,
                                                   int64_t scap, int64_t cap,
                                                   const uint32_t* __restrict__ scnt,
                                                   const uint32_t* __restrict__ soff,
                                                   const float* __restrict__ gpair,
                                                   float* __restrict__ ssum,
                                                   uint32_t* __restrict__ long_list,
                                                   uint32_t* __restrict__ long_count) {
  constexpr int GSC = ((10 + C) + 3) & ~3;
  constexpr int Q = GSC / 4;
  const int64_t S = min((int64_t)misc[kMiscVisible], scap);
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = t / Q;
  const int q = (int)(t - k * Q);
  if (k >= S) return;
  const uint32_t n = scnt[k], o = soff[k];
  if (n > kLongRows) {
    if (q == 0) long_list[atomicAdd(long_count, 1u)] = (uint32_t)k;
    return;
  }
  // after a pair-capacity overflow the records past the capacity were never written
  const uint32_t m = ((int64_t)o + n <= cap) ? n : (((int64_t)o < cap) ? (uint32_t)(cap - o) : 0u);
  const float4* col = reinterpret_cast<const float4*>(gpair) + (size_t)o * Q + q;
  // rows in groups of four whose loads are issued together, the last group
  // padded with +0 (the sum starts at +0 and never becomes -0, so adding +0
  // changes no bit): the records are added in row order as before
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (uint32_t r = 0; r < m; r += 4) {
    float4 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      a[u] = r + u < m ? col[(size_t)(r + u) * Q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc.x += a[u].x; acc.y += a[u].y; acc.z += a[u].z; acc.w += a[u].w;
    }
  }
  reinterpret_cast<float4*>(ssum)[(size_t)k * Q + q] = acc;
}

// Long slots: one wave each; the grid loops over the list (every wave exits).
template <int C>
__global__ __launch_bounds__(64) void k_slot_sums_long(const uint32_t* __restrict__ long_list,
                                                       const uint32_t* __restrict__ long_count,
                                                       int64_t cap,
                                                       const uint32_t* __restrict__ scnt,
                                                       const uint32_t* __restrict__ soff,
                                                       const float* __restrict__ gpair,
                                                       float* __restrict__ ssum) {
  constexpr int NV = 10 + C;
  constexpr int GSC = ((10 + C) + 3) & ~3;
  const int lane = threadIdx.x;
  const uint32_t nl = *long_count;
  const int my_comp = rs_comp(lane, NV);
  const bool writer = my_comp >= 0 && (lane & rs_dup_bits(NV)) == 0;
  for (uint32_t it = blockIdx.x; it < nl; it += gridDim.x) {
    const uint32_t k = long_list[it];
    const uint32_t n = scnt[k], o = soff[k];
    const uint32_t m = ((int64_t)o + n <= cap) ? n : (((int64_t)o < cap) ? (uint32_t)(cap - o) : 0u);
    constexpr int Q = GSC / 4;
    float acc[GSC];
#pragma unroll
    for (int c = 0; c < GSC; ++c) acc[c] = 0.0f;
    for (uint32_t r = lane; r < m; r += 64) {
      const float4* row = reinterpret_cast<const float4*>(gpair) + (size_t)(o + r) * Q;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const float4 a = row[j];
        acc[4 * j] += a.x; acc[4 * j + 1] += a.y; acc[4 * j + 2] += a.z; acc[4 * j + 3] += a.w;
      }
    }
    const float tot = wave_reduce_scatter<NV>(acc, lane);
    if (writer) ssum[(size_t)k * GSC + my_comp] = tot;
  }
}

// Projection adjoint of surfel i summed over the batch's views: each visible
// (view, surfel) slot's gradient sum is chained through the projection of
// that view and accumulated.  vals[11 + C]: dL/d(z, q, s, alpha, rgb, sem)
// w.r.t. the activated values; alpha is the activated opacity the forward
// used.
template <int C>
__device__ __forceinline__ void surfel_grads(int i, const ViewDev* __restrict__ views, int V,
                                             int N, float eps, float x, float y, float z,
                                             const float q[4], float sx, float sy, float alpha,
                                             const uint32_t* __restrict__ pos, int64_t scap,
                                             const uint32_t* __restrict__ partv,
                                             uint32_t vis_total, int nb, int blk,
                                             const float* __restrict__ ssum,
                                             const float4* __restrict__ rec, float* vals) {
  constexpr int GSC = ((10 + C) + 3) & ~3;
  constexpr int Q = GSC / 4;
  const float ha = -0.5f * alpha;
  float dz = 0.0f, dq[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dsx = 0.0f, dsy = 0.0f, dal = 0.0f;
  float dft[3 + C];
#pragma unroll
  for (int c = 0; c < 3 + C; ++c) dft[c] = 0.0f;
  // the slots' positions (0xffffffff for a culled slot; after a slot-capacity
  // overflow a visible slot may have none either, and the results are flagged
  // invalid) are requested kPre views at a time, ahead of their sums.  Where
  // the projection block blk (kProjBlock surfels) has no visible slot in a
  // view (its scanned visible count, partv, does not grow), the slots have no
  // position and are culled.
  const size_t nparts = (size_t)V * nb;
  auto block_vis = [&](int v) {
    const size_t pb = (size_t)v * nb + blk;
    return (pb + 1 < nparts ? partv[pb + 1] : vis_total) != partv[pb];
  };
  constexpr int kPre = 8;
  uint32_t pv[kPre];
  for (int v = 0; v < V; ++v) {
    const int k = v & (kPre - 1);
    if (k == 0) {
#pragma unroll
      for (int j = 0; j < kPre; ++j)
        pv[j] = (v + j < V && block_vis(v + j)) ? pos[(size_t)(v + j) * N + i] : 0xffffffffu;
    }
    uint32_t p = pv[0];
#pragma unroll
    for (int j = 1; j < kPre; ++j) p = (k == j) ? pv[j] : p;
    if ((int64_t)p >= scap) continue;
    const size_t slot = (size_t)v * N + i;
    const float4* r4 = reinterpret_cast<const float4*>(ssum) + (size_t)p * Q;
    float rg[4 * Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const float4 a = r4[j];
      rg[4 * j] = a.x; rg[4 * j + 1] = a.y; rg[4 * j + 2] = a.z; rg[4 * j + 3] = a.w;
    }
    // this view's contribution first, then one add per component into the
    // running sum, so summing views here or across calls gives the same bits
    // the records hold moments of gda = dL/d(alpha) per pixel over the
    // pixel offsets (dx, dy); dL/dq = -(alpha / 2) gda, so the moments of
    // dL/dq are m = -(alpha / 2) times them, and with the conic the forward
    // used du = -(2A m_x + 2B m_y), dv = -(2C m_y + 2B m_x), dA = m_xx,
    // dB = 2 m_xy, dC = m_yy
    const float4 cn = rec[2 * slot + 1];
    const float mx = ha * rg[0], my = ha * rg[1];
    const float A2 = 2.0f * cn.x, B2 = 2.0f * cn.y, C2 = 2.0f * cn.z;
    const float du = -(A2 * mx + B2 * my);
    const float dv = -(C2 * my + B2 * mx);
    float dzv = 0.0f, dqv[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dsxv = 0.0f, dsyv = 0.0f;
    proj_adjoint(views[v], eps, x, y, z, q, sx, sy, du, dv, ha * rg[2], 2.0f * (ha * rg[3]),
                 ha * rg[4], rg[6], dzv, dqv, dsxv, dsyv);
    dz += dzv;
#pragma unroll
    for (int c = 0; c < 4; ++c) dq[c] += dqv[c];
    dsx += dsxv;
    dsy += dsyv;
    dal += rg[5];
#pragma unroll
    for (int c = 0; c < 3 + C; ++c) dft[c] += rg[7 + c];
  }
  vals[0] = dz;
  vals[1] = dq[0]; vals[2] = dq[1]; vals[3] = dq[2]; vals[4] = dq[3];
  vals[5] = dsx; vals[6] = dsy; vals[7] = dal;
#pragma unroll
  for (int c = 0; c < 3 + C; ++c) vals[8 + c] = dft[c];
}

template <int C>
__global__ __launch_bounds__(kProjBlock) void k_proj_bwd(
    const ViewDev* __restrict__ views, int V, int N, float eps, const float* __restrict__ px,
    const float* __restrict__ py, const float* __restrict__ pz, const float* __restrict__ pq,
    const float* __restrict__ ps, const float* __restrict__ pa,
    const uint32_t* __restrict__ pos, int64_t scap, const uint32_t* __restrict__ partv,
    const uint32_t* __restrict__ misc, const float* __restrict__ ssum,
    const float4* __restrict__ rec, float* __restrict__ grads, int accumulate) {
  const int i = blockIdx.x * kProjBlock + threadIdx.x;
  if (i >= N) return;
  const float q[4] = {pq[i], pq[N + i], pq[2 * (size_t)N + i], pq[3 * (size_t)N + i]};
  float vals[11 + C];
  surfel_grads<C>(i, views, V, N, eps, px[i], py[i], pz[i], q, ps[i], ps[N + i], pa[i], pos,
                  scap, partv, misc[kMiscVisible], (int)gridDim.x, (int)blockIdx.x, ssum, rec,
                  vals);
  const size_t Nn = (size_t)N;
#pragma unroll
  for (int r = 0; r < 11 + C; ++r) {
    float* g = grads + r * Nn + i;
    *g = accumulate ? (*g + vals[r]) : vals[r];
  }
}

// Fused: projection adjoint + Adam of each surfel (the parameters read for
// the adjoint are the ones the forward used; each thread updates only its own
// surfel after reading it).
template <int C>
__global__ __launch_bounds__(kProjBlock) void k_proj_bwd_adam(
    const ViewDev* __restrict__ views, int V, int N, float eps, const float* __restrict__ px,
    const float* __restrict__ py, float* __restrict__ P, float* __restrict__ M,
    float* __restrict__ Vv, float* __restrict__ s_act, float* __restrict__ a_act,
    const uint32_t* __restrict__ pos, int64_t scap, const uint32_t* __restrict__ partv,
    const float* __restrict__ ssum, const float4* __restrict__ rec, const float* __restrict__ dzr,
    float* __restrict__ grads_out, AdamArgs aa) {
  const int i = blockIdx.x * kProjBlock + threadIdx.x;
  if (i >= N) return;
  if (aa.misc[kMiscOverflow]) return;
  const size_t Nn = (size_t)N;
  const float q[4] = {P[Nn + i], P[2 * Nn + i], P[3 * Nn + i], P[4 * Nn + i]};
  float vals[11 + C];
  surfel_grads<C>(i, views, V, N, eps, px[i], py[i], P[i], q, s_act[i], s_act[Nn + i], a_act[i],
                  pos, scap, partv, aa.misc[kMiscVisible], (int)gridDim.x, (int)blockIdx.x, ssum,
                  rec, vals);
  if (dzr) vals[0] += dzr[i];
  if (grads_out) {
#pragma unroll
    for (int r = 0; r < 11 + C; ++r) grads_out[r * Nn + i] = vals[r];
  }
  const int64_t step = aa.state->step + 1;
  float bc1, bc2s;
  adam_bias(aa.b1, aa.b2, step, bc1, bc2s);
  adam_surfel<C>(i, Nn, P, M, Vv, s_act, a_act, vals, aa.lr, z_rate(aa, step), aa.b1, aa.b2,
                 aa.eps, bc1, bc2s);
}

template <int C>
void proj_bwd_launch(const Layout& L, void* ws, const rogs_surfels* s, float* grads, bool acc,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_proj_bwd<C>), dim3(L.nb), dim3(kProjBlock), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.eps2d, s->x, s->y, s->z, s->q,
                     s->s, s->alpha, at<const uint32_t>(ws, L.o_pos),
                     L.scap, at<const uint32_t>(ws, L.o_partv), at<const uint32_t>(ws, L.o_misc),
                     at<const float>(ws, L.o_ssum), at<const float4>(ws, L.o_rec), grads,
                     acc ? 1 : 0);
}

// One thread per pixel; grid.y = view, so a block never straddles views.
// Writes dL/dO (all 5 + C channels; D and A rows 0) and per-block partial
// sums (loss, da, db) that k_loss_final adds in a fixed order.
template <int C>
__global__ __launch_bounds__(kLossBlock) void k_loss_v(
    const ViewDev* __restrict__ views, int V, const int64_t* __restrict__ first_blk,
    const float* __restrict__ out, const float* __restrict__ tgt,
    const uint8_t* __restrict__ label, const uint8_t* __restrict__ mask,
    const float* __restrict__ expo, const uint32_t* __restrict__ mcount, float lam_c, float lam_s,
    float scale, float* __restrict__ G, float* __restrict__ part) {
  constexpr int NO = 5 + C;
  __shared__ float s_w[3][kLossBlock / 64];
  const int v = blockIdx.y;
  const ViewDev& vw = views[v];
  const int64_t npix = (int64_t)vw.w * vw.h;
  const int64_t q = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
  const int64_t nbv = first_blk[v + 1] - first_blk[v];
  if ((int64_t)blockIdx.x >= nbv) return;
  float l = 0.0f, da = 0.0f, db = 0.0f;
  if (q < npix) {
    const size_t HW = (size_t)npix;
    const float* o = out + (size_t)NO * vw.pix_off + q;
    float* g = G + (size_t)NO * vw.pix_off + q;
    const int64_t p = vw.pix_off + q;
    float gv[NO];
#pragma unroll
    for (int c = 0; c < NO; ++c) gv[c] = 0.0f;
    const LossView lv = loss_view(expo, mcount, v, lam_c, lam_s, scale);
    // a pixel outside the mask is evaluated with zero weights: its gradient
    // and loss terms are +-0, as in the fused forward epilogue
    const bool in = mask[p] != 0;
    float ov[3 + C], tv[3];
#pragma unroll
    for (int c = 0; c < 3 + C; ++c) ov[c] = o[c * HW];
    const float* t = tgt + 3 * (size_t)vw.pix_off + q;
#pragma unroll
    for (int c = 0; c < 3; ++c) tv[c] = t[c * HW];
    pixel_loss<C>(ov, tv, label[p], in ? lv.wc : 0.0f, in ? lv.ws : 0.0f, lv.ea, lv.b, gv, l, da,
                  db);
#pragma unroll
    for (int c = 0; c < NO; ++c) g[c * HW] = gv[c];
  }
  l = wave_sum_f(l);
  da = wave_sum_f(da);
  db = wave_sum_f(db);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { s_w[0][wv] = l; s_w[1][wv] = da; s_w[2][wv] = db; }
  __syncthreads();
  if (threadIdx.x < 3) {
    float s = 0.0f;
    for (int w = 0; w < kLossBlock / 64; ++w) s += s_w[threadIdx.x][w];
    part[3 * (size_t)(first_blk[v] + blockIdx.x) + threadIdx.x] = s;
  }
}

template <int C>
void loss_launch(const Layout& L, void* ws, const float* out, const rogs_targets* t, float* G,
                 hipStream_t st) {
  const int64_t maxb = (L.max_view_pix + kLossBlock - 1) / kLossBlock;
  hipLaunchKernelGGL((k_loss_v<C>), dim3((unsigned)maxb, (unsigned)L.V), dim3(kLossBlock), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, at<const int64_t>(ws, L.o_lpart), out,
                     t->rgb, t->label, t->mask, t->exposure, at<const uint32_t>(ws, L.o_mcount),
                     t->lambda_c, t->lambda_s, t->view_scale, G,
                     at<float>(ws, L.o_lpart) + 2 * (L.V + 1));
}

// ------------------------------------------------------------ Adam

template <int C>
__global__ __launch_bounds__(256) void k_adam(int N, float* __restrict__ P,
                                              const float* __restrict__ Gd, float* __restrict__ M,
                                              float* __restrict__ Vv, float* __restrict__ s_act,
                                              float* __restrict__ a_act, AdamArgs aa) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const size_t Nn = (size_t)N;
  float g[11 + C];
#pragma unroll
  for (int r = 0; r < 11 + C; ++r) g[r] = Gd[r * Nn + i];
  float bc1, bc2s;
  adam_bias(aa.b1, aa.b2, aa.step, bc1, bc2s);
  adam_surfel<C>(i, Nn, P, M, Vv, s_act, a_act, g, aa.lr, z_rate(aa, aa.step), aa.b1, aa.b2,
                 aa.eps, bc1, bc2s);
}

// Adam on a plain array (the per-view exposure (a, b)).  With a step state
// the step comes from the device and an overflow skips the update.
__device__ __forceinline__ void adam_plain_elem(int i, float g, float* __restrict__ P,
                                                float* __restrict__ M, float* __restrict__ Vv,
                                                const AdamArgs& aa) {
  if (aa.misc && aa.misc[kMiscOverflow]) return;
  const int64_t step = aa.state ? aa.state->step + 1 : aa.step;
  float bc1, bc2s;
  adam_bias(aa.b1, aa.b2, step, bc1, bc2s);
  const float m = aa.b1 * M[i] + (1.0f - aa.b1) * g;
  const float v = aa.b2 * Vv[i] + (1.0f - aa.b2) * g * g;
  M[i] = m;
  Vv[i] = v;
  P[i] -= (aa.lr.exposure / bc1) * (m / (sqrtf(v) / bc2s + aa.eps));
}

__global__ void k_adam_plain(int n, float* __restrict__ P, const float* __restrict__ Gd,
                             float* __restrict__ M, float* __restrict__ Vv, AdamArgs aa) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  adam_plain_elem(i, Gd[i], P, M, Vv, aa);
}

// Per-view sums of the fused step's per-tile partials (loss, dL/da, dL/db)
// in two fixed-order stages: block (c, v) adds tiles c * kTileChunk ... of
// view v (8 per thread, then a fixed tree), and one wave per view adds the
// chunks in order (lane-strided, then a fixed tree), overwrites dL/d(a, b)
// and applies Adam to the view's exposure (a, b).  The result does not
// depend on scheduling.
constexpr int kTileChunk = 8 * 256;

__global__ __launch_bounds__(256) void k_loss_tiles(const ViewDev* __restrict__ views, int V,
                                                    int64_t total_tiles,
                                                    const float* __restrict__ part, int nchunk,
                                                    float* __restrict__ cpart) {
  __shared__ float s[3][256];
  const int v = blockIdx.y, c = blockIdx.x;
  const int64_t t0 = views[v].tile_off;
  const int64_t t1 = (v + 1 < V) ? views[v + 1].tile_off : total_tiles;
  const int64_t k0 = t0 + (int64_t)c * kTileChunk;
  float l = 0.0f, a = 0.0f, b = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t k = k0 + threadIdx.x + 256 * i;
    if (k < t1) {
      l += part[3 * k];
      a += part[3 * k + 1];
      b += part[3 * k + 2];
    }
  }
  s[0][threadIdx.x] = l;
  s[1][threadIdx.x] = a;
  s[2][threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
      s[2][threadIdx.x] += s[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) cpart[((size_t)v * nchunk + c) * 3 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_loss_chunks(const float* __restrict__ cpart, int nchunk,
                                                    float* __restrict__ per_view,
                                                    float* __restrict__ d_exp,
                                                    float* __restrict__ expo,
                                                    float* __restrict__ m_exp,
                                                    float* __restrict__ v_exp, AdamArgs aa) {
  const int v = blockIdx.x, lane = threadIdx.x;
  float l = 0.0f, a = 0.0f, b = 0.0f;
  for (int c = lane; c < nchunk; c += 64) {
    const float* q = cpart + ((size_t)v * nchunk + c) * 3;
    l += q[0];
    a += q[1];
    b += q[2];
  }
  l = wave_sum_f(l);
  a = wave_sum_f(a);
  b = wave_sum_f(b);
  if (lane == 0) {
    per_view[v] = l;
    if (d_exp) {
      d_exp[2 * v] = a;
      d_exp[2 * v + 1] = b;
    }
  }
  if (expo && lane < 2) adam_plain_elem(2 * v + lane, lane == 0 ? a : b, expo, m_exp, v_exp, aa);
}

// Closes a fused step: counts it (or its skip on overflow) and keeps its loss;
// then copies misc[0..3] and the step state side by side into status (for
// one read-back).
__global__ void k_step_end(StepState* __restrict__ st, const uint32_t* __restrict__ misc,
                           const float* __restrict__ per_view, int V,
                           const float* __restrict__ reg_total, AdamArgs aa,
                           uint32_t* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (misc[kMiscOverflow]) {
    st->skipped += 1;
  } else {
    float t = 0.0f;
    for (int v = 0; v < V; ++v) t += per_view[v];
    if (reg_total) t += *reg_total;
    const int64_t step = st->step + 1;
    st->lr_z = z_rate(aa, step);
    st->loss = t;
    st->step = step;
  }
  if (status) {
    for (int k = 0; k < 4; ++k) status[k] = misc[k];
    *reinterpret_cast<StepState*>(status + 4) = *st;
  }
}

}  // namespace

void launch_loss(const Layout& L, void* ws, const float* out, const rogs_targets* t, float* G,
                 float* loss_out, float* d_exp, hipStream_t st) {
  launch_mask_count(L, ws, t->mask, st);
  switch (L.C) {
    case 1: loss_launch<1>(L, ws, out, t, G, st); break;
    case 2: loss_launch<2>(L, ws, out, t, G, st); break;
    case 3: loss_launch<3>(L, ws, out, t, G, st); break;
    case 4: loss_launch<4>(L, ws, out, t, G, st); break;
    case 5: loss_launch<5>(L, ws, out, t, G, st); break;
    case 6: loss_launch<6>(L, ws, out, t, G, st); break;
    case 7: loss_launch<7>(L, ws, out, t, G, st); break;
    case 8: loss_launch<8>(L, ws, out, t, G, st); break;
    case 16: loss_launch<16>(L, ws, out, t, G, st); break;
    default: return;
  }
  float* per_view = reinterpret_cast<float*>(at<uint32_t>(ws, L.o_mcount) + L.V);
  hipLaunchKernelGGL(k_loss_views, dim3((unsigned)L.V), dim3(256), 0, st,
                     at<const int64_t>(ws, L.o_lpart), at<const float>(ws, L.o_lpart) + 2 * (L.V + 1),
                     per_view, d_exp);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, st, L.V, per_view, loss_out);
}

void launch_proj_bwd(const Layout& L, void* ws, const rogs_surfels* s, float* grads,
                     bool accumulate, hipStream_t st) {
  switch (L.C) {
    case 1: proj_bwd_launch<1>(L, ws, s, grads, accumulate, st); break;
    case 2: proj_bwd_launch<2>(L, ws, s, grads, accumulate, st); break;
    case 3: proj_bwd_launch<3>(L, ws, s, grads, accumulate, st); break;
    case 4: proj_bwd_launch<4>(L, ws, s, grads, accumulate, st); break;
    case 5: proj_bwd_launch<5>(L, ws, s, grads, accumulate, st); break;
    case 6: proj_bwd_launch<6>(L, ws, s, grads, accumulate, st); break;
    case 7: proj_bwd_launch<7>(L, ws, s, grads, accumulate, st); break;
    case 8: proj_bwd_launch<8>(L, ws, s, grads, accumulate, st); break;
    case 16: proj_bwd_launch<16>(L, ws, s, grads, accumulate, st); break;
    default: break;
  }
}

namespace {
template <int C>
void adam_launch(int n, float* params, const float* grads, float* m, float* v, float* s_act,
                 float* a_act, const AdamArgs& aa, hipStream_t st) {
  hipLaunchKernelGGL((k_adam<C>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, params,
                     grads, m, v, s_act, a_act, aa);
}

template <int C>
void proj_bwd_adam_launch(const Layout& L, void* ws, const float* x, const float* y,
                          float* params, float* m, float* v, float* s_act, float* a_act,
                          float* grads_out, const AdamArgs& aa, const float* dzr, hipStream_t st) {
  hipLaunchKernelGGL((k_proj_bwd_adam<C>), dim3(L.nb), dim3(kProjBlock), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.eps2d, x, y, params, m, v,
                     s_act, a_act, at<const uint32_t>(ws, L.o_pos),
                     L.scap, at<const uint32_t>(ws, L.o_partv), at<const float>(ws, L.o_ssum),
                     at<const float4>(ws, L.o_rec), dzr, grads_out, aa);
}
}  // namespace

#define ROGS_SEM_SWITCH(C_, CALL)      \
  switch (C_) {                        \
    case 1: { constexpr int KC = 1; CALL; } break;   \
    case 2: { constexpr int KC = 2; CALL; } break;   \
    case 3: { constexpr int KC = 3; CALL; } break;   \
    case 4: { constexpr int KC = 4; CALL; } break;   \
    case 5: { constexpr int KC = 5; CALL; } break;   \
    case 6: { constexpr int KC = 6; CALL; } break;   \
    case 7: { constexpr int KC = 7; CALL; } break;   \
    case 8: { constexpr int KC = 8; CALL; } break;   \
    case 16: { constexpr int KC = 16; CALL; } break; \
    default: break;                    \
  }

void launch_adam(int n, int C, float* params, const float* grads, float* m, float* v,
                 float* s_act, float* a_act, const rogs_optim& o, int64_t step, float* expo,
                 const float* dexpo, float* me, float* ve, int nv, hipStream_t st) {
  AdamArgs aa{};
  aa.lr = o.lr;
  aa.b1 = o.beta1;
  aa.b2 = o.beta2;
  aa.eps = o.eps;
  aa.z_start = o.z_start;
  aa.z_end = o.z_end;
  aa.total_steps = o.total_steps;
  aa.step = step;
  aa.state = nullptr;
  aa.misc = nullptr;
  ROGS_SEM_SWITCH(C, (adam_launch<KC>(n, params, grads, m, v, s_act, a_act, aa, st)));
  if (expo && nv > 0)
    hipLaunchKernelGGL(k_adam_plain, dim3((unsigned)((2 * nv + 63) / 64)), dim3(64), 0, st, 2 * nv,
                       expo, dexpo, me, ve, aa);
}

void launch_proj_bwd_adam(const Layout& L, void* ws, const float* x, const float* y, float* params,
                          float* m, float* v, float* s_act, float* a_act, float* grads_out,
                          const AdamArgs& aa, float* expo, const float* dexpo, float* me,
                          float* ve, const float* dzr, hipStream_t st) {
  ROGS_SEM_SWITCH(L.C, (proj_bwd_adam_launch<KC>(L, ws, x, y, params, m, v, s_act, a_act,
                                                  grads_out, aa, dzr, st)));
  if (expo)
    hipLaunchKernelGGL(k_adam_plain, dim3((unsigned)((2 * L.V + 63) / 64)), dim3(64), 0, st,
                       2 * L.V, expo, dexpo, me, ve, aa);
}

namespace {
template <int C>
void slot_sums_launch(const Layout& L, void* ws, hipStream_t st, bool clear) {
  uint32_t* misc = at<uint32_t>(ws, L.o_misc);
  const int64_t s_grid = L.scap;
  if (s_grid <= 0) return;
  if (clear) fill_u32(misc + kMiscLong, 0u, 1, st);
  constexpr int Q = (((10 + C) + 3) & ~3) / 4;
  hipLaunchKernelGGL((k_slot_sums<C>), dim3((unsigned)((s_grid * Q + 255) / 256)), dim3(256), 0, st,
                     misc, L.scap, L.cap, at<const uint32_t>(ws, L.o_scnt),
                     at<const uint32_t>(ws, L.o_soff), at<const float>(ws, L.o_gpair),
                     at<float>(ws, L.o_ssum), at<uint32_t>(ws, L.o_long), misc + kMiscLong);
  hipLaunchKernelGGL((k_slot_sums_long<C>), dim3(16384), dim3(64), 0, st,
                     at<const uint32_t>(ws, L.o_long), misc + kMiscLong, L.cap,
                     at<const uint32_t>(ws, L.o_scnt), at<const uint32_t>(ws, L.o_soff),
                     at<const float>(ws, L.o_gpair), at<float>(ws, L.o_ssum));
}
}  // namespace

void launch_slot_sums(const Layout& L, void* ws, hipStream_t st, bool clear) {
  ROGS_SEM_SWITCH(L.C, (slot_sums_launch<KC>(L, ws, st, clear)));
}

void launch_loss_tiles(const Layout& L, void* ws, float* d_exp, float* expo, float* m_exp,
                       float* v_exp, const AdamArgs& aa, hipStream_t st) {
  float* per_view = reinterpret_cast<float*>(at<uint32_t>(ws, L.o_mcount) + L.V);
  // the plain loss's block partials are unused on the fused path: chunk sums go there
  float* cpart = at<float>(ws, L.o_lpart) + 2 * (L.V + 1);
  const int nchunk = (int)((L.max_view_tiles + kTileChunk - 1) / kTileChunk);
  hipLaunchKernelGGL(k_loss_tiles, dim3((unsigned)nchunk, (unsigned)L.V), dim3(256), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.total_tiles,
                     at<const float>(ws, L.o_tpart), nchunk, cpart);
  hipLaunchKernelGGL(k_loss_chunks, dim3((unsigned)L.V), dim3(64), 0, st, cpart, nchunk, per_view,
                     d_exp, expo, m_exp, v_exp, aa);
}

void launch_mask_count(const Layout& L, void* ws, const uint8_t* mask, hipStream_t st) {
  uint32_t* mcount = at<uint32_t>(ws, L.o_mcount);
  fill_u32(mcount, 0u, L.V, st);
  hipLaunchKernelGGL(k_mask_count,
                     dim3((unsigned)((L.max_view_pix + kMaskPerBlock - 1) / kMaskPerBlock),
                          (unsigned)L.V),
                     dim3(kLossBlock), 0, st, at<const ViewDev>(ws, L.o_views), mask, mcount);
}

void launch_step_end(const Layout& L, void* ws, StepState* state, const AdamArgs& aa,
                     const float* reg_total, hipStream_t st) {
  const float* per_view = reinterpret_cast<const float*>(at<uint32_t>(ws, L.o_mcount) + L.V);
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, state, at<const uint32_t>(ws, L.o_misc),
                     per_view, L.V, reg_total, aa, L.o_status ? at<uint32_t>(ws, L.o_status) : nullptr);
}

}  // namespace rogs
