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
// kMaskPerBlock pixels and adds its count with one integer atomic (exact).
constexpr int kMaskPerBlock = 16 * kLossBlock;

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
  for (int k = threadIdx.x; k < kMaskPerBlock; k += kLossBlock) {
    const int64_t p = base + k;
    if (p < npix) c += m[p] ? 1u : 0u;
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

template <int C>
__global__ __launch_bounds__(kProjBlock) void k_proj_bwd(
    const ViewDev* __restrict__ views, int V, int N, float eps, const float* __restrict__ px,
    const float* __restrict__ py, const float* __restrict__ pz, const float* __restrict__ pq,
    const float* __restrict__ ps, const uint32_t* __restrict__ cnt,
    const uint32_t* __restrict__ off, const float* __restrict__ gpair, int GS, int64_t cap,
    float* __restrict__ grads, int accumulate) {
  constexpr int NV = 10 + C;
  const int i = blockIdx.x * kProjBlock + threadIdx.x;
  if (i >= N) return;
  const float x = px[i], y = py[i], z = pz[i];
  const float q[4] = {pq[i], pq[N + i], pq[2 * (size_t)N + i], pq[3 * (size_t)N + i]};
  const float sx = ps[i], sy = ps[N + i];
  float dz = 0.0f, dq[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dsx = 0.0f, dsy = 0.0f, dal = 0.0f;
  float dft[3 + C];
#pragma unroll
  for (int c = 0; c < 3 + C; ++c) dft[c] = 0.0f;
  for (int v = 0; v < V; ++v) {
    const size_t slot = (size_t)v * N + i;
    const uint32_t n = cnt[slot];
    if (!n) continue;
    const uint32_t o = off[slot];
    // after a pair-capacity overflow the records past the capacity were never written
    const uint32_t m = ((int64_t)o + n <= cap) ? n : (((int64_t)o < cap) ? (uint32_t)(cap - o) : 0u);
    float rg[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) rg[c] = 0.0f;
    for (uint32_t k = 0; k < m; ++k) {
      const float* r = gpair + (size_t)(o + k) * GS;
#pragma unroll
      for (int c = 0; c < NV; ++c) rg[c] += r[c];
    }
    // this view's contribution first, then one add per component into the
    // running sum, so summing views here or across calls gives the same bits
    float dzv = 0.0f, dqv[4] = {0.0f, 0.0f, 0.0f, 0.0f}, dsxv = 0.0f, dsyv = 0.0f;
    proj_adjoint(views[v], eps, x, y, z, q, sx, sy, rg[0], rg[1], rg[2], rg[3], rg[4], rg[6], dzv,
                 dqv, dsxv, dsyv);
    dz += dzv;
#pragma unroll
    for (int c = 0; c < 4; ++c) dq[c] += dqv[c];
    dsx += dsxv;
    dsy += dsyv;
    dal += rg[5];
#pragma unroll
    for (int c = 0; c < 3 + C; ++c) dft[c] += rg[7 + c];
  }
  const size_t Nn = (size_t)N;
  float vals[11 + C];
  vals[0] = dz;
  vals[1] = dq[0]; vals[2] = dq[1]; vals[3] = dq[2]; vals[4] = dq[3];
  vals[5] = dsx; vals[6] = dsy; vals[7] = dal;
#pragma unroll
  for (int c = 0; c < 3 + C; ++c) vals[8 + c] = dft[c];
#pragma unroll
  for (int r = 0; r < 11 + C; ++r) {
    float* g = grads + r * Nn + i;
    *g = accumulate ? (*g + vals[r]) : vals[r];
  }
}

template <int C>
void proj_bwd_launch(const Layout& L, void* ws, const rogs_surfels* s, float* grads, bool acc,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_proj_bwd<C>), dim3(L.nb), dim3(kProjBlock), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.eps2d, s->x, s->y, s->z, s->q,
                     s->s, at<const uint32_t>(ws, L.o_cnt), at<const uint32_t>(ws, L.o_off),
                     at<const float>(ws, L.o_gpair), L.GS, L.cap, grads, acc ? 1 : 0);
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
    const uint32_t mc = mcount[v];
    float gv[NO];
#pragma unroll
    for (int c = 0; c < NO; ++c) gv[c] = 0.0f;
    if (mask[p] && mc > 0) {
      const float wc = lam_c * scale / (float)mc;
      const float ws = lam_s * scale / (float)mc;
      const float a = expo[2 * v], b = expo[2 * v + 1];
      const float ea = expf(a);
      const float* t = tgt + 3 * (size_t)vw.pix_off + q;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float cc = o[c * HW];
        const float r = (ea * cc + b) - t[c * HW];
        const float sg = (r > 0.0f) ? 1.0f : ((r < 0.0f) ? -1.0f : 0.0f);
        l += wc * fabsf(r);
        gv[c] = wc * sg * ea;
        da += wc * sg * ea * cc;
        db += wc * sg;
      }
      float sv[C], ov[C];
      float mx = -INFINITY;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        ov[c] = o[(3 + c) * HW];
        mx = fmaxf(mx, ov[c]);
      }
      float se = 0.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        sv[c] = expf(ov[c] - mx);
        se += sv[c];
      }
      const int lb = label[p];
      float olb = 0.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) olb = (c == lb) ? ov[c] : olb;
      l += ws * ((mx + logf(se)) - olb);
      const float inv = 1.0f / se;
#pragma unroll
      for (int c = 0; c < C; ++c) gv[3 + c] = ws * (sv[c] * inv - ((c == lb) ? 1.0f : 0.0f));
    }
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

__global__ __launch_bounds__(256) void k_adam(int N, int K, float* __restrict__ P,
                                              const float* __restrict__ Gd, float* __restrict__ M,
                                              float* __restrict__ Vv, float* __restrict__ s_act,
                                              float* __restrict__ a_act, rogs_lr lr, float b1,
                                              float b2, float eps, float bc1, float bc2s) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const size_t Nn = (size_t)N;
  const float sx = s_act[i], sy = s_act[Nn + i], al = a_act[i];
  for (int r = 0; r < K; ++r) {
    const size_t j = r * Nn + i;
    float g = Gd[j];
    float lrr;
    if (r == 0) lrr = lr.z;
    else if (r <= 4) lrr = lr.q;
    else if (r <= 6) { lrr = lr.s; g *= (r == 5) ? sx : sy; }        // d/d log s = s d/ds
    else if (r == 7) { lrr = lr.alpha; g *= al * (1.0f - al); }     // d/d logit = a(1-a) d/da
    else if (r <= 10) lrr = lr.rgb;
    else lrr = lr.sem;
    const float m = b1 * M[j] + (1.0f - b1) * g;
    const float v = b2 * Vv[j] + (1.0f - b2) * g * g;
    M[j] = m;
    Vv[j] = v;
    const float denom = sqrtf(v) / bc2s + eps;
    P[j] -= (lrr / bc1) * (m / denom);
  }
  s_act[i] = expf(P[5 * Nn + i]);
  s_act[Nn + i] = expf(P[6 * Nn + i]);
  a_act[i] = 1.0f / (1.0f + expf(-P[7 * Nn + i]));
}

__global__ void k_adam_plain(int n, float* __restrict__ P, const float* __restrict__ Gd,
                             float* __restrict__ M, float* __restrict__ Vv, float lr, float b1,
                             float b2, float eps, float bc1, float bc2s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = Gd[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * Vv[i] + (1.0f - b2) * g * g;
  M[i] = m;
  Vv[i] = v;
  P[i] -= (lr / bc1) * (m / (sqrtf(v) / bc2s + eps));
}

}  // namespace

void launch_loss(const Layout& L, void* ws, const float* out, const rogs_targets* t, float* G,
                 float* loss_out, float* d_exp, hipStream_t st) {
  uint32_t* mcount = at<uint32_t>(ws, L.o_mcount);
  fill_u32(mcount, 0u, L.V, st);
  hipLaunchKernelGGL(k_mask_count,
                     dim3((unsigned)((L.max_view_pix + kMaskPerBlock - 1) / kMaskPerBlock),
                          (unsigned)L.V),
                     dim3(kLossBlock), 0, st, at<const ViewDev>(ws, L.o_views), t->mask, mcount);
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

void launch_adam(int n, int C, float* params, const float* grads, float* m, float* v,
                 float* s_act, float* a_act, const rogs_lr* lr, int64_t step, float b1, float b2,
                 float eps, float* expo, const float* dexpo, float* me, float* ve, int nv,
                 hipStream_t st) {
  const double bc1 = 1.0 - pow((double)b1, (double)step);
  const double bc2 = 1.0 - pow((double)b2, (double)step);
  const float bc2s = (float)sqrt(bc2);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, 11 + C,
                     params, grads, m, v, s_act, a_act, *lr, b1, b2, eps, (float)bc1, bc2s);
  if (expo && nv > 0)
    hipLaunchKernelGGL(k_adam_plain, dim3((unsigned)((2 * nv + 63) / 64)), dim3(64), 0, st, 2 * nv,
                       expo, dexpo, me, ve, lr->exposure, b1, b2, eps, (float)bc1, bc2s);
}

}  // namespace rogs
