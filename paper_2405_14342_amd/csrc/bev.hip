// Chunked orthographic BEV export (Sec. 4.2 "rendered in chunks and then
// stitched"; supp. Sec. 2.2): the map's top-down image is covered by square
// orthographic cameras of chunk_px x chunk_px pixels; each is rendered with
// the same project / bin / composite calls as training and copied into its
// place in the stitched image, together with the elevation (camera height
// minus the opacity-weighted depth).
#include <algorithm>
#include <string>

#include "rogs_internal.h"

namespace {

// Copies the requested planes of one rendered chunk (5 + C planes) into the
// stitched image (planes of W x H) at column ox, row oy.
__global__ __launch_bounds__(256) void k_stitch(const float* __restrict__ img, int cw, int ch,
                                                int C, uint32_t chans, float elev_ref,
                                                float* __restrict__ out, int W, int H, int ox,
                                                int oy) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t np = (int64_t)cw * ch;
  if (p >= np) return;
  const int u = (int)(p % cw), v = (int)(p / cw);
  const int64_t g = (int64_t)(oy + v) * W + (ox + u);
  const int64_t GP = (int64_t)W * H;
  int o = 0;
  if (chans & ROGS_CH_RGB)
    for (int c = 0; c < 3; ++c) out[(o++) * GP + g] = img[c * np + p];
  if (chans & ROGS_CH_SEM)
    for (int c = 0; c < C; ++c) out[(o++) * GP + g] = img[(3 + c) * np + p];
  const float D = img[(3 + C) * np + p], A = img[(4 + C) * np + p];
  if (chans & ROGS_CH_D) out[(o++) * GP + g] = D;
  if (chans & ROGS_CH_A) out[(o++) * GP + g] = A;
  if (chans & ROGS_CH_ELEV)
    out[(o++) * GP + g] = (A > 0.0f) ? elev_ref - D / A : __int_as_float(0x7fc00000);
}

}  // namespace

extern "C" {

void rogs_bev_camera(double x0, double y0, int32_t W, int32_t H, float m_per_px, int32_t ox,
                     int32_t oy, int32_t cw, int32_t ch, float height, rogs_camera* cam) {
  if (!cam) return;
  rogs_camera c{};
  c.w = cw;
  c.h = ch;
  c.model = ROGS_ORTHO;
  c.fx = c.fy = 1.0f / m_per_px;
  c.cx = 0.5f * (float)cw;
  c.cy = 0.5f * (float)ch;
  // chunk centre in the world: the image's top edge is y0 + H * m_per_px
  const double cxw = x0 + ((double)ox + 0.5 * cw) * (double)m_per_px;
  const double cyw = y0 + ((double)H - (double)oy - 0.5 * ch) * (double)m_per_px;
  const float R[9] = {1.0f, 0.0f, 0.0f, 0.0f, -1.0f, 0.0f, 0.0f, 0.0f, -1.0f};
  for (int k = 0; k < 9; ++k) c.R_cw[k] = R[k];
  c.t_cw[0] = (float)(-cxw);
  c.t_cw[1] = (float)(cyw);
  c.t_cw[2] = height;
  c.z_near = 0.1f;
  c.cull_lat = 0.0f;                 // no ground rectangle: the chunk is the range
  (void)W;
  *cam = c;
}

int rogs_bev_workspace_size(const rogs_surfels* s, int32_t chunk_px, const rogs_render_opts* opts,
                            int64_t pair_capacity, size_t* bytes) {
  if (!s || !opts || !bytes || chunk_px < 1 || chunk_px > 16384) return ROGS_EINVAL;
  rogs_camera cam;
  rogs_bev_camera(0.0, 0.0, chunk_px, chunk_px, 0.05f, 0, 0, chunk_px, chunk_px, 100.0f, &cam);
  size_t ws = 0;
  int r = rogs_workspace_size(s, &cam, 1, opts, pair_capacity, 0, &ws);
  if (r != ROGS_OK) return r;
  *bytes = ws + (size_t)(5 + s->n_sem) * chunk_px * chunk_px * 4 + 256;
  return ROGS_OK;
}

int rogs_bev_export(rogs_ctx* c, const rogs_surfels* s, const rogs_render_opts* opts, double x0,
                    double y0, int32_t W, int32_t H, float m_per_px, int32_t chunk_px,
                    float height, uint32_t channels, float* out, void* ws, size_t ws_bytes,
                    int64_t pair_capacity, int64_t* n_pairs_max, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (!s || !opts || !out || !ws || W < 1 || H < 1 || (int64_t)W * H >= (int64_t(1) << 40) ||
      !(m_per_px > 0.0f) || chunk_px < 1 || channels == 0 || (channels & ~ROGS_CH_ALL) != 0)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_bev_export: invalid argument");
  size_t need = 0;
  int r = rogs_bev_workspace_size(s, chunk_px, opts, pair_capacity, &need);
  if (r != ROGS_OK) return rogs::ctx_fail(c, r, "rogs_bev_export: invalid surfels or options");
  if (ws_bytes < need) return rogs::ctx_fail(c, ROGS_ENOMEM, "rogs_bev_export: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t worst = 0;
  for (int oy = 0; oy < H; oy += chunk_px) {
    for (int ox = 0; ox < W; ox += chunk_px) {
      const int cw = std::min(chunk_px, W - ox), ch = std::min(chunk_px, H - oy);
      rogs_camera cam;
      rogs_bev_camera(x0, y0, W, H, m_per_px, ox, oy, cw, ch, height, &cam);
      size_t wsb = 0;
      r = rogs_workspace_size(s, &cam, 1, opts, pair_capacity, 0, &wsb);
      if (r != ROGS_OK) return rogs::ctx_fail(c, r, "rogs_bev_export: chunk layout");
      float* img = reinterpret_cast<float*>(static_cast<uint8_t*>(ws) + (wsb + 255) / 256 * 256);
      r = rogs_project(c, s, &cam, 1, opts, ws, wsb, pair_capacity, 0, stream);
      int64_t n = 0;
      if (r == ROGS_OK) r = rogs_bin_sort(c, ws, &n, ROGS_SYNC_COUNT, stream);
      worst = std::max(worst, n);
      if (n_pairs_max) *n_pairs_max = worst;
      if (r != ROGS_OK) return r;
      // only the planes the export asks for are composited
      r = rogs_render_fwd(c, s, ws, img, channels, stream);
      if (r != ROGS_OK) return r;
      const int64_t np = (int64_t)cw * ch;
      hipLaunchKernelGGL(k_stitch, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, img, cw,
                         ch, s->n_sem, channels, height, out, W, H, ox, oy);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess)
        return rogs::ctx_fail(c, ROGS_EHIP, std::string("rogs_bev_export: ") + hipGetErrorString(e));
    }
  }
  return ROGS_OK;
}

}  // extern "C"
