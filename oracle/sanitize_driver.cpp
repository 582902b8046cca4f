// Host sanitizer run of the test oracle (TEST INFRASTRUCTURE ONLY).
//
// Built by tests/test_oracle_sanitize.py together with rogs_oracle.cpp and
// rogs_oracle_grid.cpp under AddressSanitizer and UndefinedBehaviorSanitizer
// (g++, host code only) and run as its own executable: it calls every entry
// point of the oracle on a small deterministic scene (a 12 x 12 grid of
// surfels under a pinhole camera and a top-down orthographic one, four
// semantic classes) and on the empty cases (no surfel in view, an empty loss
// mask), so that any out-of-bounds access, use of freed memory or undefined
// arithmetic in the oracle stops the run.  It also checks two facts of
// Eq. 6 that hold whatever the inputs: A = 1 - T_final and 0 <= A < 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void orc_q32(int n, const float* rec7, int npix, const int32_t* px, const int32_t* py, float* q);
void orc_row_spans(const float* rec7, int x0, int x1, int y0, int y1, float qcut, int tw, int th,
                   int W, int H, int32_t* lo, int32_t* hi);
int orc_contract(int n, int C, const float* f32, const double* f64, const float* cam,
                 const int* iopts, const float* fopts, float* rec, int32_t* rect, uint8_t* vis);
void orc_geo64(int n, int C, const float* f32, const double* f64, const float* cam,
               const int* iopts, const float* fopts, double* out);
void orc_geo64_adjoint(int n, int C, const float* f32, const double* f64, const float* cam,
                       const int* iopts, const float* fopts, int i, const double* dgeo,
                       double* dout);
int64_t orc_tile_lists(int n, int C, const float* f32, const double* f64, const float* cam,
                       const int* iopts, const float* fopts, int64_t cap, uint64_t* keys,
                       int32_t* ids, int32_t* ranges);
void orc_render_fwd(int n, int C, const float* f32, const double* f64, const float* cam,
                    const int* iopts, const float* fopts, const int32_t* pix, int64_t npix,
                    double* out, double* tfinal, int32_t* nlast);
void orc_render_bwd(int n, int C, const float* f32, const double* f64, const float* cam,
                    const int* iopts, const float* fopts, const int32_t* pix, int64_t npix,
                    const double* G, const double* tfinal, const int32_t* nlast, double* grads);
double orc_loss(int C, int64_t npix, const double* O, const float* tgt, const uint8_t* label,
                const uint8_t* mask, int64_t mcount, double exp_a, double exp_b, double lam_c,
                double lam_s, double scale, double* G, double* d_exp);
void orc_adam_raw(int n, int C, double* p, const double* g_act, double* m, double* v,
                  const double* lr, double z_start, double z_end, int64_t total_steps,
                  int64_t step, double b1, double b2, double eps, double* s_act, double* a_act,
                  int n_views, double* expo, const double* d_expo, double* m_e, double* v_e);
double orc_smooth(int64_t n, const double* z, const int32_t* nbr, double lambda, double* dz);
double orc_lidar_loss(int64_t n, const double* z, const double* zbar, double lambda, double* dz);
void orc_lidar_nn(int64_t n, const float* x, const float* y, int64_t m, const float* px,
                  const float* py, int32_t* idx);
void orc_pose_pixels(int n_poses, const float* pose, double x0, double y0, float h, int32_t* pix);
int64_t orc_layout_mask(int W, int H, int n_poses, const int32_t* pix, int r, uint8_t* mask);
void orc_layout_build(int W, int H, const uint8_t* mask, double x0, double y0, float h,
                      int n_poses, const float* pose, int64_t n, int32_t* idx, float* x, float* y,
                      float* z, double* q, int32_t* nbr);
}

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "check failed: %s\n", what);
    ++failures;
  }
}

// Camera record of the oracle: w h model fx fy cx cy R[9] t[3] znear o[2]
// ex[2] ez[2] lat fwd.  Pinhole 1.5 m above (0, 0), looking along +x and
// 20 degrees down; orthographic 10 m above (0.6, 0), looking straight down.
std::vector<float> camera(bool ortho) {
  std::vector<float> c(28, 0.0f);
  if (!ortho) {
    const double p = 20.0 * M_PI / 180.0;
    const double fwd[3] = {std::cos(p), 0.0, -std::sin(p)};
    const double right[3] = {0.0, -1.0, 0.0};
    const double down[3] = {right[1] * fwd[2] - right[2] * fwd[1],
                            right[2] * fwd[0] - right[0] * fwd[2],
                            right[0] * fwd[1] - right[1] * fwd[0]};
    const double pos[3] = {0.0, 0.0, 1.5};
    const double* rows[3] = {right, down, fwd};
    c[0] = 48; c[1] = 40; c[2] = 0;
    c[3] = c[4] = 40.0f; c[5] = 24.0f; c[6] = 20.0f;
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) c[7 + 3 * r + k] = (float)rows[r][k];
      c[16 + r] = (float)-(rows[r][0] * pos[0] + rows[r][1] * pos[1] + rows[r][2] * pos[2]);
    }
    c[19] = 0.1f;
    c[22] = 0.0f; c[23] = -1.0f;         // ground direction of camera x
    c[24] = 1.0f; c[25] = 0.0f;          // ground direction of camera z
    c[26] = 20.0f; c[27] = 40.0f;
  } else {
    const float R[9] = {1, 0, 0, 0, -1, 0, 0, 0, -1};
    c[0] = 32; c[1] = 32; c[2] = 1;
    c[3] = c[4] = 20.0f; c[5] = c[6] = 16.0f;
    for (int k = 0; k < 9; ++k) c[7 + k] = R[k];
    c[16] = -0.6f; c[17] = 0.0f; c[18] = 10.0f;
    c[19] = 0.1f;
  }
  return c;
}

}  // namespace

int main() {
  const int gx = 12, n = gx * gx, C = 4, K = 11 + C;
  std::vector<float> f32(9 * (size_t)n);
  std::vector<double> f64((13 + C) * (size_t)n);
  for (int j = 0; j < gx; ++j) {
    for (int i = 0; i < gx; ++i) {
      const int k = j * gx + i;
      const double x = 0.8 + 0.1 * i, y = 0.1 * (j - 5.5);
      const double z = 0.02 * std::sin(3.0 * x) * std::cos(2.0 * y);
      const double q[4] = {1.0, 0.02 * std::sin(7.0 * k), 0.03 * std::cos(5.0 * k), 0.0};
      const double s[2] = {0.05 + 0.01 * ((k * 7) % 5), 0.04 + 0.01 * ((k * 3) % 4)};
      const double xs[9] = {x, y, z, q[0], q[1], q[2], q[3], s[0], s[1]};
      for (int r = 0; r < 9; ++r) f32[(size_t)r * n + k] = (float)xs[r];
      for (int r = 0; r < 9; ++r) f64[(size_t)r * n + k] = (double)(float)xs[r];
      f64[9 * (size_t)n + k] = 0.3 + 0.69 * ((k * 13) % 10) / 9.0;          // alpha, up to 0.99
      for (int r = 0; r < 3 + C; ++r)
        f64[(size_t)(10 + r) * n + k] = std::sin(0.7 * k + r);            // rgb, sem
    }
  }
  const int iopts[2] = {16, 4};
  const float fopts[4] = {0.3f, 9.0f, 0.99f, 1e-6f};
  for (int which = 0; which < 3; ++which) {
    std::vector<float> cam = camera(which == 1);
    // case 2: the pinhole's ground rectangle turned backwards: nothing visible
    if (which == 2) cam[24] = -1.0f;
    const int W = (int)cam[0], H = (int)cam[1];
    const int64_t npix = (int64_t)W * H;
    std::vector<float> rec(8 * (size_t)n);
    std::vector<int32_t> rect(4 * (size_t)n);
    std::vector<uint8_t> vis(n);
    const int nv = orc_contract(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, rec.data(),
                                rect.data(), vis.data());
    expect(which == 2 ? nv == 0 : nv > 0, "visible count");
    std::vector<double> geo(6 * (size_t)n);
    orc_geo64(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, geo.data());
    const double dgeo[6] = {0.1, -0.2, 0.3, 0.05, -0.4, 0.2};
    std::vector<double> dout(7);
    orc_geo64_adjoint(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, n / 2, dgeo,
                      dout.data());
    const int TX = (W + iopts[0] - 1) / iopts[0], TY = (H + iopts[1] - 1) / iopts[1];
    std::vector<int32_t> ranges(2 * (size_t)TX * TY);
    const int64_t P = orc_tile_lists(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, 0,
                                     nullptr, nullptr, ranges.data());
    std::vector<uint64_t> keys(P > 0 ? P : 1);
    std::vector<int32_t> ids(P > 0 ? P : 1);
    orc_tile_lists(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, P, keys.data(),
                   ids.data(), ranges.data());
    for (int i = 0; i < n && which != 2; ++i) {
      if (!vis[i]) continue;
      const int rows = rect[4 * i + 3] - rect[4 * i + 2];
      std::vector<int32_t> lo(rows), hi(rows);
      orc_row_spans(&rec[8 * (size_t)i], rect[4 * i], rect[4 * i + 1], rect[4 * i + 2],
                    rect[4 * i + 3], 9.0f, iopts[0], iopts[1], W, H, lo.data(), hi.data());
      const int32_t px[2] = {0, W - 1}, py[2] = {0, H - 1};
      float q[2];
      orc_q32(1, &rec[8 * (size_t)i], 2, px, py, q);
    }
    const int NO = 5 + C;
    std::vector<double> out((size_t)NO * npix), tf(npix);
    std::vector<int32_t> nl(npix);
    orc_render_fwd(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, nullptr, npix,
                   out.data(), tf.data(), nl.data());
    for (int64_t p = 0; p < npix; ++p) {
      const double A = out[(size_t)(NO - 1) * npix + p];
      expect(std::fabs(A - (1.0 - tf[p])) <= 1e-12, "A = 1 - T_final");
      expect(A >= 0.0 && A < 1.0, "0 <= A < 1");
    }
    // loss over every pixel, then over an empty mask
    std::vector<float> tgt(3 * (size_t)npix);
    std::vector<uint8_t> label(npix), mask(npix);
    int64_t mc = 0;
    for (int64_t p = 0; p < npix; ++p) {
      for (int c = 0; c < 3; ++c) tgt[(size_t)c * npix + p] = (float)((p * (c + 3)) % 17) / 16.0f;
      label[p] = (uint8_t)(p % C);
      mask[p] = (uint8_t)((p % 5) != 0);
      mc += mask[p];
    }
    std::vector<double> G((size_t)NO * npix), dexp(2, 0.0);
    orc_loss(C, npix, out.data(), tgt.data(), label.data(), mask.data(), mc, 0.1, -0.02, 1.0, 0.06,
             0.5, G.data(), dexp.data());
    std::vector<uint8_t> none(npix, 0);
    std::vector<double> G0((size_t)NO * npix);
    const double l0 = orc_loss(C, npix, out.data(), tgt.data(), label.data(), none.data(), 0, 0.0,
                               0.0, 1.0, 0.06, 1.0, G0.data(), dexp.data());
    expect(l0 == 0.0, "empty mask: zero loss");
    // a dL/d(depth, alpha) on every pixel too, so every branch of the adjoint runs
    for (int64_t p = 0; p < npix; ++p) {
      G[(size_t)(NO - 2) * npix + p] = 0.3;
      G[(size_t)(NO - 1) * npix + p] = -0.2;
    }
    std::vector<double> grads((size_t)K * n, 0.0);
    orc_render_bwd(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, nullptr, npix, G.data(),
                   tf.data(), nl.data(), grads.data());
    // sampled pixels
    std::vector<int32_t> pix = {0, (int32_t)(npix / 2), (int32_t)(npix - 1)};
    std::vector<double> o3((size_t)NO * 3), t3(3);
    std::vector<int32_t> n3(3);
    orc_render_fwd(n, C, f32.data(), f64.data(), cam.data(), iopts, fopts, pix.data(), 3,
                   o3.data(), t3.data(), n3.data());
    // optimiser on the raw block, with exposure, over a schedule of 3 steps
    std::vector<double> raw((size_t)K * n), m((size_t)K * n, 0.0), v((size_t)K * n, 0.0);
    for (size_t k = 0; k < raw.size(); ++k) raw[k] = std::sin(0.37 * (double)k);
    std::vector<double> sa(2 * (size_t)n), aa(n), ex(2, 0.1), mex(2, 0.0), vex(2, 0.0);
    const double lr[7] = {1e-3, 1e-4, 1e-4, 1e-4, 8e-3, 0.1, 1e-3};
    for (int step = 1; step <= 3; ++step)
      orc_adam_raw(n, C, raw.data(), grads.data(), m.data(), v.data(), lr, 1e-3, 1e-5, 3, step,
                   0.9, 0.999, 1e-8, sa.data(), aa.data(), 1, ex.data(), dexp.data(), mex.data(),
                   vex.data());
  }
  // grid-side terms and the meshgrid layout
  std::vector<double> z(n), zbar(n), dz(n, 0.0);
  std::vector<int32_t> nbr(4 * (size_t)n);
  for (int j = 0; j < gx; ++j)
    for (int i = 0; i < gx; ++i) {
      const int k = j * gx + i;
      z[k] = f64[2 * (size_t)n + k];
      zbar[k] = z[k] + 0.01 * std::cos((double)k);
      nbr[k] = j > 0 ? k - gx : k;
      nbr[n + k] = j + 1 < gx ? k + gx : k;
      nbr[2 * n + k] = i > 0 ? k - 1 : k;
      nbr[3 * n + k] = i + 1 < gx ? k + 1 : k;
    }
  orc_smooth(n, z.data(), nbr.data(), 1.0, dz.data());
  orc_lidar_loss(n, z.data(), zbar.data(), 0.02, dz.data());
  std::vector<float> lx(n), ly(n), ppx(37), ppy(37);
  for (int k = 0; k < n; ++k) { lx[k] = f32[k]; ly[k] = f32[n + k]; }
  for (int k = 0; k < 37; ++k) { ppx[k] = 0.7f + 0.04f * k; ppy[k] = 0.02f * (k % 9) - 0.1f; }
  std::vector<int32_t> nn(n);
  orc_lidar_nn(n, lx.data(), ly.data(), 37, ppx.data(), ppy.data(), nn.data());
  for (int k = 0; k < n; ++k) expect(nn[k] >= 0 && nn[k] < 37, "nearest index in range");
  const int np = 9, LW = 60, LH = 30;
  std::vector<float> poses(12 * (size_t)np, 0.0f);
  for (int k = 0; k < np; ++k) {
    float* p = &poses[12 * (size_t)k];
    p[0] = 0.5f + 0.5f * k; p[1] = 1.5f; p[2] = 0.1f;
    p[3] = 1.0f; p[7] = 1.0f; p[11] = 1.0f;     // identity rotation
  }
  std::vector<int32_t> ppix(2 * np);
  orc_pose_pixels(np, poses.data(), 0.0, 0.0, 0.1f, ppix.data());
  std::vector<uint8_t> lmask((size_t)LW * LH);
  const int64_t nroad = orc_layout_mask(LW, LH, np, ppix.data(), 7, lmask.data());
  expect(nroad > 0, "road pixels");
  std::vector<int32_t> lidx((size_t)LW * LH), lnbr(4 * (size_t)nroad);
  std::vector<float> gx_(nroad), gy_(nroad), gz_(nroad);
  std::vector<double> gq(4 * (size_t)nroad);
  orc_layout_build(LW, LH, lmask.data(), 0.0, 0.0, 0.1f, np, poses.data(), nroad, lidx.data(),
                   gx_.data(), gy_.data(), gz_.data(), gq.data(), lnbr.data());
  if (failures) return 1;
  std::printf("oracle sanitizer run: ok\n");
  return 0;
}
