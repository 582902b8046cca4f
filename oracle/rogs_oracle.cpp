// Reference oracle for meshgrid-surfel splatting (RoGs, arXiv 2405.14342).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-purpose CPU
// implementation used to check the GPU library.  Only the tests, the smoke
// check and the CPU-baseline leg of the benchmark may load it; the product
// path never does.  It shares no code, header or table with the GPU library.
//
// What it computes, and where in the paper it comes from:
//   * surfel covariance Sigma = R S S^T R^T with s_z = 0            (Sec. 3.1, Eq. 2)
//   * world-to-camera W, local affine J, Sigma' = J W Sigma W^T J^T,
//     2x2 block kept; orthographic camera: J = identity (in px/m)   (Sec. 3.3.1, Eq. 5)
//   * per-view ground rectangle cull (+-20 m lateral, 40 m ahead)   (Sec. 3.3.1; supp. Sec. 2.1)
//   * surfels sorted by ascending view depth, alpha compositing      (Sec. 3.3.1, Eq. 6)
//   * semantics composited like colour                             (Sec. 3.3.1)
//   * exposure c' = e^a c + b                                       (Sec. 3.3.1, Eq. 7)
//   * masked L1 colour loss and masked cross-entropy                (Sec. 3.3.2, Eq. 8, Eq. 9)
//   * weighted sum lambda_c L_c + lambda_s L_s                      (Sec. 3.3.2, Eq. 12; Sec. 4.2)
//   * Adam                                                         (Sec. 4.2)
// Readings where the paper is silent (pixel centres, the EWA low-pass eps,
// the 3-sigma cut, the opacity clamp, the termination threshold, the
// Jacobian clamp) are fixed by the library's documented "key contract"; this
// file restates that contract on its own (FP64 projection rounded to an FP32
// record, FP32 per-pixel test) because it decides integers: which surfels
// touch which tiles and pixels, and their order.  All values are then
// computed in FP64 from the same inputs.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>
#include <omp.h>

namespace {

// ------------------------------------------------------------------ inputs

struct Cam {
  int w, h, model;
  float fx, fy, cx, cy;
  float R[9], t[3];
  float znear;
  float o[2], ex[2], ez[2];
  float lat, fwd;
};

// Flat camera layout used by the Python wrapper (28 floats):
// w h model fx fy cx cy R[9] t[3] znear o[2] ex[2] ez[2] lat fwd
Cam unpack_cam(const float* c) {
  Cam k;
  k.w = (int)c[0]; k.h = (int)c[1]; k.model = (int)c[2];
  k.fx = c[3]; k.fy = c[4]; k.cx = c[5]; k.cy = c[6];
  for (int i = 0; i < 9; ++i) k.R[i] = c[7 + i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[16 + i];
  k.znear = c[19];
  k.o[0] = c[20]; k.o[1] = c[21];
  k.ex[0] = c[22]; k.ex[1] = c[23];
  k.ez[0] = c[24]; k.ez[1] = c[25];
  k.lat = c[26]; k.fwd = c[27];
  return k;
}

struct Opts {
  int tw, th;
  float eps, qcut, amax, teps;
};

// Surfel parameters.  The *_f pointers are the FP32 inputs that take the
// discrete decisions; the double pointers carry the values.  Normally the
// doubles are the same numbers promoted; finite-difference checks perturb
// only the doubles so that the decisions stay frozen.
struct Surfels {
  int n, C;
  const float *xf, *yf, *zf, *qf, *sf;      // q: [4][n], s: [2][n]
  const double *x, *y, *z, *q, *s, *alpha, *rgb, *sem;   // rgb [3][n], sem [C][n]
};

// ------------------------------------------------------ decision contract
//
// The projection that decides integers is computed in IEEE binary64 from the
// FP32 inputs (promoted exactly), one rounded operation per step in the order
// written (the file is compiled with -ffp-contract=off so no multiply-add is
// fused), then rounded once to the binary32 record; the per-pixel test is
// binary32.  The library documents the same sequence.

struct Rec32 {
  bool vis;
  float uh, vh, ul, vl;      // centre as a binary32 pair: u = uh + ul
  float A, B, C, tz;
  int x0, x1, y0, y1;
};

int clampi_d(double f, int hi) {   // clamp a floored value into [0, hi]
  if (!(f > 0.0)) return 0;
  if (f > (double)hi) return hi;
  return (int)f;
}

// Tiles of rectangle row ty that the 3-sigma ellipse of a record can reach
// (the contract's tight culling).  The conic of the record is tested per pixel
// in binary32; its rounding error is below 2^-19.8 q / (1 - rho) with
// rho = |B| / sqrt(AC), so the ellipse is inflated to
// q <= q_cut (1 + 2^-18 / (1 - rho)) and its x-extent over the tile row's
// pixel-centre rows gives the pixel columns, hence the tiles, clipped to the
// image and to the rectangle.  A conic with 1 - rho < 2^-16 (axis ratio above
// about 360) or no positive determinant keeps the whole rectangle row.  In
// binary64 from the binary32 record, one rounding per step, no contraction.
void row_span(const Rec32& r, double qcut, int tw, int th, int W, int H, int ty, int* lo,
              int* hi) {
  *lo = r.x0;
  *hi = r.x1;
  const double A = r.A, B = r.B, C = r.C;
  if (!(A > 0.0) || !(C > 0.0)) return;
  const double det = A * C - B * B;
  const double gap = 1.0 - std::fabs(B) / std::sqrt(A * C);
  if (!(det > 0.0) || !(gap >= 0x1p-16)) return;
  *hi = r.x0;                                    // empty unless a column is reached
  const double qe = qcut * (1.0 + 0x1p-18 / gap);
  const double u = (double)r.uh + (double)r.ul;
  const double v = (double)r.vh + (double)r.vl;
  // vertical half-extent, then the tile row's pixel-centre rows inside it
  const double dym = std::sqrt((A * qe) / det);
  const int r0 = ty * th;
  const int r1 = std::min(r0 + th, H);
  double a = ((double)r0 + 0.5) - v;
  double b = ((double)r1 - 0.5) - v;
  if (b < -dym || a > dym) return;
  if (a < -dym) a = -dym;
  if (b > dym) b = dym;
  // the left boundary x(dy) = u + (-B dy - sqrt(A qe - det dy^2)) / A is convex
  // with its minimum at dy = B sqrt(qe / (C det)); the right one is its mirror
  const double dys = B * std::sqrt(qe / (C * det));
  const double tl = dys < a ? a : (dys > b ? b : dys);
  const double tr = -dys < a ? a : (-dys > b ? b : -dys);
  double dl = A * qe - det * (tl * tl);
  double dr = A * qe - det * (tr * tr);
  if (dl < 0.0) dl = 0.0;
  if (dr < 0.0) dr = 0.0;
  const double xl = u + (-(B * tl) - std::sqrt(dl)) / A;
  const double xr = u + (-(B * tr) + std::sqrt(dr)) / A;
  // pixel p is reached iff its centre p + 1/2 lies in [xl, xr]
  const double pl = std::ceil(xl - 0.5);
  const double pr = std::floor(xr - 0.5);
  if (!(pl <= pr) || pl > (double)(W - 1) || pr < 0.0) return;
  const int cl = pl < 0.0 ? 0 : (int)pl;
  const int cr = pr > (double)(W - 1) ? W - 1 : (int)pr;
  const int l = std::max(cl / tw, r.x0);
  const int h = std::min(cr / tw + 1, r.x1);
  if (l < h) {
    *lo = l;
    *hi = h;
  }
}

Rec32 contract(const Cam& c, const Opts& o, float xf, float yf, float zf, float qwf, float qxf,
               float qyf, float qzf, float sxf, float syf) {
  Rec32 r;
  r.vis = false;
  r.uh = r.vh = r.ul = r.vl = r.A = r.B = r.C = 0.0f;
  r.x0 = r.x1 = r.y0 = r.y1 = 0;
  const double x = xf, y = yf, z = zf, qw = qwf, qx = qxf, qy = qyf, qz = qzf, sx = sxf, sy = syf;
  double R[9];
  for (int k = 0; k < 9; ++k) R[k] = c.R[k];
  double tx = ((R[0] * x + R[1] * y) + R[2] * z) + (double)c.t[0];
  double ty = ((R[3] * x + R[4] * y) + R[5] * z) + (double)c.t[1];
  double tz = ((R[6] * x + R[7] * y) + R[8] * z) + (double)c.t[2];
  r.tz = (float)tz;
  if (!(tz >= (double)c.znear)) return r;
  if (c.lat > 0.0f) {
    double dx = x - (double)c.o[0];
    double dy = y - (double)c.o[1];
    double a = dx * (double)c.ex[0] + dy * (double)c.ex[1];
    double b = dx * (double)c.ez[0] + dy * (double)c.ez[1];
    if (!(std::fabs(a) <= (double)c.lat)) return r;
    if (!(b >= 0.0 && b <= (double)c.fwd)) return r;
  }
  double nn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(nn > 0.0) || !std::isfinite(nn)) return r;
  double nq = std::sqrt(nn);
  double w = qw / nq, a = qx / nq, b = qy / nq, cc = qz / nq;
  double r1x = 1.0 - 2.0 * (b * b + cc * cc);
  double r1y = 2.0 * (a * b + w * cc);
  double r1z = 2.0 * (a * cc - w * b);
  double r2x = 2.0 * (a * b - w * cc);
  double r2y = 1.0 - 2.0 * (a * a + cc * cc);
  double r2z = 2.0 * (b * cc + w * a);
  double T1[3] = {sx * r1x, sx * r1y, sx * r1z};
  double T2[3] = {sy * r2x, sy * r2y, sy * r2z};
  double c1[3], c2[3];
  for (int k = 0; k < 3; ++k) {
    c1[k] = (R[3 * k] * T1[0] + R[3 * k + 1] * T1[1]) + R[3 * k + 2] * T1[2];
    c2[k] = (R[3 * k] * T2[0] + R[3 * k + 1] * T2[1]) + R[3 * k + 2] * T2[2];
  }
  const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
  double j00, j11, j02, j12, u, v;
  if (c.model == 0) {
    double limx = (0.65 * (double)c.w) / fx;
    double limy = (0.65 * (double)c.h) / fy;
    double xr = tx / tz, yr = ty / tz;
    double xc = std::min(std::max(xr, -limx), limx);
    double yc = std::min(std::max(yr, -limy), limy);
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
  const double eps = o.eps, qcut = o.qcut;
  double m00 = j00 * c1[0] + j02 * c1[2];
  double m01 = j00 * c2[0] + j02 * c2[2];
  double m10 = j11 * c1[1] + j12 * c1[2];
  double m11 = j11 * c2[1] + j12 * c2[2];
  double g0 = m00 * m00 + m01 * m01;
  double g1 = m10 * m10 + m11 * m11;
  double s00 = g0 + eps, s11 = g1 + eps;
  double s01 = m00 * m10 + m01 * m11;
  double dm = m00 * m11 - m01 * m10;
  double det = (dm * dm + eps * (g0 + g1)) + eps * eps;
  if (!(det > 0.0) || !std::isfinite(det)) return r;
  double A = s11 / det;
  double B = -(s01 / det);
  double C = s00 / det;
  double hx = std::sqrt(qcut * s00) + 1.0;
  double hy = std::sqrt(qcut * s11) + 1.0;
  if (!std::isfinite(u) || !std::isfinite(v) || !std::isfinite(hx) || !std::isfinite(hy) ||
      !std::isfinite(A) || !std::isfinite(B) || !std::isfinite(C))
    return r;
  int TX = (c.w + o.tw - 1) / o.tw, TY = (c.h + o.th - 1) / o.th;
  r.x0 = clampi_d(std::floor((u - hx) / (double)o.tw), TX);
  r.x1 = clampi_d(std::floor((u + hx) / (double)o.tw) + 1.0, TX);
  r.y0 = clampi_d(std::floor((v - hy) / (double)o.th), TY);
  r.y1 = clampi_d(std::floor((v + hy) / (double)o.th) + 1.0, TY);
  if (r.x0 >= r.x1 || r.y0 >= r.y1) return r;
  r.uh = (float)u;
  r.ul = (float)(u - (double)r.uh);
  r.vh = (float)v;
  r.vl = (float)(v - (double)r.vh);
  r.A = (float)A;
  r.B = (float)B;
  r.C = (float)C;
  r.vis = true;
  return r;
}

// Per-pixel contribution test (binary32): q = dx (A dx + 2B dy) + C dy dy
// with two fused multiply-adds, every other product rounded on its own.
inline float q32(const Rec32& r, int px, int py) {
  const float dx = (((float)px + 0.5f) - r.uh) - r.ul;
  const float dy = (((float)py + 0.5f) - r.vh) - r.vl;
  const float t = std::fmaf(r.A, dx, (2.0f * r.B) * dy);
  return std::fmaf(dx, t, (r.C * dy) * dy);
}

inline uint32_t fbits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

// ---------------------------------------------------- FP64 value geometry
//
// The same projection in double precision, keeping every intermediate the
// adjoint needs.  Eq. 2 with s_z = 0 means only the first two rotation
// columns matter: Sigma = s_x^2 r1 r1^T + s_y^2 r2 r2^T, so the camera-space
// footprint is spanned by W(s_x r1) and W(s_y r2), and Eq. 5's 2x2 block is
// Sigma' = M M^T with M = J W [s_x r1, s_y r2] (plus the EWA low-pass eps I).

struct Geo {
  double t[3];
  double qn, qh[4];            // |q| and normalised q (w, x, y, z)
  double r1[3], r2[3];
  double T1[3], T2[3], c1[3], c2[3];
  double xr, yr, xc, yc;
  bool clx, cly;               // Jacobian clamp active
  double j00, j11, j02, j12;
  double m00, m01, m10, m11, g0, g1, s00, s01, s11, dm, det;
  double u, v, A, B, C;
};

Geo geo64(const Cam& c, const Opts& o, double x, double y, double z, const double q[4],
          double sx, double sy) {
  Geo g;
  double R[9];
  for (int i = 0; i < 9; ++i) R[i] = c.R[i];
  for (int k = 0; k < 3; ++k) g.t[k] = R[3 * k] * x + R[3 * k + 1] * y + R[3 * k + 2] * z + c.t[k];
  g.qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) g.qh[k] = q[k] / g.qn;
  double w = g.qh[0], a = g.qh[1], b = g.qh[2], cc = g.qh[3];
  // columns 1 and 2 of the rotation matrix of a unit quaternion
  g.r1[0] = 1.0 - 2.0 * (b * b + cc * cc); g.r1[1] = 2.0 * (a * b + w * cc); g.r1[2] = 2.0 * (a * cc - w * b);
  g.r2[0] = 2.0 * (a * b - w * cc); g.r2[1] = 1.0 - 2.0 * (a * a + cc * cc); g.r2[2] = 2.0 * (b * cc + w * a);
  for (int k = 0; k < 3; ++k) { g.T1[k] = sx * g.r1[k]; g.T2[k] = sy * g.r2[k]; }
  for (int k = 0; k < 3; ++k) {
    g.c1[k] = R[3 * k] * g.T1[0] + R[3 * k + 1] * g.T1[1] + R[3 * k + 2] * g.T1[2];
    g.c2[k] = R[3 * k] * g.T2[0] + R[3 * k + 1] * g.T2[1] + R[3 * k + 2] * g.T2[2];
  }
  if (c.model == 0) {
    double limx = 0.65 * c.w / (double)c.fx, limy = 0.65 * c.h / (double)c.fy;
    g.xr = g.t[0] / g.t[2];
    g.yr = g.t[1] / g.t[2];
    g.clx = (g.xr < -limx) || (g.xr > limx);
    g.cly = (g.yr < -limy) || (g.yr > limy);
    g.xc = std::min(std::max(g.xr, -limx), limx);
    g.yc = std::min(std::max(g.yr, -limy), limy);
    g.j00 = c.fx / g.t[2];
    g.j11 = c.fy / g.t[2];
    g.j02 = -g.j00 * g.xc;
    g.j12 = -g.j11 * g.yc;
    g.u = c.fx * g.xr + c.cx;
    g.v = c.fy * g.yr + c.cy;
  } else {
    g.xr = g.yr = g.xc = g.yc = 0.0;
    g.clx = g.cly = false;
    g.j00 = c.fx; g.j11 = c.fy; g.j02 = 0.0; g.j12 = 0.0;
    g.u = c.fx * g.t[0] + c.cx;
    g.v = c.fy * g.t[1] + c.cy;
  }
  g.m00 = g.j00 * g.c1[0] + g.j02 * g.c1[2];
  g.m01 = g.j00 * g.c2[0] + g.j02 * g.c2[2];
  g.m10 = g.j11 * g.c1[1] + g.j12 * g.c1[2];
  g.m11 = g.j11 * g.c2[1] + g.j12 * g.c2[2];
  const double e = o.eps;
  g.g0 = g.m00 * g.m00 + g.m01 * g.m01;
  g.g1 = g.m10 * g.m10 + g.m11 * g.m11;
  g.s00 = g.g0 + e;
  g.s11 = g.g1 + e;
  g.s01 = g.m00 * g.m10 + g.m01 * g.m11;
  g.dm = g.m00 * g.m11 - g.m01 * g.m10;
  g.det = g.dm * g.dm + e * (g.g0 + g.g1) + e * e;   // = s00 s11 - s01^2
  g.A = g.s11 / g.det;
  g.B = -g.s01 / g.det;
  g.C = g.s00 / g.det;
  return g;
}

// Adjoint of geo64: given dL/d(u, v, A, B, C, t_z) accumulate dL/d(z, q, s).
// Reverse-mode chain through every line of geo64, in reverse order.
void geo64_adjoint(const Cam& c, const Opts& o, const Geo& g, const double q[4], double sx,
                   double sy, double du, double dv, double dA, double dB, double dC,
                   double dtz_direct, double* dz, double dq[4], double* dsx, double* dsy) {
  const double e = o.eps;
  // conic: A = s11/det, B = -s01/det, C = s00/det
  double ds11 = dA / g.det, ds01 = -dB / g.det, ds00 = dC / g.det;
  double ddet = -(g.A * dA + g.B * dB + g.C * dC) / g.det;
  // det = dm^2 + e (g0 + g1) + e^2
  double ddm = 2.0 * g.dm * ddet;
  double dg0 = e * ddet + ds00, dg1 = e * ddet + ds11;
  double dm00 = 0, dm01 = 0, dm10 = 0, dm11 = 0;
  // dm = m00 m11 - m01 m10
  dm00 += g.m11 * ddm; dm11 += g.m00 * ddm; dm01 -= g.m10 * ddm; dm10 -= g.m01 * ddm;
  // s01 = m00 m10 + m01 m11
  dm00 += g.m10 * ds01; dm10 += g.m00 * ds01; dm01 += g.m11 * ds01; dm11 += g.m01 * ds01;
  // g0 = m00^2 + m01^2, g1 = m10^2 + m11^2
  dm00 += 2.0 * g.m00 * dg0; dm01 += 2.0 * g.m01 * dg0;
  dm10 += 2.0 * g.m10 * dg1; dm11 += 2.0 * g.m11 * dg1;
  // M = J [c1 c2]
  double dj00 = g.c1[0] * dm00 + g.c2[0] * dm01;
  double dj02 = g.c1[2] * dm00 + g.c2[2] * dm01;
  double dj11 = g.c1[1] * dm10 + g.c2[1] * dm11;
  double dj12 = g.c1[2] * dm10 + g.c2[2] * dm11;
  double dc1[3] = {g.j00 * dm00, g.j11 * dm10, g.j02 * dm00 + g.j12 * dm10};
  double dc2[3] = {g.j00 * dm01, g.j11 * dm11, g.j02 * dm01 + g.j12 * dm11};
  double dt[3] = {0.0, 0.0, dtz_direct};
  if (c.model == 0) {
    const double tz = g.t[2];
    // j02 = -j00 xc, j12 = -j11 yc
    dj00 += -g.xc * dj02;
    double dxc = -g.j00 * dj02;
    dj11 += -g.yc * dj12;
    double dyc = -g.j11 * dj12;
    // j00 = fx / tz, j11 = fy / tz
    dt[2] += -(g.j00 / tz) * dj00 - (g.j11 / tz) * dj11;
    // clamp
    double dxr = g.clx ? 0.0 : dxc;
    double dyr = g.cly ? 0.0 : dyc;
    // u = fx xr + cx, v = fy yr + cy
    dxr += c.fx * du;
    dyr += c.fy * dv;
    // xr = tx / tz, yr = ty / tz
    dt[0] += dxr / tz;
    dt[1] += dyr / tz;
    dt[2] += -(g.xr / tz) * dxr - (g.yr / tz) * dyr;
  } else {
    dt[0] += c.fx * du;
    dt[1] += c.fy * dv;
  }
  // t = R mu + t_cw: only z is learnable
  *dz += (double)c.R[2] * dt[0] + (double)c.R[5] * dt[1] + (double)c.R[8] * dt[2];
  // c = R T  ->  dT = R^T dc
  double dT1[3], dT2[3];
  for (int k = 0; k < 3; ++k) {
    dT1[k] = (double)c.R[k] * dc1[0] + (double)c.R[3 + k] * dc1[1] + (double)c.R[6 + k] * dc1[2];
    dT2[k] = (double)c.R[k] * dc2[0] + (double)c.R[3 + k] * dc2[1] + (double)c.R[6 + k] * dc2[2];
  }
  // T1 = sx r1, T2 = sy r2
  double dr1[3], dr2[3];
  for (int k = 0; k < 3; ++k) {
    *dsx += g.r1[k] * dT1[k];
    *dsy += g.r2[k] * dT2[k];
    dr1[k] = sx * dT1[k];
    dr2[k] = sy * dT2[k];
  }
  // rotation columns of the unit quaternion (w, a, b, c)
  const double w = g.qh[0], a = g.qh[1], b = g.qh[2], cc = g.qh[3];
  double dw = 0, da = 0, db = 0, dc = 0;
  // r1 = (1 - 2(b^2 + c^2), 2(ab + wc), 2(ac - wb))
  db += -4.0 * b * dr1[0]; dc += -4.0 * cc * dr1[0];
  da += 2.0 * b * dr1[1]; db += 2.0 * a * dr1[1]; dw += 2.0 * cc * dr1[1]; dc += 2.0 * w * dr1[1];
  da += 2.0 * cc * dr1[2]; dc += 2.0 * a * dr1[2]; dw += -2.0 * b * dr1[2]; db += -2.0 * w * dr1[2];
  // r2 = (2(ab - wc), 1 - 2(a^2 + c^2), 2(bc + wa))
  da += 2.0 * b * dr2[0]; db += 2.0 * a * dr2[0]; dw += -2.0 * cc * dr2[0]; dc += -2.0 * w * dr2[0];
  da += -4.0 * a * dr2[1]; dc += -4.0 * cc * dr2[1];
  db += 2.0 * cc * dr2[2]; dc += 2.0 * b * dr2[2]; dw += 2.0 * a * dr2[2]; da += 2.0 * w * dr2[2];
  // qh = q / |q|:  dq = (dqh - qh (qh . dqh)) / |q|
  double dqh[4] = {dw, da, db, dc};
  double dot = 0.0;
  for (int k = 0; k < 4; ++k) dot += g.qh[k] * dqh[k];
  for (int k = 0; k < 4; ++k) dq[k] += (dqh[k] - g.qh[k] * dot) / g.qn;
  (void)q;
}

// -------------------------------------------------------------- one view

struct ViewData {
  Cam cam;
  Opts opts;
  int TX, TY;
  std::vector<Rec32> rec;               // [n]
  std::vector<int> vis_ids;             // visible surfel ids, ascending
  std::vector<int> vis_index;           // surfel id -> index into vis_ids (or -1)
  std::vector<Geo> geo;                 // [n_vis]
  std::vector<std::vector<int>> lists;  // per tile: surfel ids, depth order
};

void build_view(const Surfels& S, const Cam& cam, const Opts& o, ViewData& V) {
  V.cam = cam;
  V.opts = o;
  V.TX = (cam.w + o.tw - 1) / o.tw;
  V.TY = (cam.h + o.th - 1) / o.th;
  const int n = S.n;
  V.rec.resize(n);
  V.vis_index.assign(n, -1);
  V.vis_ids.clear();
  for (int i = 0; i < n; ++i) {
    V.rec[i] = contract(cam, o, S.xf[i], S.yf[i], S.zf[i], S.qf[i], S.qf[n + i], S.qf[2 * n + i],
                        S.qf[3 * n + i], S.sf[i], S.sf[n + i]);
    if (V.rec[i].vis) {
      V.vis_index[i] = (int)V.vis_ids.size();
      V.vis_ids.push_back(i);
    }
  }
  V.geo.resize(V.vis_ids.size());
  for (size_t k = 0; k < V.vis_ids.size(); ++k) {
    int i = V.vis_ids[k];
    double q[4] = {S.q[i], S.q[n + i], S.q[2 * n + i], S.q[3 * n + i]};
    V.geo[k] = geo64(cam, o, S.x[i], S.y[i], S.z[i], q, S.s[i], S.s[n + i]);
  }
  // Brute-force tile lists: every surfel is appended to every tile of its
  // rectangle that its ellipse reaches (row spans), then each list is ordered
  // by (depth bits, id) ("ascending order of original depth", Sec. 3.3.1;
  // ties by surfel id).
  V.lists.assign((size_t)V.TX * V.TY, std::vector<int>());
  for (int i : V.vis_ids) {
    const Rec32& r = V.rec[i];
    for (int ty = r.y0; ty < r.y1; ++ty) {
      int lo, hi;
      row_span(r, o.qcut, o.tw, o.th, cam.w, cam.h, ty, &lo, &hi);
      for (int tx = lo; tx < hi; ++tx) V.lists[(size_t)ty * V.TX + tx].push_back(i);
    }
  }
  for (auto& L : V.lists) {
    std::sort(L.begin(), L.end(), [&](int a, int b) {
      uint32_t ka = fbits(V.rec[a].tz), kb = fbits(V.rec[b].tz);
      if (ka != kb) return ka < kb;
      return a < b;
    });
  }
}

// Number of output channels: RGB, C semantic logits, depth D, alpha A.
inline int n_out(int C) { return 5 + C; }

struct PixelState {
  double T;
  int nlast;
};

// Eq. 6 for one pixel (front to back along its tile's list).  Writes the
// 5 + C outputs into out[ch * stride].
PixelState pixel_forward(const Surfels& S, const ViewData& V, int px, int py, double* out,
                         size_t stride) {
  const int C = S.C, n = S.n;
  const int tile = (py / V.opts.th) * V.TX + (px / V.opts.tw);
  const std::vector<int>& L = V.lists[tile];
  for (int ch = 0; ch < n_out(C); ++ch) out[ch * stride] = 0.0;
  double T = 1.0;
  int nlast = (int)L.size();
  const double pxc = px + 0.5, pyc = py + 0.5;
  for (size_t k = 0; k < L.size(); ++k) {
    const int i = L[k];
    const Rec32& r = V.rec[i];
    if (!(q32(r, px, py) <= V.opts.qcut)) continue;
    const Geo& g = V.geo[V.vis_index[i]];
    double dx = pxc - g.u, dy = pyc - g.v;
    double q = g.A * dx * dx + g.C * dy * dy + 2.0 * g.B * dx * dy;
    double gg = std::exp(-0.5 * q);
    double a = std::min(S.alpha[i] * gg, (double)V.opts.amax);
    double w = a * T;
    for (int ch = 0; ch < 3; ++ch) out[ch * stride] += w * S.rgb[(size_t)ch * n + i];
    for (int ch = 0; ch < C; ++ch) out[(3 + ch) * stride] += w * S.sem[(size_t)ch * n + i];
    out[(3 + C) * stride] += w * g.t[2];
    T *= (1.0 - a);
    if (T < V.opts.teps) {
      nlast = (int)k + 1;
      break;
    }
  }
  out[(4 + C) * stride] = 1.0 - T;
  return PixelState{T, nlast};
}

// Number of per-visible-surfel "record" gradient slots:
// du dv dA dB dC dalpha dtz drgb[3] dsem[C]
inline int n_rg(int C) { return 10 + C; }

// Adjoint of pixel_forward for one pixel: G = dL/d(outputs) (5 + C values),
// accumulated into rg[vis_index][n_rg].
//
// Eq. 6 written out for one pixel: O = sum_k w_k f_k with w_k = a_k T_k,
// T_k = prod_{j<k} (1 - a_j), A = 1 - T_final.  For the opacity a_k after
// the clamp, d(G.O)/da_k = T_k Gf_k - S_k / (1 - a_k) with the suffix
// S_k = sum_{j>k} w_j Gf_j (every later weight carries the factor 1 - a_k),
// and dA/da_k = T_final / (1 - a_k).  The entries the pixel reached are first
// collected front to back, then the suffix is accumulated back to front.
struct Hit {
  int i, vi;
  double dx, dy, gg, a, T, w, Gf;
  bool clamped;
};

void pixel_backward(const Surfels& S, const ViewData& V, int px, int py, const double* G,
                    size_t gstride, double Tfinal, int nlast, double* rg) {
  const int C = S.C, n = S.n, NR = n_rg(C);
  const int tile = (py / V.opts.th) * V.TX + (px / V.opts.tw);
  const std::vector<int>& L = V.lists[tile];
  const double pxc = px + 0.5, pyc = py + 0.5;
  const double GA = G[(4 + C) * gstride], GD = G[(3 + C) * gstride];
  thread_local std::vector<Hit> hits;
  hits.clear();
  double T = 1.0;
  for (int k = 0; k < nlast; ++k) {
    const int i = L[k];
    const Rec32& r = V.rec[i];
    if (!(q32(r, px, py) <= V.opts.qcut)) continue;
    Hit h;
    h.i = i;
    h.vi = V.vis_index[i];
    const Geo& g = V.geo[h.vi];
    h.dx = pxc - g.u;
    h.dy = pyc - g.v;
    const double q = g.A * h.dx * h.dx + g.C * h.dy * h.dy + 2.0 * g.B * h.dx * h.dy;
    h.gg = std::exp(-0.5 * q);
    const double araw = S.alpha[i] * h.gg;
    h.clamped = araw > (double)V.opts.amax;
    h.a = h.clamped ? (double)V.opts.amax : araw;
    h.T = T;
    h.w = h.a * T;
    // Gf = dL/dO . (f_k, t_z): the pixel's output gradient against this
    // surfel's composited features and depth
    h.Gf = GD * g.t[2];
    for (int ch = 0; ch < 3; ++ch) h.Gf += G[ch * gstride] * S.rgb[(size_t)ch * n + i];
    for (int ch = 0; ch < C; ++ch) h.Gf += G[(3 + ch) * gstride] * S.sem[(size_t)ch * n + i];
    hits.push_back(h);
    T *= (1.0 - h.a);
  }
  double suffix = 0.0;   // sum over the entries behind the current one of w Gf
  for (size_t kk = hits.size(); kk-- > 0;) {
    const Hit& h = hits[kk];
    const Geo& g = V.geo[h.vi];
    double* R = rg + (size_t)h.vi * NR;
    // features: dO/df = w
    for (int ch = 0; ch < 3; ++ch) R[7 + ch] += h.w * G[ch * gstride];
    for (int ch = 0; ch < C; ++ch) R[10 + ch] += h.w * G[(3 + ch) * gstride];
    R[6] += h.w * GD;
    const double da = h.T * h.Gf - suffix / (1.0 - h.a) + GA * Tfinal / (1.0 - h.a);
    suffix += h.w * h.Gf;
    // the clamp a = min(alpha g, a_max) cuts the dependence on alpha and g
    if (!h.clamped) {
      R[5] += h.gg * da;                 // d alpha
      const double dg = S.alpha[h.i] * da;
      const double dq = -0.5 * h.gg * dg;
      R[2] += h.dx * h.dx * dq;          // dA
      R[4] += h.dy * h.dy * dq;          // dC
      R[3] += 2.0 * h.dx * h.dy * dq;    // dB
      R[0] += -(2.0 * g.A * h.dx + 2.0 * g.B * h.dy) * dq;   // du
      R[1] += -(2.0 * g.C * h.dy + 2.0 * g.B * h.dx) * dq;   // dv
    }
  }
}

Surfels make_surfels(int n, int C, const float* f32, const double* f64) {
  // f32: x[n] y[n] z[n] q[4n] s[2n]   (decision inputs)
  // f64: x y z q[4] s[2] alpha rgb[3] sem[C], each [n]   (values)
  Surfels S;
  S.n = n; S.C = C;
  S.xf = f32; S.yf = f32 + n; S.zf = f32 + 2 * (size_t)n; S.qf = f32 + 3 * (size_t)n;
  S.sf = f32 + 7 * (size_t)n;
  S.x = f64; S.y = f64 + n; S.z = f64 + 2 * (size_t)n; S.q = f64 + 3 * (size_t)n;
  S.s = f64 + 7 * (size_t)n; S.alpha = f64 + 9 * (size_t)n; S.rgb = f64 + 10 * (size_t)n;
  S.sem = f64 + 13 * (size_t)n;
  return S;
}

Opts make_opts(const int* io, const float* fo) {
  Opts o;
  o.tw = io[0]; o.th = io[1];
  o.eps = fo[0]; o.qcut = fo[1]; o.amax = fo[2]; o.teps = fo[3];
  return o;
}

}  // namespace

extern "C" {

// The per-pixel test value q32 of records rec7[n][7] (u_hi v_hi u_lo v_lo A B
// C) at pixels (px[k], py[k]) of a W x H grid: q[n][npix].
void orc_q32(int n, const float* rec7, int npix, const int32_t* px, const int32_t* py, float* q) {
  for (int i = 0; i < n; ++i) {
    Rec32 r{};
    const float* f = rec7 + 7 * (size_t)i;
    r.uh = f[0]; r.vh = f[1]; r.ul = f[2]; r.vl = f[3];
    r.A = f[4]; r.B = f[5]; r.C = f[6];
    for (int k = 0; k < npix; ++k) q[(size_t)i * npix + k] = q32(r, px[k], py[k]);
  }
}

// Row spans of one binary32 record (u_hi v_hi u_lo v_lo A B C) over the
// rectangle rows y0..y1-1: lo[k], hi[k] for row y0 + k.
void orc_row_spans(const float* rec7, int x0, int x1, int y0, int y1, float qcut, int tw, int th,
                   int W, int H, int32_t* lo, int32_t* hi) {
  Rec32 r{};
  r.vis = true;
  r.uh = rec7[0]; r.vh = rec7[1]; r.ul = rec7[2]; r.vl = rec7[3];
  r.A = rec7[4]; r.B = rec7[5]; r.C = rec7[6];
  r.x0 = x0; r.x1 = x1; r.y0 = y0; r.y1 = y1;
  for (int ty = y0; ty < y1; ++ty) {
    int l, h;
    row_span(r, (double)qcut, tw, th, W, H, ty, &l, &h);
    lo[ty - y0] = l;
    hi[ty - y0] = h;
  }
}

// Decision contract for every surfel of one view.
// rec: [n][8] = u_hi v_hi u_lo v_lo A B C tz ; rect: [n][4] = x0 x1 y0 y1 ; vis: [n]
// Returns the number of visible surfels.
int orc_contract(int n, int C, const float* f32, const double* f64, const float* cam,
                 const int* iopts, const float* fopts, float* rec, int32_t* rect, uint8_t* vis) {
  Surfels S = make_surfels(n, C, f32, f64);
  Cam c = unpack_cam(cam);
  Opts o = make_opts(iopts, fopts);
  int cnt = 0;
  for (int i = 0; i < n; ++i) {
    Rec32 r = contract(c, o, S.xf[i], S.yf[i], S.zf[i], S.qf[i], S.qf[n + i], S.qf[2 * n + i],
                       S.qf[3 * n + i], S.sf[i], S.sf[n + i]);
    vis[i] = r.vis ? 1 : 0;
    float* R = rec + 8 * (size_t)i;
    int32_t* q = rect + 4 * (size_t)i;
    if (r.vis) {
      R[0] = r.uh; R[1] = r.vh; R[2] = r.ul; R[3] = r.vl;
      R[4] = r.A; R[5] = r.B; R[6] = r.C; R[7] = r.tz;
      q[0] = r.x0; q[1] = r.x1; q[2] = r.y0; q[3] = r.y1;
    } else {
      for (int k = 0; k < 8; ++k) R[k] = 0.0f;
      R[7] = r.tz;
      q[0] = q[1] = q[2] = q[3] = 0;
    }
    cnt += r.vis;
  }
  return cnt;
}

// FP64 projection values (u v A B C tz) of every visible surfel; 0 elsewhere.
void orc_geo64(int n, int C, const float* f32, const double* f64, const float* cam,
               const int* iopts, const float* fopts, double* out) {
  Surfels S = make_surfels(n, C, f32, f64);
  Cam c = unpack_cam(cam);
  Opts o = make_opts(iopts, fopts);
  for (int i = 0; i < n; ++i) {
    double q[4] = {S.q[i], S.q[n + i], S.q[2 * n + i], S.q[3 * n + i]};
    Geo g = geo64(c, o, S.x[i], S.y[i], S.z[i], q, S.s[i], S.s[n + i]);
    double* R = out + 6 * (size_t)i;
    R[0] = g.u; R[1] = g.v; R[2] = g.A; R[3] = g.B; R[4] = g.C; R[5] = g.t[2];
  }
}

// Adjoint of orc_geo64 for one surfel (used by the Jacobian pins).
void orc_geo64_adjoint(int n, int C, const float* f32, const double* f64, const float* cam,
                       const int* iopts, const float* fopts, int i, const double* dgeo,
                       double* dout /* dz dq[4] dsx dsy */) {
  Surfels S = make_surfels(n, C, f32, f64);
  Cam c = unpack_cam(cam);
  Opts o = make_opts(iopts, fopts);
  double q[4] = {S.q[i], S.q[n + i], S.q[2 * n + i], S.q[3 * n + i]};
  Geo g = geo64(c, o, S.x[i], S.y[i], S.z[i], q, S.s[i], S.s[n + i]);
  for (int k = 0; k < 7; ++k) dout[k] = 0.0;
  geo64_adjoint(c, o, g, q, S.s[i], S.s[n + i], dgeo[0], dgeo[1], dgeo[2], dgeo[3], dgeo[4],
                dgeo[5], &dout[0], &dout[1], &dout[5], &dout[6]);
}

// Tile lists of one view.  keys = (tile << 32) | bits(t_z), ids = surfel ids,
// both in list order (tile ascending, then depth, then id); ranges [TX*TY][2].
// Returns the number of pairs P; writes at most cap of them.
int64_t orc_tile_lists(int n, int C, const float* f32, const double* f64, const float* cam,
                       const int* iopts, const float* fopts, int64_t cap, uint64_t* keys,
                       int32_t* ids, int32_t* ranges) {
  Surfels S = make_surfels(n, C, f32, f64);
  ViewData V;
  build_view(S, unpack_cam(cam), make_opts(iopts, fopts), V);
  int64_t p = 0;
  for (size_t t = 0; t < V.lists.size(); ++t) {
    if (ranges) ranges[2 * t] = (int32_t)p;
    for (int i : V.lists[t]) {
      if (p < cap) {
        keys[p] = ((uint64_t)t << 32) | fbits(V.rec[i].tz);
        ids[p] = i;
      }
      ++p;
    }
    if (ranges) ranges[2 * t + 1] = (int32_t)p;
  }
  return p;
}

// Forward render of one view.  pix: optional list of linear pixel indices
// (y * W + x); npix of them (or all W*H when pix is null).
// out: [(5 + C)][npix] (R G B sem[C] D A), tfinal [npix], nlast [npix].
void orc_render_fwd(int n, int C, const float* f32, const double* f64, const float* cam,
                    const int* iopts, const float* fopts, const int32_t* pix, int64_t npix,
                    double* out, double* tfinal, int32_t* nlast) {
  Surfels S = make_surfels(n, C, f32, f64);
  ViewData V;
  build_view(S, unpack_cam(cam), make_opts(iopts, fopts), V);
  const int W = V.cam.w;
  if (!pix) npix = (int64_t)W * V.cam.h;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t k = 0; k < npix; ++k) {
    int64_t p = pix ? pix[k] : k;
    PixelState st = pixel_forward(S, V, (int)(p % W), (int)(p / W), out + k, (size_t)npix);
    tfinal[k] = st.T;
    nlast[k] = st.nlast;
  }
}

// Backward of one view: given dL/dO, T_final and n_last at the pixels of a
// forward call (layout as orc_render_fwd), accumulate dL/d(params) into
// grads = dz[n] dq[4][n] ds[2][n] dalpha[n] drgb[3][n] dsem[C][n].
void orc_render_bwd(int n, int C, const float* f32, const double* f64, const float* cam,
                    const int* iopts, const float* fopts, const int32_t* pix, int64_t npix,
                    const double* G, const double* tfinal, const int32_t* nlast, double* grads) {
  Surfels S = make_surfels(n, C, f32, f64);
  ViewData V;
  Cam cm = unpack_cam(cam);
  Opts op = make_opts(iopts, fopts);
  build_view(S, cm, op, V);
  const int W = V.cam.w;
  if (!pix) npix = (int64_t)W * V.cam.h;
  const int NR = n_rg(C);
  const size_t nv = V.vis_ids.size();
  int nth = omp_get_max_threads();
  std::vector<std::vector<double>> part(nth);
#pragma omp parallel
  {
    int tid = omp_get_thread_num();
    part[tid].assign(nv * NR, 0.0);
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < npix; ++k) {
      int64_t p = pix ? pix[k] : k;
      pixel_backward(S, V, (int)(p % W), (int)(p / W), G + k, (size_t)npix, tfinal[k], nlast[k],
                     part[tid].data());
    }
  }
  std::vector<double> rg(nv * NR, 0.0);
  for (int t = 0; t < nth; ++t)
    if (!part[t].empty())
      for (size_t j = 0; j < rg.size(); ++j) rg[j] += part[t][j];
  double* dz = grads;
  double* dq = grads + n;
  double* ds = grads + 5 * (size_t)n;
  double* dal = grads + 7 * (size_t)n;
  double* drgb = grads + 8 * (size_t)n;
  double* dsem = grads + 11 * (size_t)n;
  for (size_t k = 0; k < nv; ++k) {
    const int i = V.vis_ids[k];
    const double* R = rg.data() + k * NR;
    double q[4] = {S.q[i], S.q[n + i], S.q[2 * n + i], S.q[3 * n + i]};
    double dzl = 0.0, dql[4] = {0, 0, 0, 0}, dsx = 0.0, dsy = 0.0;
    geo64_adjoint(cm, op, V.geo[k], q, S.s[i], S.s[n + i], R[0], R[1], R[2], R[3], R[4], R[6],
                  &dzl, dql, &dsx, &dsy);
    dz[i] += dzl;
    for (int j = 0; j < 4; ++j) dq[(size_t)j * n + i] += dql[j];
    ds[i] += dsx;
    ds[(size_t)n + i] += dsy;
    dal[i] += R[5];
    for (int j = 0; j < 3; ++j) drgb[(size_t)j * n + i] += R[7 + j];
    for (int j = 0; j < C; ++j) dsem[(size_t)j * n + i] += R[10 + j];
  }
}

// Loss of one view at npix pixels (Eq. 7, 8, 9, 12).  O: [(5+C)][npix]
// outputs; tgt: [3][npix] target RGB; label, mask: [npix]; mcount = |M_v|
// (number of mask pixels over the *whole* view).  scale = 1 / n_views.
// Writes dL/dO into G ([(5+C)][npix]; D and A entries are 0) and returns the
// loss contribution; d_exp[0..1] += dL/da, dL/db.
double orc_loss(int C, int64_t npix, const double* O, const float* tgt, const uint8_t* label,
                const uint8_t* mask, int64_t mcount, double exp_a, double exp_b, double lam_c,
                double lam_s, double scale, double* G, double* d_exp) {
  double loss = 0.0, da = 0.0, db = 0.0;
  const double ea = std::exp(exp_a);
  const double wc = mcount > 0 ? lam_c * scale / (double)mcount : 0.0;
  const double ws = mcount > 0 ? lam_s * scale / (double)mcount : 0.0;
  std::vector<double> sm(C);
  for (int64_t k = 0; k < npix; ++k) {
    for (int ch = 0; ch < 5 + C; ++ch) G[ch * npix + k] = 0.0;
    if (!mask[k] || mcount == 0) continue;
    // L1 on exposure-corrected colour
    for (int ch = 0; ch < 3; ++ch) {
      double c = O[ch * npix + k];
      double cp = ea * c + exp_b;
      double r = cp - (double)tgt[ch * npix + k];
      double sg = (r > 0.0) - (r < 0.0);
      loss += wc * std::fabs(r);
      G[ch * npix + k] = wc * sg * ea;
      da += wc * sg * ea * c;
      db += wc * sg;
    }
    // cross-entropy of the composited logits against the hard label
    double mx = -INFINITY;
    for (int j = 0; j < C; ++j) mx = std::max(mx, O[(3 + j) * npix + k]);
    double se = 0.0;
    for (int j = 0; j < C; ++j) { sm[j] = std::exp(O[(3 + j) * npix + k] - mx); se += sm[j]; }
    int lb = label[k];
    loss += ws * ((mx + std::log(se)) - O[(3 + lb) * npix + k]);
    for (int j = 0; j < C; ++j) G[(3 + j) * npix + k] = ws * (sm[j] / se - (j == lb ? 1.0 : 0.0));
  }
  d_exp[0] += da;
  d_exp[1] += db;
  return loss;
}

// Adam (torch semantics, bias-corrected) on one parameter group, in FP64.
void orc_adam(int64_t n, double* p, const double* g, double* m, double* v, double lr, double b1,
              double b2, double eps, int64_t step) {
  const double bc1 = 1.0 - std::pow(b1, (double)step);
  const double bc2 = 1.0 - std::pow(b2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / bc1, vh = v[i] / bc2;
    p[i] -= lr * mh / (std::sqrt(vh) + eps);
  }
}

// One optimiser step on the raw parameter block, as Sec. 4.2 sets it up.
// The renderer reads the activated scale s = exp(l) and opacity
// alpha = sigmoid(o); the optimiser moves the raw l and o, so their
// gradients are chained through the activations (ds/dl = s, dalpha/do =
// alpha (1 - alpha)), taken at the raw values before this step.  Rows of the
// block [11 + C][n]: z | q (4) | l (2) | o | rgb (3) | sem (C).  Every group
// has its own rate (lr[0..6] = z, q, s, alpha, rgb, sem, exposure); the z
// rate follows the schedule below.  Afterwards the activated copies are
// refreshed.  When n_views > 0 the per-view exposure (a, b) of Eq. 7 is
// stepped too, with its own rate and moments.
//
// z rate: proportional to the scene size, starting at z_start and ending at
// z_end after total_steps steps, moving linearly in log(rate) in between:
// log r(t) = (1 - t) log z_start + t log z_end, t = (step - 1) / (total - 1).
// total_steps = 1 uses z_start; total_steps = 0 (no schedule) uses lr[0].
double orc_z_rate(double lr_z, double z_start, double z_end, int64_t total_steps, int64_t step) {
  if (total_steps <= 0) return lr_z;
  if (total_steps == 1) return z_start;
  double t = (double)(step - 1) / (double)(total_steps - 1);
  t = std::min(std::max(t, 0.0), 1.0);
  return std::exp((1.0 - t) * std::log(z_start) + t * std::log(z_end));
}

void orc_adam_raw(int n, int C, double* p, const double* g_act, double* m, double* v,
                  const double* lr, double z_start, double z_end, int64_t total_steps,
                  int64_t step, double b1, double b2, double eps, double* s_act, double* a_act,
                  int n_views, double* expo, const double* d_expo, double* m_e, double* v_e) {
  const int K = 11 + C;
  const double lr_z = orc_z_rate(lr[0], z_start, z_end, total_steps, step);
  std::vector<double> graw(n);
  for (int r = 0; r < K; ++r) {
    double rate;
    if (r == 0) rate = lr_z;
    else if (r <= 4) rate = lr[1];
    else if (r <= 6) rate = lr[2];
    else if (r == 7) rate = lr[3];
    else if (r <= 10) rate = lr[4];
    else rate = lr[5];
    double* pr = p + (size_t)r * n;
    const double* gr = g_act + (size_t)r * n;
    for (int i = 0; i < n; ++i) {
      if (r == 5 || r == 6) {
        graw[i] = gr[i] * std::exp(pr[i]);            // d/dl = s d/ds
      } else if (r == 7) {
        const double a = 1.0 / (1.0 + std::exp(-pr[i]));
        graw[i] = gr[i] * a * (1.0 - a);              // d/do = alpha (1 - alpha) d/dalpha
      } else {
        graw[i] = gr[i];
      }
    }
    orc_adam(n, pr, graw.data(), m + (size_t)r * n, v + (size_t)r * n, rate, b1, b2, eps, step);
  }
  for (int i = 0; i < n; ++i) {
    s_act[i] = std::exp(p[5 * (size_t)n + i]);
    s_act[(size_t)n + i] = std::exp(p[6 * (size_t)n + i]);
    a_act[i] = 1.0 / (1.0 + std::exp(-p[7 * (size_t)n + i]));
  }
  if (n_views > 0) orc_adam(2 * (int64_t)n_views, expo, d_expo, m_e, v_e, lr[6], b1, b2, eps, step);
}

int orc_num_threads(void) { return omp_get_max_threads(); }

void orc_set_threads(int n) { omp_set_num_threads(n); }

}  // extern "C"
