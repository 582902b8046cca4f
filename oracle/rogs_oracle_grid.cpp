// Reference oracle, part 2: the grid-side terms of RoGs (arXiv 2405.14342).
//
// TEST INFRASTRUCTURE ONLY (see rogs_oracle.cpp).  Plain loops, FP64 values.
//
//   * elevation smoothness L_smooth = 1/K sum_i sum_{j in N(i)} (z_i - z_j)^2
//     over the four grid neighbours found through the pixel index of the
//     meshgrid (Sec. 3.3.2, Eq. 10; supp. Sec. 3.3), K = 4
//   * LiDAR elevation loss L_z = sum_i (z_i - zbar_i)^2, zbar_i = height of
//     the point nearest to (x_i, y_i) in the xy-plane          (Sec. 3.3.2, Eq. 11)
//   * meshgrid layout: vehicle positions projected onto a 0.1 m raster,
//     dilated into a road mask, surfels at the mask's pixels indexed by a
//     running count, neighbour indices from the adjacent pixels
//                                             (Sec. 3.1 "Meshgrid Layout"; supp. Sec. 3.3)
//   * pose-based initialisation: rotation of the nearest vehicle pose and the
//     height of the vehicle's xy-plane at the surfel   (Sec. 3.2, Eq. 4; supp. Sec. 1)
// Where the paper is silent: the raster cell of a position is the nearest
// pixel centre (round half up), the dilation is a disk of integer radius
// (dx^2 + dy^2 <= r^2), "up/down/left/right" are the rows above and below and
// the columns left and right, nearest neighbours use the squared xy distance
// in binary64 of the binary32 inputs with ties to the lower index.
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

int64_t nearest_xy(double xi, double yi, int64_t m, const float* px, const float* py) {
  double best = INFINITY;
  int64_t bi = -1;
  for (int64_t k = 0; k < m; ++k) {
    const double dx = xi - (double)px[k];
    const double dy = yi - (double)py[k];
    const double d2 = dx * dx + dy * dy;
    if (d2 < best) {
      best = d2;
      bi = k;
    }
  }
  return bi;
}

}  // namespace

extern "C" {

// Eq. 10.  nbr[4][n]: up, down, left, right (own index where there is none).
// Returns lambda * L_smooth and accumulates its gradient into dz (nullable).
double orc_smooth(int64_t n, const double* z, const int32_t* nbr, double lambda, double* dz) {
  const double K = 4.0;
  double L = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 4; ++d) {
      const int64_t j = nbr[d * n + i];
      const double r = z[i] - z[j];
      L += r * r;
      if (dz) {
        dz[i] += lambda / K * 2.0 * r;
        dz[j] -= lambda / K * 2.0 * r;
      }
    }
  }
  return lambda / K * L;
}

// Eq. 11.  Returns lambda * L_z and accumulates its gradient into dz (nullable).
double orc_lidar_loss(int64_t n, const double* z, const double* zbar, double lambda, double* dz) {
  double L = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double r = z[i] - zbar[i];
    L += r * r;
    if (dz) dz[i] += 2.0 * lambda * r;
  }
  return lambda * L;
}

// Nearest point (index) in the xy-plane for every surfel, brute force.
void orc_lidar_nn(int64_t n, const float* x, const float* y, int64_t m, const float* px,
                  const float* py, int32_t* idx) {
  for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)nearest_xy((double)x[i], (double)y[i], m, px, py);
}

// Raster cell of each pose position: col = floor((x - x0)/h + 1/2), row likewise.
void orc_pose_pixels(int n_poses, const float* pose, double x0, double y0, float h, int32_t* pix) {
  for (int k = 0; k < n_poses; ++k) {
    const float* p = pose + 12 * k;
    pix[2 * k] = (int32_t)std::floor(((double)p[0] - x0) / (double)h + 0.5);
    pix[2 * k + 1] = (int32_t)std::floor(((double)p[1] - y0) / (double)h + 0.5);
  }
}

// Road mask: a pixel is road iff some pose pixel lies within radius r (disk
// dilation).  Returns the number of road pixels.
int64_t orc_layout_mask(int W, int H, int n_poses, const int32_t* pix, int r, uint8_t* mask) {
  int64_t count = 0;
  for (int row = 0; row < H; ++row) {
    for (int col = 0; col < W; ++col) {
      uint8_t m = 0;
      for (int k = 0; k < n_poses && !m; ++k) {
        const int64_t dx = col - pix[2 * k], dy = row - pix[2 * k + 1];
        if (dx * dx + dy * dy <= (int64_t)r * r) m = 1;
      }
      mask[(int64_t)row * W + col] = m;
      count += m;
    }
  }
  return count;
}

// Surfels at the road pixels, indexed by a running count in row-major order,
// with their grid position, neighbours and pose-based initial height and
// rotation.  pose[k] = x, y, z, R (row-major 3 x 3, columns n1 n2 n3).
// Writes idx[H][W] (-1 off the road) and per surfel x, y, z (binary32),
// q[4][n] (w, x, y, z with w >= 0, binary64) and nbr[4][n].
void orc_layout_build(int W, int H, const uint8_t* mask, double x0, double y0, float h,
                      int n_poses, const float* pose, int64_t n, int32_t* idx, float* x, float* y,
                      float* z, double* q, int32_t* nbr) {
  int64_t c = 0;
  for (int64_t p = 0; p < (int64_t)W * H; ++p) idx[p] = mask[p] ? (int32_t)(c++) : -1;
  std::vector<float> px(n_poses), py(n_poses);
  for (int k = 0; k < n_poses; ++k) {
    px[k] = pose[12 * k];
    py[k] = pose[12 * k + 1];
  }
  for (int row = 0; row < H; ++row) {
    for (int col = 0; col < W; ++col) {
      const int32_t i = idx[(int64_t)row * W + col];
      if (i < 0) continue;
      x[i] = (float)(x0 + (double)col * (double)h);
      y[i] = (float)(y0 + (double)row * (double)h);
      auto at = [&](int rr, int cc) -> int32_t {
        if (rr < 0 || rr >= H || cc < 0 || cc >= W) return i;
        const int32_t j = idx[(int64_t)rr * W + cc];
        return j < 0 ? i : j;
      };
      nbr[0 * n + i] = at(row - 1, col);
      nbr[1 * n + i] = at(row + 1, col);
      nbr[2 * n + i] = at(row, col - 1);
      nbr[3 * n + i] = at(row, col + 1);
      const int64_t k = nearest_xy((double)x[i], (double)y[i], n_poses, px.data(), py.data());
      const float* P = pose + 12 * k;
      // Eq. 4: the surfel lies in the vehicle's xy-plane, n3 = third column of R_v
      const double n31 = P[3 + 2], n32 = P[3 + 5], n33 = P[3 + 8];
      const double t = (n31 * ((double)x[i] - (double)P[0]) + n32 * ((double)y[i] - (double)P[1])) / n33;
      z[i] = (float)((double)P[2] - t);
      // rotation of the nearest pose as a unit quaternion, w >= 0
      const double m00 = P[3], m01 = P[4], m02 = P[5], m10 = P[6], m11 = P[7], m12 = P[8],
                   m20 = P[9], m21 = P[10], m22 = P[11];
      double w, a, b, d;
      const double tr = m00 + m11 + m22;
      if (tr > 0.0) {
        const double s = std::sqrt(tr + 1.0) * 2.0;
        w = 0.25 * s; a = (m21 - m12) / s; b = (m02 - m20) / s; d = (m10 - m01) / s;
      } else if (m00 > m11 && m00 > m22) {
        const double s = std::sqrt(1.0 + m00 - m11 - m22) * 2.0;
        w = (m21 - m12) / s; a = 0.25 * s; b = (m01 + m10) / s; d = (m02 + m20) / s;
      } else if (m11 > m22) {
        const double s = std::sqrt(1.0 + m11 - m00 - m22) * 2.0;
        w = (m02 - m20) / s; a = (m01 + m10) / s; b = 0.25 * s; d = (m12 + m21) / s;
      } else {
        const double s = std::sqrt(1.0 + m22 - m00 - m11) * 2.0;
        w = (m10 - m01) / s; a = (m02 + m20) / s; b = (m12 + m21) / s; d = 0.25 * s;
      }
      if (w < 0.0) { w = -w; a = -a; b = -b; d = -d; }
      q[0 * n + i] = w;
      q[1 * n + i] = a;
      q[2 * n + i] = b;
      q[3 * n + i] = d;
    }
  }
}

}  // extern "C"
