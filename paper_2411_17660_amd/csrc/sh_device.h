// sh_device.h -- device helpers shared by the 3D Gaussian and 2D surfel
// paths of libgsr.so: pose loading, the quaternion gradient, the real
// spherical-harmonics colour basis and its direction gradient, and the view
// direction from the camera centre.
#pragma once
#include "gsr_device.h"

namespace gsr {

__device__ __forceinline__ void load_pose(const float* __restrict__ poses, int f, double W[9],
                                          double tf[3]) {
  const float* P = poses + f * 12;
  W[0] = P[0]; W[1] = P[1]; W[2] = P[2]; tf[0] = P[3];
  W[3] = P[4]; W[4] = P[5]; W[5] = P[6]; tf[1] = P[7];
  W[6] = P[8]; W[7] = P[9]; W[8] = P[10]; tf[2] = P[11];
}

// Gradient of a rotation R(q / |q|) (row-major R[i*3+j]) carried back to the
// raw quaternion q = qn qh, qh = (w, x, y, z) of unit length: dL/dqh from the
// entries of R, then projected on the tangent of the unit sphere and divided
// by |q|.  Writes the four FP32 components to out.
__device__ __forceinline__ void quat_grad(const double qh[4], double qn, const double dR[9],
                                          float* __restrict__ out) {
  const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  double dq[4];
  dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] +
                 w * dR[7] - 2.0 * x * dR[8]);
  dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                 z * dR[7] - 2.0 * y * dR[8]);
  dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] +
                 y * dR[5] + x * dR[6] + y * dR[7]);
  const double pr = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
  for (int a = 0; a < 4; ++a) out[a] = (float)((dq[a] - qh[a] * pr) / qn);
}

// Real spherical harmonics up to degree 3 in the order (l, m = -l..l) with
// the (-1)^|m| phase; coefficients are the textbook normalisations.
constexpr double kY0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kY1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double kY2a = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double kY2b = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double kY2c = 0.5462742152960396;   // sqrt(15/pi)/4
constexpr double kY3a = 0.5900435899266435;   // sqrt(35/(2 pi))/4
constexpr double kY3b = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double kY3c = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double kY3d = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double kY3e = 1.445305721320277;    // sqrt(105/pi)/4

// Basis values Y[k], k < (DEG+1)^2.
template <int DEG>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double* Y) {
  Y[0] = kY0;
  if (DEG < 1) return;
  Y[1] = -kY1 * y; Y[2] = kY1 * z; Y[3] = -kY1 * x;
  if (DEG < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kY2a * x * y;
  Y[5] = -kY2a * y * z;
  Y[6] = kY2b * (2.0 * zz - xx - yy);
  Y[7] = -kY2a * x * z;
  Y[8] = kY2c * (xx - yy);
  if (DEG < 3) return;
  Y[9] = -kY3a * y * (3.0 * xx - yy);
  Y[10] = kY3b * x * y * z;
  Y[11] = -kY3c * y * (4.0 * zz - xx - yy);
  Y[12] = kY3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -kY3c * x * (4.0 * zz - xx - yy);
  Y[14] = kY3e * z * (xx - yy);
  Y[15] = -kY3a * x * (xx - 3.0 * yy);
}

// ddir = sum_k w[k] * grad Y_k(x, y, z), the direction components taken as
// independent variables (the polynomials above differentiated term by term).
template <int DEG>
__device__ __forceinline__ void sh_dir_grad(double x, double y, double z, const double* w,
                                            double* dd) {
  dd[0] = dd[1] = dd[2] = 0.0;
  if (DEG < 1) return;
  dd[0] += -kY1 * w[3];
  dd[1] += -kY1 * w[1];
  dd[2] += kY1 * w[2];
  if (DEG < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  dd[0] += kY2a * y * w[4] - 2.0 * kY2b * x * w[6] - kY2a * z * w[7] + 2.0 * kY2c * x * w[8];
  dd[1] += kY2a * x * w[4] - kY2a * z * w[5] - 2.0 * kY2b * y * w[6] - 2.0 * kY2c * y * w[8];
  dd[2] += -kY2a * y * w[5] + 4.0 * kY2b * z * w[6] - kY2a * x * w[7];
  if (DEG < 3) return;
  dd[0] += -6.0 * kY3a * x * y * w[9] + kY3b * y * z * w[10] + 2.0 * kY3c * x * y * w[11] -
           6.0 * kY3d * x * z * w[12] - kY3c * (4.0 * zz - 3.0 * xx - yy) * w[13] +
           2.0 * kY3e * x * z * w[14] - 3.0 * kY3a * (xx - yy) * w[15];
  dd[1] += -3.0 * kY3a * (xx - yy) * w[9] + kY3b * x * z * w[10] -
           kY3c * (4.0 * zz - xx - 3.0 * yy) * w[11] - 6.0 * kY3d * y * z * w[12] +
           2.0 * kY3c * x * y * w[13] - 2.0 * kY3e * y * z * w[14] + 6.0 * kY3a * x * y * w[15];
  dd[2] += kY3b * x * y * w[10] - 8.0 * kY3c * y * z * w[11] +
           kY3d * (6.0 * zz - 3.0 * xx - 3.0 * yy) * w[12] - 8.0 * kY3c * x * z * w[13] +
           kY3e * (xx - yy) * w[14];
}

// Camera centre C = -R_f^T t_f and the unit direction from it to mu.
__device__ __forceinline__ double view_dir(const double W[9], const double tf[3],
                                           const double mu[3], double dir[3]) {
#pragma clang fp contract(off)
  double d[3];
  for (int i = 0; i < 3; ++i) {
    const double C = -(W[0 * 3 + i] * tf[0] + W[1 * 3 + i] * tf[1] + W[2 * 3 + i] * tf[2]);
    d[i] = mu[i] - C;
  }
  const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; ++i) dir[i] = d[i] / dist;
  return dist;
}

}  // namespace gsr
