// normals.hip -- the normal-consistency term of the surfel objective (the
// L_normal of 2D Gaussian Splatting, which the supplementary's Rendering
// settings add for surfels), forward and gradient in one pass.
//
// Per frame, on the rendered depth D, alpha and normal map n (sum_i w_i n_i):
// each pixel back-projects to P = D K^-1 (x, y, 1); on interior pixels
// (1 <= x <= W-2, 1 <= y <= H-2) the surface normal from depth is
// N = v / |v|, v = dP_y x dP_x with the central differences
// dP_x = P(x+1, y) - P(x-1, y), dP_y = P(x, y+1) - P(x, y-1) (it faces the
// camera for a surface in front of it).  As sum_i w_i = alpha, a pixel's
// sum_i w_i (1 - n_i . N) is alpha - n . N; the frame's term is its mean over
// the (W-2)(H-2) interior pixels, pixels with v = 0 adding 0, and
//   loss = weight * sum_f term_f.
// Gradients (added to the caller's buffers): dL/dalpha = s, dL/dn = -s N on
// interior pixels (s = weight / ((W-2)(H-2))); dL/dD at a pixel gathers the
// stencils of its four neighbours q, which read it through dP_x or dP_y:
// g_v = -s (n_q - N_q (N_q . n_q)) / |v_q|, dL/d(dP_y) = dP_x x g_v,
// dL/d(dP_x) = g_v x dP_y, and dP/dD = K^-1 (x, y, 1).
//
// One thread per pixel; the stencil arithmetic is FP64 (the differences of
// back-projected points cancel to ~2D/f of their size).  Loads of the
// neighbourhood hit the caches; HBM sees each input once and each gradient
// read and written once.  Per-block loss partials are summed in a fixed
// order.
#include "launch.h"

namespace gsr {

namespace {

constexpr int kNcX = 64, kNcY = 4;

struct NcFrame {
  int W, H;
  double fx, fy, cx, cy;
  const float* depth;
  const float* normal;  // 3 planes of W H
};

__device__ __forceinline__ void back_project(const NcFrame& F, int x, int y, double P[3]) {
  const double d = F.depth[(int64_t)y * F.W + x];
  P[0] = d * ((x - F.cx) / F.fx);
  P[1] = d * ((y - F.cy) / F.fy);
  P[2] = d;
}

// The stencil at interior pixel (x, y): dP_x, dP_y, N and |v|; false where
// v = 0.
__device__ __forceinline__ bool depth_normal(const NcFrame& F, int x, int y, double dPx[3],
                                             double dPy[3], double N[3], double& nv) {
  double a[3], b[3];
  back_project(F, x + 1, y, a);
  back_project(F, x - 1, y, b);
  for (int i = 0; i < 3; ++i) dPx[i] = a[i] - b[i];
  back_project(F, x, y + 1, a);
  back_project(F, x, y - 1, b);
  for (int i = 0; i < 3; ++i) dPy[i] = a[i] - b[i];
  const double v[3] = {dPy[1] * dPx[2] - dPy[2] * dPx[1], dPy[2] * dPx[0] - dPy[0] * dPx[2],
                       dPy[0] * dPx[1] - dPy[1] * dPx[0]};
  nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (!(nv > 0.0)) return false;
  for (int i = 0; i < 3; ++i) N[i] = v[i] / nv;
  return true;
}

// dL/d(dP_x) and dL/d(dP_y) of interior pixel q's term (0 where v = 0).
__device__ __forceinline__ void stencil_grad(const NcFrame& F, int qx, int qy, double s,
                                             double gx[3], double gy[3]) {
  double dPx[3], dPy[3], N[3], nv;
  for (int i = 0; i < 3; ++i) gx[i] = gy[i] = 0.0;
  if (!depth_normal(F, qx, qy, dPx, dPy, N, nv)) return;
  const int64_t plane = (int64_t)F.W * F.H;
  const int64_t p = (int64_t)qy * F.W + qx;
  const double n[3] = {F.normal[p], F.normal[plane + p], F.normal[2 * plane + p]};
  const double nn = n[0] * N[0] + n[1] * N[1] + n[2] * N[2];
  double gv[3];
  for (int i = 0; i < 3; ++i) gv[i] = -s * (n[i] - N[i] * nn) / nv;
  gy[0] = dPx[1] * gv[2] - dPx[2] * gv[1];
  gy[1] = dPx[2] * gv[0] - dPx[0] * gv[2];
  gy[2] = dPx[0] * gv[1] - dPx[1] * gv[0];
  gx[0] = gv[1] * dPy[2] - gv[2] * dPy[1];
  gx[1] = gv[2] * dPy[0] - gv[0] * dPy[2];
  gx[2] = gv[0] * dPy[1] - gv[1] * dPy[0];
}

__global__ void __launch_bounds__(kNcX * kNcY) normal_consistency_kernel(
    NcFrame F, const float* __restrict__ alpha, double s, float* __restrict__ g_depth,
    float* __restrict__ g_alpha, float* __restrict__ g_normal, double* __restrict__ part) {
  __shared__ double red[kNcY];
  const int x = blockIdx.x * kNcX + threadIdx.x;
  const int y = blockIdx.y * kNcY + threadIdx.y;
  double term = 0.0;
  if (x < F.W && y < F.H) {
    const int64_t plane = (int64_t)F.W * F.H;
    const int64_t p = (int64_t)y * F.W + x;
    const bool inner = x >= 1 && x <= F.W - 2 && y >= 1 && y <= F.H - 2;
    if (inner) {
      double dPx[3], dPy[3], N[3], nv;
      if (depth_normal(F, x, y, dPx, dPy, N, nv)) {
        const double n[3] = {F.normal[p], F.normal[plane + p], F.normal[2 * plane + p]};
        term = (double)alpha[p] - (n[0] * N[0] + n[1] * N[1] + n[2] * N[2]);
        g_alpha[p] = (float)((double)g_alpha[p] + s);
        for (int i = 0; i < 3; ++i)
          g_normal[i * plane + p] = (float)((double)g_normal[i * plane + p] - s * N[i]);
      }
    }
    // the depth at (x, y) enters the stencils of its interior neighbours
    double gP[3] = {0.0, 0.0, 0.0}, gx[3], gy[3];
    if (x - 1 >= 1 && y >= 1 && y <= F.H - 2) {  // p is q's x+1 point
      stencil_grad(F, x - 1, y, s, gx, gy);
      for (int i = 0; i < 3; ++i) gP[i] += gx[i];
    }
    if (x + 1 <= F.W - 2 && y >= 1 && y <= F.H - 2) {  // p is q's x-1 point
      stencil_grad(F, x + 1, y, s, gx, gy);
      for (int i = 0; i < 3; ++i) gP[i] -= gx[i];
    }
    if (y - 1 >= 1 && x >= 1 && x <= F.W - 2) {  // p is q's y+1 point
      stencil_grad(F, x, y - 1, s, gx, gy);
      for (int i = 0; i < 3; ++i) gP[i] += gy[i];
    }
    if (y + 1 <= F.H - 2 && x >= 1 && x <= F.W - 2) {  // p is q's y-1 point
      stencil_grad(F, x, y + 1, s, gx, gy);
      for (int i = 0; i < 3; ++i) gP[i] -= gy[i];
    }
    const double gd = gP[0] * ((x - F.cx) / F.fx) + gP[1] * ((y - F.cy) / F.fy) + gP[2];
    if (gd != 0.0) g_depth[p] = (float)((double)g_depth[p] + gd);
  }
  for (int o = 32; o > 0; o >>= 1) term += __shfl_xor(term, o, kWave);
  if (threadIdx.x == 0) red[threadIdx.y] = term;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double t = 0.0;
    for (int i = 0; i < kNcY; ++i) t += red[i];
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t * s;
  }
}

__global__ void __launch_bounds__(256) nc_total_kernel(const double* __restrict__ part,
                                                       int64_t n, float* __restrict__ loss) {
  __shared__ double red[256];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) t += part[i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)red[0];
}

}  // namespace

int64_t normal_consistency_blocks(int W, int H) {
  return (int64_t)((W + kNcX - 1) / kNcX) * ((H + kNcY - 1) / kNcY);
}

void launch_normal_consistency(hipStream_t st, int F, const gsr_camera* cams,
                               const float* depth, const float* alpha, const float* normal,
                               float weight, double* part, float* loss, float* g_depth,
                               float* g_alpha, float* g_normal) {
  int64_t off = 0, boff = 0;
  for (int f = 0; f < F; ++f) {
    const gsr_camera& c = cams[f];
    const int64_t HW = (int64_t)c.width * c.height;
    const int64_t inner = (int64_t)(c.width - 2) * (c.height - 2);
    const double s = (c.width > 2 && c.height > 2) ? (double)weight / (double)inner : 0.0;
    NcFrame fr{c.width, c.height, c.fx, c.fy, c.cx, c.cy, depth + off, normal + 3 * off};
    const dim3 grid((unsigned)((c.width + kNcX - 1) / kNcX),
                    (unsigned)((c.height + kNcY - 1) / kNcY));
    if (HW > 0)
      hipLaunchKernelGGL(normal_consistency_kernel, grid, dim3(kNcX, kNcY), 0, st, fr,
                         alpha + off, s, g_depth + off, g_alpha + off, g_normal + 3 * off,
                         part + boff);
    off += HW;
    boff += normal_consistency_blocks(c.width, c.height);
  }
  hipLaunchKernelGGL(nc_total_kernel, dim3(1), dim3(256), 0, st, part, boff, loss);
}

}  // namespace gsr
