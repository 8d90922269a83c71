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
// back-projected points cancel to ~2D/f of their size).  Each block stages
// its depths in LDS and evaluates each stencil once, so HBM sees each input
// about once and each gradient read and written once.  Per-block loss
// partials are summed in a fixed order.
#include "launch.h"

namespace gsr {

namespace {

constexpr int kNcX = 64, kNcY = 4;

struct NcFrame {
  int W, H;
  double ifx, ify, cx, cy;  // 1/f_x, 1/f_y and the principal point
  const float* depth;
  const float* normal;  // 3 planes of W H
};

// One block covers kNcX x kNcY pixels.  It stages the depths of its tile
// with a 2-pixel halo in LDS (the stencils of the pixels around the tile read
// that far), evaluates the stencil once for each pixel of the tile with a
// 1-pixel halo (N, dL/d(dP_x), dL/d(dP_y) into LDS), then each pixel takes
// its own term and gathers its depth gradient from its four neighbours'
// stencils.
constexpr int kHx = kNcX + 4, kHy = kNcY + 4;  // depth tile with halo 2
constexpr int kSx = kNcX + 2, kSy = kNcY + 2;  // stencil tile with halo 1

__global__ void __launch_bounds__(kNcX * kNcY) normal_consistency_kernel(
    NcFrame F, const float* __restrict__ alpha, double s, float* __restrict__ g_depth,
    float* __restrict__ g_alpha, float* __restrict__ g_normal, double* __restrict__ part) {
  __shared__ float dep[kHy][kHx];
  __shared__ double sgx[kSy][kSx][3], sgy[kSy][kSx][3], sN[kSy][kSx][3];
  __shared__ bool sok[kSy][kSx];
  __shared__ double red[kNcY];
  const int tid = threadIdx.y * kNcX + threadIdx.x;
  const int bx = blockIdx.x * kNcX, by = blockIdx.y * kNcY;
  const int64_t plane = (int64_t)F.W * F.H;
  // depths of the tile and its 2-pixel halo (0 outside the image: only
  // interior stencils read them, and those never reach outside)
  for (int i = tid; i < kHx * kHy; i += kNcX * kNcY) {
    const int hx = i % kHx, hy = i / kHx;
    const int x = bx + hx - 2, y = by + hy - 2;
    dep[hy][hx] = (x >= 0 && x < F.W && y >= 0 && y < F.H) ? F.depth[(int64_t)y * F.W + x]
                                                           : 0.0f;
  }
  __syncthreads();
  // the stencils of the tile and its 1-pixel halo
  for (int i = tid; i < kSx * kSy; i += kNcX * kNcY) {
    const int sx = i % kSx, sy = i / kSx;
    const int x = bx + sx - 1, y = by + sy - 1;
    bool ok = false;
    double gx[3] = {0, 0, 0}, gy[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    if (x >= 1 && x <= F.W - 2 && y >= 1 && y <= F.H - 2) {
      const int hx = sx + 1, hy = sy + 1;  // (x, y) in the depth tile
      double P1[3], P0[3], dPx[3], dPy[3];
      auto bp = [&](int ox, int oy, double* P) {
        const double d = dep[hy + oy][hx + ox];
        P[0] = d * ((x + ox - F.cx) * F.ifx);
        P[1] = d * ((y + oy - F.cy) * F.ify);
        P[2] = d;
      };
      bp(1, 0, P1);
      bp(-1, 0, P0);
      for (int k = 0; k < 3; ++k) dPx[k] = P1[k] - P0[k];
      bp(0, 1, P1);
      bp(0, -1, P0);
      for (int k = 0; k < 3; ++k) dPy[k] = P1[k] - P0[k];
      const double v[3] = {dPy[1] * dPx[2] - dPy[2] * dPx[1], dPy[2] * dPx[0] - dPy[0] * dPx[2],
                           dPy[0] * dPx[1] - dPy[1] * dPx[0]};
      const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (nv > 0.0) {
        ok = true;
        const double inv = 1.0 / nv;
        for (int k = 0; k < 3; ++k) N[k] = v[k] * inv;
        const int64_t p = (int64_t)y * F.W + x;
        const double n[3] = {F.normal[p], F.normal[plane + p], F.normal[2 * plane + p]};
        const double nn = n[0] * N[0] + n[1] * N[1] + n[2] * N[2];
        double gv[3];
        for (int k = 0; k < 3; ++k) gv[k] = -s * (n[k] - N[k] * nn) * inv;
        gy[0] = dPx[1] * gv[2] - dPx[2] * gv[1];
        gy[1] = dPx[2] * gv[0] - dPx[0] * gv[2];
        gy[2] = dPx[0] * gv[1] - dPx[1] * gv[0];
        gx[0] = gv[1] * dPy[2] - gv[2] * dPy[1];
        gx[1] = gv[2] * dPy[0] - gv[0] * dPy[2];
        gx[2] = gv[0] * dPy[1] - gv[1] * dPy[0];
      }
    }
    sok[sy][sx] = ok;
    for (int k = 0; k < 3; ++k) {
      sgx[sy][sx][k] = gx[k];
      sgy[sy][sx][k] = gy[k];
      sN[sy][sx][k] = N[k];
    }
  }
  __syncthreads();
  const int x = bx + threadIdx.x, y = by + threadIdx.y;
  double term = 0.0;
  if (x < F.W && y < F.H) {
    const int64_t p = (int64_t)y * F.W + x;
    const int sx = threadIdx.x + 1, sy = threadIdx.y + 1;
    if (sok[sy][sx]) {
      const double* N = sN[sy][sx];
      const double n[3] = {F.normal[p], F.normal[plane + p], F.normal[2 * plane + p]};
      term = (double)alpha[p] - (n[0] * N[0] + n[1] * N[1] + n[2] * N[2]);
      g_alpha[p] = (float)((double)g_alpha[p] + s);
      for (int k = 0; k < 3; ++k)
        g_normal[k * plane + p] = (float)((double)g_normal[k * plane + p] - s * N[k]);
    }
    // p is the x+1 point of its left neighbour's stencil, the x-1 point of
    // its right neighbour's, and likewise in y (non-interior stencils are 0)
    double gP[3];
    for (int k = 0; k < 3; ++k)
      gP[k] = sgx[sy][sx - 1][k] - sgx[sy][sx + 1][k] + sgy[sy - 1][sx][k] - sgy[sy + 1][sx][k];
    const double gd = gP[0] * ((x - F.cx) * F.ifx) + gP[1] * ((y - F.cy) * F.ify) + gP[2];
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

constexpr int kNcTotalThreads = 1024;

// One block: thread t sums the partials t, t + 1024, ...; each wave sums its
// lanes with a butterfly and the 16 wave totals are added in wave order.
__global__ void __launch_bounds__(kNcTotalThreads) nc_total_kernel(const double* __restrict__ part,
                                                                  int64_t n,
                                                                  float* __restrict__ loss) {
  __shared__ double red[kNcTotalThreads / kWave];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kNcTotalThreads) t += part[i];
  for (int o = kWave / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, kWave);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kNcTotalThreads / kWave; ++i) s += red[i];
    loss[0] = (float)s;
  }
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
    NcFrame fr{c.width,      c.height, 1.0 / (double)c.fx, 1.0 / (double)c.fy, c.cx, c.cy,
               depth + off, normal + 3 * off};
    const dim3 grid((unsigned)((c.width + kNcX - 1) / kNcX),
                    (unsigned)((c.height + kNcY - 1) / kNcY));
    if (HW > 0)
      hipLaunchKernelGGL(normal_consistency_kernel, grid, dim3(kNcX, kNcY), 0, st, fr,
                         alpha + off, s, g_depth + off, g_alpha + off, g_normal + 3 * off,
                         part + boff);
    off += HW;
    boff += normal_consistency_blocks(c.width, c.height);
  }
  hipLaunchKernelGGL(nc_total_kernel, dim3(1), dim3(kNcTotalThreads), 0, st, part, boff, loss);
}

}  // namespace gsr
