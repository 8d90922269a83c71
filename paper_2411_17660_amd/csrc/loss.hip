// loss.hip -- L1 rendering loss and its upstream gradient (A7).
//
// The mapper's rendering objective (DROID-Splat eqn rnd_loss) mixes an L1
// colour term, an SSIM term and an L1 depth term.  This kernel computes the
// L1 parts for a batch of frames:
//   L = sum_f [ mean_{c,p} |RGB - RGB*| + w_d * mean_{p in m_f} |D - D*| ],
//   m_f = {p : D*_p > 0},  sign(0) = 0,
// and writes dL/dRGB = sign(RGB - RGB*) / (3 H W), dL/dD = w_d sign(D - D*)
// [p in m_f] / |m_f|, dL/dAlpha = 0.  Per-block partial sums are combined in
// FP64 in a fixed order.
#include "launch.h"

namespace gsr {

constexpr int kLossThreads = 256;
constexpr int kLossItems = 8;

__global__ void __launch_bounds__(kLossThreads) loss_partial_kernel(
    const FrameDesc* __restrict__ frames, const float* __restrict__ rgb,
    const float* __restrict__ depth, const float* __restrict__ t_rgb,
    const float* __restrict__ t_depth, int blocks_x, double* __restrict__ part) {
  __shared__ double red[3][kLossThreads];
  const int f = blockIdx.y;
  const FrameDesc fr = frames[f];
  const int64_t HW = (int64_t)fr.width * fr.height;
  double s_rgb = 0.0, s_d = 0.0, s_m = 0.0;
  for (int k = 0; k < kLossItems; ++k) {
    const int64_t p = ((int64_t)blockIdx.x * kLossItems + k) * kLossThreads + threadIdx.x;
    if (p >= HW) break;
    const int64_t q = fr.pixel_offset + p;
    const int64_t qc = 3 * fr.pixel_offset + p;
    for (int c = 0; c < 3; ++c) s_rgb += fabs((double)rgb[qc + c * HW] - (double)t_rgb[qc + c * HW]);
    if (t_depth[q] > 0.0f) {
      s_d += fabs((double)depth[q] - (double)t_depth[q]);
      s_m += 1.0;
    }
  }
  red[0][threadIdx.x] = s_rgb;
  red[1][threadIdx.x] = s_d;
  red[2][threadIdx.x] = s_m;
  __syncthreads();
  for (int o = kLossThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int j = 0; j < 3; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[((int64_t)f * blocks_x + blockIdx.x) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// One block: per-frame totals -> loss and per-frame scale factors.
__global__ void __launch_bounds__(kLossThreads) loss_finalize_kernel(
    const FrameDesc* __restrict__ frames, int n_frames, int blocks_x,
    const double* __restrict__ part, float depth_weight, float* __restrict__ loss,
    float* __restrict__ scale /* [F][2]: 1/(3HW), w_d/|m| */) {
  __shared__ double red[3][kLossThreads];
  double total = 0.0;
  for (int f = 0; f < n_frames; ++f) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < blocks_x; b += kLossThreads)
      for (int j = 0; j < 3; ++j) s[j] += part[((int64_t)f * blocks_x + b) * 3 + j];
    for (int j = 0; j < 3; ++j) red[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int o = kLossThreads / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o)
        for (int j = 0; j < 3; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + o];
      __syncthreads();
    }
    const double HW = (double)frames[f].width * frames[f].height;
    const double m = red[2][0];
    total += red[0][0] / (3.0 * HW) + (m > 0.0 ? (double)depth_weight * red[1][0] / m : 0.0);
    if (threadIdx.x == 0) {
      scale[2 * f] = (float)(1.0 / (3.0 * HW));
      scale[2 * f + 1] = m > 0.0 ? (float)((double)depth_weight / m) : 0.0f;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)total;
}

__device__ __forceinline__ float sgnf(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

__global__ void __launch_bounds__(kLossThreads) loss_grad_kernel(
    const FrameDesc* __restrict__ frames, const float* __restrict__ rgb,
    const float* __restrict__ depth, const float* __restrict__ t_rgb,
    const float* __restrict__ t_depth, const float* __restrict__ scale,
    float* __restrict__ g_rgb, float* __restrict__ g_depth, float* __restrict__ g_alpha) {
  const int f = blockIdx.y;
  const FrameDesc fr = frames[f];
  const int64_t HW = (int64_t)fr.width * fr.height;
  const float sc = scale[2 * f], sd = scale[2 * f + 1];
  for (int k = 0; k < kLossItems; ++k) {
    const int64_t p = ((int64_t)blockIdx.x * kLossItems + k) * kLossThreads + threadIdx.x;
    if (p >= HW) break;
    const int64_t q = fr.pixel_offset + p;
    const int64_t qc = 3 * fr.pixel_offset + p;
    for (int c = 0; c < 3; ++c) g_rgb[qc + c * HW] = sgnf(rgb[qc + c * HW] - t_rgb[qc + c * HW]) * sc;
    g_depth[q] = t_depth[q] > 0.0f ? sgnf(depth[q] - t_depth[q]) * sd : 0.0f;
    g_alpha[q] = 0.0f;
  }
}

int loss_blocks_x(int64_t max_hw) {
  return (int)((max_hw + (int64_t)kLossThreads * kLossItems - 1) / ((int64_t)kLossThreads * kLossItems));
}

void launch_loss_l1(hipStream_t st, int F, int blocks_x, const FrameDesc* frames,
                    const float* rgb, const float* depth, const float* t_rgb,
                    const float* t_depth, float depth_weight, double* part, float* scale,
                    float* loss, float* g_rgb, float* g_depth, float* g_alpha) {
  const dim3 grid((unsigned)blocks_x, (unsigned)F);
  hipLaunchKernelGGL(loss_partial_kernel, grid, dim3(kLossThreads), 0, st, frames, rgb, depth,
                     t_rgb, t_depth, blocks_x, part);
  hipLaunchKernelGGL(loss_finalize_kernel, dim3(1), dim3(kLossThreads), 0, st, frames, F,
                     blocks_x, part, depth_weight, loss, scale);
  hipLaunchKernelGGL(loss_grad_kernel, grid, dim3(kLossThreads), 0, st, frames, rgb, depth,
                     t_rgb, t_depth, scale, g_rgb, g_depth, g_alpha);
}

}  // namespace gsr
