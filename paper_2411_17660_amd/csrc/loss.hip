// loss.hip -- L1 rendering loss and its upstream gradient (A7).
//
// The mapper's rendering objective (DROID-Splat eqn rnd_loss) mixes an L1
// colour term, an SSIM term and an L1 depth term.  This kernel computes the
// L1 parts for a batch of frames:
//   L = sum_f [ mean_{c,p} |RGB - RGB*| + w_d * mean_{p in m_f} |D - D*| ],
//   m_f = {p : D*_p > 0},  sign(0) = 0,
// and writes dL/dRGB = sign(RGB - RGB*) / (3 H W), dL/dD = w_d sign(D - D*)
// [p in m_f] / |m_f|, dL/dAlpha = 0.  Per-block partial sums are combined in
// FP64 in a fixed order.  The gradients need only the signs and |m_f|, so a
// first pass counts m_f from the target depths alone, and one pass over the
// images then writes the gradients and the loss partials together.
#include "launch.h"

#include <mutex>

namespace gsr {

// Fixed scratch of the allocation-free L1 loss (gsr_loss_l1_noalloc): the
// per-block partial sums and the per-frame scale factors of launch_loss_l1,
// in a static device array (one copy per GPU, held until the process ends)
// instead of context workspace.  Every byte a call reads was written by that
// call's own kernels first, so nothing needs clearing between calls; calls
// that overlap on one GPU share the array and race.
constexpr size_t kLossScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Resolves the device address of `scratch` on `device` (which must be the
// current device) once and caches it; later calls return the cached address.
hipError_t loss_scratch_init(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

size_t loss_scratch_bytes() { return kLossScratchBytes; }

constexpr int kLossThreads = 256;
constexpr int kLossItems = 8;

__device__ __forceinline__ float sgnf(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

// Sums v[0..2] over a block's 256 threads into red[j][0] (FP64, fixed
// order): a butterfly per wave, then the four wave totals in wave order.
__device__ __forceinline__ void block_sum3(double (*red)[kLossThreads], double v[3]) {
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  for (int j = 0; j < 3; ++j)
    for (int o = kWave / 2; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o, kWave);
  if (lane == 0)
    for (int j = 0; j < 3; ++j) red[j][wv] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
      for (int i = 0; i < kLossThreads / kWave; ++i) t += red[j][i];
      red[j][0] = t;
    }
  __syncthreads();
}

// |m_f| per block: part[f][b][2] = #{p : D*_p > 0}
__global__ void __launch_bounds__(kLossThreads) loss_mask_kernel(
    const FrameDesc* __restrict__ frames, const float* __restrict__ t_depth, int blocks_x,
    double* __restrict__ part) {
  __shared__ double red[3][kLossThreads];
  const int f = blockIdx.y;
  const FrameDesc fr = frames[f];
  const int64_t HW = (int64_t)fr.width * fr.height;
  double s_m = 0.0;
  for (int k = 0; k < kLossItems; ++k) {
    const int64_t p = ((int64_t)blockIdx.x * kLossItems + k) * kLossThreads + threadIdx.x;
    if (p >= HW) break;
    if (t_depth[fr.pixel_offset + p] > 0.0f) s_m += 1.0;
  }
  double v[3] = {0.0, 0.0, s_m};
  block_sum3(red, v);
  if (threadIdx.x == 0) part[((int64_t)f * blocks_x + blockIdx.x) * 3 + 2] = red[2][0];
}

// Sum over b of part[f][b][j] by one wave (lanes stride over the blocks,
// then a butterfly), in FP64.
__device__ __forceinline__ double wave_part_sum(const double* __restrict__ part, int f,
                                                int blocks_x, int j, int lane) {
  double s = 0.0;
  for (int b = lane; b < blocks_x; b += kWave) s += part[((int64_t)f * blocks_x + b) * 3 + j];
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  return s;
}

constexpr int kLossWaves = kLossThreads / kWave;

// One block, one wave per frame in turn: per-frame scale factors from the
// mask counts.
__global__ void __launch_bounds__(kLossThreads) loss_scale_kernel(
    const FrameDesc* __restrict__ frames, int n_frames, int blocks_x,
    const double* __restrict__ part, float depth_weight,
    float* __restrict__ scale /* [F][2]: 1/(3HW), w_d/|m| */) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (int f = w; f < n_frames; f += kLossWaves) {
    const double m = wave_part_sum(part, f, blocks_x, 2, lane);
    if (lane == 0) {
      const double HW = (double)frames[f].width * frames[f].height;
      scale[2 * f] = (float)(1.0 / (3.0 * HW));
      scale[2 * f + 1] = m > 0.0 ? (float)((double)depth_weight / m) : 0.0f;
    }
  }
}

// The gradients, and the L1 partial sums part[f][b][0..1].
__global__ void __launch_bounds__(kLossThreads) loss_partial_grad_kernel(
    const FrameDesc* __restrict__ frames, const float* __restrict__ rgb,
    const float* __restrict__ depth, const float* __restrict__ t_rgb,
    const float* __restrict__ t_depth, const float* __restrict__ scale, int blocks_x,
    double* __restrict__ part, float* __restrict__ g_rgb, float* __restrict__ g_depth,
    float* __restrict__ g_alpha) {
  __shared__ double red[3][kLossThreads];
  const int f = blockIdx.y;
  const FrameDesc fr = frames[f];
  const int64_t HW = (int64_t)fr.width * fr.height;
  const float sc = scale[2 * f], sd = scale[2 * f + 1];
  double s_rgb = 0.0, s_d = 0.0;
  for (int k = 0; k < kLossItems; ++k) {
    const int64_t p = ((int64_t)blockIdx.x * kLossItems + k) * kLossThreads + threadIdx.x;
    if (p >= HW) break;
    const int64_t q = fr.pixel_offset + p;
    const int64_t qc = 3 * fr.pixel_offset + p;
    for (int c = 0; c < 3; ++c) {
      const float x = rgb[qc + c * HW], t = t_rgb[qc + c * HW];
      s_rgb += fabs((double)x - (double)t);
      g_rgb[qc + c * HW] = sgnf(x - t) * sc;
    }
    const float d = depth[q], td = t_depth[q];
    if (td > 0.0f) s_d += fabs((double)d - (double)td);
    g_depth[q] = td > 0.0f ? sgnf(d - td) * sd : 0.0f;
    g_alpha[q] = 0.0f;
  }
  double v[3] = {s_rgb, s_d, 0.0};
  block_sum3(red, v);
  if (threadIdx.x < 2) part[((int64_t)f * blocks_x + blockIdx.x) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// One block: the loss.  Wave w sums the terms of frames w, w + 4, ... in
// order, and the four wave totals are added in wave order.
__global__ void __launch_bounds__(kLossThreads) loss_finalize_kernel(
    const FrameDesc* __restrict__ frames, int n_frames, int blocks_x,
    const double* __restrict__ part, float depth_weight, float* __restrict__ loss) {
  __shared__ double wsum[kLossWaves];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double total = 0.0;
  for (int f = w; f < n_frames; f += kLossWaves) {
    const double s_rgb = wave_part_sum(part, f, blocks_x, 0, lane);
    const double s_d = wave_part_sum(part, f, blocks_x, 1, lane);
    const double m = wave_part_sum(part, f, blocks_x, 2, lane);
    const double HW = (double)frames[f].width * frames[f].height;
    total += s_rgb / (3.0 * HW) + (m > 0.0 ? (double)depth_weight * s_d / m : 0.0);
  }
  if (lane == 0) wsum[w] = total;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kLossWaves; ++i) t += wsum[i];
    *loss = (float)t;
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
  hipLaunchKernelGGL(loss_mask_kernel, grid, dim3(kLossThreads), 0, st, frames, t_depth, blocks_x,
                     part);
  hipLaunchKernelGGL(loss_scale_kernel, dim3(1), dim3(kLossThreads), 0, st, frames, F, blocks_x,
                     part, depth_weight, scale);
  hipLaunchKernelGGL(loss_partial_grad_kernel, grid, dim3(kLossThreads), 0, st, frames, rgb,
                     depth, t_rgb, t_depth, scale, blocks_x, part, g_rgb, g_depth, g_alpha);
  hipLaunchKernelGGL(loss_finalize_kernel, dim3(1), dim3(kLossThreads), 0, st, frames, F,
                     blocks_x, part, depth_weight, loss);
}

}  // namespace gsr
