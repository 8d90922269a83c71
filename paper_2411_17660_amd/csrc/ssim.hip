// ssim.hip -- the mapper's rendering loss with its SSIM term, forward and
// backward (DROID-Splat eqn rnd_loss, Sec. 3.3; lambda2 = 0.2 in
// supplementary S1.2).  Per frame f of the batch,
//   L_f = l1 [ (1 - l2) mean|I - I*| + l2 (1 - SSIM(I, I*)) ]
//       + (1 - l1) mean_{Z* > 0} |Z - Z*|,
// SSIM being Wang et al.'s index with an 11 x 11 Gaussian window
// (sigma 1.5, weights summing to 1), C1 = 0.01^2, C2 = 0.03^2, window sums
// taken with zero padding, averaged over the 3 channels and all pixels.
//
// Two passes over 32 x 16 output tiles of one colour plane each:
//  - ssim_fwd_kernel stages the plane and its target with a 5-pixel halo in
//    LDS, takes the five window sums (w*x, w*y, w*x^2, w*y^2, w*xy) as a
//    horizontal then a vertical 11-tap pass, evaluates the SSIM map and
//    writes, per pixel, its derivatives A = dS/dmu_x, B = dS/d(w*x^2) and
//    C = dS/d(w*xy); it also sums S, |x - y| and (channel 0) the depth
//    terms of its tile into a per-tile record;
//  - ssim_loss_finalize_kernel sums the records of each frame in a fixed
//    order into the loss and the per-frame gradient scales;
//  - ssim_bwd_kernel applies the adjoint window: with the window symmetric,
//    d(sum S)/dx = w*A + 2 x (w*B) + y (w*C), the window sums again taken
//    as two 11-tap passes over A, B, C staged with a halo.
// The window sums and the map are evaluated in FP64: E[x^2] - mu^2 and the
// adjoint's sum of +-(2 x B + y C) terms cancel by up to three orders of
// magnitude where the image is flat (B, C ~ 1/C2), which FP32 would turn
// into errors of 1e-4 relative to the gradient.  Inputs and outputs are FP32.
#include <cmath>

#include "launch.h"

namespace gsr {

namespace {

constexpr int kR = 5;                  // window radius (11 x 11)
constexpr int kTaps = 2 * kR + 1;
constexpr int kTW = 32, kTH = 16;      // output tile
constexpr int kInW = kTW + 2 * kR;     // 42: staged columns
constexpr int kInH = kTH + 2 * kR;     // 26: staged rows
constexpr int kThreads = 256;
constexpr int kRowsPerThread = kTW * kTH / kThreads;  // 2 outputs per thread, one column
static_assert(kRowsPerThread * kThreads == kTW * kTH, "tile must split evenly");
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

struct Window {
  double g[kTaps];
};

// Tile t of a frame's plane: grid x is padded to a multiple of 8 and
// remapped so that each XCD (block id mod 8) takes one contiguous run of
// tiles, whose halos then meet in that XCD's L2.
__device__ __forceinline__ int tile_of(int bx, int tiles_pad) {
  return (bx & 7) * (tiles_pad >> 3) + (bx >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums n values per thread over the block; thread 0 gets the totals.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double (*red)[N]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) red[wv][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kThreads / 64; ++w)
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] += red[w][k];
}

__device__ __forceinline__ double sgn(double d) { return d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0); }

__global__ void __launch_bounds__(kThreads) ssim_fwd_kernel(
    const FrameDesc* __restrict__ frames, int tiles_pad, Window win,
    const float* __restrict__ rgb, const float* __restrict__ t_rgb,
    const float* __restrict__ depth, const float* __restrict__ t_depth, int64_t plane_stride,
    double* __restrict__ part, double* __restrict__ tile_sums /* [F][3][tiles_pad][4] */) {
  __shared__ float xs[kInH][kInW + 1], ys[kInH][kInW + 1];
  __shared__ double hs[5][kInH][kTW];
  __shared__ double red[kThreads / 64][4];
  const int f = blockIdx.z, c = blockIdx.y;
  const int t = tile_of(blockIdx.x, tiles_pad);
  const FrameDesc fr = frames[f];
  const int W = fr.width, H = fr.height;
  const int ntx = (W + kTW - 1) / kTW, nty = (H + kTH - 1) / kTH;
  double* out = tile_sums + (((int64_t)f * 3 + c) * tiles_pad + blockIdx.x) * 4;
  if (t >= ntx * nty) {
    if (threadIdx.x < 4) out[threadIdx.x] = 0.0;
    return;
  }
  const int x0 = (t % ntx) * kTW, y0 = (t / ntx) * kTH;
  const int64_t HW = (int64_t)W * H;
  const int64_t po = 3 * fr.pixel_offset + c * HW;  // first value of this plane
  for (int k = threadIdx.x; k < kInH * kInW; k += kThreads) {
    const int r = k / kInW, q = k % kInW;
    const int gy = y0 - kR + r, gx = x0 - kR + q;
    float xv = 0.0f, yv = 0.0f;
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      xv = rgb[po + (int64_t)gy * W + gx];
      yv = t_rgb[po + (int64_t)gy * W + gx];
    }
    xs[r][q] = xv;
    ys[r][q] = yv;
  }
  __syncthreads();
  // horizontal pass: staged rows x output columns
  for (int k = threadIdx.x; k < kInH * kTW; k += kThreads) {
    const int r = k / kTW, j = k % kTW;
    double sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
    for (int d = 0; d < kTaps; ++d) {
      const double xv = xs[r][j + d], yv = ys[r][j + d];
      const double gx = win.g[d] * xv, gy = win.g[d] * yv;
      sx += gx;
      sy += gy;
      sxx = fma(gx, xv, sxx);
      syy = fma(gy, yv, syy);
      sxy = fma(gx, yv, sxy);
    }
    hs[0][r][j] = sx;
    hs[1][r][j] = sy;
    hs[2][r][j] = sxx;
    hs[3][r][j] = syy;
    hs[4][r][j] = sxy;
  }
  __syncthreads();
  // vertical pass: one column, kRowsPerThread consecutive output rows
  const int j = threadIdx.x % kTW, i0 = (threadIdx.x / kTW) * kRowsPerThread;
  double v[5][kRowsPerThread];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
#pragma unroll
    for (int o = 0; o < kRowsPerThread; ++o) v[m][o] = 0.0;
#pragma unroll
    for (int d = 0; d < kTaps + kRowsPerThread - 1; ++d) {
      const double h = hs[m][i0 + d][j];
#pragma unroll
      for (int o = 0; o < kRowsPerThread; ++o)
        if (d - o >= 0 && d - o < kTaps) v[m][o] = fma(win.g[d - o], h, v[m][o]);
    }
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // sum S, sum |x - y|, sum |z - z*|, valid depths
  const int gx = x0 + j;
#pragma unroll
  for (int o = 0; o < kRowsPerThread; ++o) {
    const int gy = y0 + i0 + o;
    if (gx >= W || gy >= H) continue;
    const double mx = v[0][o], my = v[1][o];
    const double vx = v[2][o] - mx * mx, vy = v[3][o] - my * my, cxy = v[4][o] - mx * my;
    const double l_num = 2.0 * mx * my + kC1, l_den = mx * mx + my * my + kC1;
    const double c_num = 2.0 * cxy + kC2, c_den = vx + vy + kC2;
    const double rinv = 1.0 / (l_den * c_den);
    const double S = l_num * c_num * rinv;
    const double dS_dmu = c_num * c_den * rinv * rinv * (2.0 * my * l_den - 2.0 * mx * l_num);
    const double dS_dvar = -S * l_den * rinv;
    const double dS_dcov = 2.0 * l_num * rinv;
    const int64_t idx = po + (int64_t)gy * W + gx;
    part[idx] = dS_dmu - 2.0 * mx * dS_dvar - my * dS_dcov;
    part[idx + plane_stride] = dS_dvar;
    part[idx + 2 * plane_stride] = dS_dcov;
    acc[0] += S;
    acc[1] += fabs((double)xs[i0 + o + kR][j + kR] - (double)ys[i0 + o + kR][j + kR]);
    if (c == 0) {
      const int64_t q = fr.pixel_offset + (int64_t)gy * W + gx;
      const float tz = t_depth[q];
      if (tz > 0.0f) {
        acc[2] += fabs((double)depth[q] - (double)tz);
        acc[3] += 1.0;
      }
    }
  }
  block_sums<4>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out[k] = acc[k];
}

// One block: per-frame totals in a fixed order -> loss, per-frame SSIM and
// the gradient scales [F][3] = (l1 (1-l2) / 3HW, l1 l2 / 3HW, (1-l1) / |m|).
__global__ void __launch_bounds__(kThreads) ssim_loss_finalize_kernel(
    const FrameDesc* __restrict__ frames, int n_frames, int tiles_pad,
    const double* __restrict__ tile_sums, double lambda1, double lambda2,
    float* __restrict__ loss, float* __restrict__ ssim, double* __restrict__ scale) {
  __shared__ double red[kThreads / 64][4];
  double total = 0.0;
  const int per_frame = 3 * tiles_pad;
  for (int f = 0; f < n_frames; ++f) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < per_frame; b += kThreads)
      for (int k = 0; k < 4; ++k) s[k] += tile_sums[((int64_t)f * per_frame + b) * 4 + k];
    block_sums<4>(s, red);
    if (threadIdx.x == 0) {
      const double n3 = 3.0 * (double)frames[f].width * (double)frames[f].height;
      const double ss = s[0] / n3;
      total += lambda1 * ((1.0 - lambda2) * s[1] / n3 + lambda2 * (1.0 - ss)) +
               (s[3] > 0.0 ? (1.0 - lambda1) * s[2] / s[3] : 0.0);
      if (ssim) ssim[f] = (float)ss;
      scale[3 * f] = lambda1 * (1.0 - lambda2) / n3;
      scale[3 * f + 1] = lambda1 * lambda2 / n3;
      scale[3 * f + 2] = s[3] > 0.0 ? (1.0 - lambda1) / s[3] : 0.0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)total;
}

__global__ void __launch_bounds__(kThreads) ssim_bwd_kernel(
    const FrameDesc* __restrict__ frames, int tiles_pad, Window win,
    const float* __restrict__ rgb, const float* __restrict__ t_rgb,
    const float* __restrict__ depth, const float* __restrict__ t_depth, int64_t plane_stride,
    const double* __restrict__ part, const double* __restrict__ scale,
    float* __restrict__ g_rgb, float* __restrict__ g_depth, float* __restrict__ g_alpha) {
  __shared__ double as[3][kInH][kInW];
  __shared__ double hs[3][kInH][kTW];
  const int f = blockIdx.z, c = blockIdx.y;
  const int t = tile_of(blockIdx.x, tiles_pad);
  const FrameDesc fr = frames[f];
  const int W = fr.width, H = fr.height;
  const int ntx = (W + kTW - 1) / kTW, nty = (H + kTH - 1) / kTH;
  if (t >= ntx * nty) return;
  const int x0 = (t % ntx) * kTW, y0 = (t / ntx) * kTH;
  const int64_t HW = (int64_t)W * H;
  const int64_t po = 3 * fr.pixel_offset + c * HW;
  for (int k = threadIdx.x; k < kInH * kInW; k += kThreads) {
    const int r = k / kInW, q = k % kInW;
    const int gy = y0 - kR + r, gx = x0 - kR + q;
    double a = 0.0, b = 0.0, cc = 0.0;
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      const int64_t idx = po + (int64_t)gy * W + gx;
      a = part[idx];
      b = part[idx + plane_stride];
      cc = part[idx + 2 * plane_stride];
    }
    as[0][r][q] = a;
    as[1][r][q] = b;
    as[2][r][q] = cc;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kInH * kTW; k += kThreads) {
    const int r = k / kTW, j = k % kTW;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int d = 0; d < kTaps; ++d) {
      s0 = fma(win.g[d], as[0][r][j + d], s0);
      s1 = fma(win.g[d], as[1][r][j + d], s1);
      s2 = fma(win.g[d], as[2][r][j + d], s2);
    }
    hs[0][r][j] = s0;
    hs[1][r][j] = s1;
    hs[2][r][j] = s2;
  }
  __syncthreads();
  const int j = threadIdx.x % kTW, i0 = (threadIdx.x / kTW) * kRowsPerThread;
  double v[3][kRowsPerThread];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
#pragma unroll
    for (int o = 0; o < kRowsPerThread; ++o) v[m][o] = 0.0;
#pragma unroll
    for (int d = 0; d < kTaps + kRowsPerThread - 1; ++d) {
      const double h = hs[m][i0 + d][j];
#pragma unroll
      for (int o = 0; o < kRowsPerThread; ++o)
        if (d - o >= 0 && d - o < kTaps) v[m][o] = fma(win.g[d - o], h, v[m][o]);
    }
  }
  const double s_l1 = scale[3 * f], s_ss = scale[3 * f + 1], s_d = scale[3 * f + 2];
  const int gx = x0 + j;
#pragma unroll
  for (int o = 0; o < kRowsPerThread; ++o) {
    const int gy = y0 + i0 + o;
    if (gx >= W || gy >= H) continue;
    const int64_t idx = po + (int64_t)gy * W + gx;
    const double x = rgb[idx], y = t_rgb[idx];
    const double dssim = v[0][o] + 2.0 * x * v[1][o] + y * v[2][o];
    g_rgb[idx] = (float)(s_l1 * sgn(x - y) - s_ss * dssim);
    if (c == 0) {
      const int64_t q = fr.pixel_offset + (int64_t)gy * W + gx;
      const float tz = t_depth[q];
      g_depth[q] = tz > 0.0f ? (float)(s_d * sgn((double)depth[q] - (double)tz)) : 0.0f;
      g_alpha[q] = 0.0f;
    }
  }
}

Window make_window() {
  Window w;
  double s = 0.0;
  for (int d = 0; d < kTaps; ++d) {
    const double k = d - kR;
    w.g[d] = std::exp(-(k * k) / (2.0 * 1.5 * 1.5));
    s += w.g[d];
  }
  for (int d = 0; d < kTaps; ++d) w.g[d] /= s;
  return w;
}

}  // namespace

int ssim_tiles_pad(int max_w, int max_h) {
  const int n = ((max_w + kTW - 1) / kTW) * ((max_h + kTH - 1) / kTH);
  return (n + 7) & ~7;
}

void launch_loss_render(hipStream_t st, int F, int tiles_pad, const FrameDesc* frames,
                        int64_t total_px, const float* rgb, const float* depth,
                        const float* t_rgb, const float* t_depth, float lambda1, float lambda2,
                        double* part, double* tile_sums, double* scale, float* loss,
                        float* ssim, float* g_rgb, float* g_depth, float* g_alpha) {
  static const Window win = make_window();
  const dim3 grid((unsigned)tiles_pad, 3u, (unsigned)F);
  const int64_t stride = 3 * total_px;
  hipLaunchKernelGGL(ssim_fwd_kernel, grid, dim3(kThreads), 0, st, frames, tiles_pad, win, rgb,
                     t_rgb, depth, t_depth, stride, part, tile_sums);
  hipLaunchKernelGGL(ssim_loss_finalize_kernel, dim3(1), dim3(kThreads), 0, st, frames, F,
                     tiles_pad, tile_sums, (double)lambda1, (double)lambda2, loss, ssim, scale);
  hipLaunchKernelGGL(ssim_bwd_kernel, grid, dim3(kThreads), 0, st, frames, tiles_pad, win, rgb,
                     t_rgb, depth, t_depth, stride, part, scale, g_rgb, g_depth, g_alpha);
}

}  // namespace gsr
