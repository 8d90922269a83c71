// ssim.hip -- the mapper's rendering loss with its SSIM term, forward and
// backward (DROID-Splat eqn rnd_loss, Sec. 3.3; lambda2 = 0.2 in
// supplementary S1.2).  Per frame f of the batch,
//   L_f = l1 [ (1 - l2) mean|I - I*| + l2 (1 - SSIM(I, I*)) ]
//       + (1 - l1) mean_{Z* > 0} |Z - Z*|,
// SSIM being Wang et al.'s index with an 11 x 11 Gaussian window
// (sigma 1.5, weights summing to 1), C1 = 0.01^2, C2 = 0.03^2, window sums
// taken with zero padding, averaged over the 3 channels and all pixels.
//
// Three launches:
//  - ssim_fwd_kernel takes the window sums w*x, w*y, w*(x^2 + y^2) and
//    w*xy, evaluates the SSIM map and writes, per colour value, its
//    derivatives A = dS/dmu_x, B = dS/d(w*x^2) and C = dS/d(w*xy); it also
//    sums S, |x - y| and (channel 0) the depth terms of its block;
//  - ssim_frame_kernel sums each frame's block records in a fixed order
//    into the frame's loss term and gradient scales, and the last block
//    of ssim_total_kernel adds the frame terms;
//  - ssim_bwd_kernel applies the adjoint window: the window being
//    symmetric, d(sum S)/dx = w*A + 2 x (w*B) + y (w*C).
// Both window passes walk down image columns: each wave owns 64 adjacent
// columns and a run of rows of one colour plane; lane j computes column j.
// Input rows are staged one at a time in a per-wave LDS double buffer (the
// global loads of the next rows are in flight while the current row is
// processed); the horizontal 11-tap sum reads the staged row, and the
// vertical 11-tap sum accumulates in a ring of 11 output rows held in
// registers (slot = output row mod 11, static because the row loop is
// unrolled by 11), so no intermediate map goes through LDS or HBM.
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
constexpr int kLanes = 64;             // output columns per wave
constexpr int kRowW = kLanes + 2 * kR; // 74 staged columns
constexpr int kWaves = 4;              // waves per block, stacked vertically
constexpr int kThreads = 64 * kWaves;
constexpr int kChunks = 5;             // row loop: kChunks x 11 staged rows per wave
constexpr int kStaged = kChunks * kTaps;   // 55
constexpr int kSeg = kStaged - 2 * kR;     // 45 output rows per wave
constexpr int kBlockRows = kSeg * kWaves;  // 180 output rows per block
// staged rows whose global loads are in flight while a row is processed
constexpr int kAheadFwd = 3, kAheadBwd = 1;
// forward window sums: w*x, w*y, w*(x^2 + y^2), w*xy (the two second
// moments enter the map only through var_x + var_y)
constexpr int kMaps = 4;
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

struct Window {
  double g[kTaps];
};

// Block tile t of a plane: grid x is padded to a multiple of 8 and remapped
// so that each XCD (block id mod 8) takes one contiguous run of tiles.
__device__ __forceinline__ int tile_of(int bx, int tiles_pad) {
  return (bx & 7) * (tiles_pad >> 3) + (bx >> 3);
}

// Orders this wave's LDS writes before its later LDS reads (the staging
// buffers are private to a wave).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums N values per thread over the block; thread 0 gets the totals.
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
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] += red[w][k];
}

__device__ __forceinline__ double sgn(double d) { return d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0); }

// Geometry of one wave's work: plane, columns [x0, x0 + 64), output rows
// [y0, y0 + kSeg) (clipped to the image by the callers).
struct WaveTile {
  int W, H, x0, y0;
  int64_t po;        // first value of the colour plane
  int64_t pix0;      // first pixel of the frame
  bool valid;        // the block's tile exists
};

__device__ __forceinline__ WaveTile wave_tile(const FrameDesc* frames, int tiles_pad) {
  const int f = blockIdx.z, c = blockIdx.y;
  const int t = tile_of(blockIdx.x, tiles_pad);
  const FrameDesc fr = frames[f];
  WaveTile w;
  w.W = fr.width;
  w.H = fr.height;
  const int ntx = (w.W + kLanes - 1) / kLanes, nty = (w.H + kBlockRows - 1) / kBlockRows;
  w.valid = t < ntx * nty;
  w.x0 = (t % ntx) * kLanes;
  w.y0 = (t / ntx) * kBlockRows + (int)(threadIdx.x >> 6) * kSeg;
  w.po = 3 * fr.pixel_offset + (int64_t)c * w.W * w.H;
  w.pix0 = fr.pixel_offset;
  return w;
}

// Staged row rho of a wave covers image row y0 - kR + rho, columns
// x0 - kR .. x0 - kR + 73: lane j holds column j and lanes 0..9 also
// column 64 + j.  Out-of-image values are 0 (zero padding).  The same
// fetch brings the values of output row rho - kR at the lane's own column
// that the loss terms need: depth and target depth (channel 0; tz = 0
// where there is no such pixel), and, for the backward, both colours.
struct RowFetch {
  float a0, b0, a1, b1;  // staged colour values (forward)
  float x, y, dz, tz;    // output pixel: colours (backward), depths (channel 0)
};

__device__ __forceinline__ void fetch_out_px(const WaveTile& w, int rho, int lane, int c,
                                             bool colours, const float* __restrict__ rgb,
                                             const float* __restrict__ t_rgb,
                                             const float* __restrict__ depth,
                                             const float* __restrict__ t_depth, RowFetch& r) {
  const int i = rho - kR;
  const int gy = w.y0 + i, gx = w.x0 + lane;
  if (i < 0 || i >= kSeg || gy >= w.H || gx >= w.W) return;
  if (colours) {
    const int64_t idx = w.po + (int64_t)gy * w.W + gx;
    r.x = rgb[idx];
    r.y = t_rgb[idx];
  }
  if (c == 0) {
    const int64_t q = w.pix0 + (int64_t)gy * w.W + gx;
    r.dz = depth[q];
    r.tz = t_depth[q];
  }
}

__device__ __forceinline__ RowFetch fetch_row_f(const WaveTile& w, int rho, int lane, int c,
                                                const float* __restrict__ a,
                                                const float* __restrict__ b,
                                                const float* __restrict__ depth,
                                                const float* __restrict__ t_depth) {
  RowFetch r{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  const int gy = w.y0 - kR + rho;
  if (gy < 0 || gy >= w.H) return r;
  const int64_t row = w.po + (int64_t)gy * w.W;
  const int gx0 = w.x0 - kR + lane, gx1 = gx0 + kLanes;
  if (gx0 >= 0 && gx0 < w.W) {
    r.a0 = a[row + gx0];
    r.b0 = b[row + gx0];
  }
  if (lane < 2 * kR && gx1 < w.W) {
    r.a1 = a[row + gx1];
    r.b1 = b[row + gx1];
  }
  fetch_out_px(w, rho, lane, c, false, a, b, depth, t_depth, r);
  return r;
}

__global__ void __launch_bounds__(kThreads) ssim_fwd_kernel(
    const FrameDesc* __restrict__ frames, int tiles_pad, Window win,
    const float* __restrict__ rgb, const float* __restrict__ t_rgb,
    const float* __restrict__ depth, const float* __restrict__ t_depth, int64_t plane_stride,
    double* __restrict__ part, double* __restrict__ tile_sums /* [F][3][tiles_pad][4] */) {
  __shared__ double stage[kWaves][2][2][kRowW + 2];  // [wave][buffer][x | y][column]
  __shared__ double red[kWaves][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.y;
  const WaveTile w = wave_tile(frames, tiles_pad);
  double* out = tile_sums + (((int64_t)blockIdx.z * 3 + c) * tiles_pad + blockIdx.x) * 4;
  if (!w.valid) {
    if (threadIdx.x < 4) out[threadIdx.x] = 0.0;
    return;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // sum S, sum |x - y|, sum |z - z*|, valid depths
  if (w.y0 < w.H) {
    double (*buf)[2][kRowW + 2] = stage[wv];
    const int gx = w.x0 + lane;
    RowFetch nx = fetch_row_f(w, 0, lane, c, rgb, t_rgb, depth, t_depth);
    buf[0][0][lane] = nx.a0;
    buf[0][1][lane] = nx.b0;
    if (lane < 2 * kR) {
      buf[0][0][kLanes + lane] = nx.a1;
      buf[0][1][kLanes + lane] = nx.b1;
    }
    // rows 1 .. kAheadFwd in flight; row rho + kAheadFwd + 1 is fetched while
    // row rho is processed
    RowFetch ahead[kAheadFwd];
#pragma unroll
    for (int a = 0; a < kAheadFwd; ++a)
      ahead[a] = fetch_row_f(w, 1 + a, lane, c, rgb, t_rgb, depth, t_depth);
    wave_sync();
    // ring[s] accumulates output row s (mod 11); its first term (t = 0)
    // assigns, so slots need no clearing
    double ring[kTaps][kMaps];
    for (int k = 0; k < kChunks; ++k) {
#pragma unroll
      for (int u = 0; u < kTaps; ++u) {
        const int rho = k * kTaps + u;
        const int cur = rho & 1;
        nx = ahead[0];
#pragma unroll
        for (int a = 0; a + 1 < kAheadFwd; ++a) ahead[a] = ahead[a + 1];
        ahead[kAheadFwd - 1] =
            fetch_row_f(w, rho + kAheadFwd + 1, lane, c, rgb, t_rgb, depth, t_depth);
        // horizontal sums of row rho at this lane's column; the centre tap is
        // the output pixel of row rho - kR, whose |x - y| is summed here
        const bool l1_row = rho >= kR && rho - kR < kSeg && w.y0 + rho - kR < w.H;
        double h[kMaps] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < kTaps; ++d) {
          const double xv = buf[cur][0][lane + d], yv = buf[cur][1][lane + d];
          if (d == kR && l1_row && gx < w.W) acc[1] += fabs(xv - yv);
          const double gxv = win.g[d] * xv, gyv = win.g[d] * yv;
          h[0] += gxv;
          h[1] += gyv;
          h[2] = fma(gyv, yv, fma(gxv, xv, h[2]));
          h[3] = fma(gxv, yv, h[3]);
        }
        // vertical: row rho feeds output rows rho - t, t = 0..10, weight g[t]
#pragma unroll
        for (int m = 0; m < kMaps; ++m) ring[u][m] = win.g[0] * h[m];
#pragma unroll
        for (int t = 1; t < kTaps; ++t) {
          const int s = (u - t + kTaps) % kTaps;
#pragma unroll
          for (int m = 0; m < kMaps; ++m) ring[s][m] = fma(win.g[t], h[m], ring[s][m]);
        }
        // output row rho - 10 is complete
        const int s_out = (u + 1) % kTaps;
        const int i = rho - 2 * kR;
        const int gy = w.y0 + i;
        if (i >= 0 && gy < w.H && gx < w.W) {
          const double mx = ring[s_out][0], my = ring[s_out][1];
          const double cxy = ring[s_out][3] - mx * my;
          const double l_num = 2.0 * mx * my + kC1, l_den = mx * mx + my * my + kC1;
          const double c_num = 2.0 * cxy + kC2;
          const double c_den = ring[s_out][2] - mx * mx - my * my + kC2;  // var_x + var_y + C2
          const double rinv = 1.0 / (l_den * c_den);
          const double S = l_num * c_num * rinv;
          const double dS_dmu =
              c_num * c_den * rinv * rinv * (2.0 * my * l_den - 2.0 * mx * l_num);
          const double dS_dvar = -S * l_den * rinv;
          const double dS_dcov = 2.0 * l_num * rinv;
          const int64_t idx = w.po + (int64_t)gy * w.W + gx;
          part[idx] = dS_dmu - 2.0 * mx * dS_dvar - my * dS_dcov;
          part[idx + plane_stride] = dS_dvar;
          part[idx + 2 * plane_stride] = dS_dcov;
          acc[0] += S;
        }
        // publish row rho + 1 into the other buffer; its output pixel's depths
        if (rho + 1 < kStaged) {
          buf[cur ^ 1][0][lane] = nx.a0;
          buf[cur ^ 1][1][lane] = nx.b0;
          if (lane < 2 * kR) {
            buf[cur ^ 1][0][kLanes + lane] = nx.a1;
            buf[cur ^ 1][1][kLanes + lane] = nx.b1;
          }
          if (nx.tz > 0.0f) {
            acc[2] += fabs((double)nx.dz - (double)nx.tz);
            acc[3] += 1.0;
          }
        }
        wave_sync();
      }
    }
  }
  block_sums<4>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out[k] = acc[k];
}

// One block per frame: its block records in a fixed order -> the frame's
// loss term, SSIM and gradient scales, stored as
// fs[f] = (l1 (1-l2) / 3HW, l1 l2 / 3HW, (1-l1) / |m|, L_f).
__global__ void __launch_bounds__(256) ssim_frame_kernel(
    const FrameDesc* __restrict__ frames, int tiles_pad, const double* __restrict__ tile_sums,
    double lambda1, double lambda2, float* __restrict__ ssim, double* __restrict__ fs) {
  __shared__ double red[4][4];
  const int f = blockIdx.x;
  const int per_frame = 3 * tiles_pad;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < per_frame; b += blockDim.x)
    for (int k = 0; k < 4; ++k) s[k] += tile_sums[((int64_t)f * per_frame + b) * 4 + k];
  block_sums<4>(s, red);
  if (threadIdx.x == 0) {
    const double n3 = 3.0 * (double)frames[f].width * (double)frames[f].height;
    const double ss = s[0] / n3;
    if (ssim) ssim[f] = (float)ss;
    fs[4 * f] = lambda1 * (1.0 - lambda2) / n3;
    fs[4 * f + 1] = lambda1 * lambda2 / n3;
    fs[4 * f + 2] = s[3] > 0.0 ? (1.0 - lambda1) / s[3] : 0.0;
    fs[4 * f + 3] = lambda1 * ((1.0 - lambda2) * s[1] / n3 + lambda2 * (1.0 - ss)) +
                    (s[3] > 0.0 ? (1.0 - lambda1) * s[2] / s[3] : 0.0);
  }
}

// One wave: sum of the frame terms in frame order.
__global__ void __launch_bounds__(64) ssim_total_kernel(int n_frames,
                                                        const double* __restrict__ fs,
                                                        float* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  double total = 0.0;
  for (int f = 0; f < n_frames; ++f) total += fs[4 * f + 3];
  *loss = (float)total;
}

struct RowFetchD {
  double a0, b0, c0, a1, b1, c1;  // staged A, B, C
  RowFetch px;                    // output pixel of row rho - kR
};

__device__ __forceinline__ RowFetchD fetch_row_d(const WaveTile& w, int rho, int lane, int c,
                                                 const double* __restrict__ part,
                                                 int64_t stride, const float* __restrict__ rgb,
                                                 const float* __restrict__ t_rgb,
                                                 const float* __restrict__ depth,
                                                 const float* __restrict__ t_depth) {
  RowFetchD r{0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
              {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f}};
  const int gy = w.y0 - kR + rho;
  if (gy < 0 || gy >= w.H) return r;
  const int64_t row = w.po + (int64_t)gy * w.W;
  const int gx0 = w.x0 - kR + lane, gx1 = gx0 + kLanes;
  if (gx0 >= 0 && gx0 < w.W) {
    r.a0 = part[row + gx0];
    r.b0 = part[row + gx0 + stride];
    r.c0 = part[row + gx0 + 2 * stride];
  }
  if (lane < 2 * kR && gx1 < w.W) {
    r.a1 = part[row + gx1];
    r.b1 = part[row + gx1 + stride];
    r.c1 = part[row + gx1 + 2 * stride];
  }
  fetch_out_px(w, rho, lane, c, true, rgb, t_rgb, depth, t_depth, r.px);
  return r;
}

// Output rows whose pixel values wait in LDS between their fetch (with
// staged row i + kR) and their use (after staged row i + 2 kR).
constexpr int kPxRing = 8;
static_assert(kPxRing > kR + 1, "pixel ring too short");

__global__ void __launch_bounds__(kThreads) ssim_bwd_kernel(
    const FrameDesc* __restrict__ frames, int tiles_pad, Window win,
    const float* __restrict__ rgb, const float* __restrict__ t_rgb,
    const float* __restrict__ depth, const float* __restrict__ t_depth, int64_t plane_stride,
    const double* __restrict__ part, const double* __restrict__ fs,
    float* __restrict__ g_rgb, float* __restrict__ g_depth, float* __restrict__ g_alpha) {
  __shared__ double stage[kWaves][2][3][kRowW + 2];  // [wave][buffer][A | B | C][column]
  __shared__ float4 pxr[kWaves][kPxRing][kLanes];    // (x, y, z, z*) of pending output rows
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int f = blockIdx.z, c = blockIdx.y;
  const WaveTile w = wave_tile(frames, tiles_pad);
  if (!w.valid || w.y0 >= w.H) return;
  const double s_l1 = fs[4 * f], s_ss = fs[4 * f + 1], s_d = fs[4 * f + 2];
  double (*buf)[3][kRowW + 2] = stage[wv];
  float4 (*px)[kLanes] = pxr[wv];
  const int gx = w.x0 + lane;
  RowFetchD nx = fetch_row_d(w, 0, lane, c, part, plane_stride, rgb, t_rgb, depth, t_depth);
  buf[0][0][lane] = nx.a0;
  buf[0][1][lane] = nx.b0;
  buf[0][2][lane] = nx.c0;
  if (lane < 2 * kR) {
    buf[0][0][kLanes + lane] = nx.a1;
    buf[0][1][kLanes + lane] = nx.b1;
    buf[0][2][kLanes + lane] = nx.c1;
  }
  RowFetchD ahead[kAheadBwd];
#pragma unroll
  for (int a = 0; a < kAheadBwd; ++a)
    ahead[a] = fetch_row_d(w, 1 + a, lane, c, part, plane_stride, rgb, t_rgb, depth, t_depth);
  wave_sync();
  double ring[kTaps][3];  // as in the forward: the t = 0 term assigns
  for (int k = 0; k < kChunks; ++k) {
#pragma unroll
    for (int u = 0; u < kTaps; ++u) {
      const int rho = k * kTaps + u;
      const int cur = rho & 1;
      nx = ahead[0];
#pragma unroll
      for (int a = 0; a + 1 < kAheadBwd; ++a) ahead[a] = ahead[a + 1];
      ahead[kAheadBwd - 1] = fetch_row_d(w, rho + kAheadBwd + 1, lane, c, part, plane_stride,
                                         rgb, t_rgb, depth, t_depth);
      double h[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int d = 0; d < kTaps; ++d)
#pragma unroll
        for (int m = 0; m < 3; ++m) h[m] = fma(win.g[d], buf[cur][m][lane + d], h[m]);
#pragma unroll
      for (int m = 0; m < 3; ++m) ring[u][m] = win.g[0] * h[m];
#pragma unroll
      for (int t = 1; t < kTaps; ++t) {
        const int s = (u - t + kTaps) % kTaps;
#pragma unroll
        for (int m = 0; m < 3; ++m) ring[s][m] = fma(win.g[t], h[m], ring[s][m]);
      }
      const int s_out = (u + 1) % kTaps;
      const int i = rho - 2 * kR;
      const int gy = w.y0 + i;
      if (i >= 0 && gy < w.H && gx < w.W) {
        const float4 pv = px[i % kPxRing][lane];
        const int64_t idx = w.po + (int64_t)gy * w.W + gx;
        const double x = pv.x, y = pv.y;
        const double dssim = ring[s_out][0] + 2.0 * x * ring[s_out][1] + y * ring[s_out][2];
        g_rgb[idx] = (float)(s_l1 * sgn(x - y) - s_ss * dssim);
        if (c == 0) {
          const int64_t q = w.pix0 + (int64_t)gy * w.W + gx;
          g_depth[q] = pv.w > 0.0f ? (float)(s_d * sgn((double)pv.z - (double)pv.w)) : 0.0f;
          g_alpha[q] = 0.0f;
        }
      }
      if (rho + 1 < kStaged) {
        buf[cur ^ 1][0][lane] = nx.a0;
        buf[cur ^ 1][1][lane] = nx.b0;
        buf[cur ^ 1][2][lane] = nx.c0;
        if (lane < 2 * kR) {
          buf[cur ^ 1][0][kLanes + lane] = nx.a1;
          buf[cur ^ 1][1][kLanes + lane] = nx.b1;
          buf[cur ^ 1][2][kLanes + lane] = nx.c1;
        }
        const int i_px = rho + 1 - kR;  // output row whose pixel values came with it
        if (i_px >= 0 && i_px < kSeg)
          px[i_px % kPxRing][lane] = make_float4(nx.px.x, nx.px.y, nx.px.dz, nx.px.tz);
      }
      wave_sync();
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
  const int n = ((max_w + kLanes - 1) / kLanes) * ((max_h + kBlockRows - 1) / kBlockRows);
  return (n + 7) & ~7;
}

void launch_loss_render(hipStream_t st, int F, int tiles_pad, const FrameDesc* frames,
                        int64_t total_px, const float* rgb, const float* depth,
                        const float* t_rgb, const float* t_depth, float lambda1, float lambda2,
                        double* part, double* tile_sums, double* frame_sums, float* loss,
                        float* ssim, float* g_rgb, float* g_depth, float* g_alpha) {
  static const Window win = make_window();
  const dim3 grid((unsigned)tiles_pad, 3u, (unsigned)F);
  const int64_t stride = 3 * total_px;
  hipLaunchKernelGGL(ssim_fwd_kernel, grid, dim3(kThreads), 0, st, frames, tiles_pad, win, rgb,
                     t_rgb, depth, t_depth, stride, part, tile_sums);
  hipLaunchKernelGGL(ssim_frame_kernel, dim3((unsigned)F), dim3(256), 0, st, frames, tiles_pad,
                     tile_sums, (double)lambda1, (double)lambda2, ssim, frame_sums);
  hipLaunchKernelGGL(ssim_total_kernel, dim3(1), dim3(64), 0, st, F, frame_sums, loss);
  hipLaunchKernelGGL(ssim_bwd_kernel, grid, dim3(kThreads), 0, st, frames, tiles_pad, win, rgb,
                     t_rgb, depth, t_depth, stride, part, frame_sums, g_rgb, g_depth, g_alpha);
}

}  // namespace gsr
