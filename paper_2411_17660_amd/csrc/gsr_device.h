// gsr_device.h -- device-side layouts and helpers of the MI355X (gfx950)
// tile rasterizer.  Internal to libgsr.so; the public boundary is
// include/gsr.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_check.h"  // FrameDesc

namespace gsr {

// Per-pair thresholds of the compositing loop (FP32 compares).
constexpr float kAlphaMin = 1.0f / 255.0f;  // skip entries with alpha < 1/255
constexpr float kAlphaMax = 0.99f;          // alpha is clamped to 0.99
constexpr float kTMin = 1e-4f;              // stop before T drops below 1e-4
// EWA screen-space low-pass (px^2), Jacobian guard, 3-sigma extent.
constexpr double kLowpass = 0.3;
constexpr double kJGuard = 1.3;
constexpr double kExtent = 3.0;
// -0.5 * log2(e): alpha = opacity * 2^(q * kNegHalfLog2e)
constexpr float kNegHalfLog2e = -0.72134752044448170368f;

constexpr int kWave = 64;

// Per (Gaussian, frame) record written by the preprocess and staged through
// LDS by the compositing kernels: 64 bytes, read with 4 x 16-byte loads.
//  - (u, v) as FP32 hi/lo pairs so that u - i is exact to FP32 rounding even
//    at 1900 px;
//  - the conic in completed-square form q = (a1 dx + a2 dy)^2 + (a3 dy)^2,
//    a1 = sqrt(A), a2 = B / sqrt(A), a3 = sqrt(C - B^2/A) = 1/sqrt(s_yy):
//    both terms are non-negative, so anisotropic Gaussians do not cancel;
//  - the pixel bounds, 16 bits each: the 3-sigma square clipped to the box
//    where alpha can reach 1/255 (outside it alpha < 1/255).
struct alignas(16) Record {
  float u_hi, u_lo, v_hi, v_lo;
  float a1, a2, a3, opacity;
  float c0, c1, c2, z;
  uint32_t sqx, sqy;      // lo | hi << 16
  uint32_t reserved0, reserved1;
};
static_assert(sizeof(Record) == 64, "record layout");

// A record's tile rect (trect[r]): tx0 | tx1 << 16, ty0 | ty1 << 16, the tiles
// of the square clipped to the region where alpha can reach 1/255.  keyoff[r]
// is the first key slot of record r (written by keygen; all-ones if the record
// overflowed a fixed key capacity).

// Gradient of one (tile, entry) key: du, dv, dSigma'_xx, dSigma'_xy, dSigma'_yy
// (symmetric-matrix gradient), dopacity, dc0..2, dz
constexpr int kNG = 10;

// The frame of a global tile id: the last frame whose first tile is <= tile
// (every frame has at least one tile, so the first tiles increase), by
// binary search over the frame table.
__device__ __forceinline__ int frame_of_tile(const FrameDesc* fr, int n_frames, int tile) {
  int lo = 0, hi = n_frames - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fr[mid].tile_offset <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Alpha of an entry at one pixel, the single definition used by the forward
// and backward compositing kernels so that both take identical decisions.
// dx, dy: Gaussian centre minus pixel.  Explicit fma, no contraction.
struct AlphaEval {
  float dx, dy, g, a;  // g = exp(-q/2); a = min(kAlphaMax, opacity * g)
  bool clamped;
};

__device__ __forceinline__ float dx_of(float hi, float lo, int px) {
#pragma clang fp contract(off)
  return (hi - (float)px) + lo;  // hi - px is exact (Sterbenz / integer grid)
}

__device__ __forceinline__ float q_of(float a1, float a2, float a3, float dx, float dy) {
#pragma clang fp contract(off)
  const float m = __builtin_fmaf(a2, dy, a1 * dx);
  const float b = a3 * dy;
  return __builtin_fmaf(m, m, b * b);
}

__device__ __forceinline__ float gauss_of(float q) {
#pragma clang fp contract(off)
  return __builtin_amdgcn_exp2f(q * kNegHalfLog2e);
}

}  // namespace gsr
