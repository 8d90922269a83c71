// wave_util.h -- wave-level helpers shared by the kernels of the 3D Gaussian
// and 2D surfel paths: the FP64 cross-lane swaps and DPP moves, the
// transposing and LDS wave sums built on them, and the XCD-grouped tile
// schedule.
#pragma once
#include "gsr_device.h"

namespace gsr {

// Tile schedule groups: one per XCD (workgroup b runs on XCD b % kQueues).
constexpr int kQueues = 8;

// The tile of workgroup `bid` under the grouped, longest-first schedule
// `order` (tile ids, group after group); -1 for the padding workgroups.
__device__ __forceinline__ int tile_of_block(int bid, int n_tiles, int groups,
                                             const uint32_t* __restrict__ order) {
  const int per = (n_tiles + groups - 1) / groups;
  const int q = bid % groups, i = bid / groups;
  const int pos = q * per + i;
  if (i >= per || pos >= n_tiles) return -1;
  return (int)order[pos];
}

// Cross-lane helpers of the FP64 wave reduction (all VALU, no LDS traffic).
//
// swap_sum<32>(a, b): with v_permlane32_swap the upper half-wave of a trades
// places with the lower half-wave of b, so that afterwards a' + b' is
// a(l) + a(l ^ 32) on lanes l < 32 and b(l ^ 32) + b(l) on lanes l >= 32: the
// butterfly step over lane bit 5 that keeps a on the lower and b on the
// upper half, in one swap and one add.  swap_sum<16> does the same over lane
// bit 4 with v_permlane16_swap (odd 16-lane rows of a trade with even rows
// of b).
template <int W>
__device__ __forceinline__ double swap_sum(double a, double b) {
  const uint64_t ua = (uint64_t)__double_as_longlong(a), ub = (uint64_t)__double_as_longlong(b);
  uint32_t lo0, lo1, hi0, hi1;
  if constexpr (W == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32),
                                                     false, false);
    lo0 = lo[0]; lo1 = lo[1]; hi0 = hi[0]; hi1 = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32),
                                                     false, false);
    lo0 = lo[0]; lo1 = lo[1]; hi0 = hi[0]; hi1 = hi[1];
  }
  return __longlong_as_double((long long)(((uint64_t)hi0 << 32) | lo0)) +
         __longlong_as_double((long long)(((uint64_t)hi1 << 32) | lo1));
}

// The value of v on a partner lane inside the lane's 16-lane row: DPP row
// mirror (partner 15 - l) for lane bit 3, half-row mirror (7 - l) for bit 2,
// quad permutes (l ^ 2, l ^ 1) for bits 1 and 0.  The mirrors also flip the
// lower lane bits; the rounds that follow sum over those anyway.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  // every lane's partner lies in its own row, so no lane reads out of
  // bounds and no old value is needed (bound_ctrl)
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf,
                                                         true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kDppRowMirror = 0x140, kDppHalfMirror = 0x141, kDppQuadXor2 = 0x4e,
              kDppQuadXor1 = 0xb1;

// Sum over the wave of N <= 16 FP64 values per lane through LDS: every
// lane stores its values, lane 4 v + p (v < N) adds the 16 lanes
// 16 p .. 16 p + 15 of value v in a fixed pairwise order, and the quad adds
// its four parts by DPP moves.  Returns the total of value
// min(lane >> 2, N - 1) on every lane of the quad.  `red` holds
// N * kRedValue doubles used by this wave only; a wave's LDS operations
// complete in issue order, so calls may follow each other on one buffer.
// Value v, part p, term t live at v kRedValue + p kRedPart + t: the padding
// (17 and 68 doubles instead of 16 and 64) spreads the summing lanes' reads
// over the LDS banks (at most 4 lanes share one; 64 without it).
constexpr int kRedPart = 17, kRedValue = 4 * kRedPart;

template <int N>
__device__ __forceinline__ double lds_wave_sum(double* red, const double (&v)[N], int lane) {
  static_assert(N >= 1 && N <= 16, "four lanes per value");
  double* dst = red + (lane >> 4) * kRedPart + (lane & 15);
#pragma unroll
  for (int i = 0; i < N; ++i) dst[i * kRedValue] = v[i];
  const int rv = lane >> 2 < N ? lane >> 2 : N - 1, rp = lane & 3;
  const double* src = red + rv * kRedValue + rp * kRedPart;
  double s4[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
    s4[t] = (src[4 * t] + src[4 * t + 1]) + (src[4 * t + 2] + src[4 * t + 3]);
  double tot = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  tot += dpp<kDppQuadXor2>(tot);
  tot += dpp<kDppQuadXor1>(tot);
  return tot;
}

// Sum over the wave of N FP64 values per lane by recursive halving: at lane
// bit b a lane keeps the lower or the upper half of its values (by that bit)
// and adds its partner's copy of the same half.  The partners are those of
// the swaps and DPP moves above (bit 5: permlane32 swap, bit 4: permlane16
// swap, bits 3..0: row mirror, half-row mirror, quad xor 2, quad xor 1); a
// mirror also flips the lower bits, which later rounds sum over anyway, so
// after six rounds each total covers all 64 lanes and sits on exactly one
// lane.  Returns that lane's total, its index `idx` and `writer` = true on
// the N lanes that hold one (the rest hold padding).  All VALU, fixed order.
template <int C, int B>
__device__ __forceinline__ void halve_round(const double* in, double* out, int lane, int& base,
                                            int& cnt) {
  constexpr int H = (C + 1) / 2;
  const bool hi = (lane >> B) & 1;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double lo_v = in[j];
    const double hi_v = (H + j < C) ? in[H + j] : 0.0;
    if constexpr (B == 5) {
      out[j] = swap_sum<32>(lo_v, hi_v);
    } else if constexpr (B == 4) {
      out[j] = swap_sum<16>(lo_v, hi_v);
    } else {
      const double keep = hi ? hi_v : lo_v;
      const double send = hi ? lo_v : hi_v;
      constexpr int ctrl = B == 3 ? kDppRowMirror
                         : B == 2 ? kDppHalfMirror
                         : B == 1 ? kDppQuadXor2 : kDppQuadXor1;
      out[j] = keep + dpp<ctrl>(send);
    }
  }
  if (hi) {
    base += H;
    cnt = cnt > H ? cnt - H : 0;
  } else {
    cnt = cnt < H ? cnt : H;
  }
}

template <int N>
__device__ __forceinline__ double wave_transpose_sum(const double (&v)[N], int lane, int& idx,
                                                     bool& writer) {
  static_assert(N >= 1 && N <= kWave, "one total per lane");
  constexpr int C4 = (N + 1) / 2, C3 = (C4 + 1) / 2, C2 = (C3 + 1) / 2, C1 = (C2 + 1) / 2,
                C0 = (C1 + 1) / 2;
  double r4[C4], r3[C3], r2[C2], r1[C1], r0[C0], rr[(C0 + 1) / 2];
  int base = 0, cnt = N;
  halve_round<N, 5>(v, r4, lane, base, cnt);
  halve_round<C4, 4>(r4, r3, lane, base, cnt);
  halve_round<C3, 3>(r3, r2, lane, base, cnt);
  halve_round<C2, 2>(r2, r1, lane, base, cnt);
  halve_round<C1, 1>(r1, r0, lane, base, cnt);
  halve_round<C0, 0>(r0, rr, lane, base, cnt);
  idx = base;
  writer = cnt > 0;
  return rr[0];
}

}  // namespace gsr
