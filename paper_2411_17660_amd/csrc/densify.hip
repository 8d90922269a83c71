// densify.hip -- per-Gaussian pieces of map densification (DROID-Splat
// Sec. 3.3: adaptive density control or MCMC densification; lr_noise and
// the Gaussian cap in supplementary S1.2).
//
//  - densify_stats_kernel: the ADC statistic of the last backward, per
//    Gaussian the sum over its kept (Gaussian, frame) records of
//    |dL/d(u, v)|_2 (pixel units, from the FP64 per-record screen-space
//    gradient) and the number of such records, added to the caller's
//    accumulators;
//  - mcmc_noise_kernel: means += s * gate(o) * Sigma eps, Sigma = R diag(s^2)
//    R^T, gate(o) = 1 / (1 + exp(100 (o - 0.995)));
//  - relocation (MCMC): a live source chosen c times is split into N = c + 1
//    copies with o' = 1 - (1 - o)^(1/N) and scales times
//    o / sum_{m=1}^{N} C(N, m) (-1)^(m-1) o'^m / sqrt(m), the copies taking
//    the dead slots.  (The double sum over j <= N, k < j of
//    C(j-1, k) (-1)^k o'^(k+1) / sqrt(k+1) collapses to this single sum by
//    sum_{j=k+1}^{N} C(j-1, k) = C(N, k+1).)
// One thread per Gaussian; all arithmetic FP64, results rounded to FP32.
#include <cmath>

#include "launch.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr double kGateK = 100.0;
constexpr double kGateT = 1.0 - 0.005;
constexpr int kMaxCopies = 1024;  // N beyond this is computed as 1024

__global__ void __launch_bounds__(kThreads) densify_stats_kernel(
    int64_t n, int F, const uint32_t* __restrict__ ntiles, const double* __restrict__ grad2d,
    float* __restrict__ grad_accum, float* __restrict__ count) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  double s = 0.0, c = 0.0;
  for (int f = 0; f < F; ++f) {
    const int64_t r = (int64_t)f * n + g;
    if (ntiles[r] == 0) continue;
    const double du = grad2d[r * kNG], dv = grad2d[r * kNG + 1];
    s += sqrt(du * du + dv * dv);
    c += 1.0;
  }
  grad_accum[g] = (float)((double)grad_accum[g] + s);
  count[g] = (float)((double)count[g] + c);
}

__device__ __forceinline__ void quat_rot(const float* q4, double R[9]) {
  double w = q4[0], x = q4[1], y = q4[2], z = q4[3];
  const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= inv; x *= inv; y *= inv; z *= inv;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

__global__ void __launch_bounds__(kThreads) mcmc_noise_kernel(
    int64_t n, float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ opac,
    const float* __restrict__ eps, double scale) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  double R[9];
  quat_rot(quats + 4 * g, R);
  const double o = 1.0 / (1.0 + exp(-(double)opac[g]));
  const double gate = 1.0 / (1.0 + exp(kGateK * (o - kGateT)));
  double s2[3], e[3], u[3];
  for (int a = 0; a < 3; ++a) {
    s2[a] = exp(2.0 * (double)log_scales[3 * g + a]);
    e[a] = eps[3 * g + a];
  }
  // Sigma e = R diag(s^2) R^T e
  for (int a = 0; a < 3; ++a) u[a] = s2[a] * (R[a] * e[0] + R[3 + a] * e[1] + R[6 + a] * e[2]);
  for (int a = 0; a < 3; ++a) {
    const double step = R[3 * a] * u[0] + R[3 * a + 1] * u[1] + R[3 * a + 2] * u[2];
    means[3 * g + a] = (float)((double)means[3 * g + a] + scale * gate * step);
  }
}

__device__ __forceinline__ bool valid_src(const int32_t* src, int64_t n, int64_t g, int64_t& i) {
  i = src[g];
  return i >= 0 && i < n;
}

__global__ void __launch_bounds__(kThreads) relocate_count_kernel(int64_t n,
                                                                  const int32_t* __restrict__ src,
                                                                  uint32_t* __restrict__ cnt) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  int64_t i;
  if (valid_src(src, n, g, i)) atomicAdd(&cnt[i], 1u);
}

// New opacity logit and log-scales of every source (cnt > 0), rule[g][0..3].
__global__ void __launch_bounds__(kThreads) relocate_rule_kernel(
    int64_t n, const uint32_t* __restrict__ cnt, const float* __restrict__ opac,
    const float* __restrict__ log_scales, double* __restrict__ rule) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n || cnt[g] == 0) return;
  const int N = (int)min(cnt[g] + 1u, (uint32_t)kMaxCopies);
  const double o = 1.0 / (1.0 + exp(-(double)opac[g]));
  const double on = 1.0 - pow(1.0 - o, 1.0 / N);
  // t = C(N, m) o'^m built up term by term (o' ~ o / N keeps it bounded)
  double denom = 0.0, t = 1.0;
  for (int m = 1; m <= N; ++m) {
    t = t * (double)(N - m + 1) / (double)m * on;
    denom += ((m & 1) ? 1.0 : -1.0) * t / sqrt((double)m);
  }
  const double dls = log(o / denom);
  rule[4 * g] = log(on / (1.0 - on));
  for (int a = 0; a < 3; ++a) rule[4 * g + 1 + a] = (double)log_scales[3 * g + a] + dls;
}

__global__ void __launch_bounds__(kThreads) relocate_apply_kernel(
    int64_t n, int ksh3, const int32_t* __restrict__ src, const uint32_t* __restrict__ cnt,
    const double* __restrict__ rule, float* __restrict__ means, float* __restrict__ log_scales,
    float* __restrict__ quats, float* __restrict__ opac, float* __restrict__ sh) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n) return;
  int64_t i;
  if (valid_src(src, n, g, i)) {
    // a dead slot takes a copy of its (updated) source
    for (int a = 0; a < 3; ++a) means[3 * g + a] = means[3 * i + a];
    for (int a = 0; a < 4; ++a) quats[4 * g + a] = quats[4 * i + a];
    for (int a = 0; a < ksh3; ++a) sh[(int64_t)ksh3 * g + a] = sh[(int64_t)ksh3 * i + a];
  } else if (cnt[g] > 0) {
    i = g;
  } else {
    return;
  }
  opac[g] = (float)rule[4 * i];
  for (int a = 0; a < 3; ++a) log_scales[3 * g + a] = (float)rule[4 * i + 1 + a];
}

unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void launch_densify_stats(hipStream_t st, int64_t n, int F, const uint32_t* ntiles,
                          const double* grad2d, float* grad_accum, float* count) {
  if (n <= 0) return;
  hipLaunchKernelGGL(densify_stats_kernel, dim3(blocks(n)), dim3(kThreads), 0, st, n, F, ntiles,
                     grad2d, grad_accum, count);
}

void launch_mcmc_noise(hipStream_t st, int64_t n, float* means, const float* log_scales,
                       const float* quats, const float* opac, const float* eps, float scale) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mcmc_noise_kernel, dim3(blocks(n)), dim3(kThreads), 0, st, n, means,
                     log_scales, quats, opac, eps, (double)scale);
}

void launch_mcmc_relocate(hipStream_t st, int64_t n, int ksh3, float* means, float* log_scales,
                          float* quats, float* opac, float* sh, const int32_t* src,
                          uint32_t* cnt, double* rule) {
  if (n <= 0) return;
  launch_fill_u32(st, cnt, (uint64_t)n, 0u);
  hipLaunchKernelGGL(relocate_count_kernel, dim3(blocks(n)), dim3(kThreads), 0, st, n, src, cnt);
  hipLaunchKernelGGL(relocate_rule_kernel, dim3(blocks(n)), dim3(kThreads), 0, st, n, cnt, opac,
                     log_scales, rule);
  // the apply pass takes new opacities and scales from `rule` only, and
  // reads the sources' means, quaternions and SH, which it does not write
  hipLaunchKernelGGL(relocate_apply_kernel, dim3(blocks(n)), dim3(kThreads), 0, st, n, ksh3, src,
                     cnt, (const double*)rule, means, log_scales, quats, opac, sh);
}

}  // namespace gsr
