// adam.hip -- fused optimiser step of the mapping loop (A13).
//
// The mapper runs a fixed number of optimisation iterations per call
// (DROID-Splat supplementary S1.2: 100 iterations, positional learning rate
// annealed, other parameters as in MonoGS), optimising the Gaussians and,
// when pose refinement is on, the keyframe poses (Sec. 3.3, S1.3).  One
// launch updates the three groups the workload optimises:
//   means      (lr_means)   Adam
//   SH colours (lr_sh)      Adam
//   pose twist (lr_pose)    Adam on xi in se(3), then T_f <- Exp(xi) T_f and
//                           xi <- 0 (the twist is always evaluated at zero)
// with bias-corrected moments m, v and an iteration counter held in device
// memory (incremented by the kernel, so a captured iteration advances it on
// every replay).  The pose fold is FP64.
#include "launch.h"

namespace gsr {

struct AdamHyper {
  float lr_means, lr_sh, lr_pose, beta1, beta2, eps;
};

__device__ __forceinline__ float adam_delta(float g, float& m, float& v, float b1, float b2,
                                            float c1, float c2, float eps) {
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * g * g;
  const float mh = m / c1;
  const float vh = v / c2;
  return mh / (sqrtf(vh) + eps);
}

// Gaussians: elements [0, n3) are means, [n3, n3 + nsh) SH coefficients.
__global__ void __launch_bounds__(256) adam_gauss_kernel(
    uint64_t n3, uint64_t nsh, float* __restrict__ means, const float* __restrict__ g_means,
    float* __restrict__ m_means, float* __restrict__ v_means, float* __restrict__ sh,
    const float* __restrict__ g_sh, float* __restrict__ m_sh, float* __restrict__ v_sh,
    AdamHyper h, const int32_t* __restrict__ step) {
  const int t = *step + 1;  // the pose kernel of the same launch sequence bumps it
  const float c1 = 1.0f - powf(h.beta1, (float)t);
  const float c2 = 1.0f - powf(h.beta2, (float)t);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3 + nsh;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (i < n3) {
      float m = m_means[i], v = v_means[i];
      means[i] -= h.lr_means * adam_delta(g_means[i], m, v, h.beta1, h.beta2, c1, c2, h.eps);
      m_means[i] = m;
      v_means[i] = v;
    } else {
      const uint64_t j = i - n3;
      float m = m_sh[j], v = v_sh[j];
      sh[j] -= h.lr_sh * adam_delta(g_sh[j], m, v, h.beta1, h.beta2, c1, c2, h.eps);
      m_sh[j] = m;
      v_sh[j] = v;
    }
  }
}

// One thread per frame: Adam on the twist, then T <- Exp(xi) T with
// Exp(rho, phi) = [R(phi), V(phi) rho], R by Rodrigues, V the SE(3) left
// Jacobian; the last thread advances the iteration counter.
__global__ void adam_pose_kernel(int n_frames, float* __restrict__ poses,
                                 const float* __restrict__ g_twist, float* __restrict__ m_tw,
                                 float* __restrict__ v_tw, AdamHyper h,
                                 int32_t* __restrict__ step) {
  const int f = threadIdx.x;
  const int t = *step + 1;
  if (f < n_frames) {
    const float c1 = 1.0f - powf(h.beta1, (float)t);
    const float c2 = 1.0f - powf(h.beta2, (float)t);
    double xi[6];
    for (int k = 0; k < 6; ++k) {
      float m = m_tw[f * 6 + k], v = v_tw[f * 6 + k];
      xi[k] = -(double)h.lr_pose *
              (double)adam_delta(g_twist[f * 6 + k], m, v, h.beta1, h.beta2, c1, c2, h.eps);
      m_tw[f * 6 + k] = m;
      v_tw[f * 6 + k] = v;
    }
    const double* rho = xi;
    const double* phi = xi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double A, B, Cc;  // sin(th)/th, (1-cos)/th^2, (th - sin)/th^3
    if (th < 1e-5) {
      A = 1.0 - th2 / 6.0;
      B = 0.5 - th2 / 24.0;
      Cc = 1.0 / 6.0 - th2 / 120.0;
    } else {
      A = sin(th) / th;
      B = (1.0 - cos(th)) / th2;
      Cc = (th - sin(th)) / (th2 * th);
    }
    const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int l = 0; l < 3; ++l) acc += K[i * 3 + l] * K[l * 3 + j];
        K2[i * 3 + j] = acc;
      }
    double R[9], V[9];
    for (int i = 0; i < 9; ++i) {
      const double id = (i % 4 == 0) ? 1.0 : 0.0;
      R[i] = id + A * K[i] + B * K2[i];
      V[i] = id + B * K[i] + Cc * K2[i];
    }
    double tr[3];
    for (int i = 0; i < 3; ++i) tr[i] = V[i * 3 + 0] * rho[0] + V[i * 3 + 1] * rho[1] + V[i * 3 + 2] * rho[2];
    float* P = poses + f * 12;
    double Rf[9], tf[3];
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) Rf[i * 3 + j] = P[i * 4 + j];
      tf[i] = P[i * 4 + 3];
    }
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j)
        P[i * 4 + j] = (float)(R[i * 3 + 0] * Rf[0 * 3 + j] + R[i * 3 + 1] * Rf[1 * 3 + j] +
                               R[i * 3 + 2] * Rf[2 * 3 + j]);
      P[i * 4 + 3] = (float)(R[i * 3 + 0] * tf[0] + R[i * 3 + 1] * tf[1] + R[i * 3 + 2] * tf[2] +
                             tr[i]);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *step = t;
}

void launch_adam(hipStream_t st, uint64_t n3, uint64_t nsh, float* means, const float* g_means,
                 float* m_means, float* v_means, float* sh, const float* g_sh, float* m_sh,
                 float* v_sh, int n_frames, float* poses, const float* g_twist, float* m_tw,
                 float* v_tw, float lr_means, float lr_sh, float lr_pose, float beta1,
                 float beta2, float eps, int32_t* step) {
  const AdamHyper h{lr_means, lr_sh, lr_pose, beta1, beta2, eps};
  const uint64_t total = n3 + nsh;
  if (total > 0) {
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(adam_gauss_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n3, nsh,
                       means, g_means, m_means, v_means, sh, g_sh, m_sh, v_sh, h, step);
  }
  const int threads = n_frames > 0 ? ((n_frames + 63) / 64) * 64 : 64;
  hipLaunchKernelGGL(adam_pose_kernel, dim3(1), dim3(threads), 0, st, n_frames, poses, g_twist,
                     m_tw, v_tw, h, step);
}

}  // namespace gsr
