// preprocess.hip -- per (Gaussian, frame) projection (forward) and its chain
// rule (backward), FP64 on gfx950.
//
// Forward (DROID-Splat Sec. 3.3: parameters P, r, s, sigma, SH; alpha_i =
// sigma_i * G(R, t, P_i, r_i, s_i) with the EWA projection of the 3DGS
// rasterizer the paper builds on; Sec. 3.1 pinhole Pi_c):
//   s = exp(l), R(q/|q|), Sigma = R diag(s^2) R^T, sigma = 1/(1+e^-o);
//   t = R_f mu + t_f, keep iff t_z > near;
//   (u, v) = (fx t_x/t_z + cx, fy t_y/t_z + cy);
//   Sigma' = J R_f Sigma R_f^T J^T + 0.3 I (J with the 1.3x frustum guard);
//   r = 3 sqrt(lambda_max(Sigma')); square = [ceil(u-r), floor(u+r)] x ...;
//   colour = max(0, sum_k sh_k Y_k(dir) + 1/2), dir from the camera centre.
// Every integer decision (cull, square, tile rect, depth key) is taken in
// FP64 with contraction off, in a fixed operation order, so that it is
// reproducible on any IEEE-754 double implementation.
//
// The forward takes one thread per (Gaussian, frame) record, each building
// the Gaussian's world covariance itself (the parameters come from HBM about
// once, then from cache).  The backward takes one thread per Gaussian, which
// walks all frames of the batch and sums the Gaussian's gradients over them
// in frame order.
#include "launch.h"
#include "sh_device.h"
#include "wave_util.h"

#include <algorithm>

namespace gsr {

struct GaussSetup {
  double s[3], qn, qh[4], R[9], Sig[9], opacity;
};

__device__ __forceinline__ void gaussian_setup(const float* __restrict__ log_scales,
                                               const float* __restrict__ quats,
                                               const float* __restrict__ opac, int64_t g,
                                               GaussSetup& G) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a) G.s[a] = exp((double)log_scales[g * 3 + a]);
  double q[4];
  for (int a = 0; a < 4; ++a) q[a] = (double)quats[g * 4 + a];
  G.qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int a = 0; a < 4; ++a) G.qh[a] = q[a] / G.qn;
  const double w = G.qh[0], x = G.qh[1], y = G.qh[2], z = G.qh[3];
  G.R[0] = 1.0 - 2.0 * (y * y + z * z);
  G.R[1] = 2.0 * (x * y - w * z);
  G.R[2] = 2.0 * (x * z + w * y);
  G.R[3] = 2.0 * (x * y + w * z);
  G.R[4] = 1.0 - 2.0 * (x * x + z * z);
  G.R[5] = 2.0 * (y * z - w * x);
  G.R[6] = 2.0 * (x * z - w * y);
  G.R[7] = 2.0 * (y * z + w * x);
  G.R[8] = 1.0 - 2.0 * (x * x + y * y);
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = G.R[i * 3 + j] * G.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += M[i * 3 + k] * M[j * 3 + k];
      G.Sig[i * 3 + j] = acc;
    }
  G.opacity = 1.0 / (1.0 + exp(-(double)opac[g]));
}

// A Gaussian takes part only if all its parameters (means, log-scales,
// quaternion, opacity logit, the SH coefficients of the rendered degree) are
// finite numbers; otherwise every one of its records is culled and all its
// gradients are 0.  The 11 geometric values are tested here; the SH
// coefficients through the FP64 colour sum of a kept record: a finite
// coefficient times |Y_k| <= 1 cannot overflow FP64, and a NaN or infinite
// one makes the sum NaN or infinite (0 * inf is NaN), so the sum is finite
// exactly when every coefficient is.  The colour of a kept record does not
// depend on the frame's decisions, so the rule culls all frames alike.
__device__ __forceinline__ bool geometry_finite(const float* __restrict__ means,
                                                const float* __restrict__ log_scales,
                                                const float* __restrict__ quats,
                                                const float* __restrict__ opac, int64_t g) {
  bool ok = isfinite(opac[g]);
  for (int a = 0; a < 3; ++a) ok = ok && isfinite(means[g * 3 + a]) && isfinite(log_scales[g * 3 + a]);
  for (int a = 0; a < 4; ++a) ok = ok && isfinite(quats[g * 4 + a]);
  return ok;
}

// Projection of one Gaussian into one frame (FP64).
struct Proj {
  bool keep;
  double t[3], u, v, J[6], Sc[9], cov[3], det;
  int clamp_x, clamp_y;
  int32_t x_lo, x_hi, y_lo, y_hi;      // 3-sigma pixel square
  int32_t bx_lo, bx_hi, by_lo, by_hi;  // its part that can reach alpha >= 1/255
};

__device__ __forceinline__ void project(const FrameDesc& fr, const double W[9],
                                        const double tf[3], const double mu[3],
                                        const GaussSetup& G, Proj& p) {
#pragma clang fp contract(off)
  p.keep = false;
  for (int i = 0; i < 3; ++i)
    p.t[i] = W[i * 3 + 0] * mu[0] + W[i * 3 + 1] * mu[1] + W[i * 3 + 2] * mu[2] + tf[i];
  const double tx = p.t[0], ty = p.t[1], tz = p.t[2];
  if (!(tz > (double)fr.near_z)) return;
  const double fx = fr.fx, fy = fr.fy, cx = fr.cx, cy = fr.cy;
  p.u = fx * tx / tz + cx;
  p.v = fy * ty / tz + cy;
  const double limx = kJGuard * (double)fr.width / (2.0 * fx);
  const double limy = kJGuard * (double)fr.height / (2.0 * fy);
  double rx = tx / tz, ry = ty / tz;
  p.clamp_x = 0;
  p.clamp_y = 0;
  if (rx < -limx) { rx = -limx; p.clamp_x = -1; }
  if (rx > limx) { rx = limx; p.clamp_x = 1; }
  if (ry < -limy) { ry = -limy; p.clamp_y = -1; }
  if (ry > limy) { ry = limy; p.clamp_y = 1; }
  const double txc = tz * rx, tyc = tz * ry;
  p.J[0] = fx / tz; p.J[1] = 0.0; p.J[2] = -fx * txc / (tz * tz);
  p.J[3] = 0.0; p.J[4] = fy / tz; p.J[5] = -fy * tyc / (tz * tz);
  double T1[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += W[i * 3 + k] * G.Sig[k * 3 + j];
      T1[i * 3 + j] = acc;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += T1[i * 3 + k] * W[j * 3 + k];
      p.Sc[i * 3 + j] = acc;
    }
  double JS[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += p.J[i * 3 + k] * p.Sc[k * 3 + j];
      JS[i * 3 + j] = acc;
    }
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += JS[i * 3 + k] * p.J[j * 3 + k];
      S2[i * 2 + j] = acc;
    }
  p.cov[0] = S2[0] + kLowpass;
  p.cov[1] = S2[1];
  p.cov[2] = S2[3] + kLowpass;
  p.det = p.cov[0] * p.cov[2] - p.cov[1] * p.cov[1];
  if (!(p.det > 0.0)) return;
  const double mid = 0.5 * (p.cov[0] + p.cov[2]);
  const double hd = 0.5 * (p.cov[0] - p.cov[2]);
  const double lmax = mid + sqrt(hd * hd + p.cov[1] * p.cov[1]);
  const double r = kExtent * sqrt(lmax);
  const double xa = ceil(p.u - r), xb = floor(p.u + r);
  const double ya = ceil(p.v - r), yb = floor(p.v + r);
  const double Wm1 = (double)(fr.width - 1), Hm1 = (double)(fr.height - 1);
  if (!(xa <= Wm1 && xb >= 0.0 && xa <= xb)) return;
  if (!(ya <= Hm1 && yb >= 0.0 && ya <= yb)) return;
  p.x_lo = (int32_t)(xa > 0.0 ? xa : 0.0);
  p.x_hi = (int32_t)(xb < Wm1 ? xb : Wm1);
  p.y_lo = (int32_t)(ya > 0.0 ? ya : 0.0);
  p.y_hi = (int32_t)(yb < Hm1 ? yb : Hm1);
  // Tile rect: the square clipped to the bounding box of {q <= Qa}, the region
  // where alpha can reach 1/255, Qa = 2 ln(opacity / (1/255)); half-widths
  // sqrt(Qa s_xx), sqrt(Qa s_yy).  Outside it alpha < 1/255, so dropping
  // those tiles leaves the images unchanged.
  const double Qa = 2.0 * log(G.opacity / (double)kAlphaMin) * (1.0 + 1e-9);
  if (!(Qa > 0.0)) return;
  const double hx = sqrt(Qa * p.cov[0]), hy = sqrt(Qa * p.cov[2]);
  const double ba = ceil(p.u - hx), bb = floor(p.u + hx);
  const double ca = ceil(p.v - hy), cb = floor(p.v + hy);
  p.bx_lo = ba > (double)p.x_lo ? (int32_t)ba : p.x_lo;
  p.bx_hi = bb < (double)p.x_hi ? (int32_t)bb : p.x_hi;
  p.by_lo = ca > (double)p.y_lo ? (int32_t)ca : p.y_lo;
  p.by_hi = cb < (double)p.y_hi ? (int32_t)cb : p.y_hi;
  if (!(p.bx_lo <= p.bx_hi && p.by_lo <= p.by_hi)) return;
  p.keep = true;
}

// --------------------------------------------------------------------------
// A1: forward preprocess, one thread per (Gaussian, frame): blockIdx.y is the
// frame (striding by gridDim.y past 65535 frames), so a block's records
// r = f n + g are consecutive.  Each of a Gaussian's threads computes its
// activations (its parameters are read once per frame, mostly from cache).
// --------------------------------------------------------------------------
template <int DEG>
__global__ void __launch_bounds__(256) preprocess_fwd_kernel(
    int64_t n, int n_frames, const FrameDesc* __restrict__ frames,
    const float* __restrict__ poses, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, int tile_w,
    int tile_h, Record* __restrict__ rec, uint2* __restrict__ trect,
    uint32_t* __restrict__ depth_key, uint32_t* __restrict__ rec_id,
    uint32_t* __restrict__ ntiles) {
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  GaussSetup G;
  gaussian_setup(log_scales, quats, opac, g, G);
  const double mu[3] = {means[g * 3 + 0], means[g * 3 + 1], means[g * 3 + 2]};
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const bool finite = geometry_finite(means, log_scales, quats, opac, g);
  for (int f = (int)blockIdx.y; f < n_frames; f += (int)gridDim.y) {
    const int64_t r = (int64_t)f * n + g;
    const FrameDesc fr = frames[f];
    double W[9], tf[3];
    load_pose(poses, f, W, tf);
    Proj p;
    p.keep = false;
    if (finite) project(fr, W, tf, mu, G, p);
    rec_id[r] = (uint32_t)r;
    double raw[3] = {0.0, 0.0, 0.0};
    if (p.keep) {
      double dir[3];
      view_dir(W, tf, mu, dir);
      double Y[16];
      sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
      const float* shg = sh + g * nb * 3;
      for (int k = 0; k < nb; ++k)
        for (int c = 0; c < 3; ++c) raw[c] += (double)shg[k * 3 + c] * Y[k];
    }
    if (!p.keep || !isfinite(raw[0] + raw[1] + raw[2])) {
      depth_key[r] = 0xffffffffu;
      ntiles[r] = 0;
      continue;
    }
    const int tx0 = p.bx_lo / tile_w, tx1 = p.bx_hi / tile_w;
    const int ty0 = p.by_lo / tile_h, ty1 = p.by_hi / tile_h;
    ntiles[r] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    trect[r] = make_uint2((uint32_t)tx0 | ((uint32_t)tx1 << 16),
                          (uint32_t)ty0 | ((uint32_t)ty1 << 16));
    const float zf = (float)p.t[2];
    depth_key[r] = __float_as_uint(zf);
    Record o;
    o.u_hi = (float)p.u;
    o.u_lo = (float)(p.u - (double)o.u_hi);
    o.v_hi = (float)p.v;
    o.v_lo = (float)(p.v - (double)o.v_hi);
    o.a1 = (float)sqrt(p.cov[2] / p.det);
    o.a2 = (float)(-p.cov[1] / sqrt(p.cov[2] * p.det));
    o.a3 = (float)(1.0 / sqrt(p.cov[2]));
    o.opacity = (float)G.opacity;
    const double c0 = raw[0] + 0.5, c1 = raw[1] + 0.5, c2 = raw[2] + 0.5;
    o.c0 = (float)(c0 > 0.0 ? c0 : 0.0);
    o.c1 = (float)(c1 > 0.0 ? c1 : 0.0);
    o.c2 = (float)(c2 > 0.0 ? c2 : 0.0);
    o.z = zf;
    // pixel bounds tested per pixel: the square clipped to the alpha box
    // (outside it alpha < 1/255, so the contribution rule is unchanged)
    o.sqx = (uint32_t)p.bx_lo | ((uint32_t)p.bx_hi << 16);
    o.sqy = (uint32_t)p.by_lo | ((uint32_t)p.by_hi << 16);
    o.reserved0 = 0;
    o.reserved1 = 0;
    rec[r] = o;
  }
}

// --------------------------------------------------------------------------
// A9: per-record reduction of the key partials.  A group of 4 lanes owns one
// record and strides over its contiguous key slots (coalesced stamp and
// partial reads), 16 slots per round with all of a lane's loads of a round in
// flight together; slots not stamped with this backward's epoch belong to
// keys behind every pixel's stop and are skipped.  Lane sums are FP64 and the
// group combines them with a fixed butterfly, so the result is deterministic.
// The records are visited in order of their key count (a one-pass radix sort
// by floor(log2(count)), `order`), largest first: a wave's records then
// have similar counts, instead of waiting on the one Gaussian among them that
// covers hundreds of tiles, and the longest waves start first instead of
// running alone at the end; records with kWideSlots or more slots get a whole
// wave each.
// --------------------------------------------------------------------------
// Records with at least kWideSlots key slots are reduced by a whole wave each
// (slot_reduce_wide_kernel), the others by groups of kSlotGroup lanes.
constexpr uint32_t kWideSlots = 128;
constexpr uint64_t kWideWaves = 8192;  // the wide pass's grid (32 waves per CU)

// The class of kWideSlots slots: records of this class or above are wide.
constexpr uint32_t kWideClass = 8;  // 1 + log2(kWideSlots)
static_assert((1u << (kWideClass - 1)) == kWideSlots, "wide class");

// *first_wide (pre-filled with m) = the first position of the ascending
// class keys with class >= kWideClass: the one position where the class
// crosses it is written by its own thread.
__global__ void __launch_bounds__(256) wide_boundary_kernel(uint64_t m,
                                                            const uint32_t* __restrict__ cls,
                                                            uint32_t* __restrict__ first_wide) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (cls[i] >= kWideClass && (i == 0 || cls[i - 1] < kWideClass)) *first_wide = (uint32_t)i;
}

__global__ void __launch_bounds__(256) size_class_kernel(uint64_t m,
                                                         const uint32_t* __restrict__ ntiles,
                                                         uint32_t* __restrict__ cls,
                                                         uint32_t* __restrict__ idx) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const uint32_t c = ntiles[r];
  cls[r] = c == 0 ? 0u : 32u - (uint32_t)__clz(c);  // 1 + floor(log2 c)
  idx[r] = (uint32_t)r;
}

constexpr int kSlotGroup = 4;
constexpr int kSlotUnroll = 4;
static_assert(kNG % 2 == 0, "partials are read as float pairs");

// The wide pass takes the w-th largest records, w < n_wide = m - *first_wide
// (capped at wide_max), a wave each in turn (grid stride); 64 lanes stride
// over a record's slots, kSlotUnroll per lane per round.
__device__ __forceinline__ void slot_reduce_wide(
    unsigned block, unsigned n_blocks, uint64_t m, const uint32_t* __restrict__ order,
    const uint32_t* __restrict__ keyoff, const uint32_t* __restrict__ ntiles,
    const float* __restrict__ partial, const uint32_t* __restrict__ stamp, uint32_t epoch,
    uint64_t key_capacity, const uint32_t* __restrict__ first_wide, uint64_t wide_max,
    double* __restrict__ grad2d) {
  const uint64_t n_wide = min(m - *first_wide, wide_max);
  const uint64_t stride = ((uint64_t)n_blocks * blockDim.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  for (uint64_t w = ((uint64_t)block * blockDim.x + threadIdx.x) / kWave; w < n_wide;
       w += stride) {  // uniform per wave
  const uint64_t r = order[m - 1 - w];
  uint32_t cnt = ntiles[r];
  const uint32_t off = keyoff[r];
  if ((uint64_t)off + cnt > key_capacity) cnt = 0;  // overflowed the key capacity
  double acc[kNG];
#pragma unroll
  for (int j = 0; j < kNG; ++j) acc[j] = 0.0;
  for (uint32_t s0 = 0; s0 < cnt; s0 += kWave * kSlotUnroll) {
    uint32_t st[kSlotUnroll];
#pragma unroll
    for (int u = 0; u < kSlotUnroll; ++u) {
      const uint32_t s = s0 + lane + u * kWave;
      st[u] = s < cnt ? stamp[off + s] : 0u;
    }
    float2 v[kSlotUnroll][kNG / 2];
#pragma unroll
    for (int u = 0; u < kSlotUnroll; ++u) {
#pragma unroll
      for (int j = 0; j < kNG / 2; ++j) v[u][j] = make_float2(0.0f, 0.0f);
      const uint32_t s = s0 + lane + u * kWave;
      if (s < cnt && st[u] == epoch) {
        const float2* pp = reinterpret_cast<const float2*>(partial + (size_t)(off + s) * kNG);
#pragma unroll
        for (int j = 0; j < kNG / 2; ++j) v[u][j] = pp[j];
      }
    }
#pragma unroll
    for (int u = 0; u < kSlotUnroll; ++u)
#pragma unroll
      for (int j = 0; j < kNG / 2; ++j) {
        acc[2 * j] += v[u][j].x;
        acc[2 * j + 1] += v[u][j].y;
      }
  }
  // the record's ten totals by the transposing VALU reduction (no LDS
  // round trips), total idx on lane `writer`
  int idx;
  bool writer;
  const double v = wave_transpose_sum<kNG>(acc, lane, idx, writer);
  if (writer) grad2d[r * kNG + idx] = v;
  }
}

// Group k (4 lanes) takes the k-th largest record after the ones the wide
// pass took.
__device__ __forceinline__ void slot_reduce_groups(
    unsigned block, uint64_t m, const uint32_t* __restrict__ order,
    const uint32_t* __restrict__ keyoff, const uint32_t* __restrict__ ntiles,
    const float* __restrict__ partial, const uint32_t* __restrict__ stamp, uint32_t epoch,
    uint64_t key_capacity, const uint32_t* __restrict__ first_wide, uint64_t wide_max,
    double* __restrict__ grad2d /* [m][kNG] */) {
  const uint64_t gid = (uint64_t)block * blockDim.x + threadIdx.x;
  const uint64_t k = gid / kSlotGroup + min(m - *first_wide, wide_max);
  const int sub = threadIdx.x & (kSlotGroup - 1);
  // `order` ascends in key count: walk it from the end, so that the records
  // with the most slots (a wave of them runs longest) start first and the
  // small ones fill in around them
  const bool active = k < m;
  const uint64_t r = active ? order[m - 1 - k] : 0;
  uint32_t cnt = active ? ntiles[r] : 0u;
  const uint32_t off = cnt ? keyoff[r] : 0u;
  if (cnt && (uint64_t)off + cnt > key_capacity) cnt = 0;  // overflowed the key capacity
  double acc[kNG];
#pragma unroll
  for (int j = 0; j < kNG; ++j) acc[j] = 0.0;
  // kSlotUnroll slots per lane per round: all their stamps are loaded at
  // once, then the partials of the stamped ones (independent loads, all in
  // flight), then they are added in slot order
  for (uint32_t s0 = 0; s0 < cnt; s0 += kSlotGroup * kSlotUnroll) {
    uint32_t st[kSlotUnroll];
#pragma unroll
    for (int u = 0; u < kSlotUnroll; ++u) {
      const uint32_t s = s0 + sub + u * kSlotGroup;
      st[u] = s < cnt ? stamp[off + s] : 0u;
    }
    float2 v[kSlotUnroll][kNG / 2];
#pragma unroll
    for (int u = 0; u < kSlotUnroll; ++u) {
#pragma unroll
      for (int j = 0; j < kNG / 2; ++j) v[u][j] = make_float2(0.0f, 0.0f);
      const uint32_t s = s0 + sub + u * kSlotGroup;
      // 40-byte partials are 8-byte aligned: five 8-byte loads, issued only
      // by the lanes whose slot is stamped
      if (s < cnt && st[u] == epoch) {
        const float2* pp = reinterpret_cast<const float2*>(partial + (size_t)(off + s) * kNG);
#pragma unroll
        for (int j = 0; j < kNG / 2; ++j) v[u][j] = pp[j];
      }
    }
#pragma unroll
    for (int u = 0; u < kSlotUnroll; ++u)
#pragma unroll
      for (int j = 0; j < kNG / 2; ++j) {
        acc[2 * j] += v[u][j].x;
        acc[2 * j + 1] += v[u][j].y;
      }
  }
  // sum over the group's 4 lanes: quad DPP moves (partners l ^ 2, l ^ 1),
  // the butterfly order of a shuffle reduction without its LDS round trips
#pragma unroll
  for (int j = 0; j < kNG; ++j) acc[j] += dpp<kDppQuadXor2>(acc[j]);
#pragma unroll
  for (int j = 0; j < kNG; ++j) acc[j] += dpp<kDppQuadXor1>(acc[j]);
  static_assert(kSlotGroup == 4, "the group reduction is a quad permute");
  if (!active) return;
  if (cnt == 0) {
    for (int j = sub; j < kNG; j += kSlotGroup) grad2d[r * kNG + j] = 0.0;
    return;
  }
  // lane sub writes values sub, sub + kSlotGroup, ...
#pragma unroll
  for (int j0 = 0; j0 < kNG; j0 += kSlotGroup) {
    double v = acc[j0];
#pragma unroll
    for (int t = 1; t < kSlotGroup; ++t)
      if (j0 + t < kNG) v = sub == t ? acc[j0 + t] : v;
    if (j0 + sub < kNG) grad2d[r * kNG + j0 + sub] = v;
  }
}

// One launch for both passes: the first `wide_blocks` workgroups take the
// wide records (a wave each, grid stride), the rest the groups.  Workgroups
// start in order, so the long wide records start first and the group work
// fills the machine around them instead of waiting for them to finish.
__global__ void __launch_bounds__(256) slot_reduce_kernel(
    uint64_t m, const uint32_t* __restrict__ order, const uint32_t* __restrict__ keyoff,
    const uint32_t* __restrict__ ntiles, const float* __restrict__ partial,
    const uint32_t* __restrict__ stamp, const uint32_t* __restrict__ epoch_dev,
    uint64_t key_capacity, const uint32_t* __restrict__ first_wide, uint64_t wide_max,
    unsigned wide_blocks, double* __restrict__ grad2d) {
  const uint32_t epoch = *epoch_dev;
  if (blockIdx.x < wide_blocks)
    slot_reduce_wide(blockIdx.x, wide_blocks, m, order, keyoff, ntiles, partial, stamp, epoch,
                     key_capacity, first_wide, wide_max, grad2d);
  else
    slot_reduce_groups(blockIdx.x - wide_blocks, m, order, keyoff, ntiles, partial, stamp,
                       epoch, key_capacity, first_wide, wide_max, grad2d);
}

// --------------------------------------------------------------------------
// A10: chain rule to the parameters; per (Gaussian, frame) twist partials
// reduced per wave in FP64.
// --------------------------------------------------------------------------

template <int DEG>
__global__ void __launch_bounds__(256) preprocess_bwd_kernel(
    int64_t n, int n_frames, const FrameDesc* __restrict__ frames,
    const float* __restrict__ poses, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh,
    const uint32_t* __restrict__ ntiles, const double* __restrict__ grad2d,
    float* __restrict__ g_means, float* __restrict__ g_log_scales,
    float* __restrict__ g_quats, float* __restrict__ g_opac, float* __restrict__ g_sh,
    double* __restrict__ twist_partial /* [F][n_waves][6] */) {
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = g0 < n;
  const int64_t g = active ? g0 : 0;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t wave_id = g0 / kWave;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  GaussSetup G;
  if (active) gaussian_setup(log_scales, quats, opac, g, G);
  const double mu[3] = {active ? (double)means[g * 3 + 0] : 0.0,
                        active ? (double)means[g * 3 + 1] : 0.0,
                        active ? (double)means[g * 3 + 2] : 0.0};
  const float* shg = sh + g * nb * 3;
  double dmu[3] = {0, 0, 0}, dSig[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dsig = 0.0;
  float dsh[nb * 3];
  for (int i = 0; i < nb * 3; ++i) dsh[i] = 0.0f;
  bool kept = false;
  for (int f = 0; f < n_frames; ++f) {
    double tw[6] = {0, 0, 0, 0, 0, 0};
    const int64_t r = (int64_t)f * n + g;
    const uint32_t cnt = active ? ntiles[r] : 0u;
    if (cnt > 0) {
      kept = true;
      double gr[kNG];
      for (int j = 0; j < kNG; ++j) gr[j] = grad2d[r * kNG + j];
      const FrameDesc fr = frames[f];
      double W[9], tf[3];
      load_pose(poses, f, W, tf);
      Proj p;
      project(fr, W, tf, mu, G, p);
      const double fx = fr.fx, fy = fr.fy;
      const double tx = p.t[0], ty = p.t[1], tz = p.t[2];
      const double tz2 = tz * tz, tz3 = tz2 * tz;
      double dt[3];
      dt[0] = gr[0] * fx / tz;
      dt[1] = gr[1] * fy / tz;
      dt[2] = -gr[0] * fx * tx / tz2 - gr[1] * fy * ty / tz2 + gr[9];
      dsig += gr[5];
      // the key partials carry dL/dSigma' (symmetric: xx, xy, yy) directly
      const double GS[4] = {gr[2], gr[3], gr[3], gr[4]};
      // Sigma' = J Sc J^T + lowpass: G_J = 2 GS J Sc, G_Sc = J^T GS J
      double JSc[6];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
          JSc[i * 3 + j] = p.J[i * 3 + 0] * p.Sc[0 * 3 + j] + p.J[i * 3 + 1] * p.Sc[1 * 3 + j] +
                           p.J[i * 3 + 2] * p.Sc[2 * 3 + j];
      double GJ[6];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
          GJ[i * 3 + j] = 2.0 * (GS[i * 2 + 0] * JSc[0 * 3 + j] + GS[i * 2 + 1] * JSc[1 * 3 + j]);
      double GJt[6];  // GS J (2x3)
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
          GJt[i * 3 + j] = GS[i * 2 + 0] * p.J[0 * 3 + j] + GS[i * 2 + 1] * p.J[1 * 3 + j];
      double GSc[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          GSc[a * 3 + b] = p.J[0 * 3 + a] * GJt[0 * 3 + b] + p.J[1 * 3 + a] * GJt[1 * 3 + b];
      // J -> t (the guard clamp freezes t_x/t_z where active)
      dt[2] += -GJ[0] * fx / tz2 - GJ[4] * fy / tz2;
      if (p.clamp_x == 0) {
        dt[0] += -GJ[2] * fx / tz2;
        dt[2] += GJ[2] * 2.0 * fx * tx / tz3;
      } else {
        const double txc = tz * (p.clamp_x * kJGuard * (double)fr.width / (2.0 * fx));
        dt[2] += GJ[2] * fx * txc / tz3;
      }
      if (p.clamp_y == 0) {
        dt[1] += -GJ[5] * fy / tz2;
        dt[2] += GJ[5] * 2.0 * fy * ty / tz3;
      } else {
        const double tyc = tz * (p.clamp_y * kJGuard * (double)fr.height / (2.0 * fy));
        dt[2] += GJ[5] * fy * tyc / tz3;
      }
      // Sc = W Sigma W^T -> G_Sigma += W^T G_Sc W
      double T2[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          T2[i * 3 + j] = W[0 * 3 + i] * GSc[0 * 3 + j] + W[1 * 3 + i] * GSc[1 * 3 + j] +
                          W[2 * 3 + i] * GSc[2 * 3 + j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          dSig[i * 3 + j] += T2[i * 3 + 0] * W[0 * 3 + j] + T2[i * 3 + 1] * W[1 * 3 + j] +
                             T2[i * 3 + 2] * W[2 * 3 + j];
      // colour: c = max(0, raw), raw = sum_k sh_k Y_k(dir) + 1/2
      double dir[3];
      const double dist = view_dir(W, tf, mu, dir);
      double Y[16];
      sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
      double raw[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < nb; ++k)
        for (int c = 0; c < 3; ++c) raw[c] += (double)shg[k * 3 + c] * Y[k];
      double draw[3];
      for (int c = 0; c < 3; ++c) draw[c] = raw[c] + 0.5 > 0.0 ? gr[6 + c] : 0.0;
      double wk[16];
      for (int k = 0; k < nb; ++k) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) {
          dsh[k * 3 + c] += (float)(Y[k] * draw[c]);
          acc += (double)shg[k * 3 + c] * draw[c];
        }
        wk[k] = acc;
      }
      double ddir[3];
      sh_dir_grad<DEG>(dir[0], dir[1], dir[2], wk, ddir);
      const double pr = dir[0] * ddir[0] + dir[1] * ddir[1] + dir[2] * ddir[2];
      double dd[3];
      for (int a = 0; a < 3; ++a) dd[a] = (ddir[a] - dir[a] * pr) / dist;
      for (int a = 0; a < 3; ++a)
        dmu[a] += W[0 * 3 + a] * dt[0] + W[1 * 3 + a] * dt[1] + W[2 * 3 + a] * dt[2] + dd[a];
      // twist (rho, phi), left perturbation at zero:
      //   dt = rho + phi x t, dSc = [phi]x Sc - Sc [phi]x, dC = -W^T rho
      for (int a = 0; a < 3; ++a)
        tw[a] = dt[a] + W[a * 3 + 0] * dd[0] + W[a * 3 + 1] * dd[1] + W[a * 3 + 2] * dd[2];
      tw[3] = ty * dt[2] - tz * dt[1];
      tw[4] = tz * dt[0] - tx * dt[2];
      tw[5] = tx * dt[1] - ty * dt[0];
      // <G_Sc, [e_k]x Sc - Sc [e_k]x> for k = x, y, z
      const double* S = p.Sc;
      const double* Gm = GSc;
      // [e_x]x = [[0,0,0],[0,0,-1],[0,1,0]]
      {
        double E[3][9] = {{0, 0, 0, 0, 0, -1, 0, 1, 0},
                          {0, 0, 1, 0, 0, 0, -1, 0, 0},
                          {0, -1, 0, 1, 0, 0, 0, 0, 0}};
        for (int k = 0; k < 3; ++k) {
          double acc = 0.0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              double es = 0.0, se = 0.0;
              for (int l = 0; l < 3; ++l) {
                es += E[k][i * 3 + l] * S[l * 3 + j];
                se += S[i * 3 + l] * E[k][l * 3 + j];
              }
              acc += Gm[i * 3 + j] * (es - se);
            }
          tw[3 + k] += acc;
        }
      }
    }
    {
      // the wave's six twist sums by a transposing VALU reduction (DPP and
      // permlane moves: no LDS round trips), total j on one lane each
      int idx;
      bool writer;
      const double s = wave_transpose_sum<6>(tw, threadIdx.x & (kWave - 1), idx, writer);
      if (writer) twist_partial[((int64_t)f * n_waves + wave_id) * 6 + idx] = s;
    }
  }
  if (!active) return;
  float* gs = g_sh + g * nb * 3;
  if (!kept) {  // no frame sees it (culled, or a non-finite parameter)
    for (int a = 0; a < 3; ++a) g_means[g * 3 + a] = g_log_scales[g * 3 + a] = 0.0f;
    for (int a = 0; a < 4; ++a) g_quats[g * 4 + a] = 0.0f;
    g_opac[g] = 0.0f;
    for (int i = 0; i < nb * 3; ++i) gs[i] = 0.0f;
    return;
  }
  // Sigma = M M^T, M = R diag(s)
  double Gs[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Gs[i * 3 + j] = 0.5 * (dSig[i * 3 + j] + dSig[j * 3 + i]);
  double GM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Gs[i * 3 + k] * G.R[k * 3 + j] * G.s[j];
      GM[i * 3 + j] = 2.0 * acc;
    }
  double dR[9], ds[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      dR[i * 3 + j] = GM[i * 3 + j] * G.s[j];
      ds[j] += GM[i * 3 + j] * G.R[i * 3 + j];
    }
  for (int a = 0; a < 3; ++a) g_log_scales[g * 3 + a] = (float)(ds[a] * G.s[a]);
  quat_grad(G.qh, G.qn, dR, g_quats + g * 4);
  for (int a = 0; a < 3; ++a) g_means[g * 3 + a] = (float)dmu[a];
  g_opac[g] = (float)(dsig * G.opacity * (1.0 - G.opacity));
  for (int i = 0; i < nb * 3; ++i) gs[i] = dsh[i];
}

// Advances the backward epoch held in device memory (so a captured sequence
// gets a fresh epoch on every replay); 0 is skipped because fresh stamp
// memory is zero.
__global__ void bump_epoch_kernel(uint32_t* epoch) {
  const uint32_t e = *epoch + 1u;
  *epoch = e == 0u ? 1u : e;
}

// Counts for gsr_debug_stats (integer atomics, so the totals do not depend
// on the order): culled records, and Gaussians with a non-finite parameter.
__global__ void __launch_bounds__(256) cull_stats_kernel(
    uint64_t m, const uint32_t* __restrict__ ntiles, int64_t n, const float* __restrict__ means,
    const float* __restrict__ log_scales, int log_per, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, int nb3,
    unsigned long long* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool culled = i < m && ntiles[i] == 0;
  bool bad = false;
  if (i < (uint64_t)n) {
    bool ok = isfinite(opac[i]);
    for (int a = 0; a < 3; ++a) ok = ok && isfinite(means[i * 3 + a]);
    for (int a = 0; a < log_per; ++a) ok = ok && isfinite(log_scales[i * log_per + a]);
    for (int a = 0; a < 4; ++a) ok = ok && isfinite(quats[i * 4 + a]);
    for (int a = 0; a < nb3; ++a) ok = ok && isfinite(sh[i * nb3 + a]);
    bad = !ok;
  }
  const uint64_t c = __ballot(culled), b = __ballot(bad);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (c) atomicAdd(&out[0], (unsigned long long)__popcll(c));
    if (b) atomicAdd(&out[1], (unsigned long long)__popcll(b));
  }
}

void launch_cull_stats(hipStream_t st, uint64_t m, const uint32_t* ntiles, int64_t n,
                       const float* means, const float* log_scales, int log_per,
                       const float* quats, const float* opac, const float* sh, int nb3,
                       unsigned long long* out) {
  const uint64_t items = std::max<uint64_t>(m, (uint64_t)n);
  if (items == 0) return;
  hipLaunchKernelGGL(cull_stats_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st,
                     m, ntiles, n, means, log_scales, log_per, quats, opac, sh, nb3, out);
}

void launch_size_class(hipStream_t st, uint64_t m, const uint32_t* ntiles, uint32_t* cls,
                       uint32_t* idx) {
  if (m == 0) return;
  hipLaunchKernelGGL(size_class_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m,
                     ntiles, cls, idx);
}

void launch_wide_boundary(hipStream_t st, uint64_t m, const uint32_t* sorted_cls,
                          uint32_t* first_wide) {
  launch_fill_u32(st, first_wide, 1, (uint32_t)m);
  if (m == 0) return;
  hipLaunchKernelGGL(wide_boundary_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                     m, sorted_cls, first_wide);
}

void launch_bump_epoch(hipStream_t st, uint32_t* epoch) {
  hipLaunchKernelGGL(bump_epoch_kernel, dim3(1), dim3(1), 0, st, epoch);
}

// A11: per-frame sum of the per-wave twist partials (FP64, fixed order).
constexpr int kTwistThreads = 1024;

// One block per frame: thread t sums all six components of the partials
// t, t + 1024, ..., then each wave sums its lanes with a butterfly and the
// 16 wave totals are added in wave order, a fixed order for a given n.
__global__ void __launch_bounds__(kTwistThreads) twist_reduce_kernel(
    const double* __restrict__ part, int64_t n_waves, float* __restrict__ g_twist) {
  __shared__ double red[kTwistThreads / 64][6];
  const int f = blockIdx.x;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t w = threadIdx.x; w < n_waves; w += kTwistThreads) {
    const double* p = part + ((int64_t)f * n_waves + w) * 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) s[j] += p[j];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j)
    for (int o = 32; o > 0; o >>= 1) s[j] += __shfl_xor(s[j], o, 64);
  if (lane == 0)
    for (int j = 0; j < 6; ++j) red[wv][j] = s[j];
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
    for (int i = 0; i < kTwistThreads / 64; ++i) t += red[i][threadIdx.x];
    g_twist[f * 6 + threadIdx.x] = (float)t;
  }
}

void launch_preprocess_fwd(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                           const float* poses, const float* means, const float* log_scales,
                           const float* quats, const float* opac, const float* sh, int deg,
                           int tile_w, int tile_h, Record* rec, uint2* trect,
                           uint32_t* depth_key, uint32_t* rec_id, uint32_t* ntiles) {
  if (n <= 0 || F <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)std::min(F, 65535));
#define GSR_PRE_FWD(D)                                                                      \
  hipLaunchKernelGGL(preprocess_fwd_kernel<D>, grid, dim3(256), 0, st, n, F, frames, poses, \
                     means, log_scales, quats, opac, sh, tile_w, tile_h, rec, trect,        \
                     depth_key, rec_id, ntiles)
  switch (deg) {
    case 0: GSR_PRE_FWD(0); break;
    case 1: GSR_PRE_FWD(1); break;
    case 2: GSR_PRE_FWD(2); break;
    default: GSR_PRE_FWD(3); break;
  }
#undef GSR_PRE_FWD
}

int64_t preprocess_bwd_waves(int64_t n) { return ((n + 255) / 256) * 4; }

void launch_preprocess_bwd(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                           const float* poses, const float* means, const float* log_scales,
                           const float* quats, const float* opac, const float* sh, int deg,
                           const uint32_t* order, const uint32_t* first_wide,
                           const uint32_t* keyoff, const uint32_t* ntiles, const float* partial,
                           const uint32_t* stamp, const uint32_t* epoch, uint64_t key_capacity,
                           double* grad2d, float* g_means, float* g_log_scales, float* g_quats,
                           float* g_opac, float* g_sh, double* twist_partial, float* g_twist) {
  const dim3 grid((unsigned)((n + 255) / 256));
#define GSR_PRE_BWD(D)                                                                       \
  hipLaunchKernelGGL(preprocess_bwd_kernel<D>, grid, dim3(256), 0, st, n, F, frames, poses,  \
                     means, log_scales, quats, opac, sh, ntiles, grad2d, g_means,            \
                     g_log_scales, g_quats, g_opac, g_sh, twist_partial)
  if (n > 0) {
    const uint64_t m = (uint64_t)n * F;
    // wide records come first in the largest-first order and there are at
    // most K / kWideSlots of them; the wide grid covers the first
    // min(m, capacity / kWideSlots + 1) (all of them unless the keys
    // overflow the capacity), the group pass every record after those
    const uint64_t wide_max = std::min<uint64_t>(m, key_capacity / kWideSlots + 1);
    // a fixed grid of kWideWaves waves strides over the wide records
    const uint64_t wide_waves = std::min<uint64_t>(wide_max, kWideWaves);
    const unsigned wide_blocks = (unsigned)((wide_waves + 3) / 4);
    const uint64_t threads = m * kSlotGroup;
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(wide_blocks + (unsigned)((threads + 255) / 256)),
                       dim3(256), 0, st, m, order, keyoff, ntiles, partial, stamp, epoch,
                       key_capacity, first_wide, wide_max, wide_blocks, grad2d);
    switch (deg) {
      case 0: GSR_PRE_BWD(0); break;
      case 1: GSR_PRE_BWD(1); break;
      case 2: GSR_PRE_BWD(2); break;
      default: GSR_PRE_BWD(3); break;
    }
  }
#undef GSR_PRE_BWD
  launch_twist_reduce(st, F, twist_partial, n > 0 ? preprocess_bwd_waves(n) : 0, g_twist);
}

void launch_twist_reduce(hipStream_t st, int F, const double* twist_partial, int64_t n_waves,
                         float* g_twist) {
  if (F <= 0) return;
  hipLaunchKernelGGL(twist_reduce_kernel, dim3(F), dim3(kTwistThreads), 0, st, twist_partial,
                     n_waves, g_twist);
}

}  // namespace gsr
