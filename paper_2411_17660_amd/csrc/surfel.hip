// surfel.hip -- the 2D Gaussian surfel (2DGS) variant of the rasterizer
// (DROID-Splat Sec. 3.3 compares 2D surfels with its 3D Gaussians in
// tab:renderer; the 2DGS method it cites).  The key, sort and range stages
// (A2-A5) and the batching are those of the 3D path; the preprocess and the
// compositing differ.
//
// A surfel is a flat disk: mean mu, two scales (s_u, s_v), rotation q whose
// first two axes t_u, t_v span it and whose third t_w is its normal, opacity
// and SH colour.  With the frame's world->camera [R_f | t_f] and intrinsics K,
//   M = K [s_u R_f t_u | s_v R_f t_v | R_f mu + t_f]     (rows M0, M1, M2)
// maps disk coordinates (u, v, 1) to homogeneous pixels, and the ray through
// pixel (x, y) meets the disk at (u, v) = (p0/p2, p1/p2), p = h_u x h_v,
// h_u = x M2 - M0, h_v = y M2 - M1, at depth M2 . (u, v, 1).  The record
// holds M2 and k_u = c_x M2 - M0, k_v = c_y M2 - M1 (c the projected centre,
// whose third components vanish), so that a pixel forms
//   h_u = (x - c_x) M2 + k_u,   h_v = (y - c_y) M2 + k_v
// from its small offset to the centre, which FP32 keeps exact to rounding;
// the centre is stored as FP32 hi/lo pairs.  Per pixel:
//   G = exp(-(u^2 + v^2)/2), G_lp = exp(-|(x, y) - c|^2), G' = max(G, G_lp),
//   alpha = min(0.99, sigma G'), depth = M2 . (u, v, 1) (c's depth where
//   G_lp wins), normal = t_w in the camera frame, turned to face the camera;
// compositing thresholds and order as in the 3D path.  A surfel covers the
// pixel box of the projected corners of |u|, |v| <= sqrt(2 ln(255 sigma))
// united with the square of half width sqrt(ln(255 sigma)) around c; the
// box's integer bounds are taken in FP64.
#include <cstddef>

#include "launch.h"
#include "sh_device.h"

namespace gsr {

namespace {

struct Surfel {  // 96 bytes: six 16-byte loads
  float m2x, m2y, zc, kux;  // M2 = (m2x, m2y, zc); k_u = (kux, kuy, 0)
  float kuy, kvx, kvy, cxh;  // k_v = (kvx, kvy, 0); centre x hi
  float cxl, cyh, cyl, opacity;
  float c0, c1, c2, n0;      // colour, normal
  float n1, n2;
  uint32_t sqx, sqy;         // pixel box, lo | hi << 16
  float reserved[4];
};
static_assert(sizeof(Surfel) == 96, "surfel record layout");

template <int DEG>
__global__ void __launch_bounds__(256) surfel_preprocess_kernel(
    int64_t n, int n_frames, const FrameDesc* __restrict__ frames,
    const float* __restrict__ poses, const float* __restrict__ means,
    const float* __restrict__ log_scales /* [n,2] */, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, int tile_w, int tile_h,
    Surfel* __restrict__ rec, uint2* __restrict__ trect, uint32_t* __restrict__ depth_key,
    uint32_t* __restrict__ rec_id, uint32_t* __restrict__ ntiles) {
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double su = exp((double)log_scales[2 * g]), sv = exp((double)log_scales[2 * g + 1]);
  double q[4];
  for (int a = 0; a < 4; ++a) q[a] = quats[4 * g + a];
  const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  const double Rg[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                        2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                        2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
  const double o = 1.0 / (1.0 + exp(-(double)opac[g]));
  const double mu[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const double amin = (double)kAlphaMin;
  for (int f = 0; f < n_frames; ++f) {
    const int64_t r = (int64_t)f * n + g;
    const FrameDesc fr = frames[f];
    double W[9], tf[3];
    load_pose(poses, f, W, tf);
    rec_id[r] = (uint32_t)r;
    depth_key[r] = 0xffffffffu;
    ntiles[r] = 0;
    double mc[3], T[9];  // T = R_f R_g: columns t_u, t_v, t_w in the camera frame
    for (int i = 0; i < 3; ++i) {
      mc[i] = W[i * 3 + 0] * mu[0] + W[i * 3 + 1] * mu[1] + W[i * 3 + 2] * mu[2] + tf[i];
      for (int j = 0; j < 3; ++j)
        T[i * 3 + j] = W[i * 3 + 0] * Rg[0 * 3 + j] + W[i * 3 + 1] * Rg[1 * 3 + j] +
                       W[i * 3 + 2] * Rg[2 * 3 + j];
    }
    const double near = fr.near_z;
    if (!(o > amin) || !(mc[2] > near)) continue;
    const double fx = fr.fx, fy = fr.fy, cx = fr.cx, cy = fr.cy;
    // columns a = s_u t_u, b = s_v t_v, c = mc; rows of M = K [a | b | c]
    const double A[3] = {su * T[0], su * T[3], su * T[6]};
    const double B[3] = {sv * T[1], sv * T[4], sv * T[7]};
    const double M0[3] = {fx * A[0] + cx * A[2], fx * B[0] + cx * B[2], fx * mc[0] + cx * mc[2]};
    const double M1[3] = {fy * A[1] + cy * A[2], fy * B[1] + cy * B[2], fy * mc[1] + cy * mc[2]};
    const double M2[3] = {A[2], B[2], mc[2]};
    const double ccx = M0[2] / M2[2], ccy = M1[2] / M2[2];
    const double ra = sqrt(2.0 * log(o / amin)), rl = sqrt(log(o / amin));
    double lox = ccx - rl, hix = ccx + rl, loy = ccy - rl, hiy = ccy + rl;
    bool ok = true;
    for (int ia = 0; ia < 2; ++ia)
      for (int ib = 0; ib < 2; ++ib) {
        const double uu = ia ? ra : -ra, vv = ib ? ra : -ra;
        const double hx = M0[0] * uu + M0[1] * vv + M0[2];
        const double hy = M1[0] * uu + M1[1] * vv + M1[2];
        const double hz = M2[0] * uu + M2[1] * vv + M2[2];
        if (!(hz > near)) {
          ok = false;
          continue;
        }
        const double px = hx / hz, py = hy / hz;
        lox = px < lox ? px : lox;
        hix = px > hix ? px : hix;
        loy = py < loy ? py : loy;
        hiy = py > hiy ? py : hiy;
      }
    if (!ok) continue;
    const double xl = ceil(lox), xh = floor(hix), yl = ceil(loy), yh = floor(hiy);
    const int x_lo = xl > 0.0 ? (int)xl : 0;
    const int y_lo = yl > 0.0 ? (int)yl : 0;
    const int x_hi = xh < (double)(fr.width - 1) ? (int)xh : fr.width - 1;
    const int y_hi = yh < (double)(fr.height - 1) ? (int)yh : fr.height - 1;
    if (!(x_lo <= x_hi && y_lo <= y_hi)) continue;
    const int tx0 = x_lo / tile_w, tx1 = x_hi / tile_w;
    const int ty0 = y_lo / tile_h, ty1 = y_hi / tile_h;
    ntiles[r] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    trect[r] = make_uint2((uint32_t)tx0 | ((uint32_t)tx1 << 16),
                          (uint32_t)ty0 | ((uint32_t)ty1 << 16));
    const float zf = (float)mc[2];
    depth_key[r] = __float_as_uint(zf);
    double dir[3];
    view_dir(W, tf, mu, dir);
    double Y[16];
    sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
    double raw[3] = {0.0, 0.0, 0.0};
    const float* shg = sh + g * nb * 3;
    for (int k = 0; k < nb; ++k)
      for (int c = 0; c < 3; ++c) raw[c] += (double)shg[k * 3 + c] * Y[k];
    // normal turned to face the camera
    const double tw[3] = {T[2], T[5], T[8]};
    const double sgn = (tw[0] * mc[0] + tw[1] * mc[1] + tw[2] * mc[2]) < 0.0 ? 1.0 : -1.0;
    Surfel s;
    s.m2x = (float)M2[0];
    s.m2y = (float)M2[1];
    s.zc = zf;
    s.kux = (float)(ccx * M2[0] - M0[0]);
    s.kuy = (float)(ccx * M2[1] - M0[1]);
    s.kvx = (float)(ccy * M2[0] - M1[0]);
    s.kvy = (float)(ccy * M2[1] - M1[1]);
    s.cxh = (float)ccx;
    s.cxl = (float)(ccx - (double)s.cxh);
    s.cyh = (float)ccy;
    s.cyl = (float)(ccy - (double)s.cyh);
    s.opacity = (float)o;
    const double c0 = raw[0] + 0.5, c1 = raw[1] + 0.5, c2 = raw[2] + 0.5;
    s.c0 = (float)(c0 > 0.0 ? c0 : 0.0);
    s.c1 = (float)(c1 > 0.0 ? c1 : 0.0);
    s.c2 = (float)(c2 > 0.0 ? c2 : 0.0);
    s.n0 = (float)(sgn * tw[0]);
    s.n1 = (float)(sgn * tw[1]);
    s.n2 = (float)(sgn * tw[2]);
    s.sqx = (uint32_t)x_lo | ((uint32_t)x_hi << 16);
    s.sqy = (uint32_t)y_lo | ((uint32_t)y_hi << 16);
    s.reserved[0] = s.reserved[1] = s.reserved[2] = s.reserved[3] = 0.0f;
    rec[r] = s;
  }
}

// One pixel's view of one surfel: G', alpha before the clamp, depth.
struct SurfelHit {
  float Gh, z;
  bool obj;       // the disk term (not the low-pass) is the larger
  float u, v, p2, hux, huy, huz, hvx, hvy, hvz, ex, ey;  // kept for the backward
};

__device__ __forceinline__ SurfelHit surfel_eval(const Surfel& S, int px, int py) {
#pragma clang fp contract(off)
  SurfelHit h;
  h.ex = -dx_of(S.cxh, S.cxl, px);  // x - c_x
  h.ey = -dx_of(S.cyh, S.cyl, py);
  h.hux = h.ex * S.m2x + S.kux;
  h.huy = h.ex * S.m2y + S.kuy;
  h.huz = h.ex * S.zc;
  h.hvx = h.ey * S.m2x + S.kvx;
  h.hvy = h.ey * S.m2y + S.kvy;
  h.hvz = h.ey * S.zc;
  const float p0 = h.huy * h.hvz - h.huz * h.hvy;
  const float p1 = h.huz * h.hvx - h.hux * h.hvz;
  h.p2 = h.hux * h.hvy - h.huy * h.hvx;
  float G = 0.0f;
  h.u = 0.0f;
  h.v = 0.0f;
  if (h.p2 != 0.0f) {
    const float inv = 1.0f / h.p2;
    h.u = p0 * inv;
    h.v = p1 * inv;
    G = gauss_of(h.u * h.u + h.v * h.v);
  }
  const float Glp = gauss_of(2.0f * (h.ex * h.ex + h.ey * h.ey));
  h.obj = G >= Glp;
  h.Gh = h.obj ? G : Glp;
  h.z = h.obj ? (S.m2x * h.u + S.m2y * h.v + S.zc) : S.zc;
  return h;
}

template <int TW, int TH>
__global__ void __launch_bounds__(64) surfel_fwd_kernel(
    int n_frames, const FrameDesc* __restrict__ frames, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const Surfel* __restrict__ rec, float bg0, float bg1,
    float bg2, float* __restrict__ rgb, float* __restrict__ depth, float* __restrict__ alpha,
    float* __restrict__ normal, float* __restrict__ t_final, int32_t* __restrict__ n_last) {
  constexpr int PIX = TW * TH / kWave;
  constexpr int RPP = kWave / TW;
  __shared__ Surfel sm[kWave];
  const int tile = blockIdx.x;
  const int f = frame_of_tile(frames, n_frames, tile);
  const FrameDesc fr = frames[f];
  const int lt = tile - fr.tile_offset;
  const int x0 = (lt % fr.grid_x) * TW, y0 = (lt / fr.grid_x) * TH;
  const int lane = threadIdx.x;
  const int px = x0 + lane % TW;
  const int ly = lane / TW;
  const uint2 rg = ranges[tile];
  float T[PIX], C0[PIX], C1[PIX], C2[PIX], D[PIX], N0[PIX], N1[PIX], N2[PIX];
  int last[PIX];
  bool done[PIX];
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    T[k] = 1.0f;
    C0[k] = C1[k] = C2[k] = D[k] = N0[k] = N1[k] = N2[k] = 0.0f;
    last[k] = 0;
    const int py = y0 + k * RPP + ly;
    done[k] = !(px < fr.width && py < fr.height);
  }
  for (uint32_t b = rg.x; b < rg.y; b += kWave) {
    bool live = false;
#pragma unroll
    for (int k = 0; k < PIX; ++k) live |= !done[k];
    if (__ballot(live) == 0) break;
    const uint32_t e = b + lane;
    if (e < rg.y) sm[lane] = rec[vals[e]];
    __syncthreads();
    const int cnt = (int)min((uint32_t)kWave, rg.y - b);
    for (int j = 0; j < cnt; ++j) {
      const Surfel& S = sm[j];
      const int xlo = S.sqx & 0xffff, xhi = S.sqx >> 16;
      const int ylo = S.sqy & 0xffff, yhi = S.sqy >> 16;
      const bool xin = (unsigned)(px - xlo) <= (unsigned)(xhi - xlo);
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        const int row0 = y0 + k * RPP;
        if (ylo > row0 + RPP - 1 || yhi < row0) continue;
        const int py = row0 + ly;
        if (done[k] || !xin || (unsigned)(py - ylo) > (unsigned)(yhi - ylo)) continue;
        const SurfelHit h = surfel_eval(S, px, py);
        const float a = fminf(kAlphaMax, S.opacity * h.Gh);
        if (a < kAlphaMin) continue;
        const float Tn = T[k] * (1.0f - a);
        if (Tn < kTMin) {
          done[k] = true;
          continue;
        }
        const float w = a * T[k];
        C0[k] += S.c0 * w;
        C1[k] += S.c1 * w;
        C2[k] += S.c2 * w;
        D[k] += h.z * w;
        N0[k] += S.n0 * w;
        N1[k] += S.n1 * w;
        N2[k] += S.n2 * w;
        T[k] = Tn;
        last[k] = (int)(b + j + 1 - rg.x);
      }
    }
    __syncthreads();
  }
  const int64_t plane = (int64_t)fr.width * fr.height;
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    const int py = y0 + k * RPP + ly;
    if (px < fr.width && py < fr.height) {
      const int64_t p = (int64_t)py * fr.width + px;
      float* img = rgb + 3 * fr.pixel_offset;
      img[p] = C0[k] + T[k] * bg0;
      img[plane + p] = C1[k] + T[k] * bg1;
      img[2 * plane + p] = C2[k] + T[k] * bg2;
      float* nm = normal + 3 * fr.pixel_offset;
      nm[p] = N0[k];
      nm[plane + p] = N1[k];
      nm[2 * plane + p] = N2[k];
      depth[fr.pixel_offset + p] = D[k];
      alpha[fr.pixel_offset + p] = 1.0f - T[k];
      t_final[fr.pixel_offset + p] = T[k];
      n_last[fr.pixel_offset + p] = last[k];
    }
  }
}

}  // namespace

size_t surfel_record_bytes() { return sizeof(Surfel); }
size_t surfel_square_offset() { return offsetof(Surfel, sqx); }

void launch_surfel_preprocess(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                              const float* poses, const float* means, const float* log_scales,
                              const float* quats, const float* opac, const float* sh, int deg,
                              int tile_w, int tile_h, void* rec, uint2* trect,
                              uint32_t* depth_key, uint32_t* rec_id, uint32_t* ntiles) {
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256));
#define GSR_SURF_PRE(D)                                                                      \
  hipLaunchKernelGGL(surfel_preprocess_kernel<D>, grid, dim3(256), 0, st, n, F, frames,      \
                     poses, means, log_scales, quats, opac, sh, tile_w, tile_h,             \
                     (Surfel*)rec, trect, depth_key, rec_id, ntiles)
  switch (deg) {
    case 0: GSR_SURF_PRE(0); break;
    case 1: GSR_SURF_PRE(1); break;
    case 2: GSR_SURF_PRE(2); break;
    default: GSR_SURF_PRE(3); break;
  }
#undef GSR_SURF_PRE
}

void launch_surfel_fwd(hipStream_t st, int tw, int th, int n_tiles, int F,
                       const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                       const void* rec, const float* bg, float* rgb, float* depth, float* alpha,
                       float* normal, float* t_final, int32_t* n_last) {
  if (n_tiles <= 0) return;
#define GSR_SURF_FWD(W, H)                                                                  \
  hipLaunchKernelGGL((surfel_fwd_kernel<W, H>), dim3((unsigned)n_tiles), dim3(kWave), 0, st, \
                     F, frames, ranges, vals, (const Surfel*)rec, bg[0], bg[1], bg[2], rgb,  \
                     depth, alpha, normal, t_final, n_last)
  if (tw == 16 && th == 16) GSR_SURF_FWD(16, 16);
  else if (tw == 8 && th == 8) GSR_SURF_FWD(8, 8);
  else if (tw == 32 && th == 8) GSR_SURF_FWD(32, 8);
  else if (tw == 16 && th == 8) GSR_SURF_FWD(16, 8);
  else if (tw == 32 && th == 16) GSR_SURF_FWD(32, 16);
#undef GSR_SURF_FWD
}

}  // namespace gsr
