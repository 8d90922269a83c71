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
// compositing thresholds and order as in the 3D path.  The depth distortion
// of a pixel is the sum over pairs i < j of blended entries of
// w_i w_j (z_i - z_j)^2; the forward adds w_j (A z_j^2 - 2 z_j D_1 + D_2) per
// entry, A, D_1, D_2 the sums of w, w z, w z^2 in front of it, with every z
// taken relative to the pixel's first blended entry so that the FP32 sums
// stay near the spread of the depths rather than their size.  A surfel covers
// the bounding box of the image of the disk |(u, v)| <= sqrt(2 ln(255 sigma))
// (exact, from the disk's dual conic) united with the square of half width
// sqrt(ln(255 sigma)) around c, and is culled unless the disk lies beyond the
// near plane; the box's integer bounds are taken in FP64.
#include <algorithm>
#include <cstddef>

#include "launch.h"
#include "sh_device.h"
#include "wave_util.h"

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
  // a surfel with a non-finite parameter is culled in every frame: the 9
  // geometric values here, the SH coefficients through the FP64 colour sum of
  // a kept record (finite exactly when every coefficient is, as for the 3D
  // Gaussians)
  bool finite = isfinite(opac[g]) && isfinite(log_scales[2 * g]) && isfinite(log_scales[2 * g + 1]);
  for (int a = 0; a < 3; ++a) finite = finite && isfinite(means[3 * g + a]);
  for (int a = 0; a < 4; ++a) finite = finite && isfinite(quats[4 * g + a]);
  for (int f = (int)blockIdx.y; f < n_frames; f += (int)gridDim.y) {
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
    if (!finite || !(o > amin) || !(mc[2] > near)) continue;
    const double fx = fr.fx, fy = fr.fy, cx = fr.cx, cy = fr.cy;
    // columns a = s_u t_u, b = s_v t_v, c = mc; rows of M = K [a | b | c]
    const double A[3] = {su * T[0], su * T[3], su * T[6]};
    const double B[3] = {sv * T[1], sv * T[4], sv * T[7]};
    const double M0[3] = {fx * A[0] + cx * A[2], fx * B[0] + cx * B[2], fx * mc[0] + cx * mc[2]};
    const double M1[3] = {fy * A[1] + cy * A[2], fy * B[1] + cy * B[2], fy * mc[1] + cy * mc[2]};
    const double M2[3] = {A[2], B[2], mc[2]};
    const double ccx = M0[2] / M2[2], ccy = M1[2] / M2[2];
    const double r2 = 2.0 * log(o / amin);  // r_a^2
    const double ra = sqrt(r2), rl = sqrt(log(o / amin));
    // the disk's nearest point to the camera plane must be beyond the near plane
    if (!(M2[2] - ra * sqrt(M2[0] * M2[0] + M2[1] * M2[1]) > near)) continue;
    // bounding box of the image of the circle |(u, v)| = r_a: the dual conic
    // C* = M diag(r_a^2, r_a^2, -1) M^T has the vertical tangents x = x0 with
    // C*_00 - 2 x0 C*_02 + x0^2 C*_22 = 0 (and likewise in y)
    const double c22 = r2 * (M2[0] * M2[0] + M2[1] * M2[1]) - M2[2] * M2[2];
    const double c02 = r2 * (M0[0] * M2[0] + M0[1] * M2[1]) - M0[2] * M2[2];
    const double c00 = r2 * (M0[0] * M0[0] + M0[1] * M0[1]) - M0[2] * M0[2];
    const double c12 = r2 * (M1[0] * M2[0] + M1[1] * M2[1]) - M1[2] * M2[2];
    const double c11 = r2 * (M1[0] * M1[0] + M1[1] * M1[1]) - M1[2] * M1[2];
    const double dx = c02 * c02 - c00 * c22, dy = c12 * c12 - c11 * c22;
    const double sx = sqrt(dx > 0.0 ? dx : 0.0), sy = sqrt(dy > 0.0 ? dy : 0.0);
    const double xa = (c02 + sx) / c22, xb = (c02 - sx) / c22;
    const double ya = (c12 + sy) / c22, yb = (c12 - sy) / c22;
    double lox = xa < xb ? xa : xb, hix = xa < xb ? xb : xa;
    double loy = ya < yb ? ya : yb, hiy = ya < yb ? yb : ya;
    lox = ccx - rl < lox ? ccx - rl : lox;
    hix = ccx + rl > hix ? ccx + rl : hix;
    loy = ccy - rl < loy ? ccy - rl : loy;
    hiy = ccy + rl > hiy ? ccy + rl : hiy;
    const double xl = ceil(lox), xh = floor(hix), yl = ceil(loy), yh = floor(hiy);
    const int x_lo = xl > 0.0 ? (int)xl : 0;
    const int y_lo = yl > 0.0 ? (int)yl : 0;
    const int x_hi = xh < (double)(fr.width - 1) ? (int)xh : fr.width - 1;
    const int y_hi = yh < (double)(fr.height - 1) ? (int)yh : fr.height - 1;
    if (!(x_lo <= x_hi && y_lo <= y_hi)) continue;
    double dir[3];
    view_dir(W, tf, mu, dir);
    double Y[16];
    sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
    double raw[3] = {0.0, 0.0, 0.0};
    const float* shg = sh + g * nb * 3;
    for (int k = 0; k < nb; ++k)
      for (int c = 0; c < 3; ++c) raw[c] += (double)shg[k * 3 + c] * Y[k];
    if (!isfinite(raw[0] + raw[1] + raw[2])) continue;
    const int tx0 = x_lo / tile_w, tx1 = x_hi / tile_w;
    const int ty0 = y_lo / tile_h, ty1 = y_hi / tile_h;
    ntiles[r] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    trect[r] = make_uint2((uint32_t)tx0 | ((uint32_t)tx1 << 16),
                          (uint32_t)ty0 | ((uint32_t)ty1 << 16));
    const float zf = (float)mc[2];
    depth_key[r] = __float_as_uint(zf);
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
  float u, v, ip2, hux, huy, huz, hvx, hvy, hvz, ex, ey;  // kept for the backward
};

// ln 255 rounded up: beyond this squared distance from the centre the
// low-pass term is below 1/255, so alpha = sigma G_lp < 1/255 there and it
// can never be blended; skipping its exp leaves every decision unchanged
// (where G >= G_lp the disk term is taken either way, and where G < G_lp
// alpha < 1/255 either way).
constexpr float kLowpassReach = 5.6f;

// The fields of an entry that every pixel strip reads, and the part of the
// intersection fixed by the lane's pixel column (h_u = (x - c_x) M2 + k_u
// does not depend on the row): formed once per entry, in registers, instead
// of once per strip from LDS.
struct SurfelEntry {
  float cyh, cyl, m2x, m2y, kvx, kvy, zc, opacity;  // the record's row fields
  float ex, hux, huy, huz;                          // the column's part
};

__device__ __forceinline__ SurfelEntry surfel_entry(const Surfel& S, int px) {
#pragma clang fp contract(off)
  SurfelEntry e;
  e.cyh = S.cyh; e.cyl = S.cyl; e.m2x = S.m2x; e.m2y = S.m2y;
  e.kvx = S.kvx; e.kvy = S.kvy; e.zc = S.zc; e.opacity = S.opacity;
  asm volatile("" : "+v"(e.cyh), "+v"(e.cyl), "+v"(e.m2x), "+v"(e.m2y), "+v"(e.kvx),
               "+v"(e.kvy), "+v"(e.zc), "+v"(e.opacity));
  e.ex = -dx_of(S.cxh, S.cxl, px);  // x - c_x
  e.hux = e.ex * e.m2x + S.kux;
  e.huy = e.ex * e.m2y + S.kuy;
  e.huz = e.ex * e.zc;
  return e;
}

__device__ __forceinline__ SurfelHit surfel_eval(const SurfelEntry& e, int py) {
#pragma clang fp contract(off)
  SurfelHit h;
  h.ex = e.ex;
  h.ey = -dx_of(e.cyh, e.cyl, py);
  h.hux = e.hux;
  h.huy = e.huy;
  h.huz = e.huz;
  h.hvx = h.ey * e.m2x + e.kvx;
  h.hvy = h.ey * e.m2y + e.kvy;
  h.hvz = h.ey * e.zc;
  const float p0 = h.huy * h.hvz - h.huz * h.hvy;
  const float p1 = h.huz * h.hvx - h.hux * h.hvz;
  const float p2 = h.hux * h.hvy - h.huy * h.hvx;
  float G = 0.0f;
  h.u = 0.0f;
  h.v = 0.0f;
  h.ip2 = 0.0f;
  if (p2 != 0.0f) {
    // reciprocal with one Newton step (within an ulp or so of 1/p2)
    const float r0 = __builtin_amdgcn_rcpf(p2);
    h.ip2 = __builtin_fmaf(__builtin_fmaf(-p2, r0, 1.0f), r0, r0);
    h.u = p0 * h.ip2;
    h.v = p1 * h.ip2;
    G = gauss_of(h.u * h.u + h.v * h.v);
  }
  const float d2 = h.ex * h.ex + h.ey * h.ey;
  const float Glp = d2 < kLowpassReach ? gauss_of(2.0f * d2) : 0.0f;
  h.obj = G >= Glp;
  h.Gh = h.obj ? G : Glp;
  h.z = h.obj ? (e.m2x * h.u + e.m2y * h.v + e.zc) : e.zc;
  return h;
}

// COUNT: also count the evaluated (pixel, entry) pairs, those whose box
// test passes before the pixel stops (one atomic add per tile).
template <int TW, int TH, bool COUNT>
__global__ void __launch_bounds__(64) surfel_fwd_kernel(
    int n_tiles, int groups, const uint32_t* __restrict__ order, uint32_t* __restrict__ tile_nproc,
    unsigned long long* __restrict__ pair_count,
    int n_frames, const FrameDesc* __restrict__ frames, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const Surfel* __restrict__ rec, float bg0, float bg1,
    float bg2, float* __restrict__ rgb, float* __restrict__ depth, float* __restrict__ alpha,
    float* __restrict__ normal, float* __restrict__ dist, float* __restrict__ t_final,
    int32_t* __restrict__ n_last, float* __restrict__ dist_aux /* [P][4]: z_ref, A, D_1, D_2 */) {
  constexpr int PIX = TW * TH / kWave;
  constexpr int RPP = kWave / TW;
  __shared__ Surfel sm[kWave];
  const int tile = tile_of_block(blockIdx.x, n_tiles, groups, order);
  if (tile < 0) return;
  const int f = frame_of_tile(frames, n_frames, tile);
  const FrameDesc fr = frames[f];
  const int lt = tile - fr.tile_offset;
  const int x0 = (lt % fr.grid_x) * TW, y0 = (lt / fr.grid_x) * TH;
  const int lane = threadIdx.x;
  const int px = x0 + lane % TW;
  const int ly = lane / TW;
  const uint2 rg = ranges[tile];
  float T[PIX], C0[PIX], C1[PIX], C2[PIX], D[PIX], N0[PIX], N1[PIX], N2[PIX];
  // distortion sums in FP64: the backward's weights e_i = A z_i^2 -
  // 2 z_i D_1 + D_2 and z_i A - D_1 cancel where the entries lie at one
  // depth, which FP32 sums over hundreds of entries cannot resolve
  float ZR[PIX];
  double SA[PIX], S1[PIX], S2[PIX], DS[PIX];
  int last[PIX];
  bool done[PIX];
  uint32_t hits = 0;
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    T[k] = 1.0f;
    C0[k] = C1[k] = C2[k] = D[k] = N0[k] = N1[k] = N2[k] = 0.0f;
    ZR[k] = 0.0f;
    SA[k] = S1[k] = S2[k] = DS[k] = 0.0;
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
      const SurfelEntry en = surfel_entry(S, px);
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        const int row0 = y0 + k * RPP;
        if (ylo > row0 + RPP - 1 || yhi < row0) continue;
        const int py = row0 + ly;
        if (done[k] || !xin || (unsigned)(py - ylo) > (unsigned)(yhi - ylo)) continue;
        if (COUNT) ++hits;
        const SurfelHit h = surfel_eval(en, py);
        const float a = fminf(kAlphaMax, en.opacity * h.Gh);
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
        if (last[k] == 0) ZR[k] = h.z;
        const double zp = h.z - ZR[k], wd = w;
        DS[k] += wd * (SA[k] * zp * zp - 2.0 * zp * S1[k] + S2[k]);
        SA[k] += wd;
        S1[k] += wd * zp;
        S2[k] += wd * zp * zp;
        T[k] = Tn;
        last[k] = (int)(b + j + 1 - rg.x);
      }
    }
    __syncthreads();
  }
  // the tile's walk length for the backward and the next schedule: the
  // largest list position any of its pixels blended
  int most = 0;
#pragma unroll
  for (int k = 0; k < PIX; ++k) most = last[k] > most ? last[k] : most;
  for (int o = 32; o > 0; o >>= 1) {
    const int m = __shfl_xor(most, o, kWave);
    most = m > most ? m : most;
  }
  if (lane == 0) tile_nproc[tile] = (uint32_t)most;
  if (COUNT) {
    unsigned long long c = hits;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if (lane == 0) atomicAdd(pair_count, c);
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
      dist[fr.pixel_offset + p] = (float)DS[k];
      float4* ax = reinterpret_cast<float4*>(dist_aux) + (fr.pixel_offset + p);
      *ax = make_float4(ZR[k], (float)SA[k], (float)S1[k], (float)S2[k]);
    }
  }
}

// Per key (one surfel in one tile), the values the backward reduces: the
// gradients of the columns A = s_u t_u, B = s_v t_v and mc of
// M = K [A | B | mc], as sums the chain rule only scales.  With h_u =
// x M2 - M0, h_v = y M2 - M1 and (o_x, o_y) = (x - c_x^K, y - c_y^K) the
// pixel's offset from the principal point, column j's gradient is
//   (-f_x S_u[j], -f_y S_v[j], R[j]),  S_u = sum dL/dh_u, S_v = sum dL/dh_v,
//   R[j] = sum o_x dL/dh_u[j] + o_y dL/dh_v[j] + dL/dz (u, v, 1)[j],
// so no large product of a pixel position with a sum is left to cancel in
// the chain rule.  The low-pass term's gradient of the centre c =
// (M0_z, M1_z) / M2_z folds into column 2.  Order: S_u[3], S_v[3], R[3],
// opacity, colour[3], normal[3].
constexpr int kSG = 16;

template <int TW, int TH>
__global__ void __launch_bounds__(64) surfel_bwd_kernel(
    int n_tiles, int groups, const uint32_t* __restrict__ order,
    const uint32_t* __restrict__ tile_nproc,
    int n_frames, const FrameDesc* __restrict__ frames, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const Surfel* __restrict__ rec,
    const uint2* __restrict__ trect, const uint32_t* __restrict__ keyoff, float bg0, float bg1,
    float bg2, const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
    const float* __restrict__ g_alpha, const float* __restrict__ g_normal,
    const float* __restrict__ g_dist, const float* __restrict__ t_final,
    const int32_t* __restrict__ n_last, const float* __restrict__ dist_aux,
    float* __restrict__ partial, uint32_t* __restrict__ stamp,
    const uint32_t* __restrict__ epoch_dev) {
  constexpr int PIX = TW * TH / kWave;
  constexpr int RPP = kWave / TW;
  __shared__ Surfel sm[kWave];
  __shared__ uint32_t slot[kWave];
  __shared__ double red[kSG * kRedValue];  // the per-key reduction
  const int tile = tile_of_block(blockIdx.x, n_tiles, groups, order);
  if (tile < 0) return;
  const int most = (int)tile_nproc[tile];
  if (most == 0) return;
  const uint32_t epoch = *epoch_dev;
  const int f = frame_of_tile(frames, n_frames, tile);
  const FrameDesc fr = frames[f];
  const int lt = tile - fr.tile_offset;
  const int tx = lt % fr.grid_x, ty = lt / fr.grid_x;
  const int x0 = tx * TW, y0 = ty * TH;
  const int lane = threadIdx.x;
  const int px = x0 + lane % TW;
  const int ly = lane / TW;
  const uint2 rg = ranges[tile];
  const int64_t plane = (int64_t)fr.width * fr.height;
  // per pixel: T_{i+1}, the totals of the distortion sums, and the
  // transmittance seen behind the current entry (normalised by T_{i+1}).
  // dL/da_i takes the upstream-weighted difference G . (v_i - B_i) between
  // the entry's values (colour, depth, normal, distortion weight e) and
  // those seen behind it; it cancels where neighbouring surfels agree, so it
  // is formed in FP64.  G is fixed per pixel, so the recursion
  // B_i = B_{i+1} + a_i (v_i - B_{i+1}) carries over to the scalar E = G . B,
  // which the pixel keeps (FP64) together with G in FP64.
  float T[PIX], BT[PIX], AT[PIX], ZR[PIX], S1[PIX], S2[PIX];
  double E[PIX], H0[PIX], H1[PIX], H2[PIX], HD[PIX], HN0[PIX], HN1[PIX], HN2[PIX], HE[PIX];
  float G0[PIX], G1[PIX], G2[PIX], GD[PIX], GA[PIX], GN0[PIX], GN1[PIX], GN2[PIX], GE[PIX];
  int last[PIX];
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    const int py = y0 + k * RPP + ly;
    const bool valid = px < fr.width && py < fr.height;
    const int64_t p = (int64_t)py * fr.width + px;
    const int64_t q = fr.pixel_offset + p;
    last[k] = valid ? n_last[q] : 0;
    T[k] = valid ? t_final[q] : 1.0f;
    const float4 ax = valid ? reinterpret_cast<const float4*>(dist_aux)[q]
                            : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    ZR[k] = ax.x;
    AT[k] = ax.y;
    S1[k] = ax.z;
    S2[k] = ax.w;
    BT[k] = 1.0f;
    const float* gi = g_rgb + 3 * fr.pixel_offset;
    const float* gn = g_normal + 3 * fr.pixel_offset;
    G0[k] = valid ? gi[p] : 0.0f;
    G1[k] = valid ? gi[plane + p] : 0.0f;
    G2[k] = valid ? gi[2 * plane + p] : 0.0f;
    GN0[k] = valid ? gn[p] : 0.0f;
    GN1[k] = valid ? gn[plane + p] : 0.0f;
    GN2[k] = valid ? gn[2 * plane + p] : 0.0f;
    GD[k] = valid ? g_depth[q] : 0.0f;
    GA[k] = valid ? g_alpha[q] : 0.0f;
    GE[k] = valid ? g_dist[q] : 0.0f;
    H0[k] = G0[k]; H1[k] = G1[k]; H2[k] = G2[k]; HD[k] = GD[k];
    HN0[k] = GN0[k]; HN1[k] = GN1[k]; HN2[k] = GN2[k]; HE[k] = GE[k];
    // behind the last entry: the background colour, zero depth, normal and e
    E[k] = __builtin_fma(H2[k], (double)bg2, __builtin_fma(H1[k], (double)bg1, H0[k] * (double)bg0));
  }
  // Per-entry sums: the lane's own pixels sum in FP32; the lanes' sums,
  // which cancel against each other, in FP64.  A lane adds to them only past
  // the alpha test, so they are still zero after an entry no lane blended
  // and are reset only after an entry that was reduced (the empty asm keeps
  // the zeros from being rewritten on every branch of the first strip).
  float acc[kSG];
#pragma unroll
  for (int i = 0; i < kSG; ++i) {
    acc[i] = 0.0f;
    asm volatile("" : "+v"(acc[i]));
  }
  for (int hi = most; hi > 0; hi -= kWave) {
    const int lo = hi > kWave ? hi - kWave : 0;
    if (lo + lane < hi) {
      const uint32_t r = vals[rg.x + lo + lane];
      sm[lane] = rec[r];
      const uint2 tr = trect[r];
      const int rx0 = tr.x & 0xffff, rx1 = tr.x >> 16, ry0 = tr.y & 0xffff;
      slot[lane] = keyoff[r] + (uint32_t)((ty - ry0) * (rx1 - rx0 + 1) + (tx - rx0));
    }
    __syncthreads();
    for (int j = hi - lo - 1; j >= 0; --j) {
      const int pos = lo + j;
      const Surfel& S = sm[j];
      const int xlo = S.sqx & 0xffff, xhi = S.sqx >> 16;
      const int ylo = S.sqy & 0xffff, yhi = S.sqy >> 16;
      const bool xin = (unsigned)(px - xlo) <= (unsigned)(xhi - xlo);
      const SurfelEntry en = surfel_entry(S, px);
      bool any = false;
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        const int row0 = y0 + k * RPP;
        if (ylo > row0 + RPP - 1 || yhi < row0) continue;
        const int py = row0 + ly;
        if (pos >= last[k] || !xin || (unsigned)(py - ylo) > (unsigned)(yhi - ylo)) continue;
        const SurfelHit h = surfel_eval(en, py);
        const float sg = en.opacity * h.Gh;
        const float a = fminf(kAlphaMax, sg);
        if (a < kAlphaMin) continue;
        const float om = 1.0f - a;
        const float inv = __builtin_amdgcn_rcpf(om);
        float Ti = T[k] * inv;
        Ti = __builtin_fmaf(__builtin_fmaf(-Ti, om, T[k]), inv, Ti);  // Newton step
        const float w = a * Ti;
        const double zp = h.z - ZR[k];
        // dDist/dw_i: sum over the other entries m of w_m (z_i - z_m)^2
        const double e = AT[k] * zp * zp - 2.0 * zp * S1[k] + S2[k];
        // G . (v_i - B_i) = G . v_i - E
        double gv = H0[k] * (double)S.c0;
        gv = __builtin_fma(H1[k], (double)S.c1, gv);
        gv = __builtin_fma(H2[k], (double)S.c2, gv);
        gv = __builtin_fma(HD[k], (double)h.z, gv);
        gv = __builtin_fma(HN0[k], (double)S.n0, gv);
        gv = __builtin_fma(HN1[k], (double)S.n1, gv);
        gv = __builtin_fma(HN2[k], (double)S.n2, gv);
        gv = __builtin_fma(HE[k], e, gv);
        const double diff = gv - E[k];
        const float dLda = Ti * __builtin_fmaf(GA[k], BT[k], (float)diff);
        acc[10] += G0[k] * w;
        acc[11] += G1[k] * w;
        acc[12] += G2[k] * w;
        acc[13] += GN0[k] * w;
        acc[14] += GN1[k] * w;
        acc[15] += GN2[k] * w;
        // dL/dz_i: the depth map and the distortion, 2 w_i sum_m w_m (z_i - z_m)
        const float dzv = w * (GD[k] + (float)(2.0 * GE[k] * (zp * AT[k] - S1[k])));
        E[k] = __builtin_fma((double)a, diff, E[k]);
        BT[k] = BT[k] * om;
        T[k] = Ti;
        any = true;
        const bool clamped = sg > kAlphaMax;  // clamped: alpha does not move
        const float dGh = clamped ? 0.0f : dLda * en.opacity;
        if (!clamped) acc[9] += dLda * h.Gh;
        if (h.obj) {
          // z = M2 . (u, v, 1), G = exp(-(u^2 + v^2)/2), (u, v) = (p0, p1) / p2.
          // The chain through the intersection runs in FP64: its FP32
          // rounding is amplified by the conditioning 1/sin of the two
          // planes, squared for a derivative, and a tilted surfel's
          // per-pixel terms cancel in its rotation gradient.  h_u, h_v are
          // rebuilt from the stored FP32 values (the products are exact in
          // FP64); G and the decisions are the forward's.
          const double ex = h.ex, ey = h.ey;
          const double hux = ex * en.m2x + S.kux, huy = ex * en.m2y + S.kuy, huz = ex * en.zc;
          const double hvx = ey * en.m2x + en.kvx, hvy = ey * en.m2y + en.kvy, hvz = ey * en.zc;
          const double p0 = huy * hvz - huz * hvy, p1 = huz * hvx - hux * hvz;
          // 1/p2: hardware reciprocal and two Newton steps (FP64 accuracy;
          // p2 != 0 where the disk term was blended)
          const double p2 = hux * hvy - huy * hvx;
          double ip = __builtin_amdgcn_rcp(p2);
          ip = __builtin_fma(__builtin_fma(-p2, ip, 1.0), ip, ip);
          ip = __builtin_fma(__builtin_fma(-p2, ip, 1.0), ip, ip);
          const double u = p0 * ip, v = p1 * ip;
          const double gGd = (double)h.Gh * dGh, dzd = dzv;
          const double gu = -u * gGd + dzd * en.m2x;
          const double gv = -v * gGd + dzd * en.m2y;
          const double ox = (double)px - fr.cx, oy = (double)py - fr.cy;
          const double dp0 = gu * ip, dp1 = gv * ip, dp2 = -(gu * u + gv * v) * ip;
          // p = h_u x h_v: dL/dh_u = h_v x dL/dp, dL/dh_v = dL/dp x h_u
          const double a0 = hvy * dp2 - hvz * dp1, a1 = hvz * dp0 - hvx * dp2,
                       a2 = hvx * dp1 - hvy * dp0;
          const double b0 = dp1 * huz - dp2 * huy, b1 = dp2 * hux - dp0 * huz,
                       b2 = dp0 * huy - dp1 * hux;
          acc[0] += (float)a0;
          acc[1] += (float)a1;
          acc[2] += (float)a2;
          acc[3] += (float)b0;
          acc[4] += (float)b1;
          acc[5] += (float)b2;
          acc[6] += (float)(ox * a0 + oy * b0 + u * dzd);
          acc[7] += (float)(ox * a1 + oy * b1 + v * dzd);
          acc[8] += (float)(ox * a2 + oy * b2 + dzd);
        } else {
          // the low-pass: z = z_c, G_lp = exp(-|(x, y) - c|^2); its gradient
          // of c reaches M0_z, M1_z (S_u[2], S_v[2]) and, with the principal
          // point's share, R[2]
          const float t = 2.0f * h.Gh * dGh / en.zc;
          const float gx = t * h.ex, gy = t * h.ey;
          acc[2] -= gx;
          acc[5] -= gy;
          const float ocx = (S.cxh - fr.cx) + S.cxl, ocy = (S.cyh - fr.cy) + S.cyl;
          acc[8] += dzv - (gx * ocx + gy * ocy);
        }
      }
      if (__ballot(any) == 0) continue;
      double accd[kSG];
#pragma unroll
      for (int i = 0; i < kSG; ++i) accd[i] = acc[i];
      // value lane >> 2 on every lane of its quad
      const double tot = lds_wave_sum<kSG>(red, accd, lane);
#pragma unroll
      for (int i = 0; i < kSG; ++i) {
        acc[i] = 0.0f;
        asm volatile("" : "+v"(acc[i]));
      }
      const uint32_t sl = slot[j];
      if ((lane & 3) == 0) partial[(size_t)sl * kSG + (lane >> 2)] = (float)tot;
      if (lane == 0) stamp[sl] = epoch;
    }
    __syncthreads();
  }
}

// Per record (surfel, frame): the sum of its keys' partials that this
// backward stamped, FP64.  A group of kSlotGroup lanes shares a record; the
// records come in order of tile count, so the groups of one wave walk lists
// of similar length.
constexpr int kSlotGroup = 8;

__global__ void __launch_bounds__(256) surfel_slot_reduce_kernel(
    uint64_t m, const uint32_t* __restrict__ order, const uint32_t* __restrict__ keyoff,
    const uint32_t* __restrict__ ntiles, const float* __restrict__ partial,
    const uint32_t* __restrict__ stamp, const uint32_t* __restrict__ epoch_dev,
    uint64_t key_capacity, double* __restrict__ sgrad /* [m][kSG] */) {
  const uint32_t epoch = *epoch_dev;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t k = gid / kSlotGroup;
  const int sub = threadIdx.x & (kSlotGroup - 1);
  const bool active = k < m;
  const uint64_t r = active ? order[k] : 0;
  uint32_t cnt = active ? ntiles[r] : 0u;
  const uint32_t off = cnt ? keyoff[r] : 0u;
  if (cnt && (uint64_t)off + cnt > key_capacity) cnt = 0;  // overflowed the key capacity
  double acc[kSG];
#pragma unroll
  for (int j = 0; j < kSG; ++j) acc[j] = 0.0;
  for (uint32_t s = sub; s < cnt; s += kSlotGroup) {
    if (stamp[off + s] != epoch) continue;
    const float* pp = partial + (size_t)(off + s) * kSG;
#pragma unroll
    for (int j = 0; j < kSG; ++j) acc[j] += pp[j];
  }
  // sum over the group's 8 lanes by DPP moves (no LDS round trips): the
  // half-row mirror (partner 7 - l) leaves the group symmetric, then the
  // quad permutes l ^ 2 and l ^ 1 finish; all 8 lanes end with the same
  // total (each add is commutative, so mirrored lanes agree bitwise)
  static_assert(kSlotGroup == 8, "the group reduction is a half-row of DPP lanes");
#pragma unroll
  for (int j = 0; j < kSG; ++j) acc[j] += dpp<kDppHalfMirror>(acc[j]);
#pragma unroll
  for (int j = 0; j < kSG; ++j) acc[j] += dpp<kDppQuadXor2>(acc[j]);
#pragma unroll
  for (int j = 0; j < kSG; ++j) acc[j] += dpp<kDppQuadXor1>(acc[j]);
  if (!active || !ntiles[r]) return;
#pragma unroll
  for (int j0 = 0; j0 < kSG; j0 += kSlotGroup) {
    double v = acc[j0];
#pragma unroll
    for (int j = j0 + 1; j < j0 + kSlotGroup && j < kSG; ++j) v = sub == j - j0 ? acc[j] : v;
    if (j0 + sub < kSG) sgrad[r * kSG + j0 + sub] = v;
  }
}

// Chain rule from the per-key sums to the parameters (FP64), per surfel and
// frame: the record's sum of its key partials gives the gradients of the
// columns of M = K [A | B | mc]: A = s_u t_u, B = s_v t_v,
// mc = R_f mu + t_f, t_u, t_v, t_w the camera-frame axes R_f R_g.  The pose
// twist (rho, phi) moves every camera-frame vector y by phi x y and mc by
// rho as well, so dL/dphi = sum y x dL/dy.
template <int DEG>
__global__ void __launch_bounds__(256) surfel_preprocess_bwd_kernel(
    int64_t n, int n_frames, const FrameDesc* __restrict__ frames,
    const float* __restrict__ poses, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh,
    const uint32_t* __restrict__ ntiles, const uint32_t* __restrict__ keyoff,
    const double* __restrict__ sgrad, uint64_t key_capacity, float* __restrict__ g_means,
    float* __restrict__ g_log_scales, float* __restrict__ g_quats, float* __restrict__ g_opac,
    float* __restrict__ g_sh, double* __restrict__ twist_partial /* [F][n_waves][6] */) {
#pragma clang fp contract(off)
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = g0 < n;
  const int64_t g = active ? g0 : 0;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t wave_id = g0 / kWave;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const double su = active ? exp((double)log_scales[2 * g]) : 1.0;
  const double sv = active ? exp((double)log_scales[2 * g + 1]) : 1.0;
  double qh[4];
  for (int a = 0; a < 4; ++a) qh[a] = active ? quats[4 * g + a] : (a == 0 ? 1.0 : 0.0);
  const double qn = sqrt(qh[0] * qh[0] + qh[1] * qh[1] + qh[2] * qh[2] + qh[3] * qh[3]);
  for (int a = 0; a < 4; ++a) qh[a] /= qn;
  const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  const double Rg[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                        2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                        2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
  const double o = active ? 1.0 / (1.0 + exp(-(double)opac[g])) : 0.0;
  const double mu[3] = {active ? (double)means[3 * g] : 0.0,
                        active ? (double)means[3 * g + 1] : 0.0,
                        active ? (double)means[3 * g + 2] : 0.0};
  const float* shg = sh + g * nb * 3;
  double dmu[3] = {0, 0, 0}, dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dls[2] = {0, 0}, dop = 0.0;
  float dsh[nb * 3];
  for (int i = 0; i < nb * 3; ++i) dsh[i] = 0.0f;
  bool kept = false;
  for (int f = 0; f < n_frames; ++f) {
    double tw[6] = {0, 0, 0, 0, 0, 0};
    const int64_t r = (int64_t)f * n + g;
    uint32_t cnt = active ? ntiles[r] : 0u;
    kept = kept || cnt > 0;
    const uint32_t off = cnt ? keyoff[r] : 0u;
    if (cnt && (uint64_t)off + cnt > key_capacity) cnt = 0;  // overflowed the key capacity
    if (cnt > 0) {
      double K[kSG];
      for (int i = 0; i < kSG; ++i) K[i] = sgrad[r * kSG + i];
      const FrameDesc fr = frames[f];
      double W[9], tf[3];
      load_pose(poses, f, W, tf);
      double mc[3], T[9];
      for (int i = 0; i < 3; ++i) {
        mc[i] = W[i * 3 + 0] * mu[0] + W[i * 3 + 1] * mu[1] + W[i * 3 + 2] * mu[2] + tf[i];
        for (int j = 0; j < 3; ++j)
          T[i * 3 + j] = W[i * 3 + 0] * Rg[0 * 3 + j] + W[i * 3 + 1] * Rg[1 * 3 + j] +
                         W[i * 3 + 2] * Rg[2 * 3 + j];
      }
      const double fx = fr.fx, fy = fr.fy;
      // gradients of the columns A, B, mc of M = K [A | B | mc]
      double dcol[3][3];
      for (int j = 0; j < 3; ++j) {
        dcol[j][0] = -fx * K[j];
        dcol[j][1] = -fy * K[3 + j];
        dcol[j][2] = K[6 + j];
      }
      const double tu[3] = {T[0], T[3], T[6]}, tv[3] = {T[1], T[4], T[7]};
      const double tn[3] = {T[2], T[5], T[8]};
      const double sgn = (tn[0] * mc[0] + tn[1] * mc[1] + tn[2] * mc[2]) < 0.0 ? 1.0 : -1.0;
      double dT[3][3];  // dT[j] = dL/d(column j of T)
      for (int i = 0; i < 3; ++i) {
        dT[0][i] = su * dcol[0][i];
        dT[1][i] = sv * dcol[1][i];
        dT[2][i] = sgn * K[13 + i];
      }
      dls[0] += su * (dcol[0][0] * tu[0] + dcol[0][1] * tu[1] + dcol[0][2] * tu[2]);
      dls[1] += sv * (dcol[1][0] * tv[0] + dcol[1][1] * tv[1] + dcol[1][2] * tv[2]);
      // T = R_f R_g
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          dR[i * 3 + j] += W[0 * 3 + i] * dT[j][0] + W[1 * 3 + i] * dT[j][1] +
                           W[2 * 3 + i] * dT[j][2];
      dop += K[9];
      // colour: c = max(0, raw), raw = sum_k sh_k Y_k(dir) + 1/2
      double dir[3];
      const double dist = view_dir(W, tf, mu, dir);
      double Y[16];
      sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
      double raw[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < nb; ++k)
        for (int c = 0; c < 3; ++c) raw[c] += (double)shg[k * 3 + c] * Y[k];
      double draw[3];
      for (int c = 0; c < 3; ++c) draw[c] = raw[c] + 0.5 > 0.0 ? K[10 + c] : 0.0;
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
      const double* dmc = dcol[2];
      for (int a = 0; a < 3; ++a)
        dmu[a] += W[0 * 3 + a] * dmc[0] + W[1 * 3 + a] * dmc[1] + W[2 * 3 + a] * dmc[2] + dd[a];
      // twist: the camera centre moves by -R_f^T rho, so the view direction
      // adds R_f dd to rho; mc and the three axes rotate with phi
      for (int a = 0; a < 3; ++a)
        tw[a] = dmc[a] + W[a * 3 + 0] * dd[0] + W[a * 3 + 1] * dd[1] + W[a * 3 + 2] * dd[2];
      const double* ys[4] = {mc, tu, tv, tn};
      const double* gs[4] = {dmc, dT[0], dT[1], dT[2]};
      for (int m = 0; m < 4; ++m) {
        const double* Yv = ys[m];
        const double* Gv = gs[m];
        tw[3] += Yv[1] * Gv[2] - Yv[2] * Gv[1];
        tw[4] += Yv[2] * Gv[0] - Yv[0] * Gv[2];
        tw[5] += Yv[0] * Gv[1] - Yv[1] * Gv[0];
      }
    }
    {
      // the wave's six twist sums by the transposing VALU reduction
      int idx;
      bool writer;
      const double s = wave_transpose_sum<6>(tw, threadIdx.x & (kWave - 1), idx, writer);
      if (writer) twist_partial[((int64_t)f * n_waves + wave_id) * 6 + idx] = s;
    }
  }
  if (!active) return;
  if (!kept) {  // no frame sees it (culled, or a non-finite parameter)
    for (int a = 0; a < 3; ++a) g_means[g * 3 + a] = 0.0f;
    for (int a = 0; a < 4; ++a) g_quats[g * 4 + a] = 0.0f;
    g_log_scales[2 * g] = g_log_scales[2 * g + 1] = 0.0f;
    g_opac[g] = 0.0f;
    for (int i = 0; i < nb * 3; ++i) g_sh[g * nb * 3 + i] = 0.0f;
    return;
  }
  g_log_scales[2 * g] = (float)dls[0];
  g_log_scales[2 * g + 1] = (float)dls[1];
  quat_grad(qh, qn, dR, g_quats + g * 4);
  for (int a = 0; a < 3; ++a) g_means[g * 3 + a] = (float)dmu[a];
  g_opac[g] = (float)(dop * o * (1.0 - o));
  float* gsh = g_sh + g * nb * 3;
  for (int i = 0; i < nb * 3; ++i) gsh[i] = dsh[i];
}

}  // namespace

size_t surfel_record_bytes() { return sizeof(Surfel); }
size_t surfel_square_offset() { return offsetof(Surfel, sqx); }
int surfel_grad_values() { return kSG; }
int64_t surfel_preprocess_bwd_waves(int64_t n) { return ((n + 255) / 256) * 4; }

void launch_surfel_preprocess(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                              const float* poses, const float* means, const float* log_scales,
                              const float* quats, const float* opac, const float* sh, int deg,
                              int tile_w, int tile_h, void* rec, uint2* trect,
                              uint32_t* depth_key, uint32_t* rec_id, uint32_t* ntiles) {
  if (n <= 0 || F <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)std::min(F, 65535));
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
                       float* normal, float* dist, float* t_final, int32_t* n_last,
                       float* dist_aux, uint32_t* nproc, const uint32_t* prev_nproc,
                       uint32_t* order, bool xcd_groups, unsigned long long* pairs) {
  if (n_tiles <= 0) return;
  const int groups = tile_schedule_groups(xcd_groups);
  launch_tile_order(st, n_tiles, groups, prev_nproc, order);
  const dim3 grid(tile_schedule_grid(n_tiles, groups));
#define GSR_SURF_FWD_C(W, H, C)                                                             \
  hipLaunchKernelGGL((surfel_fwd_kernel<W, H, C>), grid, dim3(kWave), 0, st, n_tiles,       \
                     groups, order, nproc, pairs, F, frames, ranges, vals, (const Surfel*)rec, \
                     bg[0], bg[1], bg[2], rgb, depth, alpha, normal, dist, t_final, n_last,  \
                     dist_aux)
#define GSR_SURF_FWD(W, H)                 \
  if (pairs) GSR_SURF_FWD_C(W, H, true);   \
  else GSR_SURF_FWD_C(W, H, false)
  if (tw == 16 && th == 16) GSR_SURF_FWD(16, 16);
  else if (tw == 8 && th == 8) GSR_SURF_FWD(8, 8);
  else if (tw == 32 && th == 8) GSR_SURF_FWD(32, 8);
  else if (tw == 16 && th == 8) GSR_SURF_FWD(16, 8);
  else if (tw == 32 && th == 16) GSR_SURF_FWD(32, 16);
#undef GSR_SURF_FWD
#undef GSR_SURF_FWD_C
}

void launch_surfel_bwd(hipStream_t st, int tw, int th, int n_tiles, int F,
                       const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                       const void* rec, const uint2* trect, const uint32_t* keyoff,
                       const float* bg, const float* g_rgb, const float* g_depth,
                       const float* g_alpha, const float* g_normal, const float* g_dist,
                       const float* t_final, const int32_t* n_last, const float* dist_aux,
                       float* partial, uint32_t* stamp, const uint32_t* epoch,
                       const uint32_t* nproc, uint32_t* order, bool xcd_groups) {
  if (n_tiles <= 0) return;
  const int groups = tile_schedule_groups(xcd_groups);
  launch_tile_order(st, n_tiles, groups, nproc, order);
  const dim3 grid(tile_schedule_grid(n_tiles, groups));
#define GSR_SURF_BWD(W, H)                                                                   \
  hipLaunchKernelGGL((surfel_bwd_kernel<W, H>), grid, dim3(kWave), 0, st, n_tiles, groups,    \
                     order, nproc, F, frames, ranges, vals, (const Surfel*)rec, trect, keyoff, \
                     bg[0], bg[1], bg[2], g_rgb, g_depth, g_alpha, g_normal, g_dist, t_final,  \
                     n_last, dist_aux, partial, stamp, epoch)
  if (tw == 16 && th == 16) GSR_SURF_BWD(16, 16);
  else if (tw == 8 && th == 8) GSR_SURF_BWD(8, 8);
  else if (tw == 32 && th == 8) GSR_SURF_BWD(32, 8);
  else if (tw == 16 && th == 8) GSR_SURF_BWD(16, 8);
  else if (tw == 32 && th == 16) GSR_SURF_BWD(32, 16);
#undef GSR_SURF_BWD
}

void launch_surfel_slot_reduce(hipStream_t st, uint64_t m, const uint32_t* order,
                               const uint32_t* keyoff, const uint32_t* ntiles,
                               const float* partial, const uint32_t* stamp,
                               const uint32_t* epoch, uint64_t key_capacity, double* sgrad) {
  if (m == 0) return;
  const uint64_t threads = m * kSlotGroup;
  hipLaunchKernelGGL(surfel_slot_reduce_kernel, dim3((unsigned)((threads + 255) / 256)),
                     dim3(256), 0, st, m, order, keyoff, ntiles, partial, stamp, epoch,
                     key_capacity, sgrad);
}

void launch_surfel_preprocess_bwd(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                                  const float* poses, const float* means,
                                  const float* log_scales, const float* quats,
                                  const float* opac, const float* sh, int deg,
                                  const uint32_t* ntiles, const uint32_t* keyoff,
                                  const double* sgrad, uint64_t key_capacity, float* g_means,
                                  float* g_log_scales, float* g_quats, float* g_opac,
                                  float* g_sh, double* twist_partial, float* g_twist) {
  if (n > 0) {
    const dim3 grid((unsigned)((n + 255) / 256));
#define GSR_SURF_PRE_BWD(D)                                                                   \
  hipLaunchKernelGGL(surfel_preprocess_bwd_kernel<D>, grid, dim3(256), 0, st, n, F, frames,  \
                     poses, means, log_scales, quats, opac, sh, ntiles, keyoff, sgrad,         \
                     key_capacity, g_means, g_log_scales, g_quats, g_opac, g_sh, twist_partial)
    switch (deg) {
      case 0: GSR_SURF_PRE_BWD(0); break;
      case 1: GSR_SURF_PRE_BWD(1); break;
      case 2: GSR_SURF_PRE_BWD(2); break;
      default: GSR_SURF_PRE_BWD(3); break;
    }
#undef GSR_SURF_PRE_BWD
  }
  launch_twist_reduce(st, F, twist_partial, n > 0 ? surfel_preprocess_bwd_waves(n) : 0, g_twist);
}

}  // namespace gsr
