// raster.hip -- front-to-back compositing (forward) and its reverse-order
// backward, one wavefront per tile.
//
// Forward, per pixel, over its tile's list in (depth, index) order
// (DROID-Splat eqn:rendering, C = sum_i c_i a_i prod_{j<i}(1 - a_j), with
// a_i = sigma_i G_i): entries whose 3-sigma square misses the pixel are
// skipped; a = min(0.99, sigma exp(-q/2)); a < 1/255 is skipped; the pixel
// stops before an entry that would drop T below 1e-4.  Outputs RGB + T bg,
// the alpha-blended depth sum z_i a_i T_i and accumulated alpha 1 - T.
//
// Layout on CDNA4: a tile of TW x TH pixels is one 64-lane wave; lane l owns
// column l % TW and PIX = TW*TH/64 pixels in row strips of 64/TW rows, so a
// whole strip is skipped (wave-uniform branch) when an entry's square misses
// its rows.  64 records at a time are staged in LDS by the wave itself and
// read back as broadcasts; per-entry values stay wave-uniform.
//
// Backward: the wave walks the tile's processed prefix from the back.  Each
// lane recomputes alpha bit-identically (same helpers, explicit fma),
// rebuilds T_i = T_{i+1} / (1 - a_i) (reciprocal plus one Newton step) and
// carries what is seen behind each entry through the convex recurrence
// B_{i-1} = a_i c_i + (1 - a_i) B_i from B = background (depth from 0, the
// transmittance behind from 1), so that dC/da_i = T_i (c_i - B_i): T_i only
// scales the result and the recurrence damps rounding instead of
// accumulating it.  Colour and depth enter only through G . B (G the pixel's
// upstream gradient), which is what the lane keeps, in FP64.  The
// screen-space gradient of an entry is taken with respect to (u, v, Sigma'):
// with Q = Sigma'^-1 = L L^T (L the factor the forward already uses) and d
// the offset, dq/dd = 2 Q d and dq/dSigma' = -(Q d)(Q d)^T,
// Q d = L (L^T d); this avoids the ill-conditioned -Q dQ Q step from conic
// gradients for elongated Gaussians.  The 10 per-entry values are summed
// over the lane's pixels and then across the wave in FP64 through LDS
// (fixed order); the result for this (tile, entry) key goes to its own slot
// (no atomics), stamped with the backward's epoch so the per-record
// reduction can skip slots of keys that no pixel reached.
#include "launch.h"
#include "wave_util.h"

namespace gsr {

// Tile schedule.  The tiles are split into kQueues groups of contiguous tile
// ids (neighbouring tiles share Gaussians, so a group shares one XCD's L2);
// workgroups are dealt to the XCDs in turn, so workgroup b runs on XCD
// b % kQueues and takes the (b / kQueues)-th tile of that group.  The
// hardware dispatches workgroups in index order, so sorting each group by
// descending expected work gives a longest-first list schedule without any
// queue or atomic: long tiles start first and the short ones fill the tail.
constexpr int kOrderBins = 1024;

__device__ __forceinline__ uint32_t work_bucket(uint32_t w) {
  if (w == 0) return 0;
  const int lz = __clz(w);
  const int e = 31 - lz;                                      // floor(log2 w)
  const uint32_t frac = e > 0 ? ((w << (lz + 1)) >> 27) : 0;  // next 5 bits
  return min((uint32_t)kOrderBins - 1, 1u + (uint32_t)e * 32u + frac);
}

// One workgroup per group: a counting sort of the group's tiles by
// descending work bucket (order inside a bucket is arbitrary; results do not
// depend on it).  Work = processed entries of a previous forward over the
// same tiles (`nproc`); without it the tiles keep their spatial order.
__global__ void __launch_bounds__(1024) tile_order_kernel(int n_tiles, int groups,
                                                          const uint32_t* __restrict__ nproc,
                                                          uint32_t* __restrict__ order) {
  static_assert(kOrderBins == 1024, "one thread per bin in the offsets scan");
  __shared__ uint32_t bins[kOrderBins];
  const int q = blockIdx.x;
  const int per = (n_tiles + groups - 1) / groups;
  const int t0 = q * per, t1 = min(n_tiles, t0 + per);
  for (int i = threadIdx.x; i < kOrderBins; i += blockDim.x) bins[i] = 0;
  __syncthreads();
  if (!nproc) {
    for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) order[t] = (uint32_t)t;
    return;
  }
  for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x)
    atomicAdd(&bins[work_bucket(nproc[t])], 1u);
  __syncthreads();
  {  // exclusive offsets, largest bucket first: thread i takes bin 1023 - i
    __shared__ uint32_t wtot[kOrderBins / kWave];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int bin = kOrderBins - 1 - (int)threadIdx.x;
    const uint32_t c = bins[bin];
    uint32_t v = c;  // inclusive scan over the wave's lanes
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t u = __shfl_up(v, o, kWave);
      if (lane >= o) v += u;
    }
    if (lane == kWave - 1) wtot[wv] = v;
    __syncthreads();
    uint32_t base = 0;
    for (int k = 0; k < wv; ++k) base += wtot[k];
    bins[bin] = base + v - c;
  }
  __syncthreads();
  for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
    const uint32_t pos = atomicAdd(&bins[work_bucket(nproc[t])], 1u);
    order[t0 + pos] = (uint32_t)t;
  }
}

// The tile of workgroup `bid`, or -1 past the end of its group.

template <int TW, int TH, bool COUNT, bool MEDIAN, int BATCH>
__device__ __forceinline__ void composite_fwd_tile(
    int tile, Record* sm, int n_frames, const FrameDesc* __restrict__ frames,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const Record* __restrict__ rec, float bg0, float bg1, float bg2, float* __restrict__ rgb,
    float* __restrict__ depth, float* __restrict__ alpha, float* __restrict__ t_final,
    int32_t* __restrict__ n_last, uint32_t* __restrict__ tile_nproc,
    unsigned long long* __restrict__ pair_count, int32_t* __restrict__ med_pos) {
  constexpr int PIX = TW * TH / kWave;
  constexpr int RPP = kWave / TW;  // rows per strip
  const int f = frame_of_tile(frames, n_frames, tile);
  const FrameDesc fr = frames[f];
  const int lt = tile - fr.tile_offset;
  const int x0 = (lt % fr.grid_x) * TW, y0 = (lt / fr.grid_x) * TH;
  const int lane = threadIdx.x;
  const int px = x0 + lane % TW;
  const int ly = lane / TW;
  const uint2 rg = ranges[tile];

  // D: alpha-blended depth, or (MEDIAN) the depth of the entry after which
  // T first falls below 1/2, at list position mpos (-1: none yet)
  float T[PIX], C0[PIX], C1[PIX], C2[PIX], D[PIX];
  int last[PIX], mpos[PIX];
  bool done[PIX];
  uint32_t hits = 0;  // (pixel, entry) pairs whose square test passed (COUNT only)
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    T[k] = 1.0f; C0[k] = C1[k] = C2[k] = D[k] = 0.0f; last[k] = 0; mpos[k] = -1;
    const int py = y0 + k * RPP + ly;
    done[k] = !(px < fr.width && py < fr.height);
  }
  for (uint32_t b = rg.x; b < rg.y; b += BATCH) {
    bool live = false;
#pragma unroll
    for (int k = 0; k < PIX; ++k) live |= !done[k];
    if (__ballot(live) == 0) break;
#pragma unroll
    for (int i = lane; i < BATCH; i += kWave) {
      const uint32_t e = b + (uint32_t)i;
      if (e < rg.y) sm[i] = rec[vals[e]];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)BATCH, rg.y - b);
    for (int j = 0; j < cnt; ++j) {
      const Record& R = sm[j];
      // The fields every pixel strip reads up to the alpha test, loaded from
      // LDS once per entry (read in each strip, they would be reloaded there
      // with the address rebuilt each time).
      float e_vhi = R.v_hi, e_vlo = R.v_lo, e_a1 = R.a1, e_a2 = R.a2, e_a3 = R.a3, e_op = R.opacity;
      asm volatile("" : "+v"(e_vhi), "+v"(e_vlo), "+v"(e_a1), "+v"(e_a2), "+v"(e_a3), "+v"(e_op));
      const int xlo = R.sqx & 0xffff, xhi = R.sqx >> 16;
      const int ylo = R.sqy & 0xffff, yhi = R.sqy >> 16;
      const bool xin = (unsigned)(px - xlo) <= (unsigned)(xhi - xlo);
      const float dx = dx_of(R.u_hi, R.u_lo, px);
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        const int row0 = y0 + k * RPP;
        if (ylo > row0 + RPP - 1 || yhi < row0) continue;  // strip missed (uniform)
        const int py = row0 + ly;
        if (done[k] || !xin || (unsigned)(py - ylo) > (unsigned)(yhi - ylo)) continue;
        if (COUNT) ++hits;
        const float dy = dx_of(e_vhi, e_vlo, py);
        const float q = q_of(e_a1, e_a2, e_a3, dx, dy);
        const float g = gauss_of(q);
        const float a = fminf(kAlphaMax, e_op * g);
        if (a < kAlphaMin) continue;
        const float Tn = T[k] * (1.0f - a);
        if (Tn < kTMin) { done[k] = true; continue; }
        const float w = a * T[k];
        C0[k] += R.c0 * w;
        C1[k] += R.c1 * w;
        C2[k] += R.c2 * w;
        if (MEDIAN) {
          if (mpos[k] < 0 && Tn < 0.5f) {
            mpos[k] = (int)(b + j - rg.x);
            D[k] = R.z;
          }
        } else {
          D[k] += R.z * w;
        }
        T[k] = Tn;
        last[k] = (int)(b + j + 1 - rg.x);
      }
    }
    __syncthreads();
  }
  int mx = 0;
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
      depth[fr.pixel_offset + p] = D[k];
      alpha[fr.pixel_offset + p] = 1.0f - T[k];
      t_final[fr.pixel_offset + p] = T[k];
      n_last[fr.pixel_offset + p] = last[k];
      if (MEDIAN) med_pos[fr.pixel_offset + p] = mpos[k];
      mx = max(mx, last[k]);
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) tile_nproc[tile] = (uint32_t)mx;
  if (COUNT) {
    unsigned long long h = hits;
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
    if (lane == 0) atomicAdd(pair_count, h);
  }
}


template <int TW, int TH, bool COUNT, bool MEDIAN, int BATCH>
__global__ void __launch_bounds__(64) composite_fwd_kernel(
    int n_tiles, int groups, const uint32_t* __restrict__ order, int n_frames,
    const FrameDesc* __restrict__ frames, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const Record* __restrict__ rec, float bg0, float bg1,
    float bg2, float* __restrict__ rgb, float* __restrict__ depth, float* __restrict__ alpha,
    float* __restrict__ t_final, int32_t* __restrict__ n_last, uint32_t* __restrict__ tile_nproc,
    unsigned long long* __restrict__ pair_count, int32_t* __restrict__ med_pos) {
  __shared__ Record sm[BATCH];
  const int tile = tile_of_block(blockIdx.x, n_tiles, groups, order);
  if (tile < 0) return;
  composite_fwd_tile<TW, TH, COUNT, MEDIAN, BATCH>(tile, sm, n_frames, frames, ranges, vals, rec, bg0,
                                             bg1, bg2, rgb, depth, alpha, t_final, n_last,
                                             tile_nproc, pair_count, med_pos);
}

template <int TW, int TH, bool MEDIAN, int BATCH>
__device__ __forceinline__ void composite_bwd_tile(
    int tile, Record* sm, uint32_t* slot, double* red, uint32_t epoch, int n_frames,
    const FrameDesc* __restrict__ frames,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const Record* __restrict__ rec, const uint2* __restrict__ trect,
    const uint32_t* __restrict__ keyoff, const uint32_t* __restrict__ tile_nproc, float bg0,
    float bg1, float bg2, const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
    const float* __restrict__ g_alpha, const float* __restrict__ t_final,
    const int32_t* __restrict__ n_last, float* __restrict__ partial,
    uint32_t* __restrict__ stamp, const int32_t* __restrict__ med_pos) {
  constexpr int PIX = TW * TH / kWave;
  constexpr int RPP = kWave / TW;
  const uint32_t nproc = tile_nproc[tile];
  if (nproc == 0) return;
  const int f = frame_of_tile(frames, n_frames, tile);
  const FrameDesc fr = frames[f];
  const int lt = tile - fr.tile_offset;
  const int tx = lt % fr.grid_x, ty = lt / fr.grid_x;
  const int x0 = tx * TW, y0 = ty * TH;
  const int lane = threadIdx.x;
  const int px = x0 + lane % TW;
  const int ly = lane / TW;
  // the key reduction leaves value min(lane >> 2, 9) on each quad (lanes
  // 40..63 repeat value 9 and write nothing); the covariance sums carry
  // twice the gradient (the 1/2 is a power of two: exact)
  const int red_v = min(lane >> 2, kNG - 1);
  const bool red_writer = (lane & 3) == 0 && (lane >> 2) < kNG;
  const double red_scale = (red_v >= 2 && red_v <= 4) ? 0.5 : 1.0;
  const uint2 rg = ranges[tile];
  const int64_t plane = (int64_t)fr.width * fr.height;

  // per pixel: T_{i+1}; the transmittance seen behind the current entry
  // (normalised by T_{i+1}); upstream gradients.  dL/da_i needs the upstream-
  // weighted difference G . (c_i - B_i) between the entry's colour (and
  // depth) and what is seen behind it, B_i.  That difference cancels on
  // surfaces of uniform colour, and the gradient of a large Gaussian sums it
  // over up to 10^5 pixels, so it is formed in FP64.  G is fixed per pixel,
  // so the recursion B_i = B_{i+1} + a_i (c_i - B_{i+1}) carries over to the
  // scalar E = G . B, which is what the pixel keeps (in FP64), together with
  // G itself in FP64.
  float T[PIX], BT[PIX];
  double E[PIX], H0[PIX], H1[PIX], H2[PIX], HZ[PIX];
  float G0[PIX], G1[PIX], G2[PIX], GD[PIX], GA[PIX];
  int last[PIX];
  // MEDIAN: the depth is the z of the entry at list position mp, so G_D
  // reaches that entry's z only and no alpha
  int mp[PIX];
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    const int py = y0 + k * RPP + ly;
    const bool valid = px < fr.width && py < fr.height;
    const int64_t p = (int64_t)py * fr.width + px;
    last[k] = valid ? n_last[fr.pixel_offset + p] : 0;
    mp[k] = (MEDIAN && valid) ? med_pos[fr.pixel_offset + p] : -1;
    T[k] = valid ? t_final[fr.pixel_offset + p] : 1.0f;
    BT[k] = 1.0f;
    const float* gi = g_rgb + 3 * fr.pixel_offset;
    G0[k] = valid ? gi[p] : 0.0f;
    G1[k] = valid ? gi[plane + p] : 0.0f;
    G2[k] = valid ? gi[2 * plane + p] : 0.0f;
    GD[k] = valid ? g_depth[fr.pixel_offset + p] : 0.0f;
    GA[k] = valid ? g_alpha[fr.pixel_offset + p] : 0.0f;
    H0[k] = G0[k]; H1[k] = G1[k]; H2[k] = G2[k];
    HZ[k] = MEDIAN ? 0.0 : (double)GD[k];
    // behind the last entry: the background colour at depth 0
    E[k] = __builtin_fma(H2[k], (double)bg2, __builtin_fma(H1[k], (double)bg1, H0[k] * (double)bg0));
  }
  // Per-entry sums.  With p = a dL/da, dL/dq = -p/2: gu, gv carry
  // sum(-p Q d), the gradient of the centre, and gS* carry
  // sum(p (Q d)(Q d)^T), twice the gradient of the 2D covariance; the 1/2 is
  // applied once per key (a power of two: exact).  A lane adds to them only
  // past the alpha test, so they are still zero after an entry no lane
  // blended, and are reset only after an entry that was reduced.  The empty
  // asm hides the zeros from constant folding, so that they are set in place
  // rather than rewritten on every branch of the first strip.
  float gu = 0.f, gv = 0.f, gs = 0.f;
  double gSxx = 0.0, gSxy = 0.0, gSyy = 0.0;
  float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gz = 0.f;
  asm volatile("" : "+v"(gu), "+v"(gv), "+v"(gs), "+v"(gSxx), "+v"(gSxy), "+v"(gSyy),
               "+v"(gc0), "+v"(gc1), "+v"(gc2), "+v"(gz));
  for (int hi = (int)nproc; hi > 0; hi -= BATCH) {
    const int lo = max(0, hi - BATCH);
#pragma unroll
    for (int i = lane; i < BATCH; i += kWave) {
      if (lo + i < hi) {
        const uint32_t r = vals[rg.x + lo + i];
        const Record R = rec[r];
        sm[i] = R;
        const uint2 tr = trect[r];
        const int rx0 = tr.x & 0xffff, rx1 = tr.x >> 16, ry0 = tr.y & 0xffff;
        slot[i] = keyoff[r] + (uint32_t)((ty - ry0) * (rx1 - rx0 + 1) + (tx - rx0));
      }
    }
    __syncthreads();
    for (int j = hi - lo - 1; j >= 0; --j) {
      const int pos = lo + j;
      const Record& R = sm[j];
      // The fields every pixel strip reads, loaded from LDS once per entry
      // (read in each strip, they would be reloaded there with the address
      // rebuilt each time).
      float e_vhi = R.v_hi, e_vlo = R.v_lo, e_a1 = R.a1, e_a2 = R.a2, e_a3 = R.a3, e_op = R.opacity;
      asm volatile("" : "+v"(e_vhi), "+v"(e_vlo), "+v"(e_a1), "+v"(e_a2), "+v"(e_a3), "+v"(e_op));
      const int xlo = R.sqx & 0xffff, xhi = R.sqx >> 16;
      const int ylo = R.sqy & 0xffff, yhi = R.sqy >> 16;
      const bool xin = (unsigned)(px - xlo) <= (unsigned)(xhi - xlo);
      const float dx = dx_of(R.u_hi, R.u_lo, px);
      const float a1dx = e_a1 * dx;
      const double c0 = R.c0, c1 = R.c1, c2 = R.c2, cz = R.z;
      bool any = false;
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        const int row0 = y0 + k * RPP;
        if (ylo > row0 + RPP - 1 || yhi < row0) continue;
        const int py = row0 + ly;
        if (pos >= last[k] || !xin || (unsigned)(py - ylo) > (unsigned)(yhi - ylo)) continue;
        const float dy = dx_of(e_vhi, e_vlo, py);
        const float q = q_of(e_a1, e_a2, e_a3, dx, dy);
        const float g = gauss_of(q);
        const float sg = e_op * g;
        const float a = fminf(kAlphaMax, sg);
        if (a < kAlphaMin) continue;
        const float om = 1.0f - a;
        const float inv = __builtin_amdgcn_rcpf(om);
        float Ti = T[k] * inv;
        Ti = __builtin_fmaf(__builtin_fmaf(-Ti, om, T[k]), inv, Ti);  // Newton step
        const float w = a * Ti;
        // G . (c_i - B_i) = G . c_i - E
        double gc = __builtin_fma(H2[k], c2, __builtin_fma(H1[k], c1, H0[k] * c0));
        if (!MEDIAN) gc = __builtin_fma(HZ[k], cz, gc);
        const double diff = gc - E[k];
        // dL/da_i = T_i [G . (c_i - B_i) + G_A BT_i]
        const float dLda = Ti * __builtin_fmaf(GA[k], BT[k], (float)diff);
        gc0 += G0[k] * w;
        gc1 += G1[k] * w;
        gc2 += G2[k] * w;
        if (MEDIAN)
          gz += pos == mp[k] ? GD[k] : 0.0f;
        else
          gz += GD[k] * w;
        // step the 'behind' state in front of entry i
        E[k] = __builtin_fma((double)a, diff, E[k]);
        BT[k] = BT[k] * om;
        T[k] = Ti;
        any = true;
        if (sg > kAlphaMax) continue;  // clamped: alpha does not move
        gs += dLda * g;
        const float pa = a * dLda;
        // Q d = L (L^T d), L^T d = (a1 dx + a2 dy, a3 dy)
        const float m = __builtin_fmaf(e_a2, dy, a1dx);
        const float b = e_a3 * dy;
        const float qx = e_a1 * m;
        const float qy = __builtin_fmaf(e_a2, m, e_a3 * b);
        gu = __builtin_fmaf(-pa, qx, gu);
        gv = __builtin_fmaf(-pa, qy, gv);
        // Each pixel adds the rank-1 matrix p (Q d)(Q d)^T.  Formed in FP64
        // its three entries stay exactly rank-1; rounded one by one in FP32
        // they would not, and a Gaussian at the near plane has scale
        // gradients that read the near-null direction of the summed matrix.
        {
          const double pd = pa, qxd = qx, qyd = qy;
          const double t = pd * qxd;
          gSxx = __builtin_fma(t, qxd, gSxx);
          gSxy = __builtin_fma(t, qyd, gSxy);
          gSyy = __builtin_fma(pd * qyd, qyd, gSyy);
        }
      }
      if (__ballot(any) == 0) continue;
      // The lanes' values of one key cancel against each other: sum them in
      // FP64 (the key's total is stored as FP32; the per-record sum over its
      // keys is FP64 again)
      const double vals10[kNG] = {gu, gv, gSxx, gSxy, gSyy, gs, gc0, gc1, gc2, gz};
      const double tot = lds_wave_sum<kNG>(red, vals10, lane);
      gu = gv = gs = gc0 = gc1 = gc2 = gz = 0.f;
      gSxx = gSxy = gSyy = 0.0;
      asm volatile("" : "+v"(gu), "+v"(gv), "+v"(gs), "+v"(gSxx), "+v"(gSxy), "+v"(gSyy),
                   "+v"(gc0), "+v"(gc1), "+v"(gc2), "+v"(gz));
      const uint32_t sl = slot[j];
      if (red_writer) partial[(size_t)sl * kNG + red_v] = (float)(tot * red_scale);
      if (lane == 1) stamp[sl] = epoch;
    }
    __syncthreads();
  }
}

template <int TW, int TH, bool MEDIAN, int BATCH>
__global__ void __launch_bounds__(64, (TW * TH <= 256) ? 4 : 1) composite_bwd_kernel(
    int n_tiles, int groups, const uint32_t* __restrict__ order, int n_frames,
    const FrameDesc* __restrict__ frames, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const Record* __restrict__ rec,
    const uint2* __restrict__ trect, const uint32_t* __restrict__ keyoff,
    const uint32_t* __restrict__ tile_nproc, float bg0, float bg1, float bg2,
    const float* __restrict__ g_rgb, const float* __restrict__ g_depth,
    const float* __restrict__ g_alpha, const float* __restrict__ t_final,
    const int32_t* __restrict__ n_last, float* __restrict__ partial,
    uint32_t* __restrict__ stamp, const uint32_t* __restrict__ epoch_dev,
    const int32_t* __restrict__ med_pos) {
  __shared__ Record sm[BATCH];
  __shared__ uint32_t slot[BATCH];
  __shared__ double red[kNG * kRedValue];
  const int tile = tile_of_block(blockIdx.x, n_tiles, groups, order);
  if (tile < 0) return;
  const uint32_t epoch = *epoch_dev;
  composite_bwd_tile<TW, TH, MEDIAN, BATCH>(tile, sm, slot, red, epoch, n_frames, frames, ranges, vals, rec,
                                     trect, keyoff, tile_nproc, bg0, bg1, bg2, g_rgb, g_depth,
                                     g_alpha, t_final, n_last, partial, stamp, med_pos);
}

static void launch_order(hipStream_t st, int n_tiles, int groups, const uint32_t* nproc,
                         uint32_t* order) {
  hipLaunchKernelGGL(tile_order_kernel, dim3((unsigned)groups), dim3(1024), 0, st, n_tiles,
                     groups, nproc, order);
}

static unsigned grid_of(int n_tiles, int groups) {
  return (unsigned)(((n_tiles + groups - 1) / groups) * groups);
}

void launch_tile_order(hipStream_t st, int n_tiles, int groups, const uint32_t* nproc,
                       uint32_t* order) {
  if (n_tiles > 0) launch_order(st, n_tiles, groups, nproc, order);
}

unsigned tile_schedule_grid(int n_tiles, int groups) { return grid_of(n_tiles, groups); }
int tile_schedule_groups(bool xcd_groups) { return xcd_groups ? kQueues : 1; }

template <int TW, int TH, bool COUNT, bool MEDIAN, int BATCH>
static void launch_fwd_v(hipStream_t st, int n_tiles, int groups, const uint32_t* order, int F,
                         const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                         const Record* rec, const float* bg, float* rgb, float* depth,
                         float* alpha, float* t_final, int32_t* n_last, uint32_t* nproc,
                         unsigned long long* pairs, int32_t* med_pos) {
  auto k = composite_fwd_kernel<TW, TH, COUNT, MEDIAN, BATCH>;
  hipLaunchKernelGGL(k, dim3(grid_of(n_tiles, groups)), dim3(kWave), 0, st, n_tiles, groups,
                     order, F, frames, ranges, vals, rec, bg[0], bg[1], bg[2], rgb, depth, alpha,
                     t_final, n_last, nproc, pairs, med_pos);
}

template <int TW, int TH, int BATCH>
static void launch_fwd_b(hipStream_t st, int n_tiles, int groups, const uint32_t* order, int F,
                         const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                         const Record* rec, const float* bg, float* rgb, float* depth,
                         float* alpha, float* t_final, int32_t* n_last, uint32_t* nproc,
                         unsigned long long* pairs, int32_t* med_pos) {
#define GSR_FWD_V(C, M)                                                                         \
  launch_fwd_v<TW, TH, C, M, BATCH>(st, n_tiles, groups, order, F, frames, ranges, vals, rec,    \
                                    bg, rgb, depth, alpha, t_final, n_last, nproc, pairs,        \
                                    med_pos)
  if (pairs) {
    if (med_pos) GSR_FWD_V(true, true); else GSR_FWD_V(true, false);
  } else {
    if (med_pos) GSR_FWD_V(false, true); else GSR_FWD_V(false, false);
  }
#undef GSR_FWD_V
}

template <int TW, int TH>
static void launch_fwd_t(hipStream_t st, int batch, int n_tiles, int groups,
                         const uint32_t* order, int F, const FrameDesc* frames,
                         const uint2* ranges, const uint32_t* vals, const Record* rec,
                         const float* bg, float* rgb, float* depth, float* alpha, float* t_final,
                         int32_t* n_last, uint32_t* nproc, unsigned long long* pairs,
                         int32_t* med_pos) {
#define GSR_FWD_B(B)                                                                           \
  launch_fwd_b<TW, TH, B>(st, n_tiles, groups, order, F, frames, ranges, vals, rec, bg, rgb,     \
                          depth, alpha, t_final, n_last, nproc, pairs, med_pos)
  if (batch == 32) GSR_FWD_B(32);
  else if (batch == 128) GSR_FWD_B(128);
  else GSR_FWD_B(64);
#undef GSR_FWD_B
}

template <int TW, int TH, int BATCH>
static void launch_bwd_b(hipStream_t st, int n_tiles, int groups, const uint32_t* order, int F,
                         const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                         const Record* rec, const uint2* trect, const uint32_t* keyoff,
                         const uint32_t* nproc, const float* bg, const float* g_rgb,
                         const float* g_depth, const float* g_alpha, const float* t_final,
                         const int32_t* n_last, float* partial, uint32_t* stamp,
                         const uint32_t* epoch, const int32_t* med_pos) {
  if (med_pos) {
    auto k = composite_bwd_kernel<TW, TH, true, BATCH>;
    hipLaunchKernelGGL(k, dim3(grid_of(n_tiles, groups)), dim3(kWave), 0, st, n_tiles,
                       groups, order, F, frames, ranges, vals, rec, trect, keyoff, nproc,
                       bg[0], bg[1], bg[2], g_rgb, g_depth, g_alpha, t_final, n_last, partial,
                       stamp, epoch, med_pos);
  } else {
    auto k = composite_bwd_kernel<TW, TH, false, BATCH>;
    hipLaunchKernelGGL(k, dim3(grid_of(n_tiles, groups)), dim3(kWave), 0, st, n_tiles,
                       groups, order, F, frames, ranges, vals, rec, trect, keyoff, nproc,
                       bg[0], bg[1], bg[2], g_rgb, g_depth, g_alpha, t_final, n_last, partial,
                       stamp, epoch, med_pos);
  }
}

template <int TW, int TH>
static void launch_bwd_t(hipStream_t st, int batch, int n_tiles, int groups,
                         const uint32_t* order, int F, const FrameDesc* frames,
                         const uint2* ranges, const uint32_t* vals, const Record* rec,
                         const uint2* trect, const uint32_t* keyoff, const uint32_t* nproc,
                         const float* bg, const float* g_rgb, const float* g_depth,
                         const float* g_alpha, const float* t_final, const int32_t* n_last,
                         float* partial, uint32_t* stamp, const uint32_t* epoch,
                         const int32_t* med_pos) {
#define GSR_BWD_B(B)                                                                           \
  launch_bwd_b<TW, TH, B>(st, n_tiles, groups, order, F, frames, ranges, vals, rec, trect,     \
                          keyoff, nproc, bg, g_rgb, g_depth, g_alpha, t_final, n_last,         \
                          partial, stamp, epoch, med_pos)
  if (batch == 32) GSR_BWD_B(32);
  else if (batch == 128) GSR_BWD_B(128);
  else GSR_BWD_B(64);
#undef GSR_BWD_B
}

void launch_composite_fwd(hipStream_t st, int tw, int th, int batch, int n_tiles, int F,
                          const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                          const Record* rec, const float* bg, float* rgb, float* depth,
                          float* alpha, float* t_final, int32_t* n_last, uint32_t* nproc,
                          const uint32_t* prev_nproc, uint32_t* order, bool xcd_groups,
                          unsigned long long* pairs, int32_t* med_pos) {
  if (n_tiles <= 0) return;
  const int groups = xcd_groups ? kQueues : 1;
  launch_order(st, n_tiles, groups, prev_nproc, order);
#define GSR_FWD(W, H)                                                                         \
  launch_fwd_t<W, H>(st, batch, n_tiles, groups, order, F, frames, ranges, vals, rec, bg, rgb,  \
                     depth, alpha, t_final, n_last, nproc, pairs, med_pos)
  if (tw == 16 && th == 16) GSR_FWD(16, 16);
  else if (tw == 8 && th == 8) GSR_FWD(8, 8);
  else if (tw == 32 && th == 8) GSR_FWD(32, 8);
  else if (tw == 16 && th == 8) GSR_FWD(16, 8);
  else if (tw == 32 && th == 16) GSR_FWD(32, 16);
#undef GSR_FWD
}

void launch_composite_bwd(hipStream_t st, int tw, int th, int batch, int n_tiles, int F,
                          const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                          const Record* rec, const uint2* trect, const uint32_t* keyoff,
                          const uint32_t* nproc, const float* bg, const float* g_rgb,
                          const float* g_depth, const float* g_alpha, const float* t_final,
                          const int32_t* n_last, float* partial, uint32_t* stamp,
                          const uint32_t* epoch, uint32_t* order, bool xcd_groups,
                          const int32_t* med_pos) {
  if (n_tiles <= 0) return;
  const int groups = xcd_groups ? kQueues : 1;
  launch_order(st, n_tiles, groups, nproc, order);
#define GSR_BWD(W, H)                                                                          \
  launch_bwd_t<W, H>(st, batch, n_tiles, groups, order, F, frames, ranges, vals, rec, trect,   \
                     keyoff, nproc, bg, g_rgb, g_depth, g_alpha, t_final, n_last, partial,     \
                     stamp, epoch, med_pos)
  if (tw == 16 && th == 16) GSR_BWD(16, 16);
  else if (tw == 8 && th == 8) GSR_BWD(8, 8);
  else if (tw == 32 && th == 8) GSR_BWD(32, 8);
  else if (tw == 16 && th == 8) GSR_BWD(16, 8);
  else if (tw == 32 && th == 16) GSR_BWD(32, 16);
#undef GSR_BWD
}

}  // namespace gsr
