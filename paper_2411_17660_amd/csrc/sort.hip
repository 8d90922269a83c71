// sort.hip -- key generation and ordering of the (tile, Gaussian) lists.
//
// The compositing order of a pixel is its Gaussians by ascending (fp32 view
// depth, index) (front-to-back compositing, DROID-Splat eqn:rendering; tile
// lists of the 3DGS rasterizer it builds on).  Instead of one wide sort of
// (tile | depth) keys, the path sorts twice:
//   1. the N*F records by depth bits (stable LSD radix, 4 x 8-bit passes over
//      N*F elements), which puts each frame's Gaussians front to back with
//      ties broken by index;
//   2. keygen walks the records in that order and writes one 32-bit tile id
//      per covered tile; a stable LSD radix pass over only the tile-id bits
//      (2 passes for up to 65k tiles) then groups the keys by tile while
//      keeping the depth order inside each tile.
// This moves about 40 bytes per key instead of 6-7 passes over 12-byte
// (tile | depth, value) pairs.
//
// The radix passes use a hand-written LDS multi-split: each wave ranks its
// 64 keys per round with 8 ballots (one per digit bit), keeps running digit
// counts in LDS, and the block combines the 4 waves' counts into stable
// block offsets; no global atomics.  A pass's digit counts are stored one
// 1 KB row per block, so the histogram writes and the scatter reads them as
// whole rows, and their scan runs down the columns (3 launches); the other
// scans are reduce-then-scan in 3 launches.  All kernels read the element
// count from device memory so the sequence is capturable.
#include "launch.h"

#include <algorithm>
#include <cmath>

namespace gsr {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // elements per block

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortRounds = 16;  // 64-key rounds per wave
constexpr int kSortTile = kSortThreads * kSortRounds;  // keys per block (4096)
constexpr int kRadixBins = 256;

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one value per thread (256 threads).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    T add = tid >= o ? sh[tid - o] : (T)0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  total = sh[kScanThreads - 1];
  const T incl = sh[tid];
  __syncthreads();
  return incl - v;
}

// Loaders: element i of the scanned sequence.
struct LoadU32 {
  const uint32_t* a;
  __device__ uint32_t operator()(uint64_t i) const { return a[i]; }
};

template <typename T, typename Load>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(Load ld, const uint64_t* n_dev,
                                                                   uint64_t n_host,
                                                                   T* __restrict__ block_sums) {
  __shared__ T sh[kScanThreads];
  const uint64_t n = n_dev ? min(*n_dev, n_host) : n_host;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kScanThreads + threadIdx.x;
    if (i < n) s += (T)ld(i);
  }
  T total;
  block_exclusive_scan<T>(s, sh, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single block: exclusive scan of the block sums in place; total -> *total.
template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_spine_kernel(T* __restrict__ sums, int nb,
                                                                  T* __restrict__ total_out) {
  __shared__ T sh[kScanThreads];
  T carry = 0;
  for (int base = 0; base < nb; base += kScanThreads) {
    const int i = base + threadIdx.x;
    const T v = i < nb ? sums[i] : (T)0;
    T tot;
    const T ex = block_exclusive_scan<T>(v, sh, tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// The block's kScanTile elements pass through LDS rows of kScanItems + 1
// (padded against bank conflicts) so that global loads and stores are
// coalesced while each thread scans kScanItems consecutive elements.
template <typename T, typename Load>
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(Load ld, const uint64_t* n_dev,
                                                                 uint64_t n_host,
                                                                 const T* __restrict__ block_base,
                                                                 T* __restrict__ out) {
  constexpr int kRow = kScanItems + 1;
  __shared__ T sh[kScanThreads];
  __shared__ T stage[kScanThreads * kRow];
  const uint64_t n = n_dev ? min(*n_dev, n_host) : n_host;
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile;
  for (int k = 0; k < kScanItems; ++k) {
    const int e = k * kScanThreads + (int)threadIdx.x;  // element of the tile
    const uint64_t i = b0 + (uint64_t)e;
    stage[(e / kScanItems) * kRow + e % kScanItems] = i < n ? (T)ld(i) : (T)0;
  }
  __syncthreads();
  T v[kScanItems];
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = stage[threadIdx.x * kRow + k];
    s += v[k];
  }
  T total;
  T run = block_exclusive_scan<T>(s, sh, total) + block_base[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    stage[threadIdx.x * kRow + k] = run;
    run += v[k];
  }
  __syncthreads();
  for (int k = 0; k < kScanItems; ++k) {
    const int e = k * kScanThreads + (int)threadIdx.x;
    const uint64_t i = b0 + (uint64_t)e;
    if (i < n) out[i] = stage[(e / kScanItems) * kRow + e % kScanItems];
  }
}

// Note: scan_reduce sums a strided set of kScanTile elements and scan_down a
// thread-contiguous set; both cover exactly the block's kScanTile elements,
// so the block totals agree.

// ---------------------------------------------------------------------------
// LSD radix pass, 8-bit digit at `shift`, stable.
//
// A block owns kSortTile consecutive keys.  The scatter sees it as 4 waves x
// 16 rounds x 64 keys, wave w owning a contiguous quarter.  Per round a wave
// ranks its 64 keys by digit with 8 ballots (lanes with equal digits form
// one mask); the lowest lane of each group bumps the wave's LDS counter.  No
// atomics there, so the ranks are deterministic and the scatter is stable.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Digit counts of one block's kSortTile keys.  A count does not depend on
// the order, so each thread loads four keys with one 16-byte load and bumps
// its wave's LDS counters with atomics; the four wave histograms are summed.
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(
    const uint32_t* __restrict__ keys, const uint64_t* n_dev, uint64_t n_host, int shift,
    uint32_t* __restrict__ hist /* [nblocks][256] */) {
  __shared__ uint32_t wcnt[kSortWaves][kRadixBins];
  const uint64_t n = n_dev ? min(*n_dev, n_host) : n_host;
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kSortWaves * kRadixBins; i += kSortThreads)
    (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t bbase = (uint64_t)blockIdx.x * kSortTile;
  uint32_t* cw = wcnt[w];
#pragma unroll
  for (int j = 0; j < kSortTile / (4 * kSortThreads); ++j) {
    const uint64_t i = bbase + 4 * ((uint64_t)threadIdx.x + (uint64_t)j * kSortThreads);
    if (i + 4 <= n) {
      const uint4 k = *reinterpret_cast<const uint4*>(keys + i);  // i % 4 == 0
      atomicAdd(&cw[(k.x >> shift) & 0xffu], 1u);
      atomicAdd(&cw[(k.y >> shift) & 0xffu], 1u);
      atomicAdd(&cw[(k.z >> shift) & 0xffu], 1u);
      atomicAdd(&cw[(k.w >> shift) & 0xffu], 1u);
    } else {
      for (uint64_t t = i; t < n && t < i + 4; ++t) atomicAdd(&cw[(keys[t] >> shift) & 0xffu], 1u);
    }
  }
  __syncthreads();
  const int d = threadIdx.x;
  uint32_t c = 0;
  for (int ww = 0; ww < kSortWaves; ++ww) c += wcnt[ww][d];
  hist[(uint64_t)blockIdx.x * kRadixBins + d] = c;
}

// Exclusive offsets from the block-major counts H[b][d]: the scatter of block
// b puts its digit-d keys at sum_{d' < d} total(d') + sum_{b' < b} H[b'][d],
// the exclusive scan of the counts taken in (digit, block) order.  The blocks
// are cut into chunks of `rows`; one thread per digit walks a chunk's rows,
// so every access is a whole 1 KB row.  Rows are loaded kColBatch at a time
// so that a thread's serial walk waits on one load latency per batch.
// rows = ceil(sqrt(nb)) balances a chunk's walk against the spine's walk
// over the chunks; then there are at most ceil(sqrt(nb)) chunks (and at most
// kColMaxChunks).
constexpr unsigned kColMaxChunks = 1024;
constexpr int kColBatch = 16;
static_assert(kRadixBins == kScanThreads, "one scan thread per digit");

static inline uint64_t isqrt_ceil(uint64_t x) {
  uint64_t r = (uint64_t)std::sqrt((double)x);
  while (r * r < x) ++r;
  while (r > 0 && (r - 1) * (r - 1) >= x) --r;
  return r;
}

static inline unsigned col_rows(unsigned nb) {
  return (unsigned)std::max<uint64_t>(isqrt_ceil(nb), (nb + kColMaxChunks - 1) / kColMaxChunks);
}

// csum[c][d] = sum of H[b][d] over the rows b of chunk c
__global__ void __launch_bounds__(kRadixBins) radix_colsum_kernel(
    const uint32_t* __restrict__ hist, unsigned nb, unsigned rows, uint32_t* __restrict__ csum) {
  const unsigned d = threadIdx.x;
  const unsigned b0 = blockIdx.x * rows, b1 = min(nb, b0 + rows);
  uint32_t s = 0;
  for (unsigned b = b0; b < b1; b += kColBatch) {
    uint32_t v[kColBatch];
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      v[j] = b + j < b1 ? hist[(uint64_t)(b + j) * kRadixBins + d] : 0u;
#pragma unroll
    for (int j = 0; j < kColBatch; ++j) s += v[j];
  }
  csum[(uint64_t)blockIdx.x * kRadixBins + d] = s;
}

// One block: csum[c][d] becomes the exclusive scan over chunks of digit d;
// row nc receives the exclusive scan of the digit totals.
__global__ void __launch_bounds__(kRadixBins) radix_colspine_kernel(uint32_t* __restrict__ csum,
                                                                    unsigned nc) {
  __shared__ uint32_t sh[kScanThreads];
  const unsigned d = threadIdx.x;
  uint32_t run = 0;
  for (unsigned c = 0; c < nc; c += kColBatch) {
    uint32_t v[kColBatch];
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      v[j] = c + j < nc ? csum[(uint64_t)(c + j) * kRadixBins + d] : 0u;
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      if (c + j < nc) {
        csum[(uint64_t)(c + j) * kRadixBins + d] = run;
        run += v[j];
      }
  }
  uint32_t total;
  const uint32_t base = block_exclusive_scan<uint32_t>(run, sh, total);
  csum[(uint64_t)nc * kRadixBins + d] = base;
}

// H[b][d] becomes block b's global start of digit d
__global__ void __launch_bounds__(kRadixBins) radix_coldown_kernel(
    uint32_t* __restrict__ hist, unsigned nb, unsigned rows, const uint32_t* __restrict__ csum,
    unsigned nc) {
  const unsigned d = threadIdx.x;
  const unsigned b0 = blockIdx.x * rows, b1 = min(nb, b0 + rows);
  uint32_t run = csum[(uint64_t)blockIdx.x * kRadixBins + d] + csum[(uint64_t)nc * kRadixBins + d];
  for (unsigned b = b0; b < b1; b += kColBatch) {
    uint32_t v[kColBatch];
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      v[j] = b + j < b1 ? hist[(uint64_t)(b + j) * kRadixBins + d] : 0u;
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      if (b + j < b1) {
        hist[(uint64_t)(b + j) * kRadixBins + d] = run;
        run += v[j];
      }
  }
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const uint64_t* n_dev, uint64_t n_host, int shift,
    const uint32_t* __restrict__ offsets /* scanned [nblocks][256] */,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t wcnt[kSortWaves][kRadixBins];  // counts, then wave bases in digit
  __shared__ uint32_t dstart[kRadixBins];            // block-local start of each digit
  __shared__ uint32_t gbase[kRadixBins];             // global start of digit for the block
  __shared__ uint32_t scan_sh[kSortThreads];
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];  // block keys in local digit order
  const uint64_t n = n_dev ? min(*n_dev, n_host) : n_host;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kSortWaves * kRadixBins; i += kSortThreads)
    (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t bbase = (uint64_t)blockIdx.x * kSortTile;
  const uint64_t wbase = bbase + (uint64_t)w * (kWave * kSortRounds);
  const uint64_t lt = lanemask_lt();
  uint32_t key[kSortRounds], val[kSortRounds], rank[kSortRounds];
  for (int k = 0; k < kSortRounds; ++k) {
    const uint64_t i = wbase + (uint64_t)k * kWave + lane;
    const bool valid = i < n;
    key[k] = valid ? keys_in[i] : 0u;
    val[k] = valid ? vals_in[i] : 0u;
    const uint32_t d = (key[k] >> shift) & 0xffu;
    const uint64_t m = digit_peers(d, valid);
    // LDS ops of one wave complete in issue order: the read precedes the
    // leader's write of the same counter
    const uint32_t before = wcnt[w][d];
    rank[k] = before + (uint32_t)__popcll(m & lt);
    if (valid && (m & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
    for (int ww = 0; ww < kSortWaves; ++ww) {
      const uint32_t c = wcnt[ww][d];
      wcnt[ww][d] = run;
      run += c;
    }
    uint32_t total;
    dstart[d] = block_exclusive_scan<uint32_t>(run, scan_sh, total);
    gbase[d] = offsets[(uint64_t)blockIdx.x * kRadixBins + d];
  }
  __syncthreads();
  for (int k = 0; k < kSortRounds; ++k) {
    const uint64_t i = wbase + (uint64_t)k * kWave + lane;
    if (i < n) {
      const uint32_t d = (key[k] >> shift) & 0xffu;
      const uint32_t lp = dstart[d] + wcnt[w][d] + rank[k];
      sk[lp] = key[k];
      sv[lp] = val[k];
    }
  }
  __syncthreads();
  const uint32_t nb = (uint32_t)(n > bbase ? min((uint64_t)kSortTile, n - bbase) : 0);
  for (uint32_t idx = threadIdx.x; idx < nb; idx += kSortThreads) {
    const uint32_t kk = sk[idx];
    const uint32_t d = (kk >> shift) & 0xffu;
    const uint32_t dst = gbase[d] + (idx - dstart[d]);
    keys_out[dst] = kk;
    vals_out[dst] = sv[idx];
  }
}

// ---------------------------------------------------------------------------
// keygen: a wave owns 64 consecutive depth-sorted records; their key slots
// form one contiguous range, which the lanes write cooperatively (slot o by
// lane o % 64) after locating the owning record with a 6-step search in LDS,
// so every store instruction writes 64 consecutive keys.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) keygen_kernel(
    uint64_t m, uint64_t n, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ cnt_sorted, const uint64_t* __restrict__ offsets,
    uint32_t* __restrict__ keyoff, const uint2* __restrict__ trect,
    const FrameDesc* __restrict__ frames, uint64_t capacity,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ overflow) {
  __shared__ uint64_t s_off[4][kWave];
  __shared__ uint32_t s_r[4][kWave], s_w[4][kWave], s_gx[4][kWave], s_base[4][kWave];
  __shared__ uint8_t s_ovf[4][kWave];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const uint64_t i0 = ((uint64_t)blockIdx.x * 4 + w) * kWave;
  const uint64_t i = i0 + lane;
  uint32_t cnt = 0;
  uint64_t off = 0;
  if (i < m) {
    const uint32_t r = perm[i];
    cnt = cnt_sorted[i];
    off = offsets[i];
    s_r[w][lane] = r;
    if (cnt) {
      const FrameDesc fr = frames[r / n];
      const uint2 tr = trect[r];
      const int tx0 = tr.x & 0xffff, tx1 = tr.x >> 16;
      const int ty0 = tr.y & 0xffff;
      s_w[w][lane] = (uint32_t)(tx1 - tx0 + 1);
      s_gx[w][lane] = (uint32_t)fr.grid_x;
      s_base[w][lane] = (uint32_t)(fr.tile_offset + ty0 * fr.grid_x + tx0);
      const bool ovf = off + cnt > capacity;
      s_ovf[w][lane] = ovf ? 1 : 0;
      keyoff[r] = ovf ? 0xffffffffu : (uint32_t)off;
      if (ovf) atomicOr(overflow, 1u);
    }
  }
  s_off[w][lane] = i < m ? off : ~0ull;
  __syncthreads();  // every wave reaches the barrier; empty waves leave after it
  if (i0 >= m) return;
  // contiguous slot range of the wave's records
  const uint64_t lo = s_off[w][0];
  uint64_t hi = off + cnt;
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t h2 = __shfl_xor(hi, o, 64);
    hi = h2 > hi ? h2 : hi;
  }
  if (hi > capacity) hi = capacity;
  for (uint64_t o = lo + lane; o < hi; o += kWave) {
    // owner: the last record with s_off <= o
    int j = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (s_off[w][j + step] <= o) j += step;
    uint32_t key, val;
    if (s_ovf[w][j]) {
      key = 0xffffffffu;  // sentinel past every real tile
      val = 0u;
    } else {
      const uint32_t local = (uint32_t)(o - s_off[w][j]);
      const uint32_t wdt = s_w[w][j];
      const uint32_t row = local / wdt;
      key = s_base[w][j] + row * s_gx[w][j] + (local - row * wdt);
      val = s_r[w][j];
    }
    keys[o] = key;
    vals[o] = val;
  }
}

// [start, end) of every tile's run in the sorted keys (ranges pre-zeroed).
// Each thread scans 8 consecutive keys (two 16-byte loads) plus the key just
// before them; a run boundary writes the start of the new tile and the end
// of the previous one.
constexpr int kRangeItems = 8;

__global__ void __launch_bounds__(256) ranges_kernel(const uint32_t* __restrict__ keys,
                                                     const uint64_t* k_dev, uint64_t capacity,
                                                     uint2* __restrict__ ranges,
                                                     uint32_t n_tiles) {
  const uint64_t K = *k_dev < capacity ? *k_dev : capacity;
  const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
  if (i0 >= K) return;
  uint32_t k[kRangeItems];
  if (i0 + kRangeItems <= K) {
    const uint4 a = *reinterpret_cast<const uint4*>(keys + i0);
    const uint4 b = *reinterpret_cast<const uint4*>(keys + i0 + 4);
    k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
    k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j) k[j] = i0 + j < K ? keys[i0 + j] : 0xffffffffu;
  }
  uint32_t prev = i0 == 0 ? 0xffffffffu : keys[i0 - 1];
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t i = i0 + j;
    if (i >= K) break;
    const uint32_t t = k[j];
    if (t != prev) {
      if (t < n_tiles) ranges[t].x = (uint32_t)i;
      if (prev < n_tiles) ranges[prev].y = (uint32_t)i;
    }
    prev = t;
  }
  const uint64_t last = i0 + kRangeItems - 1 < K - 1 ? i0 + kRangeItems - 1 : K - 1;
  if (last == K - 1 && prev < n_tiles) ranges[prev].y = (uint32_t)K;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// host-side launch sequences
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(uint64_t n, uint64_t per) {
  return (unsigned)((n + per - 1) / per);
}

void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}

size_t radix_hist_elems(uint64_t n_max) { return (size_t)kRadixBins * blocks_for(n_max, kSortTile); }
size_t scan_block_elems(uint64_t n_max) { return blocks_for(n_max, kScanTile) + 1; }
// u32 elements of the column scan's chunk sums for up to n_max keys (an upper
// bound for every smaller count as well)
size_t radix_scan_elems(uint64_t n_max) {
  const uint64_t nb = blocks_for(n_max, kSortTile);
  const uint64_t nc = std::min<uint64_t>(isqrt_ceil(nb), kColMaxChunks);
  return (size_t)(nc + 1) * kRadixBins;
}

// Stable sort of (keys, vals) by the key bits [0, bits).  The element count
// is *n_dev (<= n_max).  Result ends in (keys_a, vals_a) if the number of
// passes is even, else in (keys_b, vals_b); returns true if in b.
bool launch_radix_sort(hipStream_t st, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                       uint32_t* vals_b, const uint64_t* n_dev, uint64_t n_max, int bits,
                       uint32_t* hist, uint32_t* scan_tmp) {
  if (n_max == 0) return false;
  const unsigned nb = blocks_for(n_max, kSortTile);
  const unsigned rows = col_rows(nb);
  const unsigned nc = (nb + rows - 1) / rows;
  bool in_b = false;
  for (int shift = 0; shift < bits; shift += 8) {
    uint32_t* ki = in_b ? keys_b : keys_a;
    uint32_t* vi = in_b ? vals_b : vals_a;
    uint32_t* ko = in_b ? keys_a : keys_b;
    uint32_t* vo = in_b ? vals_a : vals_b;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kSortThreads), 0, st, ki, n_dev, n_max,
                       shift, hist);
    hipLaunchKernelGGL(radix_colsum_kernel, dim3(nc), dim3(kRadixBins), 0, st, hist, nb, rows,
                       scan_tmp);
    hipLaunchKernelGGL(radix_colspine_kernel, dim3(1), dim3(kRadixBins), 0, st, scan_tmp, nc);
    hipLaunchKernelGGL(radix_coldown_kernel, dim3(nc), dim3(kRadixBins), 0, st, hist, nb, rows,
                       scan_tmp, nc);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kSortThreads), 0, st, ki, vi, n_dev,
                       n_max, shift, hist, ko, vo);
    in_b = !in_b;
  }
  return in_b;
}

// The tile counts in depth order, cnt_sorted[i] = ntiles[perm[i]], gathered
// once so that the offsets scan and keygen read them in order.
__global__ void __launch_bounds__(256) gather_counts_kernel(uint64_t m,
                                                            const uint32_t* __restrict__ ntiles,
                                                            const uint32_t* __restrict__ perm,
                                                            uint32_t* __restrict__ cnt_sorted) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) cnt_sorted[i] = ntiles[perm[i]];
}

// Exclusive scan of ntiles[perm[i]] over the m records into offsets (u64),
// total into *total; cnt_sorted[i] receives ntiles[perm[i]].
void launch_offsets_scan(hipStream_t st, const uint32_t* ntiles, const uint32_t* perm,
                         uint64_t m, uint32_t* cnt_sorted, uint64_t* offsets,
                         uint64_t* block_tmp, uint64_t* total) {
  if (m == 0) {
    launch_fill_u32(st, (uint32_t*)total, 2, 0u);
    return;
  }
  hipLaunchKernelGGL(gather_counts_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, ntiles,
                     perm, cnt_sorted);
  const unsigned sb = blocks_for(m, kScanTile);
  LoadU32 ld{cnt_sorted};
  hipLaunchKernelGGL((scan_reduce_kernel<uint64_t, LoadU32>), dim3(sb), dim3(kScanThreads), 0,
                     st, ld, (const uint64_t*)nullptr, m, block_tmp);
  hipLaunchKernelGGL((scan_spine_kernel<uint64_t>), dim3(1), dim3(kScanThreads), 0, st,
                     block_tmp, (int)sb, total);
  hipLaunchKernelGGL((scan_down_kernel<uint64_t, LoadU32>), dim3(sb), dim3(kScanThreads), 0, st,
                     ld, (const uint64_t*)nullptr, m, block_tmp, offsets);
}

void launch_keygen(hipStream_t st, uint64_t m, uint64_t n, const uint32_t* perm,
                   const uint32_t* cnt_sorted, const uint64_t* offsets, uint32_t* keyoff,
                   const uint2* trect, const FrameDesc* frames, uint64_t capacity,
                   uint32_t* keys, uint32_t* vals, uint32_t* overflow) {
  if (m == 0) return;
  hipLaunchKernelGGL(keygen_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, n, perm,
                     cnt_sorted, offsets, keyoff, trect, frames, capacity, keys, vals, overflow);
}

void launch_ranges(hipStream_t st, const uint32_t* keys, const uint64_t* k_dev, uint64_t k_max,
                   uint64_t capacity, uint2* ranges, uint64_t n_tiles) {
  launch_fill_u32(st, (uint32_t*)ranges, 2 * n_tiles, 0u);
  if (k_max == 0) return;
  hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for(k_max, 256 * kRangeItems)), dim3(256), 0, st,
                     keys, k_dev, capacity, ranges, (uint32_t)n_tiles);
}

}  // namespace gsr
