// sort.hip -- key generation and ordering of the (tile, Gaussian) lists.
//
// The compositing order of a pixel is its Gaussians by ascending (fp32 view
// depth, index) (front-to-back compositing, DROID-Splat eqn:rendering; tile
// lists of the 3DGS rasterizer it builds on).  Instead of one wide sort of
// (tile | depth) keys, the path sorts twice:
//   1. the N*F records by depth bits (stable LSD radix, 4 x 8-bit passes over
//      N*F elements), which puts each frame's Gaussians front to back with
//      ties broken by index;
//   2. keygen walks the records in that order and writes one tile id per
//      covered tile (the "slot" order), 16 bits wide while the tile ids fit
//      (up to 65,535 tiles), else 32; a stable LSD radix over only the
//      tile-id bits (two passes of <= 10 bits up to 2^20 tiles) then groups
//      the keys by tile while keeping the depth order inside each tile.
// With 16-bit keys, keygen, the two passes and the ranges move 36 bytes per
// key, instead of 6-7 passes over 12-byte (tile | depth, value) pairs.
//
// The radix passes use a hand-written LDS multi-split: each wave ranks its
// 64 keys per round with one ballot per digit bit (lanes with equal digits
// form one mask), keeps running digit counts in LDS, and the block combines
// its waves' counts into stable block offsets; no global atomics.  A
// pass's digit counts are stored one row per block, so the histogram writes
// and the scatter reads them as whole rows, and their scan runs down the
// columns (3 launches); the other scans are reduce-then-scan in 3 launches.
// Scatter blocks are dealt so that consecutive blocks run on one XCD: the
// partial cache lines at the two ends of a block's digit run are completed by
// its neighbour in the same L2 instead of leaving as partial writes.  All
// kernels read the element count from device memory so the sequence is
// capturable.
#include "launch.h"

#include <algorithm>
#include <cmath>

namespace gsr {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // elements per block

constexpr int kSortRounds = 16;  // 64-key rounds per wave in the radix passes
constexpr int kMaxDigitBits = 10;
constexpr int kMaxBins = 1 << kMaxDigitBits;
constexpr unsigned kXcds = 8;  // XCDs of an MI355X: workgroup b runs on XCD b % 8

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
// Stable LSD radix pass over the digit of `width` <= 10 bits at `shift`.
//
// A block of WAVES waves owns WAVES * 1024 consecutive keys, wave w the
// contiguous 1024 keys from w * 1024 as 16 rounds of 64.  Each lane loads
// its 16 keys and values straight into registers (fully unrolled, so all the
// loads are in flight at once).  Per round a wave ranks its 64 keys by digit
// with one ballot per digit bit, 8 or 10 whatever the width (lanes with
// equal digits form one mask); the lowest lane of each group bumps the
// wave's LDS counter.  No atomics there, so the
// ranks are deterministic and the scatter is stable.  The keys then pass
// through LDS in digit order so that each digit's run leaves the block as
// consecutive stores.  BINS (256 or 1024) sizes the LDS counters; the pass
// uses 2^width of them.
// ---------------------------------------------------------------------------

// The lanes whose digits d agree with this lane's on the bits [0, NBITS).
// A digit narrower than NBITS has zeros above its width, where every lane
// agrees, so those steps leave the mask as it is: the loop runs a fixed
// NBITS steps with no per-bit width test.
template <int NBITS>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d) {
  uint32_t m_lo = 0xffffffffu, m_hi = 0xffffffffu;
#pragma unroll
  for (int b = 0; b < NBITS; ++b) {
    // x: all ones where the lane's bit b is set; the lanes that agree with
    // it on bit b are ~(ballot ^ x), which gfx950 forms with the mask update
    // in one three-input bit operation per half (the empty asm keeps the
    // steps from being refolded into a longer xor / or chain)
    const uint32_t x = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, (uint32_t)b, 1u);
    const uint64_t bb = __ballot((int32_t)x < 0);
    asm volatile("" : "+v"(m_lo), "+v"(m_hi));
    m_lo &= ~((uint32_t)bb ^ x);
    m_hi &= ~((uint32_t)(bb >> 32) ^ x);
  }
  return ((uint64_t)m_hi << 32) | m_lo;
}

// The logical block of workgroup `bid` when the grid (kXcds * per
// workgroups) is dealt so that XCD x (workgroups x, x + kXcds, ...) runs the
// consecutive logical blocks [x per, (x + 1) per) in order.  Neighbouring
// blocks write the two ends of each digit run's cache lines; on one XCD they
// meet in one L2 instead of leaving as partial-line writes.
__device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned per) {
  return (bid % kXcds) * per + bid / kXcds;
}

// Exclusive scan of one value per thread over a block of blockDim.x threads
// (a multiple of 64, at most 1024); wsum holds 16 values.
template <typename T>
__device__ __forceinline__ T block_scan_excl(T v, T* wsum, T& total) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  T x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  T base = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    const T s = wsum[k];
    if (k < w) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

template <int WAVES>
struct RadixShape {
  static constexpr int kThreads = WAVES * kWave;
  static constexpr int kTile = kThreads * kSortRounds;  // keys per block
};

// Digit counts of one block's keys.  A count does not depend on the order,
// so each thread loads 16 bytes of keys at once and bumps its wave's LDS
// counters with atomics; the wave histograms are summed.  KeyT is uint32_t
// or uint16_t (tile ids below 2^16).
template <int BINS, int WAVES, typename KeyT>
__global__ void __launch_bounds__(256) radix_hist_kernel(
    const KeyT* __restrict__ keys, const uint64_t* n_dev, uint64_t n_host, int shift,
    int width, uint32_t* __restrict__ hist /* [nblocks][2^width] */) {
  constexpr int kTile = RadixShape<WAVES>::kTile;
  constexpr int kHW = 256 / kWave;             // waves of this kernel
  constexpr int kPer = 16 / (int)sizeof(KeyT);  // keys per 16-byte load
  __shared__ uint32_t wcnt[kHW][BINS];
  const uint64_t n = n_dev ? min(*n_dev, n_host) : n_host;
  const int bins = 1 << width;
  const uint32_t mask = (uint32_t)bins - 1u;
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kHW * BINS; i += 256) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t bbase = (uint64_t)blockIdx.x * kTile;
  uint32_t* cw = wcnt[w];
#pragma unroll
  for (int j = 0; j < kTile / (kPer * 256); ++j) {
    const uint64_t i = bbase + kPer * ((uint64_t)threadIdx.x + (uint64_t)j * 256);
    if (i + kPer <= n) {
      union {
        uint4 v;
        KeyT k[kPer];
      } u;
      u.v = *reinterpret_cast<const uint4*>(keys + i);  // i % kPer == 0
#pragma unroll
      for (int t = 0; t < kPer; ++t) atomicAdd(&cw[((uint32_t)u.k[t] >> shift) & mask], 1u);
    } else {
      for (uint64_t t = i; t < n && t < i + kPer; ++t)
        atomicAdd(&cw[((uint32_t)keys[t] >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < bins; d += 256) {
    uint32_t c = 0;
    for (int ww = 0; ww < kHW; ++ww) c += wcnt[ww][d];
    hist[(uint64_t)blockIdx.x * bins + d] = c;
  }
}

// Exclusive offsets from the block-major counts H[b][d]: the scatter of block
// b puts its digit-d keys at sum_{d' < d} total(d') + sum_{b' < b} H[b'][d],
// the exclusive scan of the counts taken in (digit, block) order.  The blocks
// are cut into chunks of `rows`; one thread per digit walks a chunk's rows,
// so every access is a whole row.  Rows are loaded kColBatch at a time so
// that a thread's serial walk waits on one load latency per batch.
// rows = ceil(sqrt(nb)) balances a chunk's walk against the spine's walk
// over the chunks; then there are at most ceil(sqrt(nb)) chunks (and at most
// kColMaxChunks).  The three kernels run max(bins, 64) threads; threads past
// the digit count only take part in the spine's block scan.
constexpr unsigned kColMaxChunks = 1024;
constexpr int kColBatch = 16;

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
__global__ void __launch_bounds__(kMaxBins) radix_colsum_kernel(
    const uint32_t* __restrict__ hist, unsigned nb, unsigned rows, int bins,
    uint32_t* __restrict__ csum) {
  const unsigned d = threadIdx.x;
  if ((int)d >= bins) return;
  const unsigned b0 = blockIdx.x * rows, b1 = min(nb, b0 + rows);
  uint32_t s = 0;
  for (unsigned b = b0; b < b1; b += kColBatch) {
    uint32_t v[kColBatch];
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      v[j] = b + j < b1 ? hist[(uint64_t)(b + j) * bins + d] : 0u;
#pragma unroll
    for (int j = 0; j < kColBatch; ++j) s += v[j];
  }
  csum[(uint64_t)blockIdx.x * bins + d] = s;
}

// One block: csum[c][d] becomes the exclusive scan over chunks of digit d;
// row nc receives the exclusive scan of the digit totals.
__global__ void __launch_bounds__(kMaxBins) radix_colspine_kernel(uint32_t* __restrict__ csum,
                                                                  unsigned nc, int bins) {
  __shared__ uint32_t wsum[kMaxBins / kWave];
  const unsigned d = threadIdx.x;
  const bool own = (int)d < bins;
  uint32_t run = 0;
  if (own) {
    for (unsigned c = 0; c < nc; c += kColBatch) {
      uint32_t v[kColBatch];
#pragma unroll
      for (int j = 0; j < kColBatch; ++j)
        v[j] = c + j < nc ? csum[(uint64_t)(c + j) * bins + d] : 0u;
#pragma unroll
      for (int j = 0; j < kColBatch; ++j)
        if (c + j < nc) {
          csum[(uint64_t)(c + j) * bins + d] = run;
          run += v[j];
        }
    }
  }
  uint32_t total;
  const uint32_t base = block_scan_excl<uint32_t>(run, wsum, total);
  if (own) csum[(uint64_t)nc * bins + d] = base;
}

// H[b][d] becomes block b's global start of digit d
__global__ void __launch_bounds__(kMaxBins) radix_coldown_kernel(
    uint32_t* __restrict__ hist, unsigned nb, unsigned rows, int bins,
    const uint32_t* __restrict__ csum, unsigned nc) {
  const unsigned d = threadIdx.x;
  if ((int)d >= bins) return;
  const unsigned b0 = blockIdx.x * rows, b1 = min(nb, b0 + rows);
  uint32_t run = csum[(uint64_t)blockIdx.x * bins + d] + csum[(uint64_t)nc * bins + d];
  for (unsigned b = b0; b < b1; b += kColBatch) {
    uint32_t v[kColBatch];
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      v[j] = b + j < b1 ? hist[(uint64_t)(b + j) * bins + d] : 0u;
#pragma unroll
    for (int j = 0; j < kColBatch; ++j)
      if (b + j < b1) {
        hist[(uint64_t)(b + j) * bins + d] = run;
        run += v[j];
      }
  }
}

template <int BINS, int WAVES>
struct ScatterLds {
  uint32_t wcnt[WAVES][BINS];  // counts, then each wave's block-local start in digit
  uint32_t gofs[BINS];         // global start of digit d minus its block-local start
  uint32_t wsum[WAVES];
  uint32_t sk[RadixShape<WAVES>::kTile], sv[RadixShape<WAVES>::kTile];
};

// Ranks the block's keys (lane's round-k key is block-local index
// w 1024 + 64 k + lane; L.wcnt zeroed and the zeroing visible to all waves),
// moves them into digit order through L.sk / L.sv and writes them to
// (global start of digit d) + (position inside the block's run of digit d).
// The combine folds the block-local digit starts into the waves' bases and
// the global offsets, so that each key reads one LDS word on its way into
// the staging rows and one on its way out.
template <int BINS, int WAVES, typename KeyT>
__device__ __forceinline__ void rank_and_scatter(ScatterLds<BINS, WAVES>& L,
                                                 const uint32_t (&key)[kSortRounds],
                                                 const uint32_t (&val)[kSortRounds],
                                                 uint32_t nkeys, int shift, int width,
                                                 const uint32_t* __restrict__ offs_row,
                                                 KeyT* __restrict__ keys_out,
                                                 uint32_t* __restrict__ vals_out) {
  constexpr int kThreads = RadixShape<WAVES>::kThreads;
  constexpr int DPT = (BINS + kThreads - 1) / kThreads;  // digits per thread in the combine
  static_assert(BINS == 256 || BINS == kMaxBins, "8- or 10-bit digit counters");
  constexpr int kBinBits = BINS == 256 ? 8 : kMaxDigitBits;
  const int bins = 1 << width;
  const uint32_t mask = (uint32_t)bins - 1u;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const uint32_t wbase = (uint32_t)w * (kWave * kSortRounds);
  const uint32_t wbase_s = __builtin_amdgcn_readfirstlane(wbase);  // wave-uniform
  uint32_t rank[kSortRounds];
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k) {
    const uint32_t i = wbase + (uint32_t)k * kWave + lane;
    const bool valid = i < nkeys;
    const uint32_t d = (key[k] >> shift) & mask;
    uint64_t m = digit_peers<kBinBits>(d);
    if (wbase_s + (uint32_t)k * kWave + kWave > nkeys) m &= __ballot(valid);  // partial round
    // LDS ops of one wave complete in issue order: the read precedes the
    // leader's write of the same counter
    const uint32_t before = L.wcnt[w][d];
    // peers below this lane: mbcnt counts the mask's bits under the lane
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    rank[k] = before + below;
    if (valid && below == 0) L.wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  {
    // thread t owns digits [t DPT, t DPT + DPT): wave bases per digit, then
    // the block-local digit starts by a scan over the threads
    uint32_t tot[DPT];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = threadIdx.x * DPT + j;
      uint32_t run = 0;
      if (d < bins) {
        for (int ww = 0; ww < WAVES; ++ww) {
          const uint32_t c = L.wcnt[ww][d];
          L.wcnt[ww][d] = run;
          run += c;
        }
      }
      tot[j] = run;
      mine += run;
    }
    uint32_t total;
    uint32_t base = block_scan_excl<uint32_t>(mine, L.wsum, total);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = threadIdx.x * DPT + j;
      if (d < bins) {
        for (int ww = 0; ww < WAVES; ++ww) L.wcnt[ww][d] += base;
        L.gofs[d] = offs_row[d] - base;  // mod 2^32: the output index adds base back
      }
      base += tot[j];
    }
  }
  __syncthreads();  // (also: every wave is done with whatever L.sk held)
  // A full block (all but the last) takes the loops without a per-key test,
  // so that the unrolled rounds' LDS reads are all in flight before the
  // dependent writes and stores; the test made each round wait for its own.
  const bool full = nkeys == (uint32_t)RadixShape<WAVES>::kTile;  // block-uniform
  if (full) {
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
      const uint32_t lp = L.wcnt[w][__builtin_amdgcn_ubfe(key[k], shift, width)] + rank[k];
      L.sk[lp] = key[k];
      L.sv[lp] = val[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
      const uint32_t i = wbase + (uint32_t)k * kWave + lane;
      if (i < nkeys) {
        const uint32_t lp = L.wcnt[w][__builtin_amdgcn_ubfe(key[k], shift, width)] + rank[k];
        L.sk[lp] = key[k];
        L.sv[lp] = val[k];
      }
    }
  }
  __syncthreads();
  // kSortRounds slots per thread: consecutive threads take consecutive
  // slots, so each digit's run leaves as consecutive stores
  if (full) {
    uint32_t kk[kSortRounds], vv[kSortRounds];
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
      const uint32_t idx = threadIdx.x + (uint32_t)k * kThreads;
      kk[k] = L.sk[idx];
      vv[k] = L.sv[idx];
    }
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
      const uint32_t idx = threadIdx.x + (uint32_t)k * kThreads;
      const uint32_t dst = L.gofs[__builtin_amdgcn_ubfe(kk[k], shift, width)] + idx;
      keys_out[dst] = (KeyT)kk[k];
      vals_out[dst] = vv[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSortRounds; ++k) {
      const uint32_t idx = threadIdx.x + (uint32_t)k * kThreads;
      if (idx < nkeys) {
        const uint32_t kk = L.sk[idx];
        const uint32_t dst = L.gofs[__builtin_amdgcn_ubfe(kk, shift, width)] + idx;
        keys_out[dst] = (KeyT)kk;
        vals_out[dst] = L.sv[idx];
      }
    }
  }
}

template <int BINS, int WAVES, typename KeyT>
__global__ void __launch_bounds__(WAVES * kWave) radix_scatter_kernel(
    const KeyT* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const uint64_t* n_dev, uint64_t n_host, int shift, int width, unsigned nb, unsigned per,
    const uint32_t* __restrict__ offsets /* scanned [nblocks][2^width] */,
    KeyT* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  constexpr int kThreads = RadixShape<WAVES>::kThreads;
  constexpr int kTile = RadixShape<WAVES>::kTile;
  __shared__ ScatterLds<BINS, WAVES> L;
  const unsigned b = xcd_block(blockIdx.x, per);
  if (b >= nb) return;  // padding workgroup: before any barrier
  const uint64_t n = n_dev ? min(*n_dev, n_host) : n_host;
  const uint64_t bbase = (uint64_t)b * kTile;
  const uint32_t nkeys = (uint32_t)(n > bbase ? min((uint64_t)kTile, n - bbase) : 0);
  for (int i = threadIdx.x; i < WAVES * BINS; i += kThreads) (&L.wcnt[0][0])[i] = 0;
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t wbase = (uint32_t)(threadIdx.x / kWave) * (kWave * kSortRounds);
  uint32_t key[kSortRounds], val[kSortRounds];
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k) {
    const uint32_t i = wbase + (uint32_t)k * kWave + lane;
    key[k] = i < nkeys ? (uint32_t)keys_in[bbase + i] : 0u;
    val[k] = i < nkeys ? vals_in[bbase + i] : 0u;
  }
  __syncthreads();
  rank_and_scatter<BINS, WAVES, KeyT>(L, key, val, nkeys, shift, width,
                                offsets + (uint64_t)b * (1u << width), keys_out, vals_out);
}

// q = floor(a / b), r = a - q b for b >= 1: a float estimate corrected by
// one step each way (exact while a < 2^21, where the estimate is off by at
// most one), else the integer division.
__device__ __forceinline__ uint32_t div_rem(uint32_t a, uint32_t b, uint32_t& r) {
  if (a >= (1u << 21)) {
    const uint32_t q = a / b;
    r = a - q * b;
    return q;
  }
  uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
  int32_t rr = (int32_t)(a - q * b);
  if (rr < 0) {
    --q;
    rr += (int32_t)b;
  } else if (rr >= (int32_t)b) {
    ++q;
    rr -= (int32_t)b;
  }
  r = (uint32_t)rr;
  return q;
}

// ---------------------------------------------------------------------------
// keygen: key slot o (0 <= o < K) belongs to the depth-ordered record i with
// offsets[i] <= o < offsets[i] + cnt[i]; its key is the global id of the
// (o - offsets[i])-th tile of the record's tile rect, row by row, and its
// value the record id perm[i].  A wave owns 64 consecutive depth-ordered
// records; their slots form one contiguous range, which the lanes write
// cooperatively (slot o by lane o % 64, every store instruction 64
// consecutive keys).  The owner of each slot of a 64-slot round comes from
// the record starts that fall in the round: those records mark their slot in
// LDS, and a slot's owner is the number of records started at or before it,
// less one (one LDS write, one read and a ballot per round; a binary search
// over the 64 starts took six dependent LDS reads and twice the VALU work,
// and this kernel is bound by VALU issue).  A record whose slots pass the key
// capacity gets the all-ones sentinel key (past every tile) on its slots
// below the capacity.
// ---------------------------------------------------------------------------
template <typename KeyT>
__global__ void __launch_bounds__(256) keygen_kernel(
    uint64_t m, uint64_t n, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ cnt_sorted, const uint64_t* __restrict__ offsets,
    uint32_t* __restrict__ keyoff, const uint2* __restrict__ trect_sorted,
    const FrameDesc* __restrict__ frames, uint64_t capacity, KeyT* __restrict__ keys,
    uint32_t* __restrict__ vals, uint32_t* __restrict__ overflow) {
  // per record: (first tile id or sentinel, rect width | grid width << 16,
  // value, first slot relative to the wave's first); per slot of a round:
  // the round's number where a record starts there.  Each wave uses its own
  // rows.
  __shared__ uint4 s_rec[4][kWave];
  __shared__ uint32_t s_mark[4][kWave];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const uint64_t i0 = ((uint64_t)blockIdx.x * 4 + w) * kWave;
  const uint64_t i = i0 + lane;
  uint32_t cnt = 0;
  uint64_t off = 0;
  if (i < m) {
    cnt = cnt_sorted[i];
    off = offsets[i];
    if (cnt) {
      const uint32_t r = perm[i];
      const uint2 tr = trect_sorted[i];
      const FrameDesc fr = frames[r / (uint32_t)n];
      const uint32_t tx0 = tr.x & 0xffffu, tx1 = tr.x >> 16, ty0 = tr.y & 0xffffu;
      const bool ovf = off + cnt > capacity;
      keyoff[r] = ovf ? 0xffffffffu : (uint32_t)off;
      if (ovf) atomicOr(overflow, 1u);
      s_rec[w][lane] =
          make_uint4(ovf ? 0xffffffffu : (uint32_t)fr.tile_offset + ty0 * (uint32_t)fr.grid_x + tx0,
                     (tx1 - tx0 + 1u) | ((uint32_t)fr.grid_x << 16), ovf ? 0u : r, 0u);
    }
  }
  // contiguous slot range [lo, hi) of the wave's records
  const uint64_t lo = __shfl(off, 0, kWave);
  uint64_t hi = i < m ? off + cnt : 0;
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t h2 = __shfl_xor(hi, o, kWave);
    hi = h2 > hi ? h2 : hi;
  }
  if (hi > capacity) hi = capacity;
  if (i0 >= m || hi <= lo) return;  // wave-uniform
  // records with a slot in the range have first slots below hi; the others
  // (culled, or past the capacity) never own a slot.  The starts of the
  // records with slots increase strictly along the lanes from 0.
  const uint32_t start = (i < m && cnt && off < hi) ? (uint32_t)(off - lo) : 0xffffffffu;
  s_rec[w][lane].w = start;
  s_mark[w][lane] = 0u;
  const uint32_t span = (uint32_t)(hi - lo);  // < 2^32: slots are 32-bit
  // the wave's output runs, from wave-uniform bases
  const uint64_t lo_s = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(lo >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)lo);
  KeyT* __restrict__ kout = keys + lo_s;
  uint32_t* __restrict__ vout = vals + lo_s;
  uint32_t before = 0;  // records starting before the round
  uint32_t round = 0;
  for (uint32_t base = 0; base < span; base += kWave) {
    // owner of slot base + lane: the last record starting at or before it.
    // Records starting inside the window mark their slot with the round's
    // number (distinct slots, so no two lanes write one word); LDS ops of
    // one wave complete in issue order, so the marks are in place when the
    // lanes read them.
    ++round;
    if (start != 0xffffffffu && start - base < (uint32_t)kWave) s_mark[w][start - base] = round;
    __builtin_amdgcn_wave_barrier();
    const uint64_t sm = __ballot(s_mark[w][lane] == round);
    const uint32_t upto =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(sm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sm, 0u)) +
        (uint32_t)((sm >> lane) & 1ull);
    const uint32_t owner = (before + upto - 1u) & (kWave - 1);
    before += (uint32_t)__popcll(sm);
    const uint32_t o = base + (uint32_t)lane;
    const uint4 R = s_rec[w][owner];
    if (o < span) {
      uint32_t key = 0xffffffffu;
      if (R.x != 0xffffffffu) {
        uint32_t col;
        const uint32_t row = div_rem(o - R.w, R.y & 0xffffu, col);
        key = R.x + row * (R.y >> 16) + col;
      }
      kout[o] = (KeyT)key;  // the sentinel stays all ones
      vout[o] = R.z;
    }
  }
}

// [start, end) of every tile's run in the sorted keys (ranges pre-zeroed).
// Each thread scans 32 consecutive keys (four 16-byte loads of 16-bit keys,
// eight of 32-bit ones) plus the key just before them; a run boundary writes
// the start of the new tile and the end of the previous one.
constexpr int kRangeItems = 32;

template <typename KeyT>
__global__ void __launch_bounds__(256) ranges_kernel(const KeyT* __restrict__ keys,
                                                     const uint64_t* k_dev, uint64_t capacity,
                                                     uint2* __restrict__ ranges,
                                                     uint32_t n_tiles) {
  constexpr int kPer = 16 / (int)sizeof(KeyT);  // keys per 16-byte load
  static_assert(kRangeItems % kPer == 0, "whole 16-byte loads");
  const uint64_t K = *k_dev < capacity ? *k_dev : capacity;
  const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
  if (i0 >= K) return;
  uint32_t k[kRangeItems];
  if (i0 + kRangeItems <= K) {
#pragma unroll
    for (int q = 0; q < kRangeItems / kPer; ++q) {
      union {
        uint4 v;
        KeyT k[kPer];
      } u;
      u.v = *reinterpret_cast<const uint4*>(keys + i0 + q * kPer);
#pragma unroll
      for (int t = 0; t < kPer; ++t) k[q * kPer + t] = u.k[t];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j) k[j] = i0 + j < K ? (uint32_t)keys[i0 + j] : 0xffffffffu;
  }
  uint32_t prev = i0 == 0 ? 0xffffffffu : (uint32_t)keys[i0 - 1];
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

// Plain copy, one 16-byte element per thread: the reference for the
// achievable HBM bandwidth that the sort's fraction is taken against.
__global__ void __launch_bounds__(256) copy16_kernel(const uint4* __restrict__ a,
                                                     uint4* __restrict__ b, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = a[i];
}

void launch_copy16(hipStream_t st, const void* src, void* dst, uint64_t n16) {
  if (n16 == 0) return;
  hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
}

// Frame descriptors passed by value as kernel arguments (at most 64 per
// launch: 3 KB of the 4 KB argument space), so that a captured graph keeps
// each forward's own table.
constexpr int kFramesPerLaunch = 64;
struct FrameBatch {
  FrameDesc f[kFramesPerLaunch];
};

__global__ void set_frames_kernel(FrameBatch b, int count, FrameDesc* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = b.f[i];
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

void launch_set_frames(hipStream_t st, const FrameDesc* host, int n, FrameDesc* dst) {
  for (int i0 = 0; i0 < n; i0 += kFramesPerLaunch) {
    FrameBatch b{};
    const int c = std::min(kFramesPerLaunch, n - i0);
    std::copy(host + i0, host + i0 + c, b.f);
    hipLaunchKernelGGL(set_frames_kernel, dim3(1), dim3(kFramesPerLaunch), 0, st, b, c,
                       dst + i0);
  }
}

void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}

// Digit widths of the tile passes: ceil(bits / kMaxDigitBits) passes of
// near-equal width, the narrower ones first (fewer digits make longer runs
// per block).
static int tile_pass_widths(int bits, int* widths) {
  const int passes = std::max(1, (bits + kMaxDigitBits - 1) / kMaxDigitBits);
  const int base = bits / passes, extra = bits % passes;
  for (int p = 0; p < passes; ++p) widths[p] = base + (p >= passes - extra ? 1 : 0);
  return passes;
}

static int max_digit_width(int bits) {
  int w[8];
  const int passes = tile_pass_widths(bits, w);
  int mx = 1;
  for (int p = 0; p < passes; ++p) mx = std::max(mx, w[p]);
  return mx;
}

// Workspace bounds use the smallest block (4 waves, 4096 keys).
size_t radix_hist_elems(uint64_t n_max, int bits) {
  const int wmax = bits > 0 ? max_digit_width(bits) : 8;
  return ((size_t)1 << std::max(wmax, 8)) * blocks_for(n_max, RadixShape<4>::kTile);
}
size_t scan_block_elems(uint64_t n_max) { return blocks_for(n_max, kScanTile) + 1; }
// u32 elements of the column scan's chunk sums for up to n_max keys (an upper
// bound for every smaller count as well)
size_t radix_scan_elems(uint64_t n_max, int bits) {
  const int wmax = bits > 0 ? max_digit_width(bits) : 8;
  const uint64_t nb = blocks_for(n_max, RadixShape<4>::kTile);
  const uint64_t nc = std::min<uint64_t>(isqrt_ceil(nb), kColMaxChunks);
  return (size_t)(nc + 1) << std::max(wmax, 8);
}

// Column scan of the block-major digit counts into per-block digit starts.
static void radix_offsets(hipStream_t st, uint32_t* hist, unsigned nb, int width,
                          uint32_t* scan_tmp) {
  const int bins = 1 << width;
  const unsigned rows = col_rows(nb);
  const unsigned nc = (nb + rows - 1) / rows;
  const unsigned thr = (unsigned)std::max(bins, kWave);
  hipLaunchKernelGGL(radix_colsum_kernel, dim3(nc), dim3(thr), 0, st, hist, nb, rows, bins,
                     scan_tmp);
  hipLaunchKernelGGL(radix_colspine_kernel, dim3(1), dim3(thr), 0, st, scan_tmp, nc, bins);
  hipLaunchKernelGGL(radix_coldown_kernel, dim3(nc), dim3(thr), 0, st, hist, nb, rows, bins,
                     scan_tmp, nc);
}

template <int BINS, int WAVES, typename KeyT>
static void radix_pass(hipStream_t st, const KeyT* ki, const uint32_t* vi, KeyT* ko,
                       uint32_t* vo, const uint64_t* n_dev, uint64_t n_max, int shift, int width,
                       uint32_t* hist, uint32_t* scan_tmp) {
  const unsigned nb = blocks_for(n_max, RadixShape<WAVES>::kTile);
  const unsigned per = (nb + kXcds - 1) / kXcds;
  hipLaunchKernelGGL((radix_hist_kernel<BINS, WAVES, KeyT>), dim3(nb), dim3(256), 0, st, ki,
                     n_dev, n_max, shift, width, hist);
  radix_offsets(st, hist, nb, width, scan_tmp);
  hipLaunchKernelGGL((radix_scatter_kernel<BINS, WAVES, KeyT>), dim3(per * kXcds),
                     dim3(RadixShape<WAVES>::kThreads), 0, st, ki, vi, n_dev, n_max, shift,
                     width, nb, per, hist, ko, vo);
}

// Large passes take 8-wave blocks (longer digit runs per block); small ones
// and 10-bit digits (LDS) take 4-wave blocks.
constexpr uint64_t kBigPass = 1ull << 24;

template <typename KeyT>
static void radix_pass_any(hipStream_t st, const KeyT* ki, const uint32_t* vi, KeyT* ko,
                           uint32_t* vo, const uint64_t* n_dev, uint64_t n_max, int shift,
                           int width, uint32_t* hist, uint32_t* scan_tmp) {
  if (width > 8)
    radix_pass<kMaxBins, 4>(st, ki, vi, ko, vo, n_dev, n_max, shift, width, hist, scan_tmp);
  else if (n_max >= kBigPass)
    radix_pass<256, 8>(st, ki, vi, ko, vo, n_dev, n_max, shift, width, hist, scan_tmp);
  else
    radix_pass<256, 4>(st, ki, vi, ko, vo, n_dev, n_max, shift, width, hist, scan_tmp);
}

// Stable sort of (keys, vals) by the key bits [0, bits), 8-bit digits.  The
// element count is *n_dev (<= n_max).  Result ends in (keys_a, vals_a) if the
// number of passes is even, else in (keys_b, vals_b); returns true if in b.
bool launch_radix_sort(hipStream_t st, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                       uint32_t* vals_b, const uint64_t* n_dev, uint64_t n_max, int bits,
                       uint32_t* hist, uint32_t* scan_tmp) {
  if (n_max == 0) return false;
  bool in_b = false;
  for (int shift = 0; shift < bits; shift += 8) {
    const int width = std::min(8, bits - shift);
    radix_pass_any<uint32_t>(st, in_b ? keys_b : keys_a, in_b ? vals_b : vals_a,
                             in_b ? keys_a : keys_b, in_b ? vals_a : vals_b, n_dev, n_max, shift,
                             width, hist, scan_tmp);
    in_b = !in_b;
  }
  return in_b;
}

bool tile_keys_16bit(int bits) { return bits <= 16; }

void launch_keygen(hipStream_t st, uint64_t m, uint64_t n, const uint32_t* perm,
                   const uint32_t* cnt_sorted, const uint64_t* offsets, uint32_t* keyoff,
                   const uint2* trect_sorted, const FrameDesc* frames, uint64_t capacity,
                   int bits, void* keys, uint32_t* vals, uint32_t* overflow) {
  if (m == 0) return;
  if (tile_keys_16bit(bits))
    hipLaunchKernelGGL(keygen_kernel<uint16_t>, dim3(blocks_for(m, 256)), dim3(256), 0, st, m,
                       n, perm, cnt_sorted, offsets, keyoff, trect_sorted, frames, capacity,
                       static_cast<uint16_t*>(keys), vals, overflow);
  else
    hipLaunchKernelGGL(keygen_kernel<uint32_t>, dim3(blocks_for(m, 256)), dim3(256), 0, st, m,
                       n, perm, cnt_sorted, offsets, keyoff, trect_sorted, frames, capacity,
                       static_cast<uint32_t*>(keys), vals, overflow);
}

template <typename KeyT>
static bool tile_sort_t(hipStream_t st, KeyT* keys_a, uint32_t* vals_a, KeyT* keys_b,
                        uint32_t* vals_b, const uint64_t* k_dev, uint64_t k_max, int bits,
                        uint32_t* hist, uint32_t* scan_tmp) {
  int widths[8];
  const int passes = tile_pass_widths(bits, widths);
  bool in_b = false;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    radix_pass_any<KeyT>(st, in_b ? keys_b : keys_a, in_b ? vals_b : vals_a,
                         in_b ? keys_a : keys_b, in_b ? vals_a : vals_b, k_dev, k_max, shift,
                         widths[p], hist, scan_tmp);
    in_b = !in_b;
    shift += widths[p];
  }
  return in_b;
}

// Stable sort of the tile keys by the tile-id bits [0, bits) in passes of
// near-equal width; 16-bit keys when bits <= 16.  Returns true if the result
// is in (keys_b, vals_b).
bool launch_tile_sort(hipStream_t st, void* keys_a, uint32_t* vals_a, void* keys_b,
                      uint32_t* vals_b, const uint64_t* k_dev, uint64_t k_max, int bits,
                      uint32_t* hist, uint32_t* scan_tmp) {
  if (k_max == 0) return false;
  if (tile_keys_16bit(bits))
    return tile_sort_t<uint16_t>(st, static_cast<uint16_t*>(keys_a), vals_a,
                                 static_cast<uint16_t*>(keys_b), vals_b, k_dev, k_max, bits,
                                 hist, scan_tmp);
  return tile_sort_t<uint32_t>(st, static_cast<uint32_t*>(keys_a), vals_a,
                               static_cast<uint32_t*>(keys_b), vals_b, k_dev, k_max, bits, hist,
                               scan_tmp);
}

// The tile counts in depth order, cnt_sorted[i] = ntiles[perm[i]], gathered
// once so that the offsets scan and keygen read them in order, together
// with the tile rects (keygen's one random read per record happens here, as
// part of the gather that has to be random anyway).  A record is kept iff its
// sorted depth key is not the all-ones of a culled record, and a kept
// record's tile count is the area of its rect (the preprocess writes the two
// together; a culled record has neither).
__global__ void __launch_bounds__(256) gather_counts_kernel(uint64_t m,
                                                            const uint32_t* __restrict__ skey,
                                                            const uint32_t* __restrict__ perm,
                                                            const uint2* __restrict__ trect,
                                                            uint32_t* __restrict__ cnt_sorted,
                                                            uint2* __restrict__ trect_sorted) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  uint2 tr = make_uint2(0u, 0u);
  uint32_t c = 0;
  if (skey[i] != 0xffffffffu) {
    tr = trect[perm[i]];
    c = ((tr.x >> 16) - (tr.x & 0xffffu) + 1u) * ((tr.y >> 16) - (tr.y & 0xffffu) + 1u);
  }
  cnt_sorted[i] = c;
  trect_sorted[i] = tr;
}

// Exclusive scan of the depth-ordered records' tile counts into offsets
// (u64), total into *total; cnt_sorted[i] and trect_sorted[i] receive the
// count and the tile rect of record perm[i] (zero for a culled record).
void launch_offsets_scan(hipStream_t st, const uint32_t* skey, const uint32_t* perm,
                         const uint2* trect, uint64_t m, uint32_t* cnt_sorted,
                         uint2* trect_sorted, uint64_t* offsets, uint64_t* block_tmp,
                         uint64_t* total) {
  if (m == 0) {
    launch_fill_u32(st, (uint32_t*)total, 2, 0u);
    return;
  }
  hipLaunchKernelGGL(gather_counts_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, skey,
                     perm, trect, cnt_sorted, trect_sorted);
  const unsigned sb = blocks_for(m, kScanTile);
  LoadU32 ld{cnt_sorted};
  hipLaunchKernelGGL((scan_reduce_kernel<uint64_t, LoadU32>), dim3(sb), dim3(kScanThreads), 0,
                     st, ld, (const uint64_t*)nullptr, m, block_tmp);
  hipLaunchKernelGGL((scan_spine_kernel<uint64_t>), dim3(1), dim3(kScanThreads), 0, st,
                     block_tmp, (int)sb, total);
  hipLaunchKernelGGL((scan_down_kernel<uint64_t, LoadU32>), dim3(sb), dim3(kScanThreads), 0, st,
                     ld, (const uint64_t*)nullptr, m, block_tmp, offsets);
}

void launch_ranges(hipStream_t st, const void* keys, int bits, const uint64_t* k_dev,
                   uint64_t k_max, uint64_t capacity, uint2* ranges, uint64_t n_tiles) {
  launch_fill_u32(st, (uint32_t*)ranges, 2 * n_tiles, 0u);
  if (k_max == 0) return;
  const dim3 grid(blocks_for(k_max, 256 * kRangeItems));
  if (tile_keys_16bit(bits))
    hipLaunchKernelGGL(ranges_kernel<uint16_t>, grid, dim3(256), 0, st,
                       static_cast<const uint16_t*>(keys), k_dev, capacity, ranges,
                       (uint32_t)n_tiles);
  else
    hipLaunchKernelGGL(ranges_kernel<uint32_t>, grid, dim3(256), 0, st,
                       static_cast<const uint32_t*>(keys), k_dev, capacity, ranges,
                       (uint32_t)n_tiles);
}

}  // namespace gsr

