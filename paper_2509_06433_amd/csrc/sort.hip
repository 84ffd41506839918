// Tile binning and the depth-keyed radix sort.
//
// Order of the instance list: (view, tile, raw float bits of depth, Gaussian
// index). It is built in two stable steps:
//   1. an LSD radix sort of the (view, Gaussian) splats by depth bits; the
//      splats start in (view, index) order, so ties keep index order;
//   2. instances are emitted in that depth order, then a stable LSD radix
//      sort on the global tile id groups them by tile while keeping the depth
//      order inside every tile.
// The radix sort is an 8-bit-digit onesweep (see below); instance offsets
// come from a reduce-then-scan over the tile counts in depth order.

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;      // 2048
// emission: output positions per workgroup, its threads, and the histogram
// words it can accumulate (4 passes of 8 bits)
constexpr int kEmitBlock = 1024;
constexpr int kEmitThreads = 256;
constexpr int kEmitHist = 1024;

constexpr int kSortThreads = 256;                          // 4 wave64
constexpr int kSortItems = 16;                             // histogram kernel
constexpr int kSortChunk = kSortThreads * kSortItems;      // 4096
// element count up to which a sort pass takes 4 keys per thread instead of
// 16 (measured on MI355X: 200k depth keys 89 -> 74 us over four passes; at
// 1.9M tile keys 4 and 8 keys per thread are 70 % and 17 % slower than 16)
constexpr int64_t kSortSmall = int64_t(1) << 19;
constexpr uint32_t kSpinLimit = 1u << 20;   // bounded waits of the look-back kernels

int blocks_for(int64_t n, int chunk) { return (int)((n + chunk - 1) / chunk); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a block of kScanThreads.
// Returns the exclusive prefix; *total receives the block total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(x);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const uint32_t v = wsum[w];
    before += (w < wave) ? v : 0u;
    all += v;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}


// Single-pass exclusive scan with decoupled look-back. Workgroups publish
// their chunk total, and the first wave looks back over the published totals
// of up to 64 predecessors per step until it meets an inclusive prefix. A
// workgroup waits only on lower workgroup indices, which the dispatcher has
// already placed: each XCD dispatches its workgroups in index order, so the
// lowest workgroup not yet placed only waits for placed ones, which finish
// and free its XCD's slots. (Ticket counters would guarantee this order too,
// but hundreds of workgroups incrementing one word serialise on it: 7 us of a
// 65 us tile sort.) A wait is still bounded: past the spin limit the error
// flag is raised and the scan goes on, so every wave exits. Status word per
// workgroup: flag (1 = chunk total, 2 = inclusive prefix) in the high half,
// the value in the low half.
constexpr unsigned long long kScanAgg = 1ull << 32;
constexpr unsigned long long kScanInc = 2ull << 32;

__global__ void __launch_bounds__(kScanThreads) scan_lookback_kernel(
    const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ n_dev,
    int64_t n_host, uint32_t* __restrict__ out, uint32_t* __restrict__ total_out,
    unsigned long long* __restrict__ status, uint32_t* __restrict__ err, uint32_t* __restrict__ block_rank,
    int64_t plan_blocks) {
  __shared__ uint32_t tile[kScanChunk];
  __shared__ uint32_t s_excl;
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  const uint32_t bid = blockIdx.x;
  const int64_t base = (int64_t)bid * kScanChunk;
  // workgroups past the element count have nothing to do, and no workgroup
  // that has looks at them
  if (base >= n && bid > 0) return;
  const bool last_block = base + kScanChunk >= n;
  // loads at in-bounds addresses for every lane (element 0 past the end),
  // all issued before the first wait
  uint32_t ld[kScanItems];
  if (idx) {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t j = base + k * kScanThreads + threadIdx.x;
      ld[k] = idx[j < n ? j : 0];
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t j = base + k * kScanThreads + threadIdx.x;
      ld[k] = in[j < n ? ld[k] : 0u];
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t j = base + k * kScanThreads + threadIdx.x;
      ld[k] = in[j < n ? j : 0];
    }
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    tile[local] = base + local < n ? ld[k] : 0u;
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = tile[threadIdx.x * kScanItems + k];
    s += v[k];
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan(s, &tot);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(status + bid, (bid == 0 ? kScanInc : kScanAgg) | tot, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    if (bid > 0) {
      int64_t p = (int64_t)bid - 1;          // nearest predecessor not yet summed
      uint32_t spins = 0;
      while (true) {
        const int64_t q = p - lane;
        const unsigned long long w =
            q >= 0 ? __hip_atomic_load(status + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kScanInc;
        const uint32_t flag = (uint32_t)(w >> 32);
        const uint64_t waiting = __ballot(flag == 0u);
        const uint64_t inc = __ballot(flag == 2u);
        const int first_inc = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint64_t need = first_inc >= 63 ? ~0ull : ((2ull << first_inc) - 1ull);
        if (waiting & need) {
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicOr(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        uint32_t val = (lane <= first_inc) ? (uint32_t)w : 0u;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) val += __shfl_xor(val, m, 64);
        excl += val;
        if (first_inc < 64) break;
        p -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(status + bid, kScanInc | (unsigned long long)(excl + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_excl = excl;
      if (last_block && total_out) *total_out = excl + tot;
    }
  }
  __syncthreads();
  uint32_t run = s_excl + ex;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    tile[threadIdx.x * kScanItems + k] = run;
    // the emission plan: element j's run [run, run + v) holds the first
    // position of every output block starting in it
    if (block_rank) {
      const uint32_t j = (uint32_t)(base + threadIdx.x * kScanItems + k);
      for (int64_t b = ((int64_t)run + kEmitBlock - 1) / kEmitBlock;
           b < plan_blocks && b * kEmitBlock < (int64_t)run + v[k]; ++b)
        block_rank[b] = j;
    }
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    const int64_t j = base + local;
    if (j < n) out[j] = tile[local];
  }
}

// Compaction of the visible splats and their instance offsets in one
// single-pass scan over all splats in index order (the order the per-tile
// depth path bins them in): vals[r] = index of the r-th splat with a nonzero
// tile count, offsets[r] = the tile counts of the visible splats before it,
// *count_out = their number, *total_out = the instance total; with block_rank
// also the emission plan (as scan_lookback_kernel writes it). Status word per
// workgroup: flag (1 = chunk totals, 2 = inclusive) in bits 62-63, the
// visible count in bits 32-61 and the instance count in bits 0-31; sums of
// such words stay exact while there are fewer than 2^30 splats and 2^32
// instances. Look-back and bounded wait as in scan_lookback_kernel.
constexpr unsigned long long kCsAgg = 1ull << 62;
constexpr unsigned long long kCsInc = 2ull << 62;
constexpr unsigned long long kCsPayload = (1ull << 62) - 1ull;

// Blocks of tiles a listed splat's tile rectangle overlaps (BlockGeo), from
// its inclusive pixel rectangle.
__device__ __forceinline__ uint32_t block_count(const int4& r, const BlockGeo& g) {
  const uint32_t bx0 = ((uint32_t)r.x >> g.twl) >> g.bwl, bx1 = ((uint32_t)r.z >> g.twl) >> g.bwl;
  const uint32_t by0 = ((uint32_t)r.y >> g.thl) >> g.bhl, by1 = ((uint32_t)r.w >> g.thl) >> g.bhl;
  return (bx1 - bx0 + 1u) * (by1 - by0 + 1u);
}

// BLOCKS: the counts scanned are the splats' block counts (binning by blocks
// of tiles; rect and geo give them), and the sum of their tile counts is
// added to *tile_total (one atomic per workgroup).
template <bool BLOCKS>
__global__ void __launch_bounds__(kScanThreads) compact_scan_kernel(
    const uint32_t* __restrict__ ntiles, int64_t n, uint32_t* __restrict__ vals, uint32_t* __restrict__ offsets,
    uint32_t* __restrict__ count_out, uint32_t* __restrict__ total_out, unsigned long long* __restrict__ status,
    uint32_t* __restrict__ err, uint32_t* __restrict__ block_rank, int64_t plan_blocks,
    const int4* __restrict__ rect, BlockGeo geo, uint32_t* __restrict__ tile_total) {
  __shared__ uint32_t tile[kScanChunk];
  __shared__ unsigned long long s_excl;
  const uint32_t bid = blockIdx.x;
  const int64_t base = (int64_t)bid * kScanChunk;
  // loads at in-bounds addresses for every lane, all issued before the
  // first wait
  uint32_t ld[kScanItems];
  int4 rct[BLOCKS ? kScanItems : 1];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = base + k * kScanThreads + threadIdx.x;
    ld[k] = ntiles[j < n ? j : 0];
    if (BLOCKS) rct[k] = rect[j < n ? j : 0];
  }
  uint32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    const uint32_t c = base + local < n ? ld[k] : 0u;
    if (BLOCKS) {
      // the rectangle of an unlisted splat is stale: only listed ones count
      tsum += c;
      tile[local] = c != 0u ? block_count(rct[k], geo) : 0u;
    } else {
      tile[local] = c;
    }
  }
  if (BLOCKS) {
    tsum = wave_incl_scan(tsum);
    if ((threadIdx.x & 63) == 63 && tsum) atomicAdd(tile_total, tsum);
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t sc = 0, st = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = tile[threadIdx.x * kScanItems + k];
    sc += v[k] != 0u ? 1u : 0u;
    st += v[k];
  }
  uint32_t totc, tott;
  const uint32_t exc = block_excl_scan(sc, &totc);
  const uint32_t ext = block_excl_scan(st, &tott);
  const unsigned long long mine = ((unsigned long long)totc << 32) | tott;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(status + bid, (bid == 0 ? kCsInc : kCsAgg) | mine, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long excl = 0;
    if (bid > 0) {
      int64_t p = (int64_t)bid - 1;          // nearest predecessor not yet summed
      uint32_t spins = 0;
      while (true) {
        const int64_t q = p - lane;
        const unsigned long long w =
            q >= 0 ? __hip_atomic_load(status + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kCsInc;
        const uint32_t flag = (uint32_t)(w >> 62);
        const uint64_t waiting = __ballot(flag == 0u);
        const uint64_t inc = __ballot(flag == 2u);
        const int first_inc = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint64_t need = first_inc >= 63 ? ~0ull : ((2ull << first_inc) - 1ull);
        if (waiting & need) {
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicOr(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        const unsigned long long val = (lane <= first_inc) ? (w & kCsPayload) : 0ull;
        uint32_t lo = (uint32_t)val, hi = (uint32_t)(val >> 32);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
          lo += __shfl_xor(lo, m, 64);
          hi += __shfl_xor(hi, m, 64);
        }
        excl += ((unsigned long long)hi << 32) + lo;
        if (first_inc < 64) break;
        p -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(status + bid, kCsInc | (excl + mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_excl = excl;
      if (bid == gridDim.x - 1) {
        *count_out = (uint32_t)((excl + mine) >> 32);
        *total_out = (uint32_t)(excl + mine);
      }
    }
  }
  __syncthreads();
  uint32_t rc = (uint32_t)(s_excl >> 32) + exc, rt = (uint32_t)s_excl + ext;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (v[k]) {
      vals[rc] = (uint32_t)(base + threadIdx.x * kScanItems + k);
      offsets[rc] = rt;
      // the emission plan: rank rc's run [rt, rt + v) holds the first position
      // of every output block starting in it
      if (block_rank)
        for (int64_t b = ((int64_t)rt + kEmitBlock - 1) / kEmitBlock; b < plan_blocks && b * kEmitBlock < (int64_t)rt + v[k];
             ++b)
          block_rank[b] = rc;
      ++rc;
    }
    rt += v[k];
  }
}

// Order-preserving compaction of the visible splats (nonzero tile count):
// out_keys[r], out_vals[r] = key and index of the r-th visible splat; the
// count -> *count_out. Single pass with the same look-back as the scan.
__global__ void __launch_bounds__(kScanThreads) compact_visible_kernel(
    const uint32_t* __restrict__ ntiles, const uint32_t* __restrict__ keys, int64_t n,
    uint32_t* __restrict__ out_keys, uint32_t* __restrict__ out_vals, uint32_t* __restrict__ count_out,
    unsigned long long* __restrict__ status, uint32_t* __restrict__ err) {
  __shared__ uint32_t s_excl;
  __shared__ uint32_t flags[kScanChunk];
  const uint32_t bid = blockIdx.x;
  const int64_t base = (int64_t)bid * kScanChunk;
  uint32_t ld[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = base + k * kScanThreads + threadIdx.x;
    ld[k] = ntiles[j < n ? j : 0];
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    flags[local] = (base + local < n && ld[k] != 0u) ? 1u : 0u;
  }
  __syncthreads();
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = flags[threadIdx.x * kScanItems + k];
    s += v[k];
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan(s, &tot);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_store(status + bid, (bid == 0 ? kScanInc : kScanAgg) | tot, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    if (bid > 0) {
      int64_t p = (int64_t)bid - 1;
      uint32_t spins = 0;
      while (true) {
        const int64_t q = p - lane;
        const unsigned long long w =
            q >= 0 ? __hip_atomic_load(status + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kScanInc;
        const uint32_t flag = (uint32_t)(w >> 32);
        const uint64_t waiting = __ballot(flag == 0u);
        const uint64_t inc = __ballot(flag == 2u);
        const int first_inc = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint64_t need = first_inc >= 63 ? ~0ull : ((2ull << first_inc) - 1ull);
        if (waiting & need) {
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicOr(err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        uint32_t val = (lane <= first_inc) ? (uint32_t)w : 0u;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) val += __shfl_xor(val, m, 64);
        excl += val;
        if (first_inc < 64) break;
        p -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(status + bid, kScanInc | (unsigned long long)(excl + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_excl = excl;
      if (bid == gridDim.x - 1) *count_out = excl + tot;
    }
  }
  __syncthreads();
  uint32_t run = s_excl + ex;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (v[k]) {
      const int64_t j = base + threadIdx.x * kScanItems + k;
      out_keys[run] = keys[j];
      out_vals[run] = (uint32_t)j;
    }
    run += v[k];
  }
}

// ---------------------------------------------------------------------------
// Onesweep LSD radix sort with RB-bit digits (RB = 8 or 11: 256 or 2048
// buckets; 11-bit digits sort 32-bit depth keys in 3 passes and up to 2048
// tiles in one).
//   global_hist: digit histograms of every pass in one read of the keys
//                (skipped when the producer of the keys accumulated them).
//   pass:        one kernel per digit. Each workgroup ranks its chunk of
//                keys (256 threads x 4 or 16 keys, 4 for small sorts so that
//                a pass spreads over more CUs) with wave ballots, publishes
//                its per-digit counts, and gets its per-digit offset by
//                looking back over the published counts of lower workgroup
//                indices (decoupled look-back; the dispatch order makes this
//                safe, as for the scan above). A wait on a predecessor is
//                bounded: past the spin limit the workgroup raises the error
//                flag and goes on, so every wave exits.
// Each thread owns R / 256 consecutive digits for the per-digit steps.
// Status word per (workgroup, digit): 2 flag bits (1 = count of this
// workgroup, 2 = inclusive prefix up to this workgroup) over a 30-bit count.
// ---------------------------------------------------------------------------
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kCountMask = (1u << 30) - 1;
constexpr int kMaxRadix = 2048;

// Digit width and pass count for a sort on `bits` key bits. 8-bit digits:
// measured on MI355X, an 11-bit pass (2048 buckets: 8x the published counts
// and look-back traffic per workgroup) costs about three 8-bit passes, so it
// never pays for the pass it saves.
__host__ __device__ inline void radix_plan(int bits, int* rb, int* passes) {
  *rb = 8;
  *passes = (bits + 7) / 8;
}

// Digit bits of the pass over block ids (at least one, so that a single
// block still gets its pass and its table).
__host__ __device__ inline int bits_for_blocks(int nblocks) {
  int b = 1;
  while (b < 8 && (1 << b) < nblocks) ++b;
  return b;
}

__global__ void __launch_bounds__(kSortThreads) global_hist_kernel(const uint32_t* __restrict__ keys,
                                                                   const uint32_t* __restrict__ n_dev, int64_t n_host,
                                                                   int rb, int passes, uint32_t* __restrict__ ghist) {
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  __shared__ uint32_t h[3 * kMaxRadix];          // passes * radix <= 3 * 2048 (11-bit) or 4 * 256 (8-bit)
  const int R = 1 << rb;
  for (int e = threadIdx.x; e < passes * R; e += kSortThreads) h[e] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t j = base + k * kSortThreads + threadIdx.x;
    if (j < n) {
      const uint32_t key = keys[j];
      for (int p = 0; p < passes; ++p) atomicAdd(&h[p * R + ((key >> (rb * p)) & (R - 1))], 1u);
    }
  }
  __syncthreads();
  uint32_t* dst = ghist + (size_t)(blockIdx.x % kHistCopies) * (passes * R);
  for (int e = threadIdx.x; e < passes * R; e += kSortThreads)
    if (h[e]) atomicAdd(&dst[e], h[e]);
}

// Counting half of a reduce-then-scan digit pass: workgroup b counts the
// digits of keys [b CHUNK, (b + 1) CHUNK) and stores them digit-major,
// counts[d * nb + b], so that one exclusive scan over the array gives each
// (digit, workgroup) run its first output position. Workgroups past the
// element count store zeros.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads) digit_count_kernel(const uint32_t* __restrict__ keys,
                                                                   const uint32_t* __restrict__ n_dev, int64_t n_host,
                                                                   int shift, int dbits,
                                                                   uint32_t* __restrict__ counts) {
  constexpr int R = 256;
  constexpr int NW = kSortThreads / 64;
  constexpr int CHUNK = kSortThreads * ITEMS;
  static_assert(R == kSortThreads, "one digit per thread");
  __shared__ uint32_t h[NW][R];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
#pragma unroll
  for (int w = 0; w < NW; ++w) h[w][tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  // all loads in flight before the first wait (in-bounds addresses, element
  // 0 past the end), then the counts of the valid items
  uint32_t k[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t j = base + r * kSortThreads + tid;
    k[r] = keys[j < n ? j : 0];
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r)
    if (base + r * kSortThreads + tid < n) atomicAdd(&h[wave][(k[r] >> shift) & ((1u << dbits) - 1u)], 1u);
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) c += h[w][tid];
  if (tid < (1 << dbits)) counts[(size_t)tid * gridDim.x + blockIdx.x] = c;
}

// One digit pass: rank each key within its workgroup, find the output
// position of the workgroup's run of each digit, scatter. The run starts
// come either from a decoupled look-back over the workgroups' published
// digit counts plus the global histogram (SCANNED false: `status` holds the
// published counts), or, SCANNED true, from the exclusive scan of
// digit_count_kernel's counts (`status` holds that scan, digit-major).
// TABLE: the pass over block ids of the binning by blocks, whose first
// workgroup also writes the block table (see launch_block_sort).
template <int RB, int ITEMS, bool SCANNED = false, bool TABLE = false>
__global__ void __launch_bounds__(kSortThreads) onesweep_pass_kernel(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, const uint32_t* __restrict__ n_dev,
    int64_t n_host, int shift, int dbits, const uint32_t* __restrict__ ghist, int ghist_stride,
    uint32_t* __restrict__ status,
    uint32_t* __restrict__ err, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const uint32_t* __restrict__ whist = nullptr, uint4* __restrict__ table = nullptr) {
  constexpr int R = 1 << RB;
  constexpr int NW = kSortThreads / 64;
  constexpr int CHUNK = kSortThreads * ITEMS;    // keys per workgroup
  constexpr int WCHUNK = 64 * ITEMS;             // keys per wave
  constexpr int DPT = R / kSortThreads;          // digits owned per thread
  static_assert(R % kSortThreads == 0, "whole digits per thread");
  // wcnt (per-wave digit counts) is dead once each key has its block-local
  // offset; the staged keys and values reuse its storage
  static_assert(NW * R >= 2 * CHUNK || RB == 8, "staging fits in the count storage");
  constexpr int kCountWords = NW * R > 2 * CHUNK ? NW * R : 2 * CHUNK;
  __shared__ uint32_t s_mem[kCountWords];
  __shared__ uint32_t gofs[R];         // global start of each digit's run of this block (minus its local start)
  __shared__ uint32_t lstart[R];       // block-local start of each digit's run
  __shared__ uint32_t s_wsum[2][NW];
  __shared__ uint32_t s_tsum[NW];
  uint32_t (*wcnt)[R] = reinterpret_cast<uint32_t (*)[R]>(s_mem);
  uint32_t* s_keys = s_mem;
  uint32_t* s_vals = s_mem + CHUNK;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  const int64_t n = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  // the digit's low `dbits` bits (all RB but in the top pass of a sort on a
  // bit count that is no multiple of RB, whose keys leave the rest zero)
  const uint32_t dmask = (1u << dbits) - 1u;
  for (int e = tid; e < NW * R; e += kSortThreads) (&wcnt[0][0])[e] = 0;
  __syncthreads();
  const uint32_t bid = blockIdx.x;
  // workgroups past the element count have nothing to do, and no workgroup
  // that has looks at them
  if ((int64_t)bid * CHUNK >= n && bid > 0) return;
  const int64_t base = (int64_t)bid * CHUNK + (int64_t)wave * WCHUNK;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t k_reg[ITEMS], v_reg[ITEMS], off[ITEMS];
  // every lane loads from an address in bounds (element 0 past the end), so
  // all of the workgroup's loads are in flight before the first wait; a
  // guarded load per item would cost one memory round trip per item
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t j = base + r * 64 + lane;
    const int64_t jc = j < n ? j : 0;
    k_reg[r] = keys[jc];
    v_reg[r] = vals[jc];
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t j = base + r * 64 + lane;
    const bool valid = j < n;
    const uint32_t key = valid ? k_reg[r] : 0u;
    k_reg[r] = key;
    const uint32_t d = (key >> shift) & dmask;
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if (b >= dbits) break;
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      mask &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(mask & lt_mask);
    const uint32_t before = wcnt[wave][d];
    off[r] = valid ? before + rank : 0xFFFFFFFFu;
    if (valid && rank == 0) wcnt[wave][d] = before + (uint32_t)__popcll(mask);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // owned digits: wave prefixes in place, block counts, aggregates published
  uint32_t mine[DPT];
#pragma unroll
  for (int t = 0; t < DPT; ++t) {
    const int d = tid * DPT + t;
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = acc;
      acc += c;
    }
    mine[t] = acc;
    if (!SCANNED)
      __hip_atomic_store(status + (size_t)bid * R + d, (bid == 0 ? kFlagInc : kFlagAgg) | acc, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  // exclusive prefixes over lower workgroups, all owned digits walking together
  uint32_t excl[DPT];
#pragma unroll
  for (int t = 0; t < DPT; ++t) excl[t] = 0;
  if (!SCANNED && bid > 0 && DPT == 1) {
    // one digit per thread: read kLookChunk predecessors per round trip and
    // take them in order until an inclusive prefix; an entry not yet
    // published stops the round, which is retried from there
    constexpr int kLookChunk = 16;
    int64_t p = (int64_t)bid - 1;
    uint32_t spins = 0;
    const int d = tid;
    while (true) {
      uint32_t v[kLookChunk];
#pragma unroll
      for (int q = 0; q < kLookChunk; ++q)
        v[q] = p - q >= 0 ? __hip_atomic_load(status + (size_t)(p - q) * R + d, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)
                          : kFlagInc;
      int used = 0;
      bool found = false;
#pragma unroll
      for (int q = 0; q < kLookChunk; ++q) {
        if (found || used < q) continue;
        const uint32_t flag = v[q] & ~kCountMask;
        if (flag == 0u) continue;
        excl[0] += v[q] & kCountMask;
        used = q + 1;
        found = flag == kFlagInc;
      }
      if (found) break;
      p -= used;
      if (used < kLookChunk) {
        if (++spins > kSpinLimit) {
          atomicOr(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __hip_atomic_store(status + (size_t)bid * R + d, kFlagInc | (excl[0] + mine[0]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else if (!SCANNED && bid > 0) {
    uint32_t pending = (DPT == 32 ? ~0u : ((1u << DPT) - 1u));
    int64_t p = (int64_t)bid - 1;
    uint32_t spins = 0;
    while (pending && p >= 0) {
      uint32_t v[DPT];
      bool wait = false;
#pragma unroll
      for (int t = 0; t < DPT; ++t) {
        v[t] = ((pending >> t) & 1u)
                   ? __hip_atomic_load(status + (size_t)p * R + tid * DPT + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : kFlagInc;
        wait = wait || ((v[t] & ~kCountMask) == 0u);
      }
      if (wait) {
        if (++spins > kSpinLimit) {
          atomicOr(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
#pragma unroll
      for (int t = 0; t < DPT; ++t) {
        if (!((pending >> t) & 1u)) continue;
        excl[t] += v[t] & kCountMask;
        if ((v[t] & ~kCountMask) == kFlagInc) pending &= ~(1u << t);
      }
      --p;
    }
#pragma unroll
    for (int t = 0; t < DPT; ++t)
      __hip_atomic_store(status + (size_t)bid * R + tid * DPT + t, kFlagInc | (excl[t] + mine[t]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  // exclusive scans over the R digits: of the global histogram (start of
  // each digit in the output) and of this block's counts (local runs)
  {
    uint32_t gs = 0, ms = 0, gpre[DPT], mpre[DPT];
#pragma unroll
    for (int t = 0; t < DPT; ++t) {
      gpre[t] = gs;
      mpre[t] = ms;
      uint32_t h = 0;
      if (!SCANNED) {
#pragma unroll
        for (int c = 0; c < kHistCopies; ++c) h += ghist[(size_t)c * ghist_stride + tid * DPT + t];
      }
      gs += h;
      ms += mine[t];
    }
    uint32_t x = gs, y = ms;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
      const uint32_t xs = __shfl_up(x, dd, 64), ys = __shfl_up(y, dd, 64);
      if (lane >= dd) {
        x += xs;
        y += ys;
      }
    }
    if (lane == 63) {
      s_wsum[0][wave] = x;
      s_wsum[1][wave] = y;
    }
    __syncthreads();
    uint32_t bx = 0, by = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      bx += (w < wave) ? s_wsum[0][w] : 0u;
      by += (w < wave) ? s_wsum[1][w] : 0u;
    }
    const uint32_t gx0 = bx + x - gs, my0 = by + y - ms;
#pragma unroll
    for (int t = 0; t < DPT; ++t) {
      const int d = tid * DPT + t;
      lstart[d] = my0 + mpre[t];
      // (the scanned starts exist for the live digits only; no key has another)
      const uint32_t start =
          SCANNED ? ((uint32_t)d <= dmask ? status[(size_t)d * gridDim.x + bid] : 0u) : gx0 + gpre[t] + excl[t];
      gofs[d] = start - (my0 + mpre[t]);
    }
    if (TABLE && !SCANNED && DPT == 1 && bid == 0) {
      // binning by blocks (one pass over the block ids): per block, its run
      // [start, end) in the sorted output and the first position of its
      // tiles' lists (the tiles of the blocks before it, summed)
      const uint32_t h = gs;     // this digit's (block's) instance count
      uint32_t w = 0;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c) w += whist[(size_t)c * R + tid];
      uint32_t z = w;
#pragma unroll
      for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t zs = __shfl_up(z, dd, 64);
        if (lane >= dd) z += zs;
      }
      if (lane == 63) s_tsum[wave] = z;
      __syncthreads();
      uint32_t bz = 0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) bz += (w2 < wave) ? s_tsum[w2] : 0u;
      const uint32_t st0 = gx0 + gpre[0];
      table[tid] = make_uint4(st0, st0 + h, bz + z - w, w);
    }
  }
  __syncthreads();
  // block-local position of every key, then the count storage becomes the
  // staging area
  uint32_t lp[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t d = (k_reg[r] >> shift) & dmask;
    lp[r] = off[r] == 0xFFFFFFFFu ? 0xFFFFFFFFu : lstart[d] + wcnt[wave][d] + off[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    if (lp[r] == 0xFFFFFFFFu) continue;
    s_keys[lp[r]] = k_reg[r];
    s_vals[lp[r]] = v_reg[r];
  }
  __syncthreads();
  // consecutive threads write consecutive positions of each digit's run
  const int64_t blk0 = (int64_t)bid * CHUNK;
  const int cnt = (int)(n - blk0 < CHUNK ? (n - blk0 > 0 ? n - blk0 : 0) : CHUNK);
  for (int j = tid; j < cnt; j += kSortThreads) {
    const uint32_t key = s_keys[j];
    const uint32_t d = (key >> shift) & dmask;
    const uint32_t pos = gofs[d] + (uint32_t)j;
    if (pos < n) {
      keys_out[pos] = key;
      vals_out[pos] = s_vals[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Binning by counting, for the per-tile depth order (each tile's list is
// sorted by (depth, index) after binning, so the binning itself only has to
// group the instances by tile). Workgroup (v, b) owns the splats [b C, (b +
// 1) C) of view v. bin_count_kernel counts its instances per tile of the view
// in LDS and stores the counts tile-major, counts[tile * nb + b] (tile =
// global tile id, nb workgroups per view); one exclusive scan over that
// matrix gives each (tile, workgroup) run its first output position, tiles in
// global order; bin_scatter_kernel walks the same instances again and puts
// each into its workgroup's run of its tile (in LDS-atomic order: the depth
// sort that follows imposes the final order) and writes the tile ranges.
// This replaces the emission, the radix sort of the tile keys and the range
// search of the general path: no global atomics, two passes over the splats'
// records and one over the instances.
// ---------------------------------------------------------------------------
constexpr int kBinThreads = 1024;        // one splat per thread per round
constexpr int kBinMaxTiles = 8192;       // tiles of one view (LDS bins, 32 KB)

struct BinArgs {
  const uint32_t* ntiles;     // [V * n] tile count per splat (0: not listed)
  const int4* rect;           // [V * n] pixel rectangle, inclusive
  const ViewDesc* views;
  int64_t n;                  // Gaussians (splats per view)
  int chunk;                  // splats per workgroup, a multiple of kBinThreads
  int nb;                     // workgroups per view
  int tw_log2, th_log2;       // tile size (powers of two)
};

// The tile rectangle of splat sidx (a listed one): its first view-local tile,
// width and height in tiles.
__device__ __forceinline__ void bin_rect(const BinArgs& a, int tiles_x, int64_t sidx, int* first, int* w, int* h) {
  const int4 r = a.rect[sidx];
  const int tx0 = r.x >> a.tw_log2, tx1 = r.z >> a.tw_log2;
  const int ty0 = r.y >> a.th_log2, ty1 = r.w >> a.th_log2;
  *first = ty0 * tiles_x + tx0;
  *w = tx1 - tx0 + 1;
  *h = ty1 - ty0 + 1;
}

__global__ void __launch_bounds__(kBinThreads) bin_count_kernel(BinArgs a, uint32_t* __restrict__ counts,
                                                                uint32_t* __restrict__ visible_out) {
  extern __shared__ uint32_t s_bins[];                 // the view's tiles
  __shared__ uint32_t s_visible;
  const int v = blockIdx.x / a.nb, b = blockIdx.x % a.nb;
  const ViewDesc& V = a.views[v];
  const int tiles_x = V.tiles_x, tiles = V.tiles_x * V.tiles_y;
  for (int t = threadIdx.x; t < tiles; t += kBinThreads) s_bins[t] = 0u;
  if (threadIdx.x == 0) s_visible = 0u;
  __syncthreads();
  uint32_t visible = 0;
  const int64_t c0 = (int64_t)b * a.chunk, c1 = min(c0 + (int64_t)a.chunk, a.n);
  for (int64_t j = c0 + threadIdx.x; j < c1; j += kBinThreads) {
    const int64_t sidx = (int64_t)v * a.n + j;
    if (a.ntiles[sidx] == 0u) continue;
    ++visible;
    int first, w, h;
    bin_rect(a, tiles_x, sidx, &first, &w, &h);
    for (int dy = 0; dy < h; ++dy)
      for (int dx = 0; dx < w; ++dx) atomicAdd(&s_bins[first + dy * tiles_x + dx], 1u);
  }
  const uint64_t any = __ballot(visible != 0u);
  if (any) {
    uint32_t x = visible;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_visible, x);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tiles; t += kBinThreads)
    counts[(int64_t)(V.tile_offset + t) * a.nb + b] = s_bins[t];
  if (threadIdx.x == 0 && s_visible) atomicAdd(visible_out, s_visible);
}

__global__ void __launch_bounds__(kBinThreads) bin_scatter_kernel(BinArgs a, const uint32_t* __restrict__ starts,
                                                                  const uint32_t* __restrict__ total_dev,
                                                                  int64_t capacity, int64_t num_tiles,
                                                                  uint32_t* __restrict__ keys,
                                                                  uint32_t* __restrict__ vals,
                                                                  uint2* __restrict__ ranges,
                                                                  uint32_t* __restrict__ overflow) {
  extern __shared__ uint32_t s_bins[];                 // next free position of each tile's run
  const int v = blockIdx.x / a.nb, b = blockIdx.x % a.nb;
  const ViewDesc& V = a.views[v];
  const int tiles_x = V.tiles_x, tiles = V.tiles_x * V.tiles_y;
  const uint32_t toff = (uint32_t)V.tile_offset;
  const uint32_t total = *total_dev;
  const uint32_t cap = (uint32_t)min(capacity, (int64_t)0xFFFFFFFF);
  if (blockIdx.x == 0 && threadIdx.x == 0 && (int64_t)total > capacity) atomicOr(overflow, 1u);
  for (int t = threadIdx.x; t < tiles; t += kBinThreads) s_bins[t] = starts[(int64_t)(toff + t) * a.nb + b];
  // the ranges of this view's tiles, spread over its workgroups; clipped to
  // the instance storage (an overflowing render lists only what fits)
  for (int t = b * kBinThreads + threadIdx.x; t < tiles; t += a.nb * kBinThreads) {
    const int64_t g = (int64_t)toff + t;
    const uint32_t st = starts[g * a.nb];
    const uint32_t en = g + 1 < num_tiles ? starts[(g + 1) * a.nb] : total;
    ranges[g] = make_uint2(min(st, cap), min(en, cap));
  }
  __syncthreads();
  const int64_t c0 = (int64_t)b * a.chunk, c1 = min(c0 + (int64_t)a.chunk, a.n);
  for (int64_t j = c0 + threadIdx.x; j < c1; j += kBinThreads) {
    const int64_t sidx = (int64_t)v * a.n + j;
    if (a.ntiles[sidx] == 0u) continue;
    int first, w, h;
    bin_rect(a, tiles_x, sidx, &first, &w, &h);
    for (int dy = 0; dy < h; ++dy)
      for (int dx = 0; dx < w; ++dx) {
        const int t = first + dy * tiles_x + dx;
        const uint32_t pos = atomicAdd(&s_bins[t], 1u);
        if (pos < cap) {
          keys[pos] = toff + (uint32_t)t;
          vals[pos] = (uint32_t)sidx;
        }
      }
  }
}

// Instance emission, balanced over the output: workgroup b writes the
// output positions [1024 b, 1024 b + 1024). emit_plan_kernel first records,
// per block, the depth rank whose instances hold the block's first position;
// the block's ranks (at most 1024, every listed splat has at least one
// instance) are staged with their offsets, and each thread writes output
// positions round-robin, finding the owning rank by binary search over the
// staged offsets. Positions past `capacity` are dropped and flagged.

__global__ void __launch_bounds__(256) emit_plan_kernel(const uint32_t* __restrict__ offsets,
                                                        const uint32_t* __restrict__ total_dev,
                                                        const uint32_t* __restrict__ count_dev, int64_t count_host,
                                                        int64_t nblocks, uint32_t* __restrict__ block_rank) {
  const int64_t count = count_dev ? min((int64_t)*count_dev, count_host) : count_host;
  const uint32_t total = *total_dev;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < count; r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t a = offsets[r], b = r + 1 < count ? offsets[r + 1] : total;
    // blocks whose first position lies in [a, b)
    for (int64_t blk = ((int64_t)a + kEmitBlock - 1) / kEmitBlock; blk * kEmitBlock < (int64_t)b && blk < nblocks; ++blk)
      block_rank[blk] = (uint32_t)r;
  }
}

// BLOCKS: one instance per (splat, block of tiles) instead of per (splat,
// tile) (binning by blocks; geo, rect and views give the blocks). Its key is
// the global block id in bits 0-15 and the part of the splat's tile
// rectangle inside the block, block-relative, in bits 16-31 (first and
// one-past-last column, then row, 4 bits each). hist receives the
// histogram of the block ids (one 8-bit pass) and whist, per block, the
// tiles its instances cover (both in kHistCopies copies).
template <bool BLOCKS>
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(const uint32_t* __restrict__ sorted_s,
                                                           const uint32_t* __restrict__ offsets,
                                                           const uint32_t* __restrict__ total_dev,
                                                           const uint32_t* __restrict__ count_dev,
                                                           const uint32_t* __restrict__ block_rank,
                                                           const Splat* __restrict__ splats, int64_t count_host,
                                                           uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                           int64_t capacity, uint32_t* __restrict__ overflow,
                                                           uint32_t* __restrict__ hist, int hist_rb, int hist_passes,
                                                           const int4* __restrict__ rect,
                                                           const ViewDesc* __restrict__ views, uint32_t num,
                                                           BlockGeo geo, uint32_t* __restrict__ whist) {
  __shared__ uint32_t s_off[kEmitBlock + 1];
  __shared__ uint32_t s_sid[kEmitBlock];
  // first tile id of the rectangle; rectangle width | view row pitch << 16.
  // BLOCKS: view-local tile rectangle (x0 | x1 << 16, y0 | y1 << 16, both
  // inclusive), the first block's global id and the splat's blocks per row |
  // the view's blocks per row << 16
  __shared__ int4 s_geo4[BLOCKS ? kEmitBlock : 1];
  __shared__ int2 s_geo2[BLOCKS ? 1 : kEmitBlock];
  __shared__ uint32_t s_hist[kEmitHist];  // hist_passes * 2^hist_rb <= kEmitHist; BLOCKS: 2 x 256
  const int tid = threadIdx.x;
  const uint32_t total = *total_dev;
  if (blockIdx.x == 0 && tid == 0 && (int64_t)total > capacity) atomicOr(overflow, 1u);
  const int64_t count = count_dev ? min((int64_t)*count_dev, count_host) : count_host;
  const int64_t o0 = (int64_t)blockIdx.x * kEmitBlock;
  const int64_t written = min((int64_t)total, capacity);
  const int64_t oend = min(o0 + kEmitBlock, written);
  if (o0 >= oend || count == 0) return;
  const int hR = 1 << hist_rb;
  const int hwords = BLOCKS ? 2 * kMaxBlocks : hist_passes * hR;
  if (hist)
    for (int e = tid; e < hwords; e += kEmitThreads) s_hist[e] = 0u;
  // ranks [r0, r_end) hold this block's positions
  // (block b + 1's start is read only if that block exists and starts
  // inside the output; it holds the rank of position 1024 (b + 1))
  const int64_t r0 = block_rank[blockIdx.x];
  const bool next = (int64_t)blockIdx.x + 1 < (int64_t)gridDim.x && o0 + kEmitBlock < written;
  const int64_t r_end = next ? min((int64_t)block_rank[blockIdx.x + 1] + 1, count) : count;
  const int nr = (int)min(r_end - r0, (int64_t)kEmitBlock);
  if (r0 >= count || nr <= 0) return;
  for (int j = tid; j < nr; j += kEmitThreads) {
    const int64_t r = r0 + j;
    s_off[j] = offsets[r];
    const uint32_t sid = sorted_s[r];
    s_sid[j] = sid;
    if (BLOCKS) {
      const int4 rc = rect[sid];
      const ViewDesc& V = views[sid / num];
      const uint32_t x0 = (uint32_t)rc.x >> geo.twl, x1 = (uint32_t)rc.z >> geo.twl;
      const uint32_t y0 = (uint32_t)rc.y >> geo.thl, y1 = (uint32_t)rc.w >> geo.thl;
      const uint32_t bx0 = x0 >> geo.bwl, by0 = y0 >> geo.bhl;
      const uint32_t bw = (x1 >> geo.bwl) - bx0 + 1u;
      s_geo4[j] = make_int4((int)(x0 | (x1 << 16)), (int)(y0 | (y1 << 16)),
                           (int)((uint32_t)V.block_offset + by0 * (uint32_t)V.blocks_x + bx0),
                           (int)(bw | ((uint32_t)V.blocks_x << 16)));
    } else {
      // the tile rectangle the projection stored in the record's spare words
      s_geo2[j] = make_int2((int)__float_as_uint(splats[sid].w1.w), (int)__float_as_uint(splats[sid].w2.w));
    }
  }
  if (tid == 0) s_off[nr] = r0 + nr < count ? offsets[r0 + nr] : total;
  __syncthreads();
  for (int64_t o = o0 + tid; o < oend; o += kEmitThreads) {
    int lo = 0, hi = nr;                  // s_off[lo] <= o < s_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= (uint32_t)o) lo = mid;
      else hi = mid;
    }
    const uint32_t local = (uint32_t)o - s_off[lo];
    uint32_t key;
    if (BLOCKS) {
      const int4 geo4 = s_geo4[lo];
      const uint32_t wdt = (uint32_t)geo4.w & 0xFFFFu, pitch = (uint32_t)geo4.w >> 16;
      const uint32_t dy = local / wdt, dx = local - dy * wdt;
      const uint32_t x0 = (uint32_t)geo4.x & 0xFFFFu, x1 = (uint32_t)geo4.x >> 16;
      const uint32_t y0 = (uint32_t)geo4.y & 0xFFFFu, y1 = (uint32_t)geo4.y >> 16;
      const uint32_t bx = (x0 >> geo.bwl) + dx, by = (y0 >> geo.bhl) + dy;
      const uint32_t cx = bx << geo.bwl, cy = by << geo.bhl;   // the block's first tile
      const uint32_t rx0 = x0 > cx ? x0 - cx : 0u, rx1 = min(x1 + 1u - cx, 1u << geo.bwl);
      const uint32_t ry0 = y0 > cy ? y0 - cy : 0u, ry1 = min(y1 + 1u - cy, 1u << geo.bhl);
      const uint32_t blk = (uint32_t)geo4.z + dy * pitch + dx;
      key = blk | (rx0 << 16) | (rx1 << 20) | (ry0 << 24) | (ry1 << 28);
      if (hist) {
        atomicAdd(&s_hist[blk & (kMaxBlocks - 1)], 1u);
        atomicAdd(&s_hist[kMaxBlocks + (blk & (kMaxBlocks - 1))], (rx1 - rx0) * (ry1 - ry0));
      }
    } else {
      const int2 geo2 = s_geo2[lo];
      const uint32_t wdt = (uint32_t)geo2.y & 0xFFFFu, pitch = (uint32_t)geo2.y >> 16;
      const uint32_t dy = local / wdt, dx = local - dy * wdt;
      key = (uint32_t)geo2.x + dy * pitch + dx;
      if (hist)
        for (int p = 0; p < hist_passes; ++p) atomicAdd(&s_hist[p * hR + ((key >> (hist_rb * p)) & (hR - 1))], 1u);
    }
    keys[o] = key;
    vals[o] = s_sid[lo];
  }
  if (hist) {
    __syncthreads();
    if (BLOCKS) {
      uint32_t* dst = hist + (size_t)(blockIdx.x % kHistCopies) * kMaxBlocks;
      uint32_t* wdst = whist + (size_t)(blockIdx.x % kHistCopies) * kMaxBlocks;
      for (int e = tid; e < kMaxBlocks; e += kEmitThreads) {
        if (s_hist[e]) atomicAdd(&dst[e], s_hist[e]);
        if (s_hist[kMaxBlocks + e]) atomicAdd(&wdst[e], s_hist[kMaxBlocks + e]);
      }
    } else {
      uint32_t* dst = hist + (size_t)(blockIdx.x % kHistCopies) * (hist_passes * hR);
      for (int e = tid; e < hist_passes * hR; e += kEmitThreads)
        if (s_hist[e]) atomicAdd(&dst[e], s_hist[e]);
    }
  }
}

__global__ void tile_ranges_kernel(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                                   int64_t n_host, uint2* __restrict__ ranges, int64_t num_tiles) {
  const int64_t count = n_dev ? min((int64_t)*n_dev, n_host) : n_host;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    // the key and both neighbours loaded together (clamped at the ends)
    const uint32_t k = keys[i];
    const uint32_t kp = keys[i > 0 ? i - 1 : 0];
    const uint32_t kn = keys[i + 1 < count ? i + 1 : i];
    if (k >= num_tiles) continue;
    if (i == 0 || kp != k) ranges[k].x = (uint32_t)i;
    if (i == count - 1 || kn != k) ranges[k].y = (uint32_t)(i + 1);
  }
}

// One workgroup: bucket the tiles by floor(log2(list length)), longest class
// first, with LDS counters.
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) tile_order_kernel(const uint2* __restrict__ ranges,
                                                                   int64_t num_tiles, uint32_t* __restrict__ order) {
  __shared__ uint32_t count[33], cursor[33];
  const int tid = threadIdx.x;
  if (tid < 33) count[tid] = 0u;
  __syncthreads();
  for (int64_t t = tid; t < num_tiles; t += kOrderThreads) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    const int cls = len ? 32 - __clz(len) : 0;      // 0 (empty) .. 32
    atomicAdd(&count[32 - cls], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int c = 0; c < 33; ++c) {
      cursor[c] = run;
      run += count[c];
    }
  }
  __syncthreads();
  for (int64_t t = tid; t < num_tiles; t += kOrderThreads) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    const int cls = len ? 32 - __clz(len) : 0;
    order[atomicAdd(&cursor[32 - cls], 1u)] = (uint32_t)t;
  }
}

// Balanced placement: the tiles sorted by weight (heaviest first; the walk
// length the previous render recorded in tile_last when there is one, else
// the list length), then dealt to consecutive rounds of `ncu` workgroups in
// snake order (round 0 heaviest to lightest, round 1 the reverse, ...). The
// dispatcher hands the first workgroups of a launch to the CUs in turn, so each
// CU starts with a mix of heavy and light tiles rather than several heavy
// ones. One workgroup, a bitonic sort in LDS of at most kBalanceMax tiles.
constexpr int kBalanceMax = 8192;
__global__ void __launch_bounds__(kOrderThreads) tile_balance_kernel(const uint2* __restrict__ ranges,
                                                                     const uint32_t* __restrict__ tile_last,
                                                                     int num_tiles, int ncu,
                                                                     uint32_t* __restrict__ order) {
  __shared__ unsigned long long key[kBalanceMax];
  int n2 = 1;
  while (n2 < num_tiles) n2 <<= 1;
  for (int t = threadIdx.x; t < n2; t += kOrderThreads) {
    unsigned long long k = 0ull;     // padding sorts last
    if (t < num_tiles) {
      const uint2 r = ranges[t];
      const uint32_t len = r.y - r.x;
      const uint32_t tl = tile_last ? tile_last[t] : 0u;
      const uint32_t w = (tl > 0u && tl <= len) ? tl : len;
      // heaviest first, ties by tile index: sort descending on (w, ~t)
      k = ((unsigned long long)(w + 1u) << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)t);
    }
    key[t] = k;
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < n2; i += kOrderThreads) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const unsigned long long a = key[i], b = key[j];
          if (desc ? (a < b) : (a > b)) {
            key[i] = b;
            key[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int b = threadIdx.x; b < num_tiles; b += kOrderThreads) {
    const int round = b / ncu, c = b - round * ncu;
    const int len = min(ncu, num_tiles - round * ncu);
    const int pos = round * ncu + ((round & 1) ? len - 1 - c : c);
    order[b] = 0xFFFFFFFFu - (uint32_t)(key[pos] & 0xFFFFFFFFull);
  }
}

// Per-tile depth order. The instances of a tile arrive in splat-index order
// (emission in index order, then a stable sort by tile); a stable LSD radix
// sort of each tile's list on the raw bits of z (positive floats order like
// their bits; zkey[s], as the projection stores them) then gives the order
// (tile, z bits, index). One workgroup per tile. Every wave ranks rows of
// 64 keys in list order with ballots (the rank among equal digits in the
// row, plus the wave's running count of that digit), so the scatter keeps
// equal digits in list order. A list of at most kTileSortCap entries is
// sorted in LDS, on its keys minus the list's smallest in 9-bit digits (as
// many passes as the range of its keys needs); a longer one in four 8-bit
// passes, chunk by chunk through the alternate key/value buffers, its tile
// keys used as scratch and rewritten at the end.
// Ranks one chunk of n <= kTileSortCap keys held in registers, wave w owning
// the chunk's entries [w R 64, (w + 1) R 64) with R = rpw, row r its entries
// w R 64 + 64 r + lane: off[r] = the entry's rank among the wave's earlier
// entries of its BITS-bit digit; wcnt[w][d] = the wave's count of digit d.
constexpr int kTileSortThreads = 256;
constexpr int kTileSortWaves = kTileSortThreads / 64;
// rows of 64 per wave per chunk: 6 keeps the kernels within five workgroups
// per CU (8 rows took 102 VGPRs and 38 KB of LDS, four workgroups;
// 640x480/200k: 43 -> 37 us)
constexpr int kTileSortRows = 6;
constexpr int kTileSortCap = kTileSortThreads * kTileSortRows;            // 1536 entries per chunk

// rpw: rows per wave in use (the chunk's entries spread evenly over the
// waves, at most kTileSortRows; rows past it are neither ranked nor set).
template <int BITS>
__device__ __forceinline__ void tile_sort_rank(const uint32_t* k, int n, int shift, uint32_t* off,
                                               uint32_t (*wcnt)[1 << BITS], int wave, int lane, int rpw) {
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kTileSortRows; ++r) {
    if (r >= rpw) break;
    const int e = wave * (64 * rpw) + r * 64 + lane;
    const bool valid = e < n;
    const uint32_t d = (k[r] >> shift) & ((1u << BITS) - 1u);
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      mask &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(mask & lt_mask);
    const uint32_t before = wcnt[wave][d];
    off[r] = valid ? before + rank : 0xFFFFFFFFu;
    if (valid && rank == 0) wcnt[wave][d] = before + (uint32_t)__popcll(mask);
    __builtin_amdgcn_wave_barrier();
  }
}

// A tile's list [0, n) sorted by depth key: each run of equal keys is put in
// splat-index order (odd-even transposition within the runs until two
// consecutive rounds change nothing; a list without equal keys costs one
// comparison per entry). The binning leaves equal depths in whatever order it
// placed them (index order for the radix path, LDS-atomic order for the
// counting path); the list order is (tile, depth, index) either way. k and v
// are LDS or global: every thread of the workgroup calls this together.
__device__ void order_equal_depths(const uint32_t* k, uint32_t* v, int n) {
  bool tie = false;
  for (int e = threadIdx.x; e + 1 < n; e += kTileSortThreads) tie = tie || (k[e] == k[e + 1]);
  if (!__syncthreads_or(tie)) return;
  bool prev = true;
  for (int round = 0;; ++round) {
    bool swapped = false;
    const int par = round & 1;
    for (int q = threadIdx.x; 2 * q + par + 1 < n; q += kTileSortThreads) {
      const int i = 2 * q + par;
      if (k[i] == k[i + 1]) {
        const uint32_t a = v[i], b = v[i + 1];
        if (a > b) {
          v[i] = b;
          v[i + 1] = a;
          swapped = true;
        }
      }
    }
    const bool any = __syncthreads_or(swapped);
    if (!any && !prev) break;
    prev = any;
  }
}

// LDS of the per-tile depth sort.
struct TileSortShared {
  union {
    struct {
      uint32_t k[kTileSortCap], v[kTileSortCap];   // the list after each pass
      uint32_t wcnt[kTileSortWaves][512];          // per wave and 9-bit digit
      uint32_t start[512];                         // the digit's first position
    } lds;                                         // the sort in LDS
    uint32_t part[kTileSortWaves][kTileSortCap];   // per-wave staging of the block filter
  };
  // the sort through global memory (8-bit digits)
  uint32_t wcnt[kTileSortWaves][256];
  uint32_t start[256];     // the digit's first position (whole list) plus earlier chunks' count
  uint32_t wsum[kTileSortWaves];
  uint32_t range[2][kTileSortWaves];   // per wave: smallest and largest key
};

// Stable LSD sort of a list of n <= kTileSortCap entries that the workgroup
// holds in registers (thread: rows r < rpw of its wave, entry w rpw 64 +
// 64 r + lane; the other rows and entries past n are padding), on the keys
// minus the list's smallest key, in 9-bit digits: as many passes as the
// largest difference needs (a 25-bit range, depths from 1 to 5, takes three
// where 8-bit digits of the raw keys take four; equal keys none). The
// sorted list ends in S.lds.k (keys minus the smallest), S.lds.v. The buffers
// must be free (a barrier since they were last read).
__device__ __forceinline__ void lds_depth_sort(TileSortShared& S, uint32_t (&k)[kTileSortRows],
                                               uint32_t (&v)[kTileSortRows], int n, int rpw) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
  for (int r = 0; r < kTileSortRows; ++r) {
    if (r >= rpw) break;
    if (wave * (64 * rpw) + r * 64 + lane < n) {
      lo = min(lo, k[r]);
      hi = max(hi, k[r]);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor(lo, d, 64));
    hi = max(hi, (uint32_t)__shfl_xor(hi, d, 64));
  }
  if (lane == 0) {
    S.range[0][wave] = lo;
    S.range[1][wave] = hi;
  }
  for (int w = 0; w < kTileSortWaves; ++w) {
    S.lds.wcnt[w][tid] = 0u;
    S.lds.wcnt[w][tid + 256] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kTileSortWaves; ++w) {
    lo = min(lo, S.range[0][w]);
    hi = max(hi, S.range[1][w]);
  }
  const uint32_t span = hi - lo;
  const int passes = span == 0u ? 0 : (32 - __clz(span) + 8) / 9;
#pragma unroll
  for (int r = 0; r < kTileSortRows; ++r) k[r] -= lo;   // (padding wraps; it is never ranked)
  uint32_t off[kTileSortRows];
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 9 * pass;
    tile_sort_rank<9>(k, n, shift, off, S.lds.wcnt, wave, lane, rpw);
    __syncthreads();
    // digits 2 tid and 2 tid + 1: the exclusive prefix over the waves, the
    // totals, and the exclusive scan of the totals over the 512 digits
    uint32_t a0 = 0, a1 = 0;
#pragma unroll
    for (int w = 0; w < kTileSortWaves; ++w) {
      uint2* c = reinterpret_cast<uint2*>(&S.lds.wcnt[w][2 * tid]);
      const uint2 cw = *c;
      *c = make_uint2(a0, a1);
      a0 += cw.x;
      a1 += cw.y;
    }
    const uint32_t pair = a0 + a1;
    uint32_t x = pair;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
      const uint32_t y = __shfl_up(x, dd, 64);
      if (lane >= dd) x += y;
    }
    if (lane == 63) S.wsum[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += S.wsum[w];
    const uint32_t s0 = base + x - pair;
    *reinterpret_cast<uint2*>(&S.lds.start[2 * tid]) = make_uint2(s0, s0 + a0);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTileSortRows; ++r) {
      if (r >= rpw) break;
      if (off[r] == 0xFFFFFFFFu) continue;
      const uint32_t d = (k[r] >> shift) & 511u;
      const uint32_t pos = S.lds.start[d] + S.lds.wcnt[wave][d] + off[r];
      if (pos < (uint32_t)n) {     // always, when the counts are right; never outside the list
        S.lds.k[pos] = k[r];
        S.lds.v[pos] = v[r];
      }
    }
    __syncthreads();
    if (pass + 1 < passes) {
      // the next pass's entries, and its counters cleared (every wave has
      // read this pass's)
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        if (r >= rpw) break;
        const int e = wave * (64 * rpw) + r * 64 + lane;
        if (e < n) {
          k[r] = S.lds.k[e];
          v[r] = S.lds.v[e];
        }
      }
      for (int w = 0; w < kTileSortWaves; ++w) {
        S.lds.wcnt[w][tid] = 0u;
        S.lds.wcnt[w][tid + 256] = 0u;
      }
      __syncthreads();
    }
  }
  if (passes == 0) {
    // every key equal: the list stays in its order
#pragma unroll
    for (int r = 0; r < kTileSortRows; ++r) {
      if (r >= rpw) break;
      const int e = wave * (64 * rpw) + r * 64 + lane;
      if (e < n) {
        S.lds.k[e] = k[r];
        S.lds.v[e] = v[r];
      }
    }
    __syncthreads();
  }
}

// Rows per wave for a list of n <= kTileSortCap entries in LDS.
__device__ __forceinline__ int lds_rows(int n) { return (n + kTileSortThreads - 1) / kTileSortThreads; }

// A list longer than kTileSortCap, [rg.x, rg.x + n), sorted through global
// memory: per pass, the digit totals of the whole list, then every chunk in
// list order scattered after the earlier chunks' entries of each digit;
// passes alternate between (keys, vals) and (keys_alt, vals_alt) over the
// range, and the list arrives in vals (its keys are scratch). Ends with the
// tile key in keys over the range.
__device__ __forceinline__ void global_depth_sort(TileSortShared& S, uint2 rg, int n, uint32_t tile, bool ties,
                                                  const uint32_t* __restrict__ zkey, uint32_t num_splats,
                                                  uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                  uint32_t* __restrict__ keys_alt, uint32_t* __restrict__ vals_alt) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t k[kTileSortRows], v[kTileSortRows], off[kTileSortRows];
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    const uint32_t* ks = (pass & 1) ? keys_alt : keys;
    const uint32_t* vs = (pass & 1) ? vals_alt : vals;
    uint32_t* kd = (pass & 1) ? keys : keys_alt;
    uint32_t* vd = (pass & 1) ? vals : vals_alt;
    // digit totals of the whole list (the ranking's counts, chunk by chunk)
    uint32_t total = 0;
    for (int c0 = 0; c0 < n; c0 += kTileSortCap) {
      const int cn = min(kTileSortCap, n - c0);
      // loads at in-bounds positions for every lane (the chunk's first
      // entry past its end), masked afterwards
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        const int e = wave * (64 * kTileSortRows) + r * 64 + lane;
        const uint32_t at = rg.x + c0 + (e < cn ? e : 0);
        k[r] = pass == 0 ? vs[at] : ks[at];
      }
      if (pass == 0) {
        // (the list holds splat indices; the clamp keeps the gather in
        // bounds regardless)
#pragma unroll
        for (int r = 0; r < kTileSortRows; ++r) k[r] = zkey[min(k[r], num_splats - 1u)];
      }
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r)
        if (wave * (64 * kTileSortRows) + r * 64 + lane >= cn) k[r] = 0xFFFFFFFFu;
      for (int w = 0; w < kTileSortWaves; ++w) S.wcnt[w][tid] = 0u;
      __syncthreads();
      tile_sort_rank<8>(k, cn, shift, off, S.wcnt, wave, lane, kTileSortRows);
      __syncthreads();
      for (int w = 0; w < kTileSortWaves; ++w) total += S.wcnt[w][tid];
      __syncthreads();
    }
    S.start[tid] = total;
    __syncthreads();
    {
      const uint32_t acc = S.start[tid];
      uint32_t x = acc;
#pragma unroll
      for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t y = __shfl_up(x, dd, 64);
        if (lane >= dd) x += y;
      }
      if (lane == 63) S.wsum[wave] = x;
      __syncthreads();
      uint32_t base = 0;
      for (int w = 0; w < wave; ++w) base += S.wsum[w];
      __syncthreads();
      S.start[tid] = base + x - acc;
    }
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += kTileSortCap) {
      const int cn = min(kTileSortCap, n - c0);
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        const int e = wave * (64 * kTileSortRows) + r * 64 + lane;
        const uint32_t at = rg.x + c0 + (e < cn ? e : 0);
        v[r] = vs[at];
        if (pass != 0) k[r] = ks[at];
      }
      if (pass == 0) {
#pragma unroll
        for (int r = 0; r < kTileSortRows; ++r) k[r] = zkey[min(v[r], num_splats - 1u)];
      }
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        if (wave * (64 * kTileSortRows) + r * 64 + lane >= cn) {
          v[r] = 0u;
          k[r] = 0xFFFFFFFFu;
        }
      }
      for (int w = 0; w < kTileSortWaves; ++w) S.wcnt[w][tid] = 0u;
      __syncthreads();
      tile_sort_rank<8>(k, cn, shift, off, S.wcnt, wave, lane, kTileSortRows);
      __syncthreads();
      uint32_t acc = 0;
      for (int w = 0; w < kTileSortWaves; ++w) {
        const uint32_t c = S.wcnt[w][tid];
        S.wcnt[w][tid] = acc;
        acc += c;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        if (off[r] == 0xFFFFFFFFu) continue;
        const uint32_t d = (k[r] >> shift) & 255u;
        const uint32_t pos = S.start[d] + S.wcnt[wave][d] + off[r];
        if (pos < (uint32_t)n) {   // always, when the counts are right; never outside the tile's range
          kd[rg.x + pos] = k[r];
          vd[rg.x + pos] = v[r];
        }
      }
      __syncthreads();
      S.start[tid] += acc;          // this chunk's entries of each digit precede the next chunk's
      __syncthreads();
    }
  }
  // four passes end in (keys, vals); the keys held depth bits: order
  // equal depths, then restore the tile key
  __syncthreads();
  if (ties) order_equal_depths(keys + rg.x, vals + rg.x, n);
  for (int e = tid; e < n; e += kTileSortThreads) keys[rg.x + e] = tile;
}

// TIES: the lists did not arrive in splat-index order (the counting
// binning): equal depths are put in index order after the passes.
template <bool TIES>
__global__ void __launch_bounds__(kTileSortThreads) tile_depth_sort_kernel(
    const uint2* __restrict__ ranges, int64_t num_tiles, const uint32_t* __restrict__ zkey, uint32_t num_splats,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ keys_alt,
    uint32_t* __restrict__ vals_alt) {
  __shared__ TileSortShared S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t tile = blockIdx.x; tile < num_tiles; tile += gridDim.x) {
    const uint2 rg = ranges[tile];
    const int n = (int)(rg.y - rg.x);
    if (n < 2) continue;
    if (n <= kTileSortCap) {
      // in LDS: load, then the passes the keys' range needs. Lanes past
      // the list read its first entry (a listed splat, so its depth key is
      // in bounds too): every row's id and key loads are in flight at once
      // rather than one guarded round trip after another
      uint32_t k[kTileSortRows], v[kTileSortRows];
      const int rpw = lds_rows(n);
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        const int e = wave * (64 * rpw) + r * 64 + lane;
        v[r] = vals[rg.x + (r < rpw && e < n ? e : 0)];
      }
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) k[r] = zkey[min(v[r], num_splats - 1u)];
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        const int e = wave * (64 * rpw) + r * 64 + lane;
        if (r >= rpw || e >= n) {
          v[r] = 0u;
          k[r] = 0xFFFFFFFFu;
        }
      }
      lds_depth_sort(S, k, v, n, rpw);
      if (TIES) order_equal_depths(S.lds.k, S.lds.v, n);
      for (int e = tid; e < n; e += kTileSortThreads) vals[rg.x + e] = S.lds.v[e];
    } else {
      global_depth_sort(S, rg, n, (uint32_t)tile, TIES, zkey, num_splats, keys, vals, keys_alt, vals_alt);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Binning by blocks of tiles, the per-tile step. The block instances arrive
// grouped by block (a stable pass over the block ids of instances emitted in
// splat-index order), so a block's list is in index order. One workgroup per
// tile reads its block's list, keeps the instances whose block-relative
// rectangle covers the tile (a stream compaction by ballots, which keeps the
// order) and sorts them stably by depth bits as tile_depth_sort_kernel does.
// The tile's list goes to the first position of its block's tiles (from the
// block table) plus the tiles of its block before it in row-major order,
// which every entry of the block's list gives arithmetically from its
// rectangle: no scan over the tiles is needed. Tiles whose list would pass
// the capacity get an empty range and raise the overflow flag.
// ---------------------------------------------------------------------------
constexpr int kBlockRows = 32;   // long lists: rows of 256 entries whose keep masks stay in LDS
constexpr int kBlockLoads = 8;   // rows whose loads are in flight together (4: same time, 16: slower)

// Whether a block instance (key) covers the block-relative tile (lx, ly), and
// how many tiles it covers before that one in the block's row-major order.
__device__ __forceinline__ void block_entry(uint32_t key, uint32_t lx, uint32_t ly, bool valid, bool& keep,
                                            uint32_t& before) {
  const uint32_t rx0 = (key >> 16) & 15u, rx1 = (key >> 20) & 15u, ry0 = (key >> 24) & 15u, ry1 = key >> 28;
  keep = valid && rx0 <= lx && lx < rx1 && ry0 <= ly && ly < ry1;
  const uint32_t ye = min(ry1, ly), xe = min(rx1, lx);
  uint32_t b = (ye > ry0 ? ye - ry0 : 0u) * (rx1 - rx0);
  if (ry0 <= ly && ly < ry1) b += xe > rx0 ? xe - rx0 : 0u;
  before = valid ? b : 0u;
}

// (five workgroups per CU, so that a 640x480 view's 1200 tiles are resident at once)
__global__ void __launch_bounds__(kTileSortThreads) __attribute__((amdgpu_waves_per_eu(5))) block_tile_sort_kernel(
    const ViewDesc* __restrict__ views, int num_views, int64_t num_tiles, BlockGeo geo,
    const uint4* __restrict__ table, const uint32_t* __restrict__ bkeys, const uint32_t* __restrict__ bvals,
    const uint32_t* __restrict__ zkey, uint32_t num_splats, int64_t capacity, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ vals, uint32_t* __restrict__ keys_alt, uint32_t* __restrict__ vals_alt,
    uint2* __restrict__ ranges, uint32_t* __restrict__ overflow) {
  __shared__ TileSortShared S;
  __shared__ unsigned long long s_mask[kBlockRows][kTileSortWaves];
  __shared__ uint32_t s_rowbase[kBlockRows + 1];
  __shared__ uint32_t s_red[2][kTileSortWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int64_t tile = blockIdx.x; tile < num_tiles; tile += gridDim.x) {
    __syncthreads();    // the previous tile's LDS is free
    int view = 0;
    while (view + 1 < num_views && tile >= views[view + 1].tile_offset) ++view;
    const ViewDesc& V = views[view];
    const uint32_t lt = (uint32_t)(tile - V.tile_offset);
    const uint32_t ty = lt / (uint32_t)V.tiles_x, tx = lt - ty * (uint32_t)V.tiles_x;
    const uint32_t bx = tx >> geo.bwl, by = ty >> geo.bhl;
    const uint32_t lx = tx - (bx << geo.bwl), ly = ty - (by << geo.bhl);
    const uint4 T = table[(uint32_t)V.block_offset + by * (uint32_t)V.blocks_x + bx];
    const uint32_t start = T.x;
    const int m = (int)(T.y - T.x);
    // one pass over the block's run: wave w takes rows [w wr, (w + 1) wr) of
    // 64 entries, so the waves' kept entries, each wave's in run order at its
    // running count in its part of LDS, concatenate in run order. Also the
    // tile's offset within the block (the covered tiles before it).
    const int wr = ((m + 63) / 64 + kTileSortWaves - 1) / kTileSortWaves;
    uint32_t cnt = 0, pre = 0;
    for (int r0 = 0; r0 < wr; r0 += kBlockLoads) {
      uint32_t kk[kBlockLoads], vv[kBlockLoads];
#pragma unroll
      for (int q = 0; q < kBlockLoads; ++q) {
        const int e = (wave * wr + r0 + q) * 64 + lane;
        const uint32_t j = start + (r0 + q < wr && e < m ? (uint32_t)e : 0u);
        kk[q] = bkeys[j];
        vv[q] = bvals[j];
      }
#pragma unroll
      for (int q = 0; q < kBlockLoads; ++q) {
        if (r0 + q >= wr) break;
        bool keep;
        uint32_t before;
        block_entry(kk[q], lx, ly, (wave * wr + r0 + q) * 64 + lane < m, keep, before);
        pre += before;
        const uint64_t bal = __ballot(keep);
        const uint32_t pos = cnt + (uint32_t)__popcll(bal & lt_mask);
        // (a part holds kTileSortCap entries: a list that fits the LDS sort
        // never passes it; a longer one is compacted again below)
        if (keep && pos < (uint32_t)kTileSortCap) S.part[wave][pos] = vv[q];
        cnt += (uint32_t)__popcll(bal);
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pre += __shfl_xor(pre, d, 64);
    if (lane == 0) {
      s_red[0][wave] = cnt;
      s_red[1][wave] = pre;
    }
    __syncthreads();
    uint32_t n = 0, P = 0;
#pragma unroll
    for (int w = 0; w < kTileSortWaves; ++w) {
      n += s_red[0][w];
      P += s_red[1][w];
    }
    const uint32_t off = T.z + P;
    if ((int64_t)off + n > capacity) {
      if (tid == 0) {
        atomicOr(overflow, 1u);
        ranges[tile] = make_uint2(0u, 0u);
      }
      continue;
    }
    if (tid == 0) ranges[tile] = make_uint2(off, off + n);
    if (n == 0) continue;
    if (n <= (uint32_t)kTileSortCap) {
      // list position e lies in the part of the wave w with c_w <= e < c_{w+1}
      const uint32_t c1 = s_red[0][0], c2 = c1 + s_red[0][1], c3 = c2 + s_red[0][2];
      uint32_t k[kTileSortRows], v[kTileSortRows];
      const int rpw = lds_rows((int)n);
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        const uint32_t e = (uint32_t)(wave * (64 * rpw) + r * 64 + lane);
        const uint32_t w = (e >= c1 ? 1u : 0u) + (e >= c2 ? 1u : 0u) + (e >= c3 ? 1u : 0u);
        const uint32_t cw = w == 0 ? 0u : (w == 1 ? c1 : (w == 2 ? c2 : c3));
        // (every kept entry is a splat index; the clamp keeps the depth-key
        // gather of the padding lanes in bounds)
        v[r] = min(S.part[w][r < rpw && e < n ? e - cw : 0u], num_splats - 1u);
      }
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) k[r] = zkey[v[r]];
#pragma unroll
      for (int r = 0; r < kTileSortRows; ++r) {
        const int e = wave * (64 * rpw) + r * 64 + lane;
        if (r >= rpw || e >= (int)n) {
          v[r] = 0u;
          k[r] = 0xFFFFFFFFu;
        }
      }
      if (n == 1) {
        if (tid == 0) vals[off] = v[0];
        continue;
      }
      __syncthreads();   // every thread holds its entries before the passes reuse the buffers
      lds_depth_sort(S, k, v, (int)n, rpw);
      for (int e = tid; e < (int)n; e += kTileSortThreads) vals[off + e] = S.lds.v[e];
    } else {
      // a list longer than the LDS sort holds: its kept entries again, in
      // run order (per-row ballots and a prefix over the rows), straight to
      // their places in vals, segment by segment of kBlockRows rows of 256,
      // then sorted through global memory
      const int nrows = (m + kTileSortThreads - 1) / kTileSortThreads;
      uint32_t segbase = 0;
      for (int rb = 0; rb < nrows; rb += kBlockRows) {
        const int rn = min(kBlockRows, nrows - rb);
        __syncthreads();   // the previous segment's masks are consumed
        for (int r0 = 0; r0 < rn; r0 += kBlockLoads) {
          uint32_t kk[kBlockLoads];
#pragma unroll
          for (int q = 0; q < kBlockLoads; ++q) {
            const int e = (rb + r0 + q) * kTileSortThreads + tid;
            kk[q] = bkeys[start + (e < m ? e : 0)];
          }
#pragma unroll
          for (int q = 0; q < kBlockLoads; ++q) {
            if (r0 + q >= rn) break;
            bool keep;
            uint32_t before;
            block_entry(kk[q], lx, ly, (rb + r0 + q) * kTileSortThreads + tid < m, keep, before);
            const uint64_t bal = __ballot(keep);
            if (lane == 0) s_mask[r0 + q][wave] = bal;
          }
        }
        __syncthreads();
        if (wave == 0) {
          uint32_t t = 0;
          if (lane < rn)
#pragma unroll
            for (int w = 0; w < kTileSortWaves; ++w) t += (uint32_t)__popcll(s_mask[lane][w]);
          uint32_t x = t;
#pragma unroll
          for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t y = __shfl_up(x, dd, 64);
            if (lane >= dd) x += y;
          }
          if (lane < rn) s_rowbase[lane] = segbase + x - t;
          if (lane == 63) s_rowbase[kBlockRows] = segbase + x;
        }
        __syncthreads();
        for (int r0 = 0; r0 < rn; r0 += kBlockLoads) {
          uint32_t vv[kBlockLoads];
#pragma unroll
          for (int q = 0; q < kBlockLoads; ++q) {
            const int e = (rb + r0 + q) * kTileSortThreads + tid;
            vv[q] = bvals[start + (e < m ? e : 0)];
          }
#pragma unroll
          for (int q = 0; q < kBlockLoads; ++q) {
            const int r = r0 + q;
            if (r >= rn) break;
            const uint64_t mk = s_mask[r][wave];
            if (!((mk >> lane) & 1ull)) continue;
            uint32_t pos = s_rowbase[r] + (uint32_t)__popcll(mk & lt_mask);
            for (int w = 0; w < wave; ++w) pos += (uint32_t)__popcll(s_mask[r][w]);
            if (pos < n) vals[off + pos] = vv[q];   // always, when the masks are right
          }
        }
        segbase = s_rowbase[kBlockRows];
      }
      __syncthreads();
      global_depth_sort(S, make_uint2(off, off + n), (int)n, (uint32_t)tile, false, zkey, num_splats, keys, vals,
                        keys_alt, vals_alt);
    }
  }
}

__global__ void clear_kernel(ClearList L) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int s = 0; s < L.count; ++s) {
    uint32_t* p = L.p[s];
    const int64_t n = L.n[s];
    // 16-byte stores over the aligned body
    const int64_t head = (int64_t)(((16u - ((uintptr_t)p & 15u)) & 15u) / 4u);
    const int64_t h = head < n ? head : n;
    for (int64_t i = t; i < h; i += stride) p[i] = 0u;
    const int64_t nv = (n - h) / 4;
    uint4* q = reinterpret_cast<uint4*>(p + h);
    for (int64_t i = t; i < nv; i += stride) q[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = h + 4 * nv + t; i < n; i += stride) p[i] = 0u;
  }
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_f32_kernel(float* __restrict__ p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void __launch_bounds__(256) count_work_kernel(const uint32_t* __restrict__ last, int64_t npix,
                                                         const uint32_t* __restrict__ ntiles, int64_t n, int num_views,
                                                         unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s_pairs;
  __shared__ unsigned int s_vis[256];
  if (threadIdx.x == 0) s_pairs = 0;
  s_vis[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x)
    acc += last[i];
  atomicAdd(&s_pairs, acc);
  const int64_t total = n * num_views;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    if (ntiles[i]) atomicAdd(&s_vis[i / n], 1u);
  __syncthreads();
  if (threadIdx.x == 0 && s_pairs) atomicAdd(&out[0], s_pairs);
  if (threadIdx.x < num_views && s_vis[threadIdx.x]) atomicAdd(&out[1 + threadIdx.x], (unsigned long long)s_vis[threadIdx.x]);
}

int grid_cap(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (int)g;
}

}  // namespace

// Keys per thread of a sort pass: small sorts take short chunks, so that the
// pass spreads over more workgroups with less serial ranking work each
// (measured at 200k keys: 2 and 8 slower than 4; at 1.5M and 12M: 12 faster
// than 16 by 1-2 %, 8 slower at 12M).
static int sort_items(int64_t n) { return n <= kSortSmall ? 4 : 12; }

static int64_t sort_chunk(int64_t n) { return (int64_t)kSortThreads * sort_items(n); }

// Reduce-then-scan passes launch three kernels per pass instead of one and
// need no global histogram. Measured on the tile sort: slower at small
// sizes (128x96, 2k Gaussians: 8.6 -> 14.1 us), faster above 2^19 keys
// (1.5M: the same sort and 2 us less emission; 11.8M: 202 -> 189 us;
// 17.5M: 296 -> 260 us).
bool radix_prefers_scan(int64_t n) { return n > kSortSmall; }

int64_t radix_scratch_elems(int64_t n, int bits) {
  int rb, passes;
  radix_plan(bits, &rb, &passes);
  const int64_t nb = blocks_for(n, sort_chunk(n));
  // status words for every pass (or the digit counts and their scan), the
  // copies of the global histograms, the look-back words of the count scans
  const int64_t words = (int64_t)(nb > 0 ? nb : 1) * (1 << rb);
  return (int64_t)(passes > 2 ? passes : 2) * words + (int64_t)kHistCopies * passes * (1 << rb) +
         (int64_t)passes * 2 * blocks_for(words, kScanChunk);
}

int64_t scan_partial_elems(int64_t n) { return 2 * (int64_t)blocks_for(n > 0 ? n : 1, kScanChunk); }

uint32_t* radix_hist(uint32_t* scratch, int64_t n, int bits, int* rb, int* passes) {
  radix_plan(bits, rb, passes);
  const int64_t nb = blocks_for(n, sort_chunk(n));
  return scratch + (int64_t)*passes * (nb > 0 ? nb : 1) * (1 << *rb);
}

void scan_gather_exclusive(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n,
                           const uint32_t* n_dev, uint32_t* total_dev, uint32_t* scratch, uint32_t* err, bool clear,
                           hipStream_t st, uint32_t* block_rank, int64_t capacity) {
  if (n == 0) {
    if (total_dev) fill_u32_kernel<<<1, 64, 0, st>>>(total_dev, 0u, 1);
    return;
  }
  const int nb = blocks_for(n, kScanChunk);
  if (clear) fill_u32_kernel<<<grid_cap(2 * nb, 256), 256, 0, st>>>(scratch, 0u, 2 * nb);
  unsigned long long* status = reinterpret_cast<unsigned long long*>(scratch);
  scan_lookback_kernel<<<nb, kScanThreads, 0, st>>>(in, idx, n_dev, n, out, total_dev, status, err, block_rank,
                                                    (capacity + kEmitBlock - 1) / kEmitBlock);
}

void launch_compact_scan(const uint32_t* ntiles, int64_t n, uint32_t* vals, uint32_t* offsets, uint32_t* count_out,
                         uint32_t* total_out, uint32_t* scratch, uint32_t* err, uint32_t* block_rank, int64_t capacity,
                         hipStream_t st) {
  if (n == 0) {
    fill_u32_kernel<<<1, 64, 0, st>>>(count_out, 0u, 1);
    fill_u32_kernel<<<1, 64, 0, st>>>(total_out, 0u, 1);
    return;
  }
  const int nb = blocks_for(n, kScanChunk);
  unsigned long long* status = reinterpret_cast<unsigned long long*>(scratch);
  compact_scan_kernel<false><<<nb, kScanThreads, 0, st>>>(ntiles, n, vals, offsets, count_out, total_out, status, err,
                                                          block_rank, (capacity + kEmitBlock - 1) / kEmitBlock, nullptr,
                                                          BlockGeo{}, nullptr);
}

void launch_compact_scan_blocks(const uint32_t* ntiles, const int4* rect, const BlockGeo& geo, int64_t n,
                                uint32_t* vals, uint32_t* offsets, uint32_t* count_out, uint32_t* block_total,
                                uint32_t* tile_total, uint32_t* scratch, uint32_t* err, uint32_t* block_rank,
                                int64_t capacity, hipStream_t st) {
  if (n == 0) {
    fill_u32_kernel<<<1, 64, 0, st>>>(count_out, 0u, 1);
    fill_u32_kernel<<<1, 64, 0, st>>>(block_total, 0u, 1);
    return;
  }
  const int nb = blocks_for(n, kScanChunk);
  unsigned long long* status = reinterpret_cast<unsigned long long*>(scratch);
  compact_scan_kernel<true><<<nb, kScanThreads, 0, st>>>(ntiles, n, vals, offsets, count_out, block_total, status, err,
                                                         block_rank, (capacity + kEmitBlock - 1) / kEmitBlock, rect,
                                                         geo, tile_total);
}

void launch_compact_visible(const uint32_t* ntiles, const uint32_t* keys, int64_t n, uint32_t* out_keys,
                            uint32_t* out_vals, uint32_t* count_out, uint32_t* scratch, uint32_t* err, bool clear,
                            hipStream_t st) {
  if (n == 0) {
    fill_u32_kernel<<<1, 64, 0, st>>>(count_out, 0u, 1);
    return;
  }
  const int nb = blocks_for(n, kScanChunk);
  if (clear) fill_u32_kernel<<<grid_cap(2 * nb, 256), 256, 0, st>>>(scratch, 0u, 2 * nb);
  unsigned long long* status = reinterpret_cast<unsigned long long*>(scratch);
  compact_visible_kernel<<<nb, kScanThreads, 0, st>>>(ntiles, keys, n, out_keys, out_vals, count_out, status, err);
}

void radix_sort_pairs(uint32_t*& keys, uint32_t*& vals, uint32_t*& keys_alt, uint32_t*& vals_alt, int64_t n,
                      const uint32_t* n_dev, int bits, uint32_t* scratch, uint32_t* err, bool clear, bool hist_ready,
                      hipStream_t st) {
  if (n <= 1 || bits <= 0) return;
  int rb, passes;
  radix_plan(bits, &rb, &passes);
  const int R = 1 << rb;
  const int items = sort_items(n);
  const int nb = blocks_for(n, sort_chunk(n));
  uint32_t* status = scratch;
  uint32_t* ghist = scratch + (int64_t)passes * nb * R;
  const int gstride = passes * R;
  const int64_t clear_n = radix_scratch_elems(n, bits);
  if (clear) fill_u32_kernel<<<grid_cap(clear_n, 256), 256, 0, st>>>(scratch, 0u, clear_n);
  if (!hist_ready)
    global_hist_kernel<<<blocks_for(n, kSortChunk), kSortThreads, 0, st>>>(keys, n_dev, n, rb, passes, ghist);
  for (int p = 0; p < passes; ++p) {
    uint32_t* stp = status + (int64_t)p * nb * R;
    const int sh = rb * p;
    if (items == 4)
      onesweep_pass_kernel<8, 4><<<nb, kSortThreads, 0, st>>>(keys, vals, n_dev, n, sh, rb, ghist + p * R, gstride, stp,
                                                              err, keys_alt, vals_alt);
    else
      onesweep_pass_kernel<8, 12><<<nb, kSortThreads, 0, st>>>(keys, vals, n_dev, n, sh, rb, ghist + p * R, gstride, stp,
                                                               err, keys_alt, vals_alt);
    uint32_t* t = keys; keys = keys_alt; keys_alt = t;
    t = vals; vals = vals_alt; vals_alt = t;
  }
}

void radix_sort_pairs_scanned(uint32_t*& keys, uint32_t*& vals, uint32_t*& keys_alt, uint32_t*& vals_alt,
                              int64_t n, const uint32_t* n_dev, int bits, uint32_t* scratch, uint32_t* err,
                              hipStream_t st) {
  if (n <= 1 || bits <= 0) return;
  int rb, passes;
  radix_plan(bits, &rb, &passes);
  const int R = 1 << rb;
  const int items = sort_items(n);
  const int nb = blocks_for(n, sort_chunk(n));
  const int64_t words = (int64_t)nb * R;
  // counts and their scan reused by every pass; the scans' look-back words
  // (cleared with the rest of the scratch) one set per pass
  uint32_t* counts = scratch;
  uint32_t* starts = scratch + words;
  uint32_t* scan_status = scratch + (int64_t)(passes > 2 ? passes : 2) * words + (int64_t)kHistCopies * passes * R;
  for (int p = 0; p < passes; ++p) {
    const int sh = rb * p;
    // digits that can occur: keys lie below 2^bits
    const int db = bits - sh < rb ? bits - sh : rb;
    const int64_t live_words = (int64_t)nb << db;
    if (items == 4)
      digit_count_kernel<4><<<nb, kSortThreads, 0, st>>>(keys, n_dev, n, sh, db, counts);
    else
      digit_count_kernel<12><<<nb, kSortThreads, 0, st>>>(keys, n_dev, n, sh, db, counts);
    scan_gather_exclusive(counts, nullptr, starts, live_words, nullptr, nullptr,
                          scan_status + (int64_t)p * 2 * blocks_for(words, kScanChunk), err, false, st);
    if (items == 4)
      onesweep_pass_kernel<8, 4, true><<<nb, kSortThreads, 0, st>>>(keys, vals, n_dev, n, sh, db, nullptr, 0, starts,
                                                                    err, keys_alt, vals_alt);
    else
      onesweep_pass_kernel<8, 12, true><<<nb, kSortThreads, 0, st>>>(keys, vals, n_dev, n, sh, db, nullptr, 0, starts,
                                                                     err, keys_alt, vals_alt);
    uint32_t* t = keys; keys = keys_alt; keys_alt = t;
    t = vals; vals = vals_alt; vals_alt = t;
  }
}

int64_t emit_plan_elems(int64_t capacity) { return (capacity + kEmitBlock - 1) / kEmitBlock + 1; }

void launch_emit(const uint32_t* sorted_s, const uint32_t* offsets, const uint32_t* total_dev,
                 const uint32_t* count_dev, const Splat* splats, int64_t count, uint32_t* keys,
                 uint32_t* vals, int64_t capacity, uint32_t* overflow, uint32_t* hist, int hist_bits,
                 uint32_t* block_rank, bool plan_ready, hipStream_t st) {
  if (count == 0) return;
  int rb = 8, hp = 0;
  if (hist_bits > 0) radix_plan(hist_bits, &rb, &hp);
  const bool fits = hp >= 1 && hp * (1 << rb) <= kEmitHist;
  const int64_t nblocks = (capacity + kEmitBlock - 1) / kEmitBlock;
  if (nblocks == 0) {
    // no instance slot: only the overflow flag can be raised
    emit_kernel<false><<<1, kEmitThreads, 0, st>>>(sorted_s, offsets, total_dev, count_dev, block_rank, splats, count,
                                                   keys, vals, capacity, overflow, nullptr, rb, hp, nullptr, nullptr,
                                                   1u, BlockGeo{}, nullptr);
    return;
  }
  if (!plan_ready)
    emit_plan_kernel<<<grid_cap(count, 256), 256, 0, st>>>(offsets, total_dev, count_dev, count, nblocks, block_rank);
  emit_kernel<false><<<(unsigned)nblocks, kEmitThreads, 0, st>>>(sorted_s, offsets, total_dev, count_dev, block_rank,
                                                                 splats, count, keys, vals, capacity, overflow,
                                                                 fits ? hist : nullptr, rb, hp, nullptr, nullptr, 1u,
                                                                 BlockGeo{}, nullptr);
}

void launch_emit_blocks(const uint32_t* visible, const uint32_t* offsets, const uint32_t* total_dev,
                        const uint32_t* count_dev, const int4* rect, const ViewDesc* views, int64_t num,
                        const BlockGeo& geo, int64_t count, uint32_t* keys, uint32_t* vals, int64_t capacity,
                        uint32_t* overflow, uint32_t* hist, uint32_t* whist, uint32_t* block_rank, bool plan_ready,
                        hipStream_t st) {
  if (count == 0) return;
  const int64_t nblocks = (capacity + kEmitBlock - 1) / kEmitBlock;
  const uint32_t n32 = (uint32_t)(num > 0 ? num : 1);
  if (nblocks == 0) {
    emit_kernel<true><<<1, kEmitThreads, 0, st>>>(visible, offsets, total_dev, count_dev, block_rank, nullptr, count,
                                                  keys, vals, capacity, overflow, nullptr, 8, 1, rect, views, n32, geo,
                                                  nullptr);
    return;
  }
  if (!plan_ready)
    emit_plan_kernel<<<grid_cap(count, 256), 256, 0, st>>>(offsets, total_dev, count_dev, count, nblocks, block_rank);
  emit_kernel<true><<<(unsigned)nblocks, kEmitThreads, 0, st>>>(visible, offsets, total_dev, count_dev, block_rank,
                                                                nullptr, count, keys, vals, capacity, overflow, hist, 8,
                                                                1, rect, views, n32, geo, whist);
}

bool emit_histogram_fits(int bits) {
  int rb, hp;
  radix_plan(bits, &rb, &hp);
  return bits > 0 && hp * (1 << rb) <= kEmitHist;
}

int bin_chunk(int64_t n) {
  // a workgroup per 1024 splats of a view fills the chip at one view; fewer
  // and longer ones (a smaller count matrix) for large maps
  const int64_t rounds = n / ((int64_t)kBinThreads * 192);
  return kBinThreads * (int)(rounds < 1 ? 1 : (rounds > 8 ? 8 : rounds));
}

bool bin_view_fits(int64_t tiles) { return tiles <= kBinMaxTiles; }

static BinArgs bin_args(const uint32_t* ntiles, const int4* rect, const ViewDesc* views, int64_t n, int tile_w,
                        int tile_h) {
  BinArgs a;
  a.ntiles = ntiles;
  a.rect = rect;
  a.views = views;
  a.n = n;
  a.chunk = bin_chunk(n);
  a.nb = (int)((n + a.chunk - 1) / a.chunk);
  a.tw_log2 = __builtin_ctz((unsigned)tile_w);
  a.th_log2 = __builtin_ctz((unsigned)tile_h);
  return a;
}

void launch_bin_count(const uint32_t* ntiles, const int4* rect, const ViewDesc* views, int num_views, int64_t n,
                      int max_view_tiles, int tile_w, int tile_h, uint32_t* counts, uint32_t* visible,
                      hipStream_t st) {
  if (n == 0 || num_views == 0) return;
  const BinArgs a = bin_args(ntiles, rect, views, n, tile_w, tile_h);
  bin_count_kernel<<<(unsigned)(num_views * a.nb), kBinThreads, sizeof(uint32_t) * (size_t)max_view_tiles, st>>>(
      a, counts, visible);
}

void launch_bin_scatter(const uint32_t* ntiles, const int4* rect, const ViewDesc* views, int num_views, int64_t n,
                        int max_view_tiles, int tile_w, int tile_h, const uint32_t* starts,
                        const uint32_t* total_dev, int64_t capacity, int64_t num_tiles, uint32_t* keys,
                        uint32_t* vals, uint2* ranges, uint32_t* overflow, hipStream_t st) {
  if (n == 0 || num_views == 0) {
    // no splat: every tile is empty
    if (num_tiles > 0)
      fill_u32_kernel<<<grid_cap(2 * num_tiles, 256), 256, 0, st>>>(reinterpret_cast<uint32_t*>(ranges), 0u,
                                                                    2 * num_tiles);
    return;
  }
  const BinArgs a = bin_args(ntiles, rect, views, n, tile_w, tile_h);
  bin_scatter_kernel<<<(unsigned)(num_views * a.nb), kBinThreads, sizeof(uint32_t) * (size_t)max_view_tiles, st>>>(
      a, starts, total_dev, capacity, num_tiles, keys, vals, ranges, overflow);
}

void launch_tile_ranges(const uint32_t* keys, const uint32_t* n_dev, int64_t count, uint2* ranges, int64_t num_tiles,
                        bool clear, hipStream_t st) {
  if (clear)
    fill_u32_kernel<<<grid_cap(2 * num_tiles, 256), 256, 0, st>>>(reinterpret_cast<uint32_t*>(ranges), 0u,
                                                                  2 * num_tiles);
  if (count == 0) return;
  tile_ranges_kernel<<<grid_cap(count, 256), 256, 0, st>>>(keys, n_dev, count, ranges, num_tiles);
}


void launch_tile_depth_sort(const uint2* ranges, int64_t num_tiles, const uint32_t* zkey, int64_t num_splats,
                            uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, bool index_order,
                            hipStream_t st) {
  if (num_tiles == 0 || num_splats == 0) return;
  const unsigned grid = (unsigned)(num_tiles < 65536 ? num_tiles : 65536);
  const uint32_t ns = (uint32_t)num_splats;
  if (index_order)
    tile_depth_sort_kernel<false><<<grid, kTileSortThreads, 0, st>>>(ranges, num_tiles, zkey, ns, keys, vals, keys_alt,
                                                                      vals_alt);
  else
    tile_depth_sort_kernel<true><<<grid, kTileSortThreads, 0, st>>>(ranges, num_tiles, zkey, ns, keys, vals, keys_alt,
                                                                     vals_alt);
}

// Binning by blocks: keys per thread of the one pass over the block ids
// (measured at 640x480/200k, about 550k block instances: 20.2 us with 4,
// 18.0 us with 12).
constexpr int kBlockSortItems = 12;
constexpr int kBlockSortChunk = kSortThreads * kBlockSortItems;

int64_t block_sort_scratch_elems(int64_t n) {
  const int64_t nb = blocks_for(n > 0 ? n : 1, kBlockSortChunk);
  return nb * kMaxBlocks + (int64_t)kHistCopies * kMaxBlocks;
}

uint32_t* block_sort_hist(uint32_t* scratch, int64_t n) {
  return scratch + (int64_t)blocks_for(n > 0 ? n : 1, kBlockSortChunk) * kMaxBlocks;
}

void launch_block_sort(const uint32_t* keys, const uint32_t* vals, const uint32_t* n_dev, int64_t n, int nblocks,
                       uint32_t* scratch, const uint32_t* whist, uint4* table, uint32_t* err, uint32_t* keys_out,
                       uint32_t* vals_out, hipStream_t st) {
  const int nb = blocks_for(n > 0 ? n : 1, kBlockSortChunk);
  const int dbits = bits_for_blocks(nblocks);
  onesweep_pass_kernel<8, kBlockSortItems, false, true><<<nb, kSortThreads, 0, st>>>(
      keys, vals, n_dev, n, 0, dbits, block_sort_hist(scratch, n), kMaxBlocks, scratch, err, keys_out, vals_out, whist,
      table);
}

void launch_block_tile_sort(const ViewDesc* views, int num_views, int64_t num_tiles, const BlockGeo& geo,
                            const uint4* table, const uint32_t* bkeys, const uint32_t* bvals, const uint32_t* zkey,
                            int64_t num_splats, int64_t capacity, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                            uint32_t* vals_alt, uint2* ranges, uint32_t* overflow, hipStream_t st) {
  if (num_tiles == 0 || num_splats == 0) return;
  const unsigned grid = (unsigned)(num_tiles < 65536 ? num_tiles : 65536);
  block_tile_sort_kernel<<<grid, kTileSortThreads, 0, st>>>(views, num_views, num_tiles, geo, table, bkeys, bvals,
                                                           zkey, (uint32_t)num_splats, capacity, keys, vals, keys_alt,
                                                           vals_alt, ranges, overflow);
}

void launch_tile_order(const uint2* ranges, int64_t num_tiles, uint32_t* order, hipStream_t st) {
  if (num_tiles == 0) return;
  tile_order_kernel<<<1, kOrderThreads, 0, st>>>(ranges, num_tiles, order);
}

bool tile_balance_supported(int64_t num_tiles) { return num_tiles > 0 && num_tiles <= kBalanceMax; }

void launch_tile_balance(const uint2* ranges, const uint32_t* tile_last, int64_t num_tiles, int ncu, uint32_t* order,
                         hipStream_t st) {
  if (num_tiles == 0) return;
  tile_balance_kernel<<<1, kOrderThreads, 0, st>>>(ranges, tile_last, (int)num_tiles, ncu > 0 ? ncu : 256, order);
}

void launch_clear(const ClearList& L, hipStream_t st) {
  int64_t most = 0;
  for (int k = 0; k < L.count; ++k) most = L.n[k] > most ? L.n[k] : most;
  if (L.count == 0) return;
  clear_kernel<<<grid_cap(most / 4 + 1, 256), 256, 0, st>>>(L);
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n == 0) return;
  fill_u32_kernel<<<grid_cap(n, 256), 256, 0, st>>>(p, v, n);
}

void launch_count_work(const uint32_t* last, int64_t npix, const uint32_t* ntiles, int64_t n, int num_views,
                       unsigned long long* out, hipStream_t st) {
  fill_u32_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(out), 0u, 2 * (1 + num_views));
  const int64_t m = npix > n * num_views ? npix : n * num_views;
  count_work_kernel<<<grid_cap(m, 256) < 2048 ? grid_cap(m, 256) : 2048, 256, 0, st>>>(last, npix, ntiles, n, num_views,
                                                                                         out);
}

void launch_fill_f32(float* p, float v, int64_t n, hipStream_t st) {
  if (n == 0) return;
  fill_f32_kernel<<<grid_cap(n, 256), 256, 0, st>>>(p, v, n);
}

}  // namespace gsr
