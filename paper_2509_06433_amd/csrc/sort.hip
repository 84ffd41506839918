// Tile binning and the depth-keyed radix sort.
//
// Order of the instance list: (view, tile, raw float bits of depth, Gaussian
// index). It is built in two stable steps:
//   1. an LSD radix sort of the (view, Gaussian) splats by depth bits; the
//      splats start in (view, index) order, so ties keep index order;
//   2. instances are emitted in that depth order, then a stable LSD radix
//      sort on the global tile id groups them by tile while keeping the depth
//      order inside every tile.
// The radix sort is reduce-then-scan with 8-bit digits: a per-block digit
// histogram, a device-wide exclusive scan of the digit-major histogram
// table, and a stable scatter that ranks keys inside wave64s with ballots.

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;      // 2048

constexpr int kSortThreads = 256;                          // 4 wave64
constexpr int kSortItems = 16;
constexpr int kSortChunk = kSortThreads * kSortItems;      // 4096
constexpr int kWaveChunk = 64 * kSortItems;                // 1024 keys per wave
constexpr int kRadix = 256;

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

__device__ __forceinline__ uint32_t load_gather(const uint32_t* in, const uint32_t* idx, int64_t j) {
  return idx ? in[idx[j]] : in[j];
}

__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                   const uint32_t* __restrict__ idx, int64_t n,
                                                                   uint32_t* __restrict__ partials) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = base + k * kScanThreads + threadIdx.x;
    if (j < n) s += load_gather(in, idx, j);
  }
  uint32_t total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Single block: exclusive scan of the partials in place; grand total -> *total.
__global__ void __launch_bounds__(kScanThreads) scan_partials_kernel(uint32_t* __restrict__ partials, int nparts,
                                                                     uint32_t* __restrict__ total_out) {
  uint32_t carry = 0;
  for (int base = 0; base < nparts; base += kScanThreads) {
    const int j = base + threadIdx.x;
    const uint32_t x = j < nparts ? partials[j] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(x, &tot);
    if (j < nparts) partials[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const uint32_t* __restrict__ in,
                                                                 const uint32_t* __restrict__ idx, int64_t n,
                                                                 const uint32_t* __restrict__ partials,
                                                                 uint32_t* __restrict__ out) {
  // blocked arrangement: thread t owns items t*kScanItems .. +kScanItems-1 of the chunk
  __shared__ uint32_t tile[kScanChunk];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    const int64_t j = base + local;
    tile[local] = j < n ? load_gather(in, idx, j) : 0u;
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
  uint32_t run = block_excl_scan(s, &tot) + partials[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    tile[threadIdx.x * kScanItems + k] = run;
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

// Per-block histogram of the digit (key >> shift) & 255, stored digit-major:
// hist[digit * nblocks + block].
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                  int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
#pragma unroll 4
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t j = base + k * kSortThreads + threadIdx.x;
    if (j < n) atomicAdd(&h[(keys[j] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter. Wave w of a block owns keys [base + w*1024, base + (w+1)*1024)
// and walks them in 16 rounds of 64 consecutive keys. Within a round, lanes with
// equal digits are found with 8 ballots; a wave-private LDS counter per digit
// carries ranks across rounds, so no block barrier is needed until the end.
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t n, int shift,
    const uint32_t* __restrict__ hist_scanned, uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
  __shared__ uint32_t gofs[kRadix];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][threadIdx.x] = 0;
  gofs[threadIdx.x] = hist_scanned[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)wave * kWaveChunk;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t k_reg[kSortItems], v_reg[kSortItems], off[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t j = base + r * 64 + lane;
    const bool valid = j < n;
    const uint32_t key = valid ? keys[j] : 0u;
    k_reg[r] = key;
    v_reg[r] = valid ? vals[j] : 0u;
    const uint32_t d = (key >> shift) & (kRadix - 1);
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      mask &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(mask & lt_mask);
    const uint32_t before = wcnt[wave][d];
    off[r] = before + rank;
    if (valid && rank == 0) wcnt[wave][d] = before + (uint32_t)__popcll(mask);
    // keep this wave's LDS read of the next round after this write
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t j = base + r * 64 + lane;
    if (j < n) {
      const uint32_t d = (k_reg[r] >> shift) & (kRadix - 1);
      const uint32_t pos = gofs[d] + wcnt[wave][d] + off[r];
      if (pos < n) {
        keys_out[pos] = k_reg[r];
        vals_out[pos] = v_reg[r];
      }
    }
  }
}

__global__ void emit_kernel(const uint32_t* __restrict__ sorted_s, const uint32_t* __restrict__ offsets,
                            const int4* __restrict__ rect, int64_t count, int64_t n,
                            const ViewDesc* __restrict__ views, int tile_w, int tile_h, uint32_t* __restrict__ keys,
                            uint32_t* __restrict__ vals, int64_t capacity) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < count; r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = sorted_s[r];
    const int4 pr = rect[s];
    if (pr.z < pr.x) continue;
    const int view = (int)(s / n);
    const ViewDesc& V = views[view];
    const int tx0 = pr.x / tile_w, tx1 = pr.z / tile_w, ty0 = pr.y / tile_h, ty1 = pr.w / tile_h;
    int64_t o = offsets[r];
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        if (o < capacity) {
          keys[o] = (uint32_t)(V.tile_offset + ty * V.tiles_x + tx);
          vals[o] = s;
        }
        ++o;
      }
  }
}

__global__ void tile_ranges_kernel(const uint32_t* __restrict__ keys, int64_t count, uint2* __restrict__ ranges,
                                   int64_t num_tiles) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (k >= num_tiles) continue;
    if (i == 0 || keys[i - 1] != k) ranges[k].x = (uint32_t)i;
    if (i == count - 1 || keys[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
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

__global__ void count_work_kernel(const uint32_t* __restrict__ last, int64_t npix, const uint32_t* __restrict__ ntiles,
                                  int64_t n, int num_views, unsigned long long* __restrict__ out) {
  unsigned long long s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x)
    s += last[i];
  if (s) atomicAdd(&out[0], s);
  const int64_t total = n * num_views;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    if (ntiles[i]) atomicAdd(&out[1 + i / n], 1ull);
}

int grid_cap(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (int)g;
}

}  // namespace

void radix_scratch_sizes(int64_t n, int64_t* hist_elems, int64_t* partial_elems) {
  const int64_t nb = blocks_for(n, kSortChunk);
  *hist_elems = (int64_t)kRadix * (nb > 0 ? nb : 1);
  const int64_t scan_n = *hist_elems > n ? *hist_elems : n;
  *partial_elems = blocks_for(scan_n, kScanChunk) + 1;
}

void scan_gather_exclusive(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n, uint32_t* total_dev,
                           uint32_t* partials, hipStream_t st) {
  if (n == 0) {
    if (total_dev) fill_u32_kernel<<<1, 64, 0, st>>>(total_dev, 0u, 1);
    return;
  }
  const int nb = blocks_for(n, kScanChunk);
  scan_reduce_kernel<<<nb, kScanThreads, 0, st>>>(in, idx, n, partials);
  scan_partials_kernel<<<1, kScanThreads, 0, st>>>(partials, nb, total_dev);
  scan_down_kernel<<<nb, kScanThreads, 0, st>>>(in, idx, n, partials, out);
}

void radix_sort_pairs(uint32_t*& keys, uint32_t*& vals, uint32_t*& keys_alt, uint32_t*& vals_alt, int64_t n,
                      int bits, uint32_t* hist, uint32_t* partials, hipStream_t st) {
  if (n <= 1) return;
  const int nb = blocks_for(n, kSortChunk);
  const int64_t hn = (int64_t)kRadix * nb;
  for (int shift = 0; shift < bits; shift += 8) {
    radix_hist_kernel<<<nb, kSortThreads, 0, st>>>(keys, n, shift, hist);
    scan_gather_exclusive(hist, nullptr, hist, hn, nullptr, partials, st);
    radix_scatter_kernel<<<nb, kSortThreads, 0, st>>>(keys, vals, n, shift, hist, keys_alt, vals_alt);
    uint32_t* t = keys; keys = keys_alt; keys_alt = t;
    t = vals; vals = vals_alt; vals_alt = t;
  }
}

void launch_emit(const uint32_t* sorted_s, const uint32_t* offsets, const int4* rect, int64_t count, int64_t n,
                 const ViewDesc* views, int tile_w, int tile_h, uint32_t* keys, uint32_t* vals, int64_t capacity,
                 hipStream_t st) {
  if (count == 0) return;
  emit_kernel<<<grid_cap(count, 256), 256, 0, st>>>(sorted_s, offsets, rect, count, n, views, tile_w, tile_h, keys,
                                                    vals, capacity);
}

void launch_tile_ranges(const uint32_t* keys, int64_t count, uint2* ranges, int64_t num_tiles, hipStream_t st) {
  fill_u32_kernel<<<grid_cap(2 * num_tiles, 256), 256, 0, st>>>(reinterpret_cast<uint32_t*>(ranges), 0u,
                                                                2 * num_tiles);
  if (count == 0) return;
  tile_ranges_kernel<<<grid_cap(count, 256), 256, 0, st>>>(keys, count, ranges, num_tiles);
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
