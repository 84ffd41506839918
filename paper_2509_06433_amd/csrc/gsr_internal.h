// Internal declarations shared by the HIP translation units of libgsr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

// Per-view constants the kernels read from device memory.
struct ViewDesc {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float campos[3];        // camera centre in world coordinates, -R^T t
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_offset;    // first global tile id of this view
  int32_t pix_offset;     // first pixel of this view in per-pixel scratch
  int32_t block_offset;   // binning by blocks of tiles: first global block id of this view
  int32_t blocks_x;       // and its blocks per row
};

// Binning by blocks of tiles: a block is 2^bwl x 2^bhl tiles of one view
// (at most 8 x 8), numbered view by view, row-major within a view; a tile is
// 2^twl x 2^thl pixels. At most kMaxBlocks blocks over all views, so that
// one 8-bit radix pass groups the block instances.
constexpr int kMaxBlocks = 256;
struct BlockGeo {
  int32_t bwl, bhl;
  int32_t twl, thl;
  int32_t nblocks;
};

// Per-view image pointers (forward outputs, backward inputs, loss targets).
struct ViewImages {
  float* rgb;
  float* depth;
  float* alpha;
};

// Projected splat of one (view, Gaussian): three 16-byte words.
//   w0 = (u, v, z, opacity)  w1 = (A, B, C, tile0) conic  w2 = (r, g, b, tgeo)
// tile0, tgeo (integer bits, for the emission only): the first global tile id
// of the splat's tile rectangle; its width | the view's tile pitch << 16.
struct Splat {
  float4 w0, w1, w2;
};

// Screen-space gradient of one (view, Gaussian), accumulated by atomics.
enum { G2_U = 0, G2_V, G2_A, G2_B, G2_C, G2_O, G2_R, G2_G, G2_BL, G2_Z, G2_N };

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTransMin = 1e-4f;

// ---- project.hip ---------------------------------------------------------
// One thread per (view, Gaussian). Writes ntiles[s] (0 when culled) and, for
// the splats it lists (ntiles[s] > 0) only, splats[s], rect[s] (pixel
// rectangle, inclusive) and the depth key zkey[s] (raw float bits of z);
// s = view * N + i.
// Projection of every (view, Gaussian) splat into splats, rect, ntiles and
// zkey (indexed view * n + Gaussian); with zhist the digit histograms of the
// visible splats' depth keys are accumulated there; with nonfinite, the number
// of Gaussians with a non-finite mean, log-scale, rotation or opacity logit,
// or a zero rotation quaternion, is added there (once per Gaussian).
void launch_project(const float* params, int64_t n, int64_t stride, int deg, int num_views,
                    const ViewDesc* views, int tile_w, int tile_h, float znear, Splat* splats,
                    int4* rect, uint32_t* ntiles, uint32_t* zkey, uint32_t* zhist, int zrb, int zpasses,
                    uint32_t* nonfinite, hipStream_t st);
// scale[k][n] = exp(log-scale k) and opacity[n] = sigmoid(logit) of the n
// Gaussians, as the projection computes them (either output may be null).
void launch_activations(const float* params, int64_t n, int64_t stride, float* scale, float* opacity,
                        hipStream_t st);
// Chain rule from screen-space gradients g2[V*N][10] to grad_params (+=, or
// with overwrite = every plane written, zero where no view contributed).
// Counters of the replayed mapping iteration (stats words).
enum : int {
  kStatAdamSteps = 0,
  kStatIterations = 1,
  kStatSkipped = 2,
  kStatMaxInstances = 3,
  kStatLastInstances = 4,
  kStatErrors = 5,
  kStatWords = 8
};
struct IterCounters {
  const uint32_t* totals;   // [0] instance count, [1] error word, [2] instance overflow flag
  uint32_t* stats;          // device counters, kStatWords
  uint32_t* host;           // device address of the pinned host copy, or null
  int adam;                 // the iteration ends with an Adam step
};
// One thread, after every kernel that can raise the error or overflow flag:
// counts the replay (as skipped when a flag is set, and then not as an Adam
// step), keeps the instance counts, and copies the counters to the host.
__device__ inline void count_iteration(const IterCounters& c) {
  // the counters are read once, updated in registers and written to the
  // device copy and the host mirror: no load waits behind a store
  uint32_t s[kStatWords];
#pragma unroll
  for (int k = 0; k < kStatWords; ++k) s[k] = c.stats[k];
  const uint32_t count = c.totals[0];
  const bool err = c.totals[1] != 0u, over = c.totals[2] != 0u;
  if (err || over) {
    s[kStatSkipped] += 1u;
    if (err) s[kStatErrors] += 1u;
  } else {
    s[kStatIterations] += 1u;
    if (c.adam) s[kStatAdamSteps] += 1u;
  }
  s[kStatMaxInstances] = max(s[kStatMaxInstances], count);
  s[kStatLastInstances] = count;
#pragma unroll
  for (int k = 0; k < kStatWords; ++k) c.stats[k] = s[k];
  if (c.host) {
#pragma unroll
    for (int k = 0; k < kStatWords; ++k) c.host[k] = s[k];
    __threadfence_system();
  }
}

// Only (view, Gaussian) pairs with a nonzero tile count (ntiles[V*N]) are
// visited: one thread per Gaussian walks its own visible views. zero_g2: the
// rows read are zeroed, so g2 is all zero again afterwards. counters (may be
// null): the first workgroup also counts the iteration (count_iteration).
void launch_project_backward(const float* params, int64_t n, int64_t stride, int deg, int num_views,
                             const ViewDesc* views, float znear, float* g2, const uint32_t* ntiles,
                             float* grad, bool overwrite, bool zero_g2, const IterCounters* counters,
                             hipStream_t st);
// Camera gradient of every view from the screen-space gradients g2:
// gcam[v][12] += dL/dR (row-major), dL/dt; twist[v][6] (may be null) += the
// gradient with respect to a left perturbation (rho, phi) of the pose.
void launch_pose_backward(const float* params, int64_t n, int64_t stride, int deg, int num_views,
                          const ViewDesc* views, const float* g2, const uint32_t* ntiles, double* gcam, double* twist,
                          hipStream_t st);
// Inspection copy of the splats of one view: out[n][16] (see gsr_copy_splats).
void launch_export_splats(const float* params, int64_t n, int64_t stride, const ViewDesc* view, float znear,
                          const Splat* splats, const int4* rect, const uint32_t* ntiles, float* out,
                          hipStream_t st);

// ---- sort.hip --------------------------------------------------------------
// The digit histograms of a sort are accumulated in kHistCopies copies
// (consecutive blocks of passes * 2^rb words): workgroup b of a producer adds
// into copy b % kHistCopies, and each sort pass sums the copies of its digit.
// Hundreds of workgroups adding into the same few hundred words serialise on
// those addresses (measured: 22 us of a 41 us emission at 1470 workgroups).
constexpr int kHistCopies = 16;
// Scratch (u32 words) of radix_sort_pairs for n elements sorted on `bits` bits.
int64_t radix_scratch_elems(int64_t n, int bits);
// Stable LSD radix sort of (keys, vals) on the low `bits` bits of the keys,
// 8 bits per pass, ping-ponging between the buffers; on return keys/vals
// point at the sorted data and keys_alt/vals_alt at the other pair. The element
// count is *n_dev when n_dev is not null (n is then the capacity the grid is
// sized for), else n. *err becomes nonzero if a look-back wait hit its bound
// (the result is then invalid). clear = false: the caller has zeroed the
// scratch; hist_ready = true: the caller has accumulated the digit
// histograms at radix_hist(scratch, n) (as the projection and the emission
// kernels do), so the histogram kernel is skipped.
void radix_sort_pairs(uint32_t*& keys, uint32_t*& vals, uint32_t*& keys_alt, uint32_t*& vals_alt, int64_t n,
                      const uint32_t* n_dev, int bits, uint32_t* scratch, uint32_t* err, bool clear, bool hist_ready,
                      hipStream_t st);
// The same sort with reduce-then-scan passes: per pass, digit counts per
// workgroup, one exclusive scan over them, then the ranking and scatter. No
// global histogram and no serial look-back between the workgroups.
void radix_sort_pairs_scanned(uint32_t*& keys, uint32_t*& vals, uint32_t*& keys_alt, uint32_t*& vals_alt,
                              int64_t n, const uint32_t* n_dev, int bits, uint32_t* scratch, uint32_t* err,
                              hipStream_t st);
// Whether a sort of n keys is faster with reduce-then-scan passes.
bool radix_prefers_scan(int64_t n);
// The digit histograms ([passes][2^rb]) inside a sort scratch for n elements
// sorted on `bits` bits; *rb and *passes receive the digit width and count.
uint32_t* radix_hist(uint32_t* scratch, int64_t n, int bits, int* rb, int* passes);
// Whether the emission kernel can accumulate the histograms of a sort on
// `bits` bits (passes * 2^rb <= 2048).
bool emit_histogram_fits(int bits);
// Scan scratch (u32 words) needed by scan_gather_exclusive for n elements.
int64_t scan_partial_elems(int64_t n);
// Exclusive scan out[r] = sum_{j<r} in[idx[r]] (idx may be null) over
// min(*n_dev, n) elements (n if n_dev is null); total -> *total_dev. Single
// pass with decoupled look-back; clear = false: the caller has zeroed the
// scratch (scan_partial_elems(n) words). *err is raised if a bounded wait
// expired. With block_rank (the emission's plan for `capacity` instance
// slots, emit_plan_elems(capacity) words) the scan also records, for every
// block of emission output positions below the capacity, the element whose
// run holds the block's first position, so that launch_emit needs no plan
// kernel (plan_ready).
void scan_gather_exclusive(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n,
                           const uint32_t* n_dev, uint32_t* total_dev, uint32_t* scratch, uint32_t* err, bool clear,
                           hipStream_t st, uint32_t* block_rank = nullptr, int64_t capacity = 0);
// Order-preserving compaction of the visible splats (nonzero tile count) and
// their instance offsets in one pass over the n splats in index order:
// vals[r] = index of the r-th visible splat, offsets[r] = the tile counts of
// the visible splats before it, *count_out = their number, *total_out = the
// instance total; with block_rank the emission plan for `capacity` slots, as
// scan_gather_exclusive writes it. Needs n < 2^30. The scratch (zeroed by
// the caller) is that of scan_gather_exclusive.
void launch_compact_scan(const uint32_t* ntiles, int64_t n, uint32_t* vals, uint32_t* offsets, uint32_t* count_out,
                         uint32_t* total_out, uint32_t* scratch, uint32_t* err, uint32_t* block_rank, int64_t capacity,
                         hipStream_t st);
// Binning by blocks of tiles (geo): the same compaction, with each visible
// splat counted by the blocks its tile rectangle overlaps (from rect):
// offsets[r] = the block instances before the r-th visible splat, their
// total -> *block_total; the visible splats' tile counts are added to
// *tile_total (the instance count of the tile lists).
void launch_compact_scan_blocks(const uint32_t* ntiles, const int4* rect, const BlockGeo& geo, int64_t n,
                                uint32_t* vals, uint32_t* offsets, uint32_t* count_out, uint32_t* block_total,
                                uint32_t* tile_total, uint32_t* scratch, uint32_t* err, uint32_t* block_rank,
                                int64_t capacity, hipStream_t st);
// Order-preserving compaction of the n splats with a nonzero tile count:
// out_keys/out_vals[r] = key and index of the r-th one, *count_out = their
// number. Same scratch size and semantics as scan_gather_exclusive.
void launch_compact_visible(const uint32_t* ntiles, const uint32_t* keys, int64_t n, uint32_t* out_keys,
                            uint32_t* out_vals, uint32_t* count_out, uint32_t* scratch, uint32_t* err, bool clear,
                            hipStream_t st);
// Binning by counting (the per-tile depth order only): splats per workgroup
// for n Gaussians per view, whether a view of `tiles` tiles fits the
// workgroup's bins, and the two passes. bin_count: per workgroup and tile of
// its view, the instance count, into counts[tile * nb + b] (nb = ceil(n /
// chunk) workgroups per view; num_tiles * nb words); *visible += the listed
// splats. After an exclusive scan of counts (in place), bin_scatter: the
// instances of each tile in positions [start, end) (those below capacity),
// the tile key and splat index of each, ranges[tile] = [start, end) clipped
// to capacity, and *overflow set when *total_dev exceeds capacity.
int bin_chunk(int64_t n);
bool bin_view_fits(int64_t tiles);
void launch_bin_count(const uint32_t* ntiles, const int4* rect, const ViewDesc* views, int num_views, int64_t n,
                      int max_view_tiles, int tile_w, int tile_h, uint32_t* counts, uint32_t* visible,
                      hipStream_t st);
void launch_bin_scatter(const uint32_t* ntiles, const int4* rect, const ViewDesc* views, int num_views, int64_t n,
                        int max_view_tiles, int tile_w, int tile_h, const uint32_t* starts,
                        const uint32_t* total_dev, int64_t capacity, int64_t num_tiles, uint32_t* keys,
                        uint32_t* vals, uint2* ranges, uint32_t* overflow, hipStream_t st);
// Instance emission in depth order; writes beyond `capacity` are dropped and
// set *overflow when the total exceeds it. With hist (and
// emit_histogram_fits(hist_bits)) the digit histograms of the written tile
// keys, for a sort on hist_bits bits, are accumulated there.
// The depth-sorted splats are sorted_s[0 .. min(*count_dev, count)).
// block_rank: scratch of emit_plan_elems(capacity) words.
int64_t emit_plan_elems(int64_t capacity);
void launch_emit(const uint32_t* sorted_s, const uint32_t* offsets, const uint32_t* total_dev,
                 const uint32_t* count_dev, const Splat* splats, int64_t count, uint32_t* keys,
                 uint32_t* vals, int64_t capacity, uint32_t* overflow, uint32_t* hist, int hist_bits,
                 uint32_t* block_rank, bool plan_ready, hipStream_t st);
// Binning by blocks: one instance per (visible splat, block it overlaps), in
// splat order at the offsets above (at most `capacity`, else *overflow):
// key = global block id | block-relative tile rectangle << 16 (x0, x1, y0,
// y1; 4 bits each, one-past-last ends), value = splat index (view * num +
// Gaussian). hist (kHistCopies x kMaxBlocks, at block_sort_hist) receives the
// block ids' histogram and whist (the same shape) the tiles they cover.
void launch_emit_blocks(const uint32_t* visible, const uint32_t* offsets, const uint32_t* total_dev,
                        const uint32_t* count_dev, const int4* rect, const ViewDesc* views, int64_t num,
                        const BlockGeo& geo, int64_t count, uint32_t* keys, uint32_t* vals, int64_t capacity,
                        uint32_t* overflow, uint32_t* hist, uint32_t* whist, uint32_t* block_rank, bool plan_ready,
                        hipStream_t st);
// The stable pass over the block ids of min(*n_dev, n) block instances, into
// keys_out/vals_out, which also writes table[b] = (first, one past last
// position of block b's run, first position of its tiles' lists, their
// instance count) for every block. scratch: block_sort_scratch_elems(n)
// words, zeroed, its histogram (block_sort_hist) filled by the emission.
int64_t block_sort_scratch_elems(int64_t n);
uint32_t* block_sort_hist(uint32_t* scratch, int64_t n);
void launch_block_sort(const uint32_t* keys, const uint32_t* vals, const uint32_t* n_dev, int64_t n, int nblocks,
                       uint32_t* scratch, const uint32_t* whist, uint4* table, uint32_t* err, uint32_t* keys_out,
                       uint32_t* vals_out, hipStream_t st);
// Per tile: its list from its block's run (bkeys, bvals), sorted by depth
// bits, in vals at [ranges[t].x, ranges[t].y); lists of more than 1536
// instances are sorted through keys, keys_alt and vals_alt. A tile whose list
// would pass `capacity` gets an empty range and sets *overflow.
void launch_block_tile_sort(const ViewDesc* views, int num_views, int64_t num_tiles, const BlockGeo& geo,
                            const uint4* table, const uint32_t* bkeys, const uint32_t* bvals, const uint32_t* zkey,
                            int64_t num_splats, int64_t capacity, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                            uint32_t* vals_alt, uint2* ranges, uint32_t* overflow, hipStream_t st);
// ranges[t] = (start, end) of global tile t in the sorted key array of
// min(*n_dev, count) instances (count if n_dev is null); clear = false: the
// caller has zeroed ranges.
void launch_tile_ranges(const uint32_t* keys, const uint32_t* n_dev, int64_t count, uint2* ranges, int64_t num_tiles,
                        bool clear, hipStream_t st);

// order[0..num_tiles) = the tiles by decreasing list length, in classes of
// equal floor(log2(length)) (order within a class unspecified), so that the
// longest tiles start first and the tail of a launch holds the short ones.
void launch_tile_order(const uint2* ranges, int64_t num_tiles, uint32_t* order, hipStream_t st);
// order[0..num_tiles) = the tiles dealt to rounds of ncu workgroups in snake
// order of decreasing weight (tile_last[t] when it is in (0, list length],
// else the list length; tile_last may be null), so that the tiles a CU starts
// with mix heavy and light ones. At most 8192 tiles (tile_balance_supported).
bool tile_balance_supported(int64_t num_tiles);
void launch_tile_balance(const uint2* ranges, const uint32_t* tile_last, int64_t num_tiles, int ncu, uint32_t* order,
                         hipStream_t st);
// Sorts each tile's instances by the raw bits of the splat's depth (zkey, per
// splat, from the projection), stably, so the list order becomes (tile, z
// bits, index) when the instances arrive in index order (index_order); else
// equal depths are put in index order afterwards. keys/vals: the
// tile-grouped instances; keys_alt/vals_alt: scratch of the same size (tiles
// of more than 1536 instances go through it).
void launch_tile_depth_sort(const uint2* ranges, int64_t num_tiles, const uint32_t* zkey, int64_t num_splats,
                            uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, bool index_order,
                            hipStream_t st);

// Zeroes up to kMaxClear segments of 32-bit words in one launch.
constexpr int kMaxClear = 10;
struct ClearList {
  uint32_t* p[kMaxClear];
  int64_t n[kMaxClear];
  int count;
  void add(void* ptr, int64_t words) {
    if (ptr && words > 0 && count < kMaxClear) {
      p[count] = static_cast<uint32_t*>(ptr);
      n[count] = words;
      ++count;
    }
  }
};
void launch_clear(const ClearList& L, hipStream_t st);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// out[0] = sum of last[0..npix); out[1+v] = number of nonzero ntiles in view v's segment of n.
void launch_count_work(const uint32_t* last, int64_t npix, const uint32_t* ntiles, int64_t n, int num_views,
                       unsigned long long* out, hipStream_t st);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t st);

// ---- blend.hip -------------------------------------------------------------
struct BlendArgs {
  const ViewDesc* views;
  const ViewImages* images;     // forward: outputs; backward: dL/dimage
  int32_t num_views;
  int32_t num_tiles;
  const uint32_t* order;        // workgroup -> tile (longest lists first); null = identity
  const uint2* ranges;
  const uint32_t* inst_vals;    // splat index per sorted instance
  const Splat* splats;
  const int4* rect;             // per splat: inclusive pixel rectangle of its binning extent
  float* tfinal;                // per pixel, all views
  uint32_t* last;               // per pixel: index (within the tile list) after the last composited
  float* g2;                    // backward: screen-space gradient accumulators [V*N][10]
  float bg[3];
  // Chunked backward (chunk_len > 0): the backward's work unit is a chunk of
  // chunk_len list positions of one tile (the last of max_chunks chunks takes
  // the rest of the list). The forward records per pixel, in
  // ckpt[(slot * kCkptFields + f) * ckpt_stride + pixel], slot s =
  // (T before chunk s, then the colour and depth composited within chunk s),
  // from which every chunk starts its reverse walk.
  float* ckpt;
  int64_t ckpt_stride;
  int32_t chunk_len;
  int32_t max_chunks;
  uint32_t* tile_last;          // per tile: largest last position of its pixels (forward writes)
  // Forward only, optional: the L1 mapping loss fused into the compositing
  // (as launch_loss_l1 computes it): targets per view (rgb, depth), gradient
  // images written per view, the loss added to *loss.
  const ViewImages* loss_target;
  const ViewImages* loss_grad;
  float depth_weight;
  float* loss;
  // Fused forward and backward (launch_blend_fused): per tile, set once its
  // forward's state is written (zero before the launch); the error word set
  // when a backward unit's bounded wait expires. The backward reads the
  // image gradients from loss_grad.
  uint32_t* tile_done;
  uint32_t* err;
  // Fused launch over a work queue (when its units outnumber the workgroups
  // the device holds at once): the next-unit counter, zero before the launch;
  // null for the plain grid. queue_grid: the workgroups it launches (as
  // many as the device holds at once).
  uint32_t* queue;
  int32_t queue_grid;
};
constexpr int kCkptFields = 5;
bool blend_supported(int tile_w, int tile_h);
// ppt: pixels per thread (1, or 2 for tiles of at least 128 pixels)
void launch_blend_forward(const BlendArgs& a, int tile_w, int tile_h, int ppt, hipStream_t st);
// depth: Gaussians per staged batch of the backward (0 = default, 16, 32 or 64;
// capped at the workgroup's thread count)
bool batch_depth_supported(int depth);
void launch_blend_backward(const BlendArgs& a, int tile_w, int tile_h, int ppt, int depth, hipStream_t st);
// The splat-parallel schedule of the same backward: one wavefront per tile,
// a Gaussian per lane, the pixels pipelined through the lanes; needs
// unchunked forward state (chunk_len 0) and a.tile_last.
void launch_blend_backward_splat(const BlendArgs& a, int tile_w, int tile_h, hipStream_t st);
// Forward (with the fused loss) and backward in one launch, at the default
// batch depth; needs loss_target, loss_grad, g2, tile_done and err.
void launch_blend_fused(const BlendArgs& a, int tile_w, int tile_h, int ppt, hipStream_t st);
// Workgroups of the fused launch the current device holds at once (its CU
// count times the kernel's occupancy per CU); 0 if the device cannot say.
int64_t blend_fused_resident(int tile_w, int tile_h, int ppt);
// Valid chunk settings: chunk_len 0 (whole tile lists) or a multiple of 16
// up to 1 << 20, with 1 <= max_chunks <= 64.
bool chunking_supported(int chunk_len, int max_chunks);
// clear_loss = false: the caller has zeroed *loss.
void launch_loss_l1(const ViewDesc* views, const ViewImages* rendered, const ViewImages* target,
                    const ViewImages* grad, int num_views, int max_pixels, float depth_weight,
                    float* loss, bool clear_loss, hipStream_t st);
// Adam; with step_dev the bias corrections are those of step *step_dev, the
// step count including this step (bc1, bc2 ignored); skip[0] or skip[1]
// nonzero (if skip is not null) leaves everything unchanged.
void launch_adam(float* p, const float* g, float* m, float* v, int64_t num, int64_t stride,
                 int planes, const float* lr_dev, float b1, float b2, float eps, float bc1,
                 float bc2, const uint32_t* step_dev, const uint32_t* skip, hipStream_t st);

}  // namespace gsr
