// Host side of the C ABI: argument checking and the order of the kernel
// launches for render, backward, loss and Adam.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "context.h"

using namespace gsr;

namespace gsr {

// Chunks of the tile lists as the backward's work unit pay off when a launch
// has too few tiles to keep every CU busy to the end (measured: 1200 tiles
// -16 % backward time, 3225 tiles -8 %, 9600 tiles +1 %, 57k tiles +6 %).
int chunk_len_for(const gsr_ctx* ctx, const RenderPlan& P) {
  if (ctx->bwd_schedule == 1) return 0;     // the splat-parallel backward walks whole lists
  if (ctx->chunk_len > 0) return ctx->chunk_len;
  if (ctx->chunk_len < 0) return 0;
  return P.ntiles < kAutoChunkTiles ? kAutoChunk : 0;
}

static int64_t scan_elems(const gsr_ctx* ctx, const Buffers& B, const RenderPlan& P);

int plan_render(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams, RenderPlan* plan) {
  RET_IF(check_gaussians(g));
  RET_IF(check_cams(cams, nv));
  RenderPlan& P = *plan;
  P.num = g->num;
  P.stride = g->stride;
  P.deg = g->sh_degree;
  P.nv = nv;
  P.total = g->num * nv;
  if (P.total > (int64_t(1) << 31)) return GSR_ERR_INVALID;
  P.views = make_views(ctx, cams, nv, &P.ntiles, &P.npix);
  if (P.ntiles >= (int64_t(1) << 31)) return GSR_ERR_INVALID;
  P.capacity = 0;
  P.sorted_splats = P.inst_keys = P.inst_vals = nullptr;
  plan_blocks(ctx, P);
  return GSR_OK;
}

// Binning by blocks of tiles applies to the per-tile depth order (option
// binning 0 or 3). The block is the smallest (at most 8 x 8 tiles; then the
// squarest, then the one giving fewer blocks) that leaves at most kMaxBlocks
// blocks over all views, so that a single 8-bit radix pass groups the block
// instances; the automatic choice also wants it to cover at least two
// tiles. Smaller blocks mean shorter block lists for every tile to filter,
// larger ones fewer block instances.
void plan_blocks(const gsr_ctx* ctx, RenderPlan& P) {
  P.use_blocks = false;
  P.blocks = BlockGeo{};
  for (ViewDesc& v : P.views) {
    v.block_offset = 0;
    v.blocks_x = 0;
  }
  if (!(ctx->binning == 0 || ctx->binning == 3) || P.num == 0 || P.nv == 0 || !per_tile_depth(ctx, P)) return;
  int bw = -1, bh = -1;
  int64_t best = 0;
  for (int area = 0; area <= 6 && bw < 0; ++area) {
    for (int w = 0; w <= 3; ++w) {
      const int h = area - w;
      if (h < 0 || h > 3) continue;
      int64_t nb = 0;
      for (int v = 0; v < P.nv; ++v)
        nb += (int64_t)((P.views[v].tiles_x + (1 << w) - 1) >> w) * ((P.views[v].tiles_y + (1 << h) - 1) >> h);
      if (nb > kMaxBlocks) continue;
      const int sq = std::abs(w - h), bsq = std::abs(bw - bh);
      if (bw < 0 || sq < bsq || (sq == bsq && nb < best)) {
        bw = w;
        bh = h;
        best = nb;
      }
    }
  }
  // single-tile blocks: as many block instances as tile instances, and the
  // per-tile filter on top; the automatic choice takes the radix path then
  if (bw < 0 || (bw + bh == 0 && ctx->binning == 0)) return;
  int32_t off = 0;
  for (ViewDesc& v : P.views) {
    v.block_offset = off;
    v.blocks_x = (v.tiles_x + (1 << bw) - 1) >> bw;
    off += v.blocks_x * ((v.tiles_y + (1 << bh) - 1) >> bh);
  }
  P.use_blocks = true;
  P.blocks = BlockGeo{bw, bh, __builtin_ctz((unsigned)ctx->tile_w), __builtin_ctz((unsigned)ctx->tile_h), off};
}

// Scratch of the tile grouping (B.hist2): the radix sort of the tile keys,
// or with blocks the pass over the block ids.
static int64_t tile_sort_scratch_elems(const RenderPlan& P) {
  return P.use_blocks ? block_sort_scratch_elems(P.capacity) : radix_scratch_elems(P.capacity, bits_for(P.ntiles - 1));
}

int size_instances(gsr_ctx* ctx, Buffers& B, const RenderPlan& P) {
  if (P.capacity >= (int64_t(1) << 30)) return GSR_ERR_CAPACITY;
  const size_t i4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(P.capacity, 1);
  RET_IF(ensure(ctx, B.ikeys, i4));
  RET_IF(ensure(ctx, B.ivals, i4));
  RET_IF(ensure(ctx, B.ikeys_alt, i4));
  RET_IF(ensure(ctx, B.ivals_alt, i4));
  RET_IF(ensure(ctx, B.hist2, sizeof(uint32_t) * (size_t)tile_sort_scratch_elems(P)));
  RET_IF(ensure(ctx, B.block_rank, sizeof(uint32_t) * (size_t)emit_plan_elems(P.capacity)));
  if (P.use_blocks) {
    RET_IF(ensure(ctx, B.bkeys, i4));
    RET_IF(ensure(ctx, B.bvals, i4));
    RET_IF(ensure(ctx, B.btab, sizeof(uint32_t) * (size_t)kBlockTabWords));
  }
  return GSR_OK;
}

int size_render(gsr_ctx* ctx, Buffers& B, RenderPlan& P, const gsr_image* out, hipStream_t st) {
  const int nv = P.nv;
  std::vector<ViewImages> ims(nv);
  for (int v = 0; v < nv; ++v) ims[v] = ViewImages{out[v].rgb, out[v].depth, out[v].alpha};
  const size_t t4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(P.total, 1);
  RET_IF(ensure(ctx, B.views, sizeof(ViewDesc) * nv));
  RET_IF(ensure(ctx, B.images, sizeof(ViewImages) * nv));
  RET_IF(ensure(ctx, B.splats, sizeof(Splat) * (size_t)std::max<int64_t>(P.total, 1)));
  RET_IF(ensure(ctx, B.rect, sizeof(int4) * (size_t)std::max<int64_t>(P.total, 1)));
  RET_IF(ensure(ctx, B.ntiles, t4));
  RET_IF(ensure(ctx, B.zkey, t4));
  RET_IF(ensure(ctx, B.svals, t4));
  RET_IF(ensure(ctx, B.zkey_alt, t4));
  RET_IF(ensure(ctx, B.svals_alt, t4));
  RET_IF(ensure(ctx, B.offsets, t4));
  RET_IF(size_instances(ctx, B, P));
  RET_IF(ensure(ctx, B.ranges, sizeof(uint2) * (size_t)std::max<int64_t>(P.ntiles, 1)));
  RET_IF(ensure(ctx, B.order, sizeof(uint32_t) * (size_t)std::max<int64_t>(P.ntiles, 1)));
  RET_IF(ensure(ctx, B.tfinal, sizeof(float) * (size_t)P.npix));
  RET_IF(ensure(ctx, B.last, sizeof(uint32_t) * (size_t)P.npix));
  RET_IF(ensure(ctx, B.tile_last, sizeof(uint32_t) * (size_t)std::max<int64_t>(P.ntiles, 1)));
  if (!P.forward_only) {
    RET_IF(ensure(ctx, B.images2, sizeof(ViewImages) * nv));
    // per tile a forward-done flag, then the work-queue counter of the fused launch
    RET_IF(ensure(ctx, B.tile_done, sizeof(uint32_t) * (size_t)(P.ntiles + 1)));
    if (chunk_len_for(ctx, P) > 0)
      RET_IF(ensure(ctx, B.ckpt, sizeof(float) * kCkptFields * (size_t)ctx->max_chunks * (size_t)P.npix));
    RET_IF(ensure(ctx, B.g2, sizeof(float) * G2_N * (size_t)std::max<int64_t>(P.total, 1)));
  }
  RET_IF(ensure(ctx, B.total, 64));
  RET_IF(ensure(ctx, B.hist, sizeof(uint32_t) * (size_t)radix_scratch_elems(P.total, 32)));
  {
    int64_t m = 0;
    int mt = 0;
    if (use_bins(ctx, B, P, &m, &mt)) RET_IF(ensure(ctx, B.bins, sizeof(uint32_t) * (size_t)m));
  }
  RET_IF(ensure(ctx, B.partials, 2 * sizeof(uint32_t) * (size_t)scan_partial_elems(scan_elems(ctx, B, P))));
  RET_IF(upload(ctx, B.views.p, P.views.data(), sizeof(ViewDesc) * nv, st));
  RET_IF(upload(ctx, B.images.p, ims.data(), sizeof(ViewImages) * nv, st));
  return GSR_OK;
}

void front_clears(const gsr_ctx* ctx, Buffers& B, const RenderPlan& P, ClearList& L) {
  L.add(B.total.p, 8);
  L.add(B.partials.p, 2 * scan_partial_elems(scan_elems(ctx, B, P)));
  if (P.total > 1) L.add(B.hist.p, radix_scratch_elems(P.total, 32));
}

void back_clears(Buffers& B, const RenderPlan& P, ClearList& L) {
  if (P.use_blocks) {
    // the block pass's look-back words and histogram, the per-block tile
    // counts; every tile's range is written by the per-tile step
    L.add(B.hist2.p, block_sort_scratch_elems(P.capacity));
    L.add(B.btab.p, (int64_t)kHistCopies * kMaxBlocks);
    return;
  }
  if (P.capacity > 1 && P.ntiles > 1) L.add(B.hist2.p, radix_scratch_elems(P.capacity, bits_for(P.ntiles - 1)));
  L.add(B.ranges.p, 2 * P.ntiles);
}

int launch_front(gsr_ctx* ctx, Buffers& B, RenderPlan& P, const float* params, hipStream_t st) {
  const int nv = P.nv;
  uint32_t* totals = as<uint32_t>(B.total);
  const bool global_depth = !per_tile_depth(ctx, P);
  int zrb = 8, zpasses = 0;
  // the global depth sort keeps look-back passes at every size, with its
  // histograms formed by the projection (reduce-then-scan passes measured
  // slower there: 16 views of 2M Gaussians, 245 -> 353 us)
  uint32_t* zhist =
      global_depth && P.total > 1 ? radix_hist(as<uint32_t>(B.hist), P.total, 32, &zrb, &zpasses) : nullptr;
  {
    StageTimer tm(ctx, GSR_STAGE_PROJECT, st);
    launch_project(params, P.num, P.stride, P.deg, nv, as<ViewDesc>(B.views), ctx->tile_w, ctx->tile_h, ctx->znear,
                   as<Splat>(B.splats), as<int4>(B.rect), as<uint32_t>(B.ntiles), as<uint32_t>(B.zkey), zhist, zrb,
                   zpasses, totals + 4, st);
  }
  CHECK_LAUNCH(ctx);
  uint32_t* zk = as<uint32_t>(B.zkey);
  uint32_t* sv = as<uint32_t>(B.svals);
  uint32_t* zka = as<uint32_t>(B.zkey_alt);
  uint32_t* sva = as<uint32_t>(B.svals_alt);
  uint32_t* cscan = as<uint32_t>(B.partials);
  uint32_t* oscan = cscan + scan_partial_elems(P.total);
  // only the visible splats (count in totals[3]) are binned. With the global
  // depth sort they are compacted, sorted by depth and then scanned for their
  // instance offsets; else they are binned in index order (each tile's list
  // is sorted after binning), and one pass compacts them and forms the
  // offsets. With the instance capacity fixed ahead (the captured iteration)
  // the offsets scan also writes the emission plan.
  int64_t bin_entries = 0;
  int bin_tiles = 0;
  if (use_bins(ctx, B, P, &bin_entries, &bin_tiles)) {
    // binning by counting: the per-(tile, workgroup) counts and their scan,
    // whose total is the instance count
    P.plan_ready = false;
    StageTimer tm(ctx, GSR_STAGE_SCAN, st);
    uint32_t* counts = as<uint32_t>(B.bins);
    launch_bin_count(as<uint32_t>(B.ntiles), as<int4>(B.rect), as<ViewDesc>(B.views), nv, P.num, bin_tiles,
                     ctx->tile_w, ctx->tile_h, counts, totals + 3, st);
    scan_gather_exclusive(counts, nullptr, counts, bin_entries, nullptr, totals, cscan, totals + 1, false, st);
    CHECK_LAUNCH(ctx);
    P.sorted_splats = nullptr;
    return GSR_OK;
  }
  P.plan_ready = P.capacity > 0;
  uint32_t* plan = P.plan_ready ? as<uint32_t>(B.block_rank) : nullptr;
  if (global_depth) {
    {
      StageTimer tm(ctx, GSR_STAGE_DEPTH_SORT, st);
      launch_compact_visible(as<uint32_t>(B.ntiles), zk, P.total, zka, sva, totals + 3, cscan, totals + 1, false, st);
      radix_sort_pairs(zka, sva, zk, sv, P.total, totals + 3, 32, as<uint32_t>(B.hist), totals + 1, false, true, st);
    }
    CHECK_LAUNCH(ctx);
    {
      StageTimer tm(ctx, GSR_STAGE_SCAN, st);
      scan_gather_exclusive(as<uint32_t>(B.ntiles), sva, as<uint32_t>(B.offsets), P.total, totals + 3, totals, oscan,
                            totals + 1, false, st, plan, P.capacity);
    }
  } else if (P.use_blocks) {
    // the offsets of the block instances; their count goes to totals[5],
    // the tile lists' instance count to totals[0]
    StageTimer tm(ctx, GSR_STAGE_SCAN, st);
    launch_compact_scan_blocks(as<uint32_t>(B.ntiles), as<int4>(B.rect), P.blocks, P.total, sva,
                               as<uint32_t>(B.offsets), totals + 3, totals + 5, totals, cscan, totals + 1, plan,
                               P.capacity, st);
  } else {
    StageTimer tm(ctx, GSR_STAGE_SCAN, st);
    launch_compact_scan(as<uint32_t>(B.ntiles), P.total, sva, as<uint32_t>(B.offsets), totals + 3, totals, cscan,
                        totals + 1, plan, P.capacity, st);
  }
  CHECK_LAUNCH(ctx);
  sv = sva;
  P.sorted_splats = sv;
  return GSR_OK;
}

// Longest-list-first tile order: worth its extra launch when views of uneven
// visibility share a launch (measured: +18% on 8 views, -4% on one view).
static bool use_lpt(const gsr_ctx* ctx, const RenderPlan& P) {
  return ctx->tile_order == 1 || (ctx->tile_order == 0 && P.nv > 1) ||
         (ctx->tile_order == 3 && !tile_balance_supported(P.ntiles));
}
static bool use_balance(const gsr_ctx* ctx, const RenderPlan& P) {
  return ctx->tile_order == 3 && tile_balance_supported(P.ntiles);
}

static void set_chunking(const gsr_ctx* ctx, Buffers& B, const RenderPlan& P, BlendArgs& ba) {
  const int cl = P.forward_only ? 0 : chunk_len_for(ctx, P);
  ba.tile_last = as<uint32_t>(B.tile_last);
  ba.chunk_len = cl;
  ba.max_chunks = cl > 0 ? ctx->max_chunks : 1;
  ba.ckpt = cl > 0 ? as<float>(B.ckpt) : nullptr;
  ba.ckpt_stride = P.npix;
}

// Automatic: fused when the backward is chunked and every tile's forward
// workgroup is resident at once, so that the backward's units fill the
// forward's tail. With more tiles the forwards run in several rounds, each
// holding its slot through its own first chunk, and the waiting units queue
// behind all of them (measured at 3225 tiles: 1336 us fused against
// 422 + 705 us in two launches; at 1200 tiles: 244 against 287).
// Automatic: per tile for at most 2^19 splats. The global sort's four passes
// are latency-bound at such sizes (14 us each at 200k), while sorting every
// tile's list in LDS costs in proportion to the instances (640x480/200k:
// 58 -> 37 us); with millions of splats the global passes are the cheaper
// (8 views, 500k: 124 against 356 us; 1200x680/1M: 92 against 494 us).
bool per_tile_depth(const gsr_ctx* ctx, const RenderPlan& P) {
  if (ctx->depth_sort != 0) return ctx->depth_sort == 1;
  return P.total <= (int64_t(1) << 19);
}

// The count matrix of the binning by counting stays below 2^26 words (256 MB);
// past that the radix path is used.
constexpr int64_t kBinMaxEntries = int64_t(1) << 26;

bool use_bins(const gsr_ctx* ctx, const Buffers& B, const RenderPlan& P, int64_t* entries, int* max_view_tiles) {
  if (ctx->binning != 1 || P.num == 0 || P.nv == 0 || !per_tile_depth(ctx, P)) return false;
  int64_t most = 0;
  for (const ViewDesc& v : P.views) most = std::max<int64_t>(most, (int64_t)v.tiles_x * v.tiles_y);
  if (!bin_view_fits(most)) return false;
  const int64_t nb = (P.num + bin_chunk(P.num) - 1) / bin_chunk(P.num);
  const int64_t m = P.ntiles * nb;
  if (m > kBinMaxEntries || m >= (int64_t(1) << 31)) return false;
  if (B.bins.fixed && sizeof(uint32_t) * (size_t)m > B.bins.cap) return false;
  *entries = m;
  *max_view_tiles = (int)most;
  return true;
}

// Elements of the largest single-pass scan of a render (the splat compaction
// or the count matrix), for its look-back scratch.
static int64_t scan_elems(const gsr_ctx* ctx, const Buffers& B, const RenderPlan& P) {
  int64_t m = 0;
  int mt = 0;
  return use_bins(ctx, B, P, &m, &mt) ? std::max(P.total, m) : P.total;
}

bool use_fused_blend(const gsr_ctx* ctx, const RenderPlan& P) {
  if (ctx->fuse_blend < 0 || ctx->batch_depth != 0 || ctx->bwd_schedule != 0) return false;
  if (ctx->fuse_blend > 0) return true;
  return chunk_len_for(ctx, P) > 0 && P.ntiles <= ctx->fused_resident;
}

static int launch_sorted_bins(gsr_ctx* ctx, Buffers& B, RenderPlan& P, hipStream_t st, uint32_t*& ik,
                              uint32_t*& iv, uint32_t*& ika, uint32_t*& iva);

// The order in which the blend workgroups take the tiles, from the tile
// ranges (where it is not the tile order).
static void launch_tile_orders(gsr_ctx* ctx, Buffers& B, const RenderPlan& P, hipStream_t st) {
  StageTimer tm(ctx, GSR_STAGE_RANGES, st);
  if (use_lpt(ctx, P)) launch_tile_order(as<uint2>(B.ranges), P.ntiles, as<uint32_t>(B.order), st);
  // the tile_last the previous render of these buffers left (a weight only)
  if (use_balance(ctx, P))
    launch_tile_balance(as<uint2>(B.ranges), as<uint32_t>(B.tile_last), P.ntiles, ctx->num_cus,
                        as<uint32_t>(B.order), st);
}
static int launch_blend_front(gsr_ctx* ctx, Buffers& B, RenderPlan& P, hipStream_t st, const FusedLoss* loss,
                              bool fused, uint32_t* ik, uint32_t* iv, uint32_t* ika, uint32_t* iva);

int launch_back(gsr_ctx* ctx, Buffers& B, RenderPlan& P, hipStream_t st, const FusedLoss* loss, bool fused) {
  uint32_t* totals = as<uint32_t>(B.total);
  uint32_t* ik = as<uint32_t>(B.ikeys);
  uint32_t* iv = as<uint32_t>(B.ivals);
  uint32_t* ika = as<uint32_t>(B.ikeys_alt);
  uint32_t* iva = as<uint32_t>(B.ivals_alt);
  int64_t bin_entries = 0;
  int bin_tiles = 0;
  if (P.use_blocks) {
    // one instance per (splat, block of tiles), grouped by block with one
    // pass that also writes the block table; the tiles' lists are formed
    // with their depth order (launch_blend_front)
    uint32_t* hist2 = as<uint32_t>(B.hist2);
    uint32_t* whist = as<uint32_t>(B.btab);
    {
      StageTimer tm(ctx, GSR_STAGE_EMIT, st);
      launch_emit_blocks(P.sorted_splats, as<uint32_t>(B.offsets), totals + 5, totals + 3, as<int4>(B.rect),
                         as<ViewDesc>(B.views), P.num, P.blocks, P.total, ika, iva, P.capacity, totals + 2,
                         block_sort_hist(hist2, P.capacity), whist, as<uint32_t>(B.block_rank), P.plan_ready, st);
    }
    CHECK_LAUNCH(ctx);
    {
      StageTimer tm(ctx, GSR_STAGE_TILE_SORT, st);
      launch_block_sort(ika, iva, totals + 5, P.capacity, P.blocks.nblocks, hist2, whist,
                        reinterpret_cast<uint4*>(whist + (int64_t)kHistCopies * kMaxBlocks), totals + 1,
                        as<uint32_t>(B.bkeys), as<uint32_t>(B.bvals), st);
    }
  } else if (use_bins(ctx, B, P, &bin_entries, &bin_tiles)) {
    StageTimer tm(ctx, GSR_STAGE_EMIT, st);
    launch_bin_scatter(as<uint32_t>(B.ntiles), as<int4>(B.rect), as<ViewDesc>(B.views), P.nv, P.num, bin_tiles,
                       ctx->tile_w, ctx->tile_h, as<uint32_t>(B.bins), totals, P.capacity, P.ntiles, ik, iv,
                       as<uint2>(B.ranges), totals + 2, st);
  } else {
    RET_IF(launch_sorted_bins(ctx, B, P, st, ik, iv, ika, iva));
  }
  CHECK_LAUNCH(ctx);
  // with blocks, the ranges exist only after the per-tile step
  if (!P.use_blocks) launch_tile_orders(ctx, B, P, st);
  return launch_blend_front(ctx, B, P, st, loss, fused, ik, iv, ika, iva);
}

// The general binning: emission of the instances in the splats' order, a
// stable radix sort of their tile keys, the tile ranges.
static int launch_sorted_bins(gsr_ctx* ctx, Buffers& B, RenderPlan& P, hipStream_t st, uint32_t*& ik,
                              uint32_t*& iv, uint32_t*& ika, uint32_t*& iva) {
  uint32_t* totals = as<uint32_t>(B.total);
  const int tbits = bits_for(P.ntiles - 1);
  // large sorts take reduce-then-scan passes; small ones the look-back
  // passes, whose global histogram the emission accumulates
  const bool scanned = radix_prefers_scan(P.capacity);
  const bool hist_in_emit = !scanned && P.capacity > 1 && tbits > 0 && emit_histogram_fits(tbits);
  int trb = 8, tpasses = 0;
  uint32_t* thist = hist_in_emit ? radix_hist(as<uint32_t>(B.hist2), P.capacity, tbits, &trb, &tpasses) : nullptr;
  {
    StageTimer tm(ctx, GSR_STAGE_EMIT, st);
    launch_emit(P.sorted_splats, as<uint32_t>(B.offsets), totals, totals + 3, as<Splat>(B.splats), P.total, ik, iv,
                P.capacity, totals + 2, thist, tbits,
                as<uint32_t>(B.block_rank), P.plan_ready, st);
  }
  CHECK_LAUNCH(ctx);
  {
    StageTimer tm(ctx, GSR_STAGE_TILE_SORT, st);
    if (scanned)
      radix_sort_pairs_scanned(ik, iv, ika, iva, P.capacity, totals, tbits, as<uint32_t>(B.hist2), totals + 1, st);
    else
      radix_sort_pairs(ik, iv, ika, iva, P.capacity, totals, tbits, as<uint32_t>(B.hist2), totals + 1, false,
                       hist_in_emit, st);
  }
  CHECK_LAUNCH(ctx);
  {
    StageTimer tm(ctx, GSR_STAGE_RANGES, st);
    launch_tile_ranges(ik, totals, P.capacity, as<uint2>(B.ranges), P.ntiles, false, st);
  }
  return GSR_OK;
}

// The per-tile depth sort (where it applies) and the forward blend (or the
// fused forward + backward launch).
static int launch_blend_front(gsr_ctx* ctx, Buffers& B, RenderPlan& P, hipStream_t st, const FusedLoss* loss,
                              bool fused, uint32_t* ik, uint32_t* iv, uint32_t* ika, uint32_t* iva) {
  uint32_t* totals = as<uint32_t>(B.total);
  CHECK_LAUNCH(ctx);
  if (P.use_blocks) {
    {
      StageTimer tm(ctx, GSR_STAGE_TILE_DEPTH, st);
      const uint32_t* whist = as<uint32_t>(B.btab);
      launch_block_tile_sort(as<ViewDesc>(B.views), P.nv, P.ntiles, P.blocks,
                             reinterpret_cast<const uint4*>(whist + (int64_t)kHistCopies * kMaxBlocks),
                             as<uint32_t>(B.bkeys), as<uint32_t>(B.bvals), as<uint32_t>(B.zkey), P.total,
                             P.capacity, ik, iv, ika, iva, as<uint2>(B.ranges), totals + 2, st);
    }
    CHECK_LAUNCH(ctx);
    launch_tile_orders(ctx, B, P, st);
  } else if (per_tile_depth(ctx, P)) {
    StageTimer tm(ctx, GSR_STAGE_TILE_DEPTH, st);
    int64_t m = 0;
    int mt = 0;
    const bool counted = use_bins(ctx, B, P, &m, &mt);   // the lists are not in index order then
    launch_tile_depth_sort(as<uint2>(B.ranges), P.ntiles, as<uint32_t>(B.zkey), P.total, ik, iv, ika, iva, !counted,
                           st);
  }
  CHECK_LAUNCH(ctx);
  P.inst_keys = ik;
  P.inst_vals = iv;

  BlendArgs ba{};
  ba.views = as<ViewDesc>(B.views);
  ba.images = as<ViewImages>(B.images);
  ba.num_views = P.nv;
  ba.num_tiles = (int32_t)P.ntiles;
  ba.order = (use_lpt(ctx, P) || use_balance(ctx, P)) ? as<uint32_t>(B.order) : nullptr;
  ba.ranges = as<uint2>(B.ranges);
  ba.inst_vals = iv;
  ba.splats = as<Splat>(B.splats);
  ba.rect = as<int4>(B.rect);
  ba.tfinal = as<float>(B.tfinal);
  ba.last = as<uint32_t>(B.last);
  ba.g2 = nullptr;
  for (int k = 0; k < 3; ++k) ba.bg[k] = ctx->bg[k];
  set_chunking(ctx, B, P, ba);
  if (loss) {
    ba.loss_target = loss->targets;
    ba.loss_grad = as<ViewImages>(B.images2);
    ba.depth_weight = loss->depth_weight;
    ba.loss = loss->loss;
  }
  if (fused && loss) {
    ba.g2 = as<float>(B.g2);
    ba.tile_done = as<uint32_t>(B.tile_done);
    ba.err = totals + 1;
    // more tiles than the device holds workgroups at once (the plain grid
    // needs every forward resident before the backward units that wait on
    // them): the work-queue form, whose counter is the word after the tiles'
    // flags
    if (P.ntiles > ctx->fused_resident && ctx->fused_resident > 0) {
      ba.queue = as<uint32_t>(B.tile_done) + P.ntiles;
      ba.queue_grid = (int32_t)ctx->fused_resident;
    }
    StageTimer tm(ctx, GSR_STAGE_BLEND, st);
    launch_blend_fused(ba, ctx->tile_w, ctx->tile_h, ctx->ppt, st);
  } else {
    StageTimer tm(ctx, GSR_STAGE_BLEND_FWD, st);
    launch_blend_forward(ba, ctx->tile_w, ctx->tile_h, ctx->ppt, st);
  }
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

int launch_bwd(gsr_ctx* ctx, Buffers& B, const RenderPlan& P, const float* params, float* grad_params,
               bool clear_g2, bool overwrite_grad, hipStream_t st, bool blend_done, const IterCounters* counters) {
  if (P.total == 0) return GSR_OK;
  if (clear_g2) {
    StageTimer tm(ctx, GSR_STAGE_ZERO, st);
    launch_fill_f32(as<float>(B.g2), 0.0f, P.total * G2_N, st);
  }
  CHECK_LAUNCH(ctx);
  BlendArgs ba{};
  ba.views = as<ViewDesc>(B.views);
  ba.images = as<ViewImages>(B.images2);
  ba.num_views = P.nv;
  ba.num_tiles = (int32_t)P.ntiles;
  ba.order = (use_lpt(ctx, P) || use_balance(ctx, P)) ? as<uint32_t>(B.order) : nullptr;
  ba.ranges = as<uint2>(B.ranges);
  ba.inst_vals = P.inst_vals;
  ba.splats = as<Splat>(B.splats);
  ba.rect = as<int4>(B.rect);
  ba.tfinal = as<float>(B.tfinal);
  ba.last = as<uint32_t>(B.last);
  ba.g2 = as<float>(B.g2);
  for (int k = 0; k < 3; ++k) ba.bg[k] = ctx->bg[k];
  set_chunking(ctx, B, P, ba);
  if (!blend_done) {
    StageTimer tm(ctx, GSR_STAGE_BLEND_BWD, st);
    if (ctx->bwd_schedule == 1) launch_blend_backward_splat(ba, ctx->tile_w, ctx->tile_h, st);
    else launch_blend_backward(ba, ctx->tile_w, ctx->tile_h, ctx->ppt, ctx->batch_depth, st);
  }
  CHECK_LAUNCH(ctx);
  if (grad_params) {
    StageTimer tm(ctx, GSR_STAGE_PROJECT_BWD, st);
    launch_project_backward(params, P.num, P.stride, P.deg, P.nv, as<ViewDesc>(B.views), ctx->znear,
                            as<float>(B.g2), as<uint32_t>(B.ntiles), grad_params, overwrite_grad,
                            overwrite_grad && !clear_g2, counters, st);
  }
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

void free_buffers(Buffers& B) {
  DevBuf* bufs[] = {&B.views, &B.images, &B.images2, &B.splats, &B.rect, &B.ntiles, &B.zkey, &B.svals,
                    &B.zkey_alt, &B.svals_alt, &B.offsets, &B.ikeys, &B.ivals, &B.ikeys_alt, &B.ivals_alt,
                    &B.hist, &B.hist2, &B.partials, &B.ranges, &B.order, &B.tfinal, &B.last, &B.g2, &B.total,
                    &B.tile_last, &B.ckpt, &B.block_rank, &B.tile_done, &B.bins, &B.bkeys, &B.bvals, &B.btab};
  for (DevBuf* b : bufs) {
    if (b->p && !b->fixed) (void)hipFree(b->p);
    b->p = nullptr;
    b->cap = 0;
  }
}

}  // namespace gsr

namespace {

// Eager forward: the instance count is read back (one stream synchronisation)
// and the instance buffers are sized to it exactly.
int render_impl(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams, const gsr_image* out,
                hipStream_t st) {
  ctx->have_forward = false;
  ctx->q_bufs = nullptr;
  ctx->q_plan = nullptr;
  RenderPlan& P = ctx->fw;
  RET_IF(plan_render(ctx, g, nv, cams, &P));
  if (!out) return GSR_ERR_INVALID;
  for (int v = 0; v < nv; ++v)
    if (!out[v].rgb || !out[v].depth || !out[v].alpha) return GSR_ERR_INVALID;
  ctx->last_stream = st;
  Buffers& B = ctx->eager;
  P.capacity = 0;
  RET_IF(size_render(ctx, B, P, out, st));
  ClearList L{};
  front_clears(ctx, B, P, L);
  launch_clear(L, st);
  RET_IF(launch_front(ctx, B, P, g->params, st));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->host_total, B.total.p, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (ctx->host_total[1] != 0) return GSR_ERR_DEVICE;
  P.capacity = (int64_t)ctx->host_total[0];
  RET_IF(size_instances(ctx, B, P));
  ClearList L2{};
  back_clears(B, P, L2);
  launch_clear(L2, st);
  RET_IF(launch_back(ctx, B, P, st));

  ctx->have_forward = true;
  ctx->fw_params = g->params;
  ctx->fw_cams.assign(cams, cams + nv);
  ctx->q_bufs = &B;
  ctx->q_plan = &P;
  ctx->q_params = g->params;
  return GSR_OK;
}

int backward_impl(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams,
                  const gsr_image* grad_out, float* grad_params, hipStream_t st) {
  RET_IF(check_gaussians(g));
  RET_IF(check_cams(cams, nv));
  if (!grad_out || (g->num > 0 && !grad_params)) return GSR_ERR_INVALID;
  const RenderPlan& P = ctx->fw;
  if (!ctx->have_forward || ctx->fw_params != g->params || P.num != g->num || P.stride != g->stride ||
      P.deg != g->sh_degree || (int)ctx->fw_cams.size() != nv ||
      std::memcmp(ctx->fw_cams.data(), cams, sizeof(gsr_camera) * nv) != 0)
    return GSR_ERR_STATE;
  ctx->last_stream = st;
  Buffers& B = ctx->eager;
  std::vector<ViewImages> ims(nv);
  for (int v = 0; v < nv; ++v) ims[v] = ViewImages{grad_out[v].rgb, grad_out[v].depth, grad_out[v].alpha};
  RET_IF(upload(ctx, B.images2.p, ims.data(), sizeof(ViewImages) * nv, st));
  return launch_bwd(ctx, B, P, g->params, grad_params, true, false, st);
}

int backward_pose_impl(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams,
                       const gsr_image* grad_out, float* grad_params, double* grad_cams, double* grad_twist,
                       hipStream_t st) {
  RET_IF(check_gaussians(g));
  RET_IF(check_cams(cams, nv));
  if (!grad_out || !grad_cams) return GSR_ERR_INVALID;
  const RenderPlan& P = ctx->fw;
  if (!ctx->have_forward || ctx->fw_params != g->params || P.num != g->num || P.stride != g->stride ||
      P.deg != g->sh_degree || (int)ctx->fw_cams.size() != nv ||
      std::memcmp(ctx->fw_cams.data(), cams, sizeof(gsr_camera) * nv) != 0)
    return GSR_ERR_STATE;
  ctx->last_stream = st;
  Buffers& B = ctx->eager;
  std::vector<ViewImages> ims(nv);
  for (int v = 0; v < nv; ++v) ims[v] = ViewImages{grad_out[v].rgb, grad_out[v].depth, grad_out[v].alpha};
  RET_IF(upload(ctx, B.images2.p, ims.data(), sizeof(ViewImages) * nv, st));
  RET_IF(launch_bwd(ctx, B, P, g->params, grad_params, true, false, st));
  if (P.total > 0) {
    launch_pose_backward(g->params, P.num, P.stride, P.deg, P.nv, as<ViewDesc>(B.views), as<float>(B.g2),
                         as<uint32_t>(B.ntiles), grad_cams, grad_twist, st);
    CHECK_LAUNCH(ctx);
  }
  return GSR_OK;
}

}  // namespace

extern "C" {

int gsr_render_backward_pose(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views, const gsr_camera* cams,
                             const gsr_image* grad_out, float* grad_params, double* grad_cams, double* grad_twist,
                             void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  try {
    return backward_pose_impl(ctx, g, num_views, cams, grad_out, grad_params, grad_cams, grad_twist,
                              (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    return GSR_ERR_OOM;
  } catch (...) {
    return GSR_ERR_INVALID;
  }
}

int gsr_create(gsr_ctx** out, const gsr_options* opt) {
  if (!out) return GSR_ERR_INVALID;
  *out = nullptr;
  gsr_ctx* ctx = new (std::nothrow) gsr_ctx();
  if (!ctx) return GSR_ERR_OOM;
  if (opt) {
    const int tw = opt->tile_w ? opt->tile_w : 16, th = opt->tile_h ? opt->tile_h : 16;
    if (!blend_supported(tw, th)) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    if (!batch_depth_supported(opt->batch_depth)) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->batch_depth = opt->batch_depth;
    ctx->tile_w = tw;
    ctx->tile_h = th;
    if (opt->pixels_per_thread < 0 || opt->pixels_per_thread > 2 ||
        (opt->pixels_per_thread == 2 && tw * th < 128)) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->ppt = opt->pixels_per_thread == 0 ? 1 : opt->pixels_per_thread;
    if (opt->tile_order < 0 || opt->tile_order > 3) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->tile_order = opt->tile_order;
    const int mc = opt->max_chunks == 0 ? ctx->max_chunks : opt->max_chunks;
    if (opt->chunk_len < -1 || !chunking_supported(opt->chunk_len > 0 ? opt->chunk_len : kAutoChunk, mc)) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->chunk_len = opt->chunk_len;
    ctx->max_chunks = mc;
    if (opt->fuse_blend < -1 || opt->fuse_blend > 1) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->fuse_blend = opt->fuse_blend;
    if (opt->depth_sort < 0 || opt->depth_sort > 2) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->depth_sort = opt->depth_sort;
    if (opt->backward_schedule < 0 || opt->backward_schedule > 1) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->bwd_schedule = opt->backward_schedule;
    if (opt->binning < 0 || opt->binning > 3) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->binning = opt->binning;
    for (int k = 0; k < 3; ++k) ctx->bg[k] = opt->bg[k];
    ctx->znear = opt->znear > 0.f ? opt->znear : 0.2f;
  }
  ctx->fused_resident = blend_fused_resident(ctx->tile_w, ctx->tile_h, ctx->ppt);
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      ctx->num_cus = cus;
    (void)hipGetLastError();
  }
  // the allocation-free render's scratch on this device (its status is
  // checked there: gsr_render_noalloc reports GSR_ERR_UNSUPPORTED without it)
  (void)noalloc_attach(ctx);
  hipError_t e = hipHostMalloc((void**)&ctx->host_total, 64, hipHostMallocDefault);
  for (int k = 0; k < kSlots && e == hipSuccess; ++k) {
    e = hipHostMalloc(&ctx->slots[k], kSlotBytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->slot_ev[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    gsr_destroy(ctx);
    return GSR_ERR_HIP;
  }
  *out = ctx;
  return GSR_OK;
}

void gsr_destroy(gsr_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  destroy_graph(ctx);
  free_buffers(ctx->eager);
  DevBuf* bufs[] = {&ctx->images3, &ctx->lr, &ctx->splat_out, &ctx->counts, &ctx->seed_buf};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (int k = 0; k < kSlots; ++k) {
    if (ctx->slots[k]) (void)hipHostFree(ctx->slots[k]);
    if (ctx->slot_ev[k]) (void)hipEventDestroy(ctx->slot_ev[k]);
  }
  if (ctx->host_total) (void)hipHostFree(ctx->host_total);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& v : ctx->ev_pending)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  delete ctx;
}

int gsr_render(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views, const gsr_camera* cams,
               const gsr_image* out, void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  try {
    return render_impl(ctx, g, num_views, cams, out, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    return GSR_ERR_OOM;
  } catch (...) {
    return GSR_ERR_INVALID;
  }
}

int gsr_render1(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cam, const gsr_image* out, void* stream) {
  return gsr_render(ctx, g, 1, cam, out, stream);
}

int gsr_render_backward(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views, const gsr_camera* cams,
                        const gsr_image* grad_out, float* grad_params, void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  try {
    return backward_impl(ctx, g, num_views, cams, grad_out, grad_params, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    return GSR_ERR_OOM;
  } catch (...) {
    return GSR_ERR_INVALID;
  }
}

int gsr_loss_l1(gsr_ctx* ctx, int32_t num_views, const gsr_camera* cams, const gsr_image* rendered,
                const gsr_image* target, float depth_weight, const gsr_image* grad_out, float* loss, void* stream) {
  if (!ctx || !rendered || !target || !grad_out) return GSR_ERR_INVALID;
  RET_IF(check_cams(cams, num_views));
  for (int v = 0; v < num_views; ++v)
    if (!rendered[v].rgb || !rendered[v].depth || !target[v].rgb || !target[v].depth || !grad_out[v].rgb ||
        !grad_out[v].depth)
      return GSR_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  ctx->last_stream = st;
  try {
    int64_t nt, np;
    std::vector<ViewDesc> views = make_views(ctx, cams, num_views, &nt, &np);
    std::vector<ViewImages> a(num_views), b(num_views), c(num_views);
    int maxpix = 0;
    for (int v = 0; v < num_views; ++v) {
      a[v] = ViewImages{rendered[v].rgb, rendered[v].depth, rendered[v].alpha};
      b[v] = ViewImages{target[v].rgb, target[v].depth, target[v].alpha};
      c[v] = ViewImages{grad_out[v].rgb, grad_out[v].depth, grad_out[v].alpha};
      maxpix = std::max(maxpix, cams[v].width * cams[v].height);
    }
    // loss descriptors live in their own buffers so a pending backward keeps its own
    RET_IF(ensure(ctx, ctx->images3, 3 * sizeof(ViewImages) * num_views + sizeof(ViewDesc) * num_views));
    char* base = static_cast<char*>(ctx->images3.p);
    ViewImages* da = reinterpret_cast<ViewImages*>(base);
    ViewImages* db = da + num_views;
    ViewImages* dc = db + num_views;
    ViewDesc* dv = reinterpret_cast<ViewDesc*>(dc + num_views);
    RET_IF(upload(ctx, da, a.data(), sizeof(ViewImages) * num_views, st));
    RET_IF(upload(ctx, db, b.data(), sizeof(ViewImages) * num_views, st));
    RET_IF(upload(ctx, dc, c.data(), sizeof(ViewImages) * num_views, st));
    RET_IF(upload(ctx, dv, views.data(), sizeof(ViewDesc) * num_views, st));
    StageTimer tm(ctx, GSR_STAGE_LOSS, st);
    launch_loss_l1(dv, da, db, dc, num_views, maxpix, depth_weight, loss, true, st);
    CHECK_LAUNCH(ctx);
  } catch (...) {
    return GSR_ERR_OOM;
  }
  return GSR_OK;
}

int gsr_adam_step(gsr_ctx* ctx, float* params, const float* grads, float* m, float* v, int64_t num, int64_t stride,
                  int32_t num_planes, const float* lr_per_plane, float beta1, float beta2, float eps, int32_t step,
                  void* stream) {
  if (!ctx || num < 0 || stride < num || num_planes < 1 || num_planes > 4096 || !lr_per_plane || step < 1)
    return GSR_ERR_INVALID;
  if (num > 0 && (!params || !grads || !m || !v)) return GSR_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  ctx->last_stream = st;
  RET_IF(ensure(ctx, ctx->lr, sizeof(float) * num_planes));
  RET_IF(upload(ctx, ctx->lr.p, lr_per_plane, sizeof(float) * num_planes, st));
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  {
    StageTimer tm(ctx, GSR_STAGE_ADAM, st);
    launch_adam(params, grads, m, v, num, stride, num_planes, as<float>(ctx->lr), beta1, beta2, eps, bc1, bc2, nullptr,
                nullptr, st);
  }
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

int gsr_query_status(gsr_ctx* ctx, int64_t* num_instances, int64_t* num_visible, int64_t* num_tiles,
                     int64_t* nonfinite_culled) {
  if (!ctx) return GSR_ERR_INVALID;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  uint32_t t[5] = {0, 0, 0, 0, 0};
  if (ctx->q_bufs) HIP_TRY(ctx, hipMemcpy(t, ctx->q_bufs->total.p, sizeof(t), hipMemcpyDeviceToHost));
  if (num_instances) *num_instances = (int64_t)t[0];
  if (num_visible) *num_visible = (int64_t)t[3];
  if (num_tiles) *num_tiles = ctx->q_plan ? ctx->q_plan->ntiles : 0;
  if (nonfinite_culled) *nonfinite_culled = (int64_t)t[4];
  if (t[1]) return GSR_ERR_DEVICE;
  // an allocation-free render that needed more instances than its fixed capacity
  if (ctx->q_bufs == &ctx->na_bufs && t[2]) return GSR_ERR_CAPACITY;
  return GSR_OK;
}

int gsr_activations(gsr_ctx* ctx, const gsr_gaussians* g, float* scale, float* opacity, void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  RET_IF(check_gaussians(g));
  hipStream_t st = (hipStream_t)stream;
  ctx->last_stream = st;
  launch_activations(g->params, g->num, g->stride, scale, opacity, st);
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

int gsr_copy_instances(gsr_ctx* ctx, uint32_t* tile, uint32_t* gid, int64_t capacity, int64_t* count) {
  if (!ctx || !count || capacity < 0) return GSR_ERR_INVALID;
  if (!ctx->q_bufs) return GSR_ERR_STATE;
  int64_t I = 0;
  RET_IF(gsr_query_status(ctx, &I, nullptr, nullptr, nullptr));
  I = std::min<int64_t>(I, ctx->q_plan->capacity);
  *count = I;
  const int64_t m = std::min(capacity, I);
  if (m == 0) return GSR_OK;
  if (!tile || !gid) return GSR_ERR_INVALID;
  const RenderPlan& P = *ctx->q_plan;
  if (P.use_blocks) {
    // the tiles' lists lie block by block: gather them in tile order
    std::vector<uint2> rg((size_t)P.ntiles);
    std::vector<uint32_t> all((size_t)I);
    HIP_TRY(ctx, hipMemcpy(rg.data(), ctx->q_bufs->ranges.p, sizeof(uint2) * rg.size(), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(all.data(), P.inst_vals, sizeof(uint32_t) * (size_t)I, hipMemcpyDeviceToHost));
    int64_t o = 0;
    for (int64_t t = 0; t < P.ntiles && o < m; ++t) {
      for (uint32_t k = rg[t].x; k < rg[t].y && o < m; ++k, ++o) {
        if ((int64_t)k >= I) return GSR_ERR_STATE;
        tile[o] = (uint32_t)t;
        gid[o] = all[k];
      }
    }
    if (o < m) return GSR_ERR_STATE;
  } else {
    HIP_TRY(ctx, hipMemcpy(tile, P.inst_keys, sizeof(uint32_t) * m, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(gid, P.inst_vals, sizeof(uint32_t) * m, hipMemcpyDeviceToHost));
  }
  const uint32_t N = (uint32_t)ctx->q_plan->num;
  for (int64_t k = 0; k < m; ++k) gid[k] = gid[k] % N;
  return GSR_OK;
}

int gsr_copy_splats(gsr_ctx* ctx, int32_t view, float* out, int64_t num) {
  if (!ctx || !out) return GSR_ERR_INVALID;
  if (!ctx->q_bufs) return GSR_ERR_STATE;
  const RenderPlan& P = *ctx->q_plan;
  Buffers& B = *ctx->q_bufs;
  if (view < 0 || view >= P.nv || num != P.num) return GSR_ERR_INVALID;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  if (num == 0) return GSR_OK;
  hipStream_t st = ctx->last_stream;
  RET_IF(ensure(ctx, ctx->splat_out, sizeof(float) * 16 * (size_t)num));
  const int64_t off = (int64_t)view * num;
  launch_export_splats(ctx->q_params, num, P.stride, as<ViewDesc>(B.views) + view, ctx->znear,
                       as<Splat>(B.splats) + off, as<int4>(B.rect) + off, as<uint32_t>(B.ntiles) + off,
                       as<float>(ctx->splat_out), st);
  CHECK_LAUNCH(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(st));
  HIP_TRY(ctx, hipMemcpy(out, ctx->splat_out.p, sizeof(float) * 16 * (size_t)num, hipMemcpyDeviceToHost));
  return GSR_OK;
}

int gsr_count_work(gsr_ctx* ctx, int64_t* pairs, int64_t* visible, int32_t num_views) {
  if (!ctx || !pairs) return GSR_ERR_INVALID;
  if (!ctx->q_bufs) return GSR_ERR_STATE;
  const RenderPlan& P = *ctx->q_plan;
  Buffers& B = *ctx->q_bufs;
  if (visible && num_views != P.nv) return GSR_ERR_INVALID;
  hipStream_t st = ctx->last_stream;
  const int nv = P.nv;
  RET_IF(ensure(ctx, ctx->counts, sizeof(unsigned long long) * (size_t)(1 + nv)));
  unsigned long long* c = as<unsigned long long>(ctx->counts);
  launch_count_work(as<uint32_t>(B.last), P.npix, as<uint32_t>(B.ntiles), P.num, nv, c, st);
  CHECK_LAUNCH(ctx);
  std::vector<unsigned long long> h(1 + nv);
  HIP_TRY(ctx, hipStreamSynchronize(st));
  HIP_TRY(ctx, hipMemcpy(h.data(), c, sizeof(unsigned long long) * (1 + nv), hipMemcpyDeviceToHost));
  *pairs = (int64_t)h[0];
  if (visible)
    for (int v = 0; v < nv; ++v) visible[v] = (int64_t)h[1 + v];
  return GSR_OK;
}

int gsr_set_profiling(gsr_ctx* ctx, uint32_t stage_mask) {
  if (!ctx) return GSR_ERR_INVALID;
  ctx->profile_mask = stage_mask;
  return GSR_OK;
}

int gsr_get_profile(gsr_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches, int32_t reset) {
  if (!ctx || stage < 0 || stage >= GSR_NUM_STAGES || !total_ms) return GSR_ERR_INVALID;
  RET_IF(harvest_graph(ctx));
  double sum = ctx->acc_ms[stage];
  auto& v = ctx->ev_pending[stage];
  for (auto& pr : v) {
    HIP_TRY(ctx, hipEventSynchronize(pr.second));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, pr.first, pr.second));
    sum += ms;
  }
  *total_ms = sum;
  if (launches) *launches = (int64_t)v.size() + ctx->acc_n[stage];
  if (reset) {
    for (auto& pr : v) {
      ctx->ev_pool.push_back(pr.first);
      ctx->ev_pool.push_back(pr.second);
    }
    v.clear();
    ctx->acc_ms[stage] = 0.0;
    ctx->acc_n[stage] = 0;
  }
  return GSR_OK;
}

int gsr_last_hip_error(gsr_ctx* ctx) { return ctx ? ctx->hip_err : ipc_last_hip_error(); }

const char* gsr_status_string(int status) {
  switch (status) {
    case GSR_OK: return "ok";
    case GSR_ERR_INVALID: return "invalid argument";
    case GSR_ERR_OOM: return "device out of memory";
    case GSR_ERR_HIP: return "HIP runtime error";
    case GSR_ERR_STATE: return "call order violated (backward without a matching forward)";
    case GSR_ERR_CAPACITY: return "fixed-capacity scratch too small";
    case GSR_ERR_UNSUPPORTED: return "unsupported option";
    case GSR_ERR_DEVICE: return "a bounded device-side wait expired (sort look-back); results invalid";
    default: return "unknown status";
  }
}

}  // extern "C"
