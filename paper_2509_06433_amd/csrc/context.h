// The context behind the C ABI: device scratch, staging, call-order state
// and per-stage timing, plus the host helpers the entry points share.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gsr.h"
#include "gsr_internal.h"

struct gsr_ctx;

namespace gsr {

inline void note_hip_failure(gsr_ctx* ctx, hipError_t e, const char* expr, const char* file, int line);

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool fixed = false;   // a window of memory the context does not own: never freed or grown
};

// Pinned staging slots for host->device uploads of small descriptor arrays;
// each slot is reused only after the event recorded behind its last copy.
constexpr int kSlots = 8;
constexpr size_t kSlotBytes = 64 * 1024;

// Device buffers of one render + backward pipeline. The eager entry points
// and a captured mapping iteration each own a set, so that growing one never
// moves memory the other's kernels (or a captured graph) refer to.
struct Buffers {
  DevBuf views, images, images2;
  DevBuf splats, rect, ntiles, zkey, svals, zkey_alt, svals_alt, offsets;
  DevBuf ikeys, ivals, ikeys_alt, ivals_alt;
  DevBuf hist, hist2, partials, ranges, order, tfinal, last, g2;   // hist: depth sort, hist2: tile sort
  DevBuf total;   // [0] instance count, [1] wait expired, [2] instance overflow, [3] visible splats,
                  // [4] Gaussians culled as non-finite or degenerate
  DevBuf tile_last, ckpt;   // per tile: longest walk; per pixel: state at the backward's chunk boundaries
  DevBuf tile_done;         // fused blend: per tile, its forward is done
  DevBuf block_rank;        // emission: first depth rank of every block of output positions
  DevBuf bins;              // binning by counting: per (tile, workgroup) counts, then run starts
  DevBuf bkeys, bvals;      // binning by blocks: the block instances grouped by block
  DevBuf btab;              // binning by blocks: per-block tile counts (kHistCopies copies), then the block table
};

// Sizes and final buffer roles of one forward render.
struct RenderPlan {
  int64_t num = 0, stride = 0;
  int deg = 0, nv = 0;
  int64_t total = 0;                   // num * nv projected splats
  int64_t ntiles = 0, npix = 0;
  int64_t capacity = 0;                // instance slots (eager: exactly the count)
  std::vector<ViewDesc> views;
  uint32_t* sorted_splats = nullptr;   // depth-sorted splat indices
  bool plan_ready = false;             // the offsets scan wrote the emission plan
  uint32_t* inst_keys = nullptr;       // sorted instance list
  uint32_t* inst_vals = nullptr;
  bool forward_only = false;           // no backward follows: no per-chunk state, no gradient scratch
  bool use_blocks = false;             // binning by blocks of tiles (blocks; views carry their block offsets)
  BlockGeo blocks{};
};

struct GraphState;   // captured mapping iteration

// Automatic backward chunking: chunks of kAutoChunk list positions when a
// launch covers fewer than kAutoChunkTiles tiles.
constexpr int kAutoChunk = 128;
constexpr int64_t kAutoChunkTiles = 4096;
int chunk_len_for(const gsr_ctx* ctx, const RenderPlan& P);

// Brackets one stage's launches with events when profiling is on. While a
// mapping iteration is being captured, the events become event-record nodes
// of the graph and the pair goes to the capture's list instead.
struct TimedPair {
  int stage;
  hipEvent_t a, b;
  hipGraphNode_t na = nullptr, nb = nullptr;   // their event-record nodes, when captured
};

struct StageTimer {
  gsr_ctx* ctx;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  hipGraphNode_t na = nullptr;
  StageTimer(gsr_ctx* c, int s, hipStream_t stream);
  ~StageTimer();
};

// Appends an event-record node behind the work captured so far on `st` and
// makes it the dependency of what is captured next (the capture-time form of
// recording an event on the stream).
inline hipError_t capture_event_node(hipStream_t st, hipEvent_t ev, hipGraphNode_t* node) {
  hipStreamCaptureStatus cs;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  hipError_t e = hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusActive || !g) return hipErrorStreamCaptureInvalidated;
  e = hipGraphAddEventRecordNode(node, g, deps, nd, ev);
  if (e != hipSuccess) return e;
  return hipStreamUpdateCaptureDependencies(st, node, 1, hipStreamSetCaptureDependencies);
}

}  // namespace gsr

struct gsr_ctx {
  using DevBuf = gsr::DevBuf;
  using ViewDesc = gsr::ViewDesc;
  int tile_w = 16, tile_h = 16;
  int ppt = 1;                          // pixels per thread in the blend kernels
  int batch_depth = 0;                  // backward batch depth (0 = default)
  int tile_order = 0;                   // 0 auto, 1 longest list first, 2 tile order, 3 balanced over the CUs
  int num_cus = 256;                    // compute units of the context's device
  int chunk_len = 0;                    // backward work unit in list positions: 0 automatic, -1 whole lists
  int max_chunks = 4;                   // chunks per tile (the last takes the rest)
  int fuse_blend = 0;                   // mapping iteration: 0 automatic, 1 fused, -1 two launches
  int64_t fused_resident = 0;           // workgroups of the fused blend launch the device holds at once
  int depth_sort = 0;                   // 0 automatic, 1 per-tile sort after binning, 2 one global sort before
  int binning = 0;                      // 0 automatic, 1 counting, 2 radix sort of tile keys, 3 blocks of tiles
  int bwd_schedule = 0;                 // blend backward: 0 pixel-parallel, 1 splat-parallel
  float bg[3] = {0.f, 0.f, 0.f};
  float znear = 0.2f;
  int hip_err = 0;
  hipStream_t last_stream = nullptr;

  gsr::Buffers eager;                   // buffers of gsr_render / gsr_render_backward
  gsr::Buffers na_bufs;                 // gsr_render_noalloc: windows of the device's static scratch
  gsr::RenderPlan na_plan;
  int na_device = -1;                   // the device whose scratch na_bufs point into
  DevBuf images3, lr, splat_out;
  DevBuf seed_buf;                      // gsr_densify: seed flags, offsets, scan scratch
  uint32_t* host_total = nullptr;
  void* slots[gsr::kSlots] = {};
  hipEvent_t slot_ev[gsr::kSlots] = {};
  bool slot_used[gsr::kSlots] = {};
  int next_slot = 0;

  // state of the last eager render, checked by the backward
  bool have_forward = false;
  const float* fw_params = nullptr;
  std::vector<gsr_camera> fw_cams;
  gsr::RenderPlan fw;

  // what the status and copy queries report on: the last eager render or
  // the last mapping iteration
  gsr::Buffers* q_bufs = nullptr;
  const gsr::RenderPlan* q_plan = nullptr;
  const float* q_params = nullptr;

  // per-stage timing
  uint32_t profile_mask = 0;          // bit k: time stage k
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[GSR_NUM_STAGES];
  DevBuf counts;

  // captured mapping iteration
  gsr::GraphState* graph = nullptr;
  std::vector<gsr::TimedPair>* capture_timed = nullptr;   // set while capturing
  // stage times harvested from replayed graphs, not yet reported
  double acc_ms[GSR_NUM_STAGES] = {};
  int64_t acc_n[GSR_NUM_STAGES] = {};
};

namespace gsr {

// A timing event from the context's pool (created when the pool is empty).
inline hipEvent_t take_event(gsr_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

inline StageTimer::StageTimer(gsr_ctx* c, int s, hipStream_t stream) : ctx(c), stage(s), st(stream) {
  if (!((ctx->profile_mask >> s) & 1u)) return;
  a = take_event(ctx);
  b = take_event(ctx);
  if (!a || !b) return;
  const hipError_t e = ctx->capture_timed ? capture_event_node(st, a, &na) : hipEventRecord(a, st);
  if (e != hipSuccess) note_hip_failure(ctx, e, "stage timer start event", __FILE__, __LINE__);
}

inline StageTimer::~StageTimer() {
  if (!a || !b) return;
  if (ctx->capture_timed) {
    hipGraphNode_t nb = nullptr;
    const hipError_t e = capture_event_node(st, b, &nb);
    if (e != hipSuccess) note_hip_failure(ctx, e, "stage timer end event", __FILE__, __LINE__);
    ctx->capture_timed->push_back(TimedPair{stage, a, b, na, nb});
  } else {
    (void)hipEventRecord(b, st);
    ctx->ev_pending[stage].emplace_back(a, b);
  }
}

}  // namespace gsr

namespace gsr {

// With GSR_DEBUG set in the environment, a failing HIP call is reported on
// stderr with its source location.
inline void note_hip_failure(gsr_ctx* ctx, hipError_t e, const char* expr, const char* file, int line) {
  ctx->hip_err = (int)e;
  static const bool verbose = std::getenv("GSR_DEBUG") != nullptr;
  if (verbose) std::fprintf(stderr, "gsr: %s:%d: %s -> %d (%s)\n", file, line, expr, (int)e, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                          \
  do {                                                              \
    hipError_t e_ = (expr);                                         \
    if (e_ != hipSuccess) {                                         \
      gsr::note_hip_failure((ctx), e_, #expr, __FILE__, __LINE__);  \
      return GSR_ERR_HIP;                                           \
    }                                                               \
  } while (0)

#define CHECK_LAUNCH(ctx) HIP_TRY(ctx, hipGetLastError())

inline int ensure(gsr_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return GSR_OK;
  if (b.fixed) return GSR_ERR_CAPACITY;
  size_t want = std::max<size_t>(bytes + bytes / 4, 256);
  if (b.p) {
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return GSR_ERR_OOM;
    }
    want = bytes;
  }
  b.cap = want;
  return GSR_OK;
}

template <class T>
inline T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}

inline int upload(gsr_ctx* ctx, void* dev, const void* host, size_t bytes, hipStream_t st) {
  if (bytes == 0) return GSR_OK;
  if (bytes > kSlotBytes) {
    HIP_TRY(ctx, hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return GSR_OK;
  }
  const int k = ctx->next_slot;
  ctx->next_slot = (k + 1) % kSlots;
  if (ctx->slot_used[k]) HIP_TRY(ctx, hipEventSynchronize(ctx->slot_ev[k]));
  std::memcpy(ctx->slots[k], host, bytes);
  HIP_TRY(ctx, hipMemcpyAsync(dev, ctx->slots[k], bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(ctx->slot_ev[k], st));
  ctx->slot_used[k] = true;
  return GSR_OK;
}

#define RET_IF(expr)            \
  do {                          \
    int r_ = (expr);            \
    if (r_ != GSR_OK) return r_; \
  } while (0)

inline int check_gaussians(const gsr_gaussians* g) {
  if (!g) return GSR_ERR_INVALID;
  if (g->num < 0 || g->num > (int64_t(1) << 27)) return GSR_ERR_INVALID;
  if (g->stride < g->num) return GSR_ERR_INVALID;
  if (g->sh_degree < 0 || g->sh_degree > 3) return GSR_ERR_INVALID;
  if (g->num > 0 && !g->params) return GSR_ERR_INVALID;
  return GSR_OK;
}

inline int num_planes(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

inline int check_cams(const gsr_camera* cams, int32_t num_views) {
  if (num_views < 1 || num_views > 256 || !cams) return GSR_ERR_INVALID;
  for (int v = 0; v < num_views; ++v) {
    const gsr_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384) return GSR_ERR_INVALID;
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.cx) || !std::isfinite(c.cy)) return GSR_ERR_INVALID;
    for (int k = 0; k < 9; ++k) if (!std::isfinite(c.R[k])) return GSR_ERR_INVALID;
    for (int k = 0; k < 3; ++k) if (!std::isfinite(c.t[k])) return GSR_ERR_INVALID;
  }
  return GSR_OK;
}

// The descriptor of one view whose tiles start at global tile toff and whose
// pixels start at poff in the per-pixel scratch.
inline void fill_view(const gsr_ctx* ctx, const gsr_camera& c, int64_t toff, int64_t poff, ViewDesc& d);

// Per-view descriptors; returns total tiles and pixels.
inline std::vector<ViewDesc> make_views(const gsr_ctx* ctx, const gsr_camera* cams, int nv, int64_t* tiles,
                                 int64_t* pixels) {
  std::vector<ViewDesc> out(nv);
  int64_t toff = 0, poff = 0;
  for (int v = 0; v < nv; ++v) {
    fill_view(ctx, cams[v], toff, poff, out[v]);
    toff += (int64_t)out[v].tiles_x * out[v].tiles_y;
    poff += (int64_t)cams[v].width * cams[v].height;
  }
  *tiles = toff;
  *pixels = poff;
  return out;
}

inline void fill_view(const gsr_ctx* ctx, const gsr_camera& c, int64_t toff, int64_t poff, ViewDesc& d) {
  std::memcpy(d.R, c.R, sizeof(d.R));
  std::memcpy(d.t, c.t, sizeof(d.t));
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i) s -= (double)c.R[i * 3 + j] * (double)c.t[i];
    d.campos[j] = (float)s;
  }
  d.width = c.width; d.height = c.height;
  d.tiles_x = (c.width + ctx->tile_w - 1) / ctx->tile_w;
  d.tiles_y = (c.height + ctx->tile_h - 1) / ctx->tile_h;
  d.tile_offset = (int32_t)toff;
  d.pix_offset = (int32_t)poff;
}

inline int bits_for(int64_t max_key) {
  int b = 0;
  while (b < 32 && (int64_t(1) << b) <= max_key) ++b;
  return b;
}

// Render pipeline shared by the eager entry points and the captured mapping
// iteration (api.hip).
//   plan_render: checks arguments, fills the plan's sizes and view descriptors.
//   size_render: grows B for the plan (instance slots: plan.capacity) and
//                uploads the view descriptors and output image pointers.
//   front_clears / back_clears: the scratch each half needs zeroed first
//                 (B.total, the scan and depth-sort scratch; the tile-sort
//                 scratch and the ranges).
//   launch_front: projection (with the depth-key histograms), depth sort,
//                 instance offsets; B.total[0] = count.
//   launch_back:  instance emission (at most plan.capacity, with the tile-key
//                 histograms), tile sort, tile ranges, compositing. Counts are
//                 read on the device. With loss, the compositing also forms
//                 the L1 loss against loss->targets and writes its image
//                 gradients through the descriptors in B.images2.
//                 With fused (needs loss), the compositing and the blend
//                 backward are one launch (launch_bwd then skips the blend
//                 backward); B.tile_done must be zero.
//   launch_bwd:   blend backward and projection backward into grad_params
//                 (added, or overwritten with overwrite_grad), image
//                 gradients from the descriptors in B.images2; g2 is zeroed
//                 first unless clear_g2 is false. With overwrite_grad and not
//                 clear_g2 (the mapping iteration) the projection backward
//                 zeroes the g2 rows it reads, so g2 stays clean between
//                 replays. With counters (and at least one Gaussian) the
//                 projection backward also counts the iteration.
// The launch_* functions make no allocation, copy or synchronisation, so a
// stream capture can record them.
int plan_render(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams, RenderPlan* plan);
int size_render(gsr_ctx* ctx, Buffers& B, RenderPlan& plan, const gsr_image* out, hipStream_t st);
void front_clears(const gsr_ctx* ctx, Buffers& B, const RenderPlan& plan, ClearList& L);
void back_clears(Buffers& B, const RenderPlan& plan, ClearList& L);
int launch_front(gsr_ctx* ctx, Buffers& B, RenderPlan& plan, const float* params, hipStream_t st);
struct FusedLoss {
  const ViewImages* targets;   // device descriptors, per view (rgb, depth)
  float depth_weight;
  float* loss;                 // added to; may be null
};
int launch_back(gsr_ctx* ctx, Buffers& B, RenderPlan& plan, hipStream_t st, const FusedLoss* loss = nullptr,
                bool fused = false);
int launch_bwd(gsr_ctx* ctx, Buffers& B, const RenderPlan& plan, const float* params, float* grad_params,
               bool clear_g2, bool overwrite_grad, hipStream_t st, bool blend_done = false,
               const IterCounters* counters = nullptr);
// Whether the mapping iteration fuses the blend forward and backward.
bool use_fused_blend(const gsr_ctx* ctx, const RenderPlan& plan);
// Whether each tile's list is sorted by depth after binning (else all visible
// splats are sorted once before binning).
bool per_tile_depth(const gsr_ctx* ctx, const RenderPlan& plan);
// Chooses the binning by blocks of tiles where it applies (plan.use_blocks,
// plan.blocks) and fills the views' block offsets; called once the plan's
// views and sizes are set.
void plan_blocks(const gsr_ctx* ctx, RenderPlan& plan);
// Words of B.btab: per-block tile counts in kHistCopies copies, then the
// block table (kMaxBlocks uint4).
constexpr int64_t kBlockTabWords = (int64_t)kHistCopies * kMaxBlocks + 4 * kMaxBlocks;
// Binning by counting for this render (per-tile depth order, every view's
// tiles within the workgroup bins, the count matrix within its bound and,
// for a fixed buffer, within that buffer): its matrix size in words (tiles x
// workgroups per view) and the largest view's tile count, else false.
bool use_bins(const gsr_ctx* ctx, const Buffers& B, const RenderPlan& plan, int64_t* entries, int* max_view_tiles);
int size_instances(gsr_ctx* ctx, Buffers& B, const RenderPlan& plan);
void free_buffers(Buffers& B);
// Points ctx->na_bufs at the current device's static scratch of the
// allocation-free render (noalloc.hip).
int noalloc_attach(gsr_ctx* ctx);
// HIP error of the calling thread's last failed gsr_ipc_* call (ipc.hip).
int ipc_last_hip_error();
// Frees the captured mapping iteration and its buffers (iteration.hip).
void destroy_graph(gsr_ctx* ctx);
// Waits for every replay still being timed and adds its stage times to the
// context's accumulators (iteration.hip).
int harvest_graph(gsr_ctx* ctx);

}  // namespace gsr
