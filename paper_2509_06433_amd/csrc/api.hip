// Host side of the C ABI: argument checking, the context's device scratch,
// and the order of the kernel launches for render, backward, loss and Adam.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gsr.h"
#include "gsr_internal.h"

using namespace gsr;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Pinned staging slots for host->device uploads of small descriptor arrays;
// each slot is reused only after the event recorded behind its last copy.
constexpr int kSlots = 8;
constexpr size_t kSlotBytes = 64 * 1024;

}  // namespace

struct gsr_ctx {
  int tile_w = 16, tile_h = 16;
  int ppt = 1;                          // pixels per thread in the blend kernels
  float bg[3] = {0.f, 0.f, 0.f};
  float znear = 0.2f;
  int hip_err = 0;
  hipStream_t last_stream = nullptr;

  DevBuf views, images, images2, images3;
  DevBuf splats, rect, ntiles, zkey, svals, zkey_alt, svals_alt, offsets;
  DevBuf ikeys, ivals, ikeys_alt, ivals_alt;
  DevBuf hist, partials, ranges, tfinal, last, g2, lr, total, splat_out;
  uint32_t* host_total = nullptr;
  void* slots[kSlots] = {};
  hipEvent_t slot_ev[kSlots] = {};
  bool slot_used[kSlots] = {};
  int next_slot = 0;

  // state of the last render, checked by the backward
  bool have_forward = false;
  const float* fw_params = nullptr;
  int64_t fw_num = 0, fw_stride = 0;
  int fw_deg = 0;
  std::vector<gsr_camera> fw_cams;
  int64_t fw_instances = 0, fw_tiles = 0, fw_pixels = 0;
  std::vector<ViewDesc> fw_views;
  uint32_t* sorted_splats = nullptr;   // depth-sorted splat indices
  uint32_t* inst_keys = nullptr;       // sorted instance list
  uint32_t* inst_vals = nullptr;

  // per-stage timing
  uint32_t profile_mask = 0;          // bit k: time stage k
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[GSR_NUM_STAGES];
  DevBuf counts;
};

namespace {

#define HIP_TRY(ctx, expr)                      \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      (ctx)->hip_err = (int)e_;                 \
      return GSR_ERR_HIP;                       \
    }                                           \
  } while (0)

#define CHECK_LAUNCH(ctx) HIP_TRY(ctx, hipGetLastError())

int ensure(gsr_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return GSR_OK;
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
T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}

int upload(gsr_ctx* ctx, void* dev, const void* host, size_t bytes, hipStream_t st) {
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

// Brackets one stage's launches with events when profiling is on.
struct StageTimer {
  gsr_ctx* ctx;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(gsr_ctx* c, int s, hipStream_t stream) : ctx(c), stage(s), st(stream) {
    if (!((ctx->profile_mask >> s) & 1u)) return;
    a = take();
    b = take();
    if (a && b) (void)hipEventRecord(a, st);
  }
  hipEvent_t take() {
    if (!ctx->ev_pool.empty()) {
      hipEvent_t e = ctx->ev_pool.back();
      ctx->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~StageTimer() {
    if (!a || !b) return;
    (void)hipEventRecord(b, st);
    ctx->ev_pending[stage].emplace_back(a, b);
  }
};

#define RET_IF(expr)            \
  do {                          \
    int r_ = (expr);            \
    if (r_ != GSR_OK) return r_; \
  } while (0)

int check_gaussians(const gsr_gaussians* g) {
  if (!g) return GSR_ERR_INVALID;
  if (g->num < 0 || g->num > (int64_t(1) << 27)) return GSR_ERR_INVALID;
  if (g->stride < g->num) return GSR_ERR_INVALID;
  if (g->sh_degree < 0 || g->sh_degree > 3) return GSR_ERR_INVALID;
  if (g->num > 0 && !g->params) return GSR_ERR_INVALID;
  return GSR_OK;
}

int num_planes(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

int check_cams(const gsr_camera* cams, int32_t num_views) {
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

// Per-view descriptors; returns total tiles and pixels.
std::vector<ViewDesc> make_views(const gsr_ctx* ctx, const gsr_camera* cams, int nv, int64_t* tiles,
                                 int64_t* pixels) {
  std::vector<ViewDesc> out(nv);
  int64_t toff = 0, poff = 0;
  for (int v = 0; v < nv; ++v) {
    const gsr_camera& c = cams[v];
    ViewDesc& d = out[v];
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
    toff += (int64_t)d.tiles_x * d.tiles_y;
    poff += (int64_t)c.width * c.height;
  }
  *tiles = toff;
  *pixels = poff;
  return out;
}

int bits_for(int64_t max_key) {
  int b = 0;
  while (b < 32 && (int64_t(1) << b) <= max_key) ++b;
  return b;
}

int render_impl(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams, const gsr_image* out,
                hipStream_t st) {
  RET_IF(check_gaussians(g));
  RET_IF(check_cams(cams, nv));
  if (!out) return GSR_ERR_INVALID;
  for (int v = 0; v < nv; ++v)
    if (!out[v].rgb || !out[v].depth || !out[v].alpha) return GSR_ERR_INVALID;
  ctx->have_forward = false;
  ctx->last_stream = st;
  const int64_t N = g->num;
  const int64_t total = N * nv;
  if (total > (int64_t(1) << 31)) return GSR_ERR_INVALID;
  int64_t ntiles = 0, npix = 0;
  std::vector<ViewDesc> views = make_views(ctx, cams, nv, &ntiles, &npix);
  if (ntiles >= (int64_t(1) << 31)) return GSR_ERR_INVALID;
  std::vector<ViewImages> ims(nv);
  for (int v = 0; v < nv; ++v) ims[v] = ViewImages{out[v].rgb, out[v].depth, out[v].alpha};

  const size_t t4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(total, 1);
  RET_IF(ensure(ctx, ctx->views, sizeof(ViewDesc) * nv));
  RET_IF(ensure(ctx, ctx->images, sizeof(ViewImages) * nv));
  RET_IF(ensure(ctx, ctx->splats, sizeof(Splat) * (size_t)std::max<int64_t>(total, 1)));
  RET_IF(ensure(ctx, ctx->rect, sizeof(int4) * (size_t)std::max<int64_t>(total, 1)));
  RET_IF(ensure(ctx, ctx->ntiles, t4));
  RET_IF(ensure(ctx, ctx->zkey, t4));
  RET_IF(ensure(ctx, ctx->svals, t4));
  RET_IF(ensure(ctx, ctx->zkey_alt, t4));
  RET_IF(ensure(ctx, ctx->svals_alt, t4));
  RET_IF(ensure(ctx, ctx->offsets, t4));
  RET_IF(ensure(ctx, ctx->ranges, sizeof(uint2) * (size_t)ntiles));
  RET_IF(ensure(ctx, ctx->tfinal, sizeof(float) * (size_t)npix));
  RET_IF(ensure(ctx, ctx->last, sizeof(uint32_t) * (size_t)npix));
  RET_IF(ensure(ctx, ctx->total, 64));
  RET_IF(ensure(ctx, ctx->hist, sizeof(uint32_t) * (size_t)radix_scratch_elems(total)));
  RET_IF(ensure(ctx, ctx->partials, sizeof(uint32_t) * (size_t)scan_partial_elems(total)));

  RET_IF(upload(ctx, ctx->views.p, views.data(), sizeof(ViewDesc) * nv, st));
  RET_IF(upload(ctx, ctx->images.p, ims.data(), sizeof(ViewImages) * nv, st));

  launch_fill_u32(as<uint32_t>(ctx->total), 0u, 2, st);
  // projection (one thread per view x Gaussian)
  {
  StageTimer tm(ctx, GSR_STAGE_PROJECT, st);
  launch_project(g->params, N, g->stride, g->sh_degree, nv, as<ViewDesc>(ctx->views), ctx->tile_w, ctx->tile_h,
                 ctx->znear, as<Splat>(ctx->splats), as<int4>(ctx->rect), as<uint32_t>(ctx->ntiles),
                 as<uint32_t>(ctx->zkey), as<uint32_t>(ctx->svals), st);
  }
  CHECK_LAUNCH(ctx);
  // depth sort of the splats
  uint32_t* zk = as<uint32_t>(ctx->zkey);
  uint32_t* sv = as<uint32_t>(ctx->svals);
  uint32_t* zka = as<uint32_t>(ctx->zkey_alt);
  uint32_t* sva = as<uint32_t>(ctx->svals_alt);
  {
    StageTimer tm(ctx, GSR_STAGE_DEPTH_SORT, st);
    radix_sort_pairs(zk, sv, zka, sva, total, nullptr, 32, as<uint32_t>(ctx->hist), as<uint32_t>(ctx->total) + 1, st);
  }
  CHECK_LAUNCH(ctx);
  // instance offsets in depth order
  uint32_t* total_dev = as<uint32_t>(ctx->total);
  {
    StageTimer tm(ctx, GSR_STAGE_SCAN, st);
    scan_gather_exclusive(as<uint32_t>(ctx->ntiles), sv, as<uint32_t>(ctx->offsets), total, total_dev,
                          as<uint32_t>(ctx->partials), st);
  }
  CHECK_LAUNCH(ctx);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->host_total, total_dev, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  const int64_t I = (int64_t)ctx->host_total[0];
  if (ctx->host_total[1] != 0) return GSR_ERR_DEVICE;

  const size_t i4 = sizeof(uint32_t) * (size_t)std::max<int64_t>(I, 1);
  RET_IF(ensure(ctx, ctx->ikeys, i4));
  RET_IF(ensure(ctx, ctx->ivals, i4));
  RET_IF(ensure(ctx, ctx->ikeys_alt, i4));
  RET_IF(ensure(ctx, ctx->ivals_alt, i4));
  if (I >= (int64_t(1) << 30)) return GSR_ERR_CAPACITY;
  RET_IF(ensure(ctx, ctx->hist, sizeof(uint32_t) * (size_t)radix_scratch_elems(std::max(I, total))));

  uint32_t* ik = as<uint32_t>(ctx->ikeys);
  uint32_t* iv = as<uint32_t>(ctx->ivals);
  uint32_t* ika = as<uint32_t>(ctx->ikeys_alt);
  uint32_t* iva = as<uint32_t>(ctx->ivals_alt);
  {
    StageTimer tm(ctx, GSR_STAGE_EMIT, st);
    launch_emit(sv, as<uint32_t>(ctx->offsets), total_dev, as<int4>(ctx->rect), total, N, as<ViewDesc>(ctx->views),
                ctx->tile_w, ctx->tile_h, ik, iv, I, st);
  }
  CHECK_LAUNCH(ctx);
  {
    StageTimer tm(ctx, GSR_STAGE_TILE_SORT, st);
    radix_sort_pairs(ik, iv, ika, iva, I, nullptr, bits_for(ntiles - 1), as<uint32_t>(ctx->hist), total_dev + 1, st);
  }
  CHECK_LAUNCH(ctx);
  {
    StageTimer tm(ctx, GSR_STAGE_RANGES, st);
    launch_tile_ranges(ik, I, as<uint2>(ctx->ranges), ntiles, st);
  }
  CHECK_LAUNCH(ctx);

  BlendArgs ba{};
  ba.views = as<ViewDesc>(ctx->views);
  ba.images = as<ViewImages>(ctx->images);
  ba.num_views = nv;
  ba.num_tiles = (int32_t)ntiles;
  ba.ranges = as<uint2>(ctx->ranges);
  ba.inst_vals = iv;
  ba.splats = as<Splat>(ctx->splats);
  ba.tfinal = as<float>(ctx->tfinal);
  ba.last = as<uint32_t>(ctx->last);
  ba.g2 = nullptr;
  for (int k = 0; k < 3; ++k) ba.bg[k] = ctx->bg[k];
  {
    StageTimer tm(ctx, GSR_STAGE_BLEND_FWD, st);
    launch_blend_forward(ba, ctx->tile_w, ctx->tile_h, ctx->ppt, st);
  }
  CHECK_LAUNCH(ctx);

  ctx->have_forward = true;
  ctx->fw_params = g->params;
  ctx->fw_num = N;
  ctx->fw_stride = g->stride;
  ctx->fw_deg = g->sh_degree;
  ctx->fw_cams.assign(cams, cams + nv);
  ctx->fw_instances = I;
  ctx->fw_tiles = ntiles;
  ctx->fw_pixels = npix;
  ctx->fw_views = views;
  ctx->sorted_splats = sv;
  ctx->inst_keys = ik;
  ctx->inst_vals = iv;
  return GSR_OK;
}

int backward_impl(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams,
                  const gsr_image* grad_out, float* grad_params, hipStream_t st) {
  RET_IF(check_gaussians(g));
  RET_IF(check_cams(cams, nv));
  if (!grad_out || (g->num > 0 && !grad_params)) return GSR_ERR_INVALID;
  if (!ctx->have_forward || ctx->fw_params != g->params || ctx->fw_num != g->num || ctx->fw_stride != g->stride ||
      ctx->fw_deg != g->sh_degree || (int)ctx->fw_cams.size() != nv ||
      std::memcmp(ctx->fw_cams.data(), cams, sizeof(gsr_camera) * nv) != 0)
    return GSR_ERR_STATE;
  ctx->last_stream = st;
  const int64_t N = g->num;
  const int64_t total = N * nv;
  std::vector<ViewImages> ims(nv);
  for (int v = 0; v < nv; ++v) ims[v] = ViewImages{grad_out[v].rgb, grad_out[v].depth, grad_out[v].alpha};
  RET_IF(ensure(ctx, ctx->images2, sizeof(ViewImages) * nv));
  RET_IF(ensure(ctx, ctx->g2, sizeof(float) * G2_N * (size_t)std::max<int64_t>(total, 1)));
  RET_IF(upload(ctx, ctx->images2.p, ims.data(), sizeof(ViewImages) * nv, st));
  if (total == 0) return GSR_OK;
  {
    StageTimer tm(ctx, GSR_STAGE_ZERO, st);
    launch_fill_f32(as<float>(ctx->g2), 0.0f, total * G2_N, st);
  }
  CHECK_LAUNCH(ctx);
  BlendArgs ba{};
  ba.views = as<ViewDesc>(ctx->views);
  ba.images = as<ViewImages>(ctx->images2);
  ba.num_views = nv;
  ba.num_tiles = (int32_t)ctx->fw_tiles;
  ba.ranges = as<uint2>(ctx->ranges);
  ba.inst_vals = ctx->inst_vals;
  ba.splats = as<Splat>(ctx->splats);
  ba.tfinal = as<float>(ctx->tfinal);
  ba.last = as<uint32_t>(ctx->last);
  ba.g2 = as<float>(ctx->g2);
  for (int k = 0; k < 3; ++k) ba.bg[k] = ctx->bg[k];
  {
    StageTimer tm(ctx, GSR_STAGE_BLEND_BWD, st);
    launch_blend_backward(ba, ctx->tile_w, ctx->tile_h, ctx->ppt, st);
  }
  CHECK_LAUNCH(ctx);
  {
    StageTimer tm(ctx, GSR_STAGE_PROJECT_BWD, st);
    launch_project_backward(g->params, N, g->stride, g->sh_degree, nv, as<ViewDesc>(ctx->views), ctx->znear,
                            as<float>(ctx->g2), grad_params, st);
  }
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

}  // namespace

extern "C" {

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
    if (opt->batch_depth != 0 && opt->batch_depth != tw * th) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->tile_w = tw;
    ctx->tile_h = th;
    if (opt->pixels_per_thread < 0 || opt->pixels_per_thread > 2 ||
        (opt->pixels_per_thread == 2 && tw * th < 128)) {
      delete ctx;
      return GSR_ERR_UNSUPPORTED;
    }
    ctx->ppt = opt->pixels_per_thread == 0 ? 1 : opt->pixels_per_thread;
    for (int k = 0; k < 3; ++k) ctx->bg[k] = opt->bg[k];
    ctx->znear = opt->znear > 0.f ? opt->znear : 0.2f;
  }
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
  DevBuf* bufs[] = {&ctx->views, &ctx->images, &ctx->images2, &ctx->images3, &ctx->splats, &ctx->rect,
                    &ctx->ntiles, &ctx->zkey, &ctx->svals, &ctx->zkey_alt, &ctx->svals_alt, &ctx->offsets,
                    &ctx->ikeys, &ctx->ivals, &ctx->ikeys_alt, &ctx->ivals_alt, &ctx->hist, &ctx->partials,
                    &ctx->ranges, &ctx->tfinal, &ctx->last, &ctx->g2, &ctx->lr, &ctx->total, &ctx->splat_out,
                    &ctx->counts};
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
    launch_loss_l1(dv, da, db, dc, num_views, maxpix, depth_weight, loss, st);
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
    launch_adam(params, grads, m, v, num, stride, num_planes, as<float>(ctx->lr), beta1, beta2, eps, bc1, bc2, st);
  }
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

int gsr_query_status(gsr_ctx* ctx, int64_t* num_instances, int64_t* num_visible, int64_t* num_tiles) {
  if (!ctx) return GSR_ERR_INVALID;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  if (ctx->total.p) {
    uint32_t flag = 0;
    HIP_TRY(ctx, hipMemcpy(&flag, as<uint32_t>(ctx->total) + 1, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (flag) return GSR_ERR_DEVICE;
  }
  if (num_instances) *num_instances = ctx->have_forward ? ctx->fw_instances : 0;
  if (num_visible) *num_visible = -1;
  if (num_tiles) *num_tiles = ctx->have_forward ? ctx->fw_tiles : 0;
  return GSR_OK;
}

int gsr_copy_instances(gsr_ctx* ctx, uint32_t* tile, uint32_t* gid, int64_t capacity, int64_t* count) {
  if (!ctx || !count || capacity < 0) return GSR_ERR_INVALID;
  if (!ctx->have_forward) return GSR_ERR_STATE;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  const int64_t I = ctx->fw_instances;
  *count = I;
  const int64_t m = std::min(capacity, I);
  if (m == 0) return GSR_OK;
  if (!tile || !gid) return GSR_ERR_INVALID;
  HIP_TRY(ctx, hipMemcpy(tile, ctx->inst_keys, sizeof(uint32_t) * m, hipMemcpyDeviceToHost));
  HIP_TRY(ctx, hipMemcpy(gid, ctx->inst_vals, sizeof(uint32_t) * m, hipMemcpyDeviceToHost));
  const uint32_t N = (uint32_t)ctx->fw_num;
  for (int64_t k = 0; k < m; ++k) gid[k] = gid[k] % N;
  return GSR_OK;
}

int gsr_copy_splats(gsr_ctx* ctx, int32_t view, float* out, int64_t num) {
  if (!ctx || !out) return GSR_ERR_INVALID;
  if (!ctx->have_forward) return GSR_ERR_STATE;
  if (view < 0 || view >= (int)ctx->fw_cams.size() || num != ctx->fw_num) return GSR_ERR_INVALID;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  if (num == 0) return GSR_OK;
  hipStream_t st = ctx->last_stream;
  RET_IF(ensure(ctx, ctx->splat_out, sizeof(float) * 16 * (size_t)num));
  const int64_t off = (int64_t)view * num;
  launch_export_splats(ctx->fw_params, num, ctx->fw_stride, as<ViewDesc>(ctx->views) + view, ctx->znear,
                       as<Splat>(ctx->splats) + off, as<int4>(ctx->rect) + off, as<float>(ctx->splat_out), st);
  CHECK_LAUNCH(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(st));
  HIP_TRY(ctx, hipMemcpy(out, ctx->splat_out.p, sizeof(float) * 16 * (size_t)num, hipMemcpyDeviceToHost));
  return GSR_OK;
}

int gsr_count_work(gsr_ctx* ctx, int64_t* pairs, int64_t* visible, int32_t num_views) {
  if (!ctx || !pairs) return GSR_ERR_INVALID;
  if (!ctx->have_forward) return GSR_ERR_STATE;
  if (visible && num_views != (int32_t)ctx->fw_cams.size()) return GSR_ERR_INVALID;
  hipStream_t st = ctx->last_stream;
  const int nv = (int)ctx->fw_cams.size();
  RET_IF(ensure(ctx, ctx->counts, sizeof(unsigned long long) * (size_t)(1 + nv)));
  unsigned long long* c = as<unsigned long long>(ctx->counts);
  launch_count_work(as<uint32_t>(ctx->last), ctx->fw_pixels, as<uint32_t>(ctx->ntiles), ctx->fw_num, nv, c, st);
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
  double sum = 0.0;
  auto& v = ctx->ev_pending[stage];
  for (auto& pr : v) {
    HIP_TRY(ctx, hipEventSynchronize(pr.second));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, pr.first, pr.second));
    sum += ms;
  }
  *total_ms = sum;
  if (launches) *launches = (int64_t)v.size();
  if (reset) {
    for (auto& pr : v) {
      ctx->ev_pool.push_back(pr.first);
      ctx->ev_pool.push_back(pr.second);
    }
    v.clear();
  }
  return GSR_OK;
}

int gsr_last_hip_error(gsr_ctx* ctx) { return ctx ? ctx->hip_err : 0; }

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
