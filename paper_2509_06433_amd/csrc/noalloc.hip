// Allocation-free forward render (gsr_render_noalloc).
//
// The same kernels as gsr_render, with every piece of device scratch taken
// from one file-scope array, `scratch`, instead of context-owned buffers that
// grow on demand, and with the instance storage at a fixed capacity instead
// of sized from a first pass. So the call makes no device allocation and no
// synchronisation. The array holds the buffers of a render at the limits
// below; each GPU the library runs on has its own copy, for the life of the
// process, shared by every context on that GPU.

#include <mutex>

#include "context.h"

using namespace gsr;

namespace {

constexpr int64_t kNaMaxSplats = int64_t(1) << 18;      // Gaussians x views
constexpr int64_t kNaMaxInstances = int64_t(1) << 21;   // (tile, Gaussian) instances over all views
constexpr int64_t kNaMaxPixels = int64_t(1) << 20;      // over all views
constexpr int64_t kNaMaxTiles = int64_t(1) << 15;       // over all views
constexpr int kNaMaxViews = 16;
// count matrix of the binning by counting (tiles x workgroups per view);
// larger renders take the radix path
constexpr int64_t kNaMaxBinEntries = int64_t(1) << 20;
constexpr size_t kNaBytes = size_t(88) << 20;

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Device address of each device's copy of `scratch`, looked up once per
// device. In host code `scratch` names a host-side stand-in, not device
// memory: only these addresses are ever handed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Carves the buffers of a forward render at the limits out of [base, base +
// kNaBytes); false if they do not fit.
bool carve(unsigned char* base, Buffers& B) {
  size_t off = 0;
  bool ok = true;
  auto take = [&](DevBuf& b, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    b.p = base + off;
    b.cap = bytes;
    b.fixed = true;
    off += bytes;
    ok = ok && off <= kNaBytes;
  };
  const size_t u4 = sizeof(uint32_t);
  int64_t hist2 = block_sort_scratch_elems(kNaMaxInstances);
  for (int bits = 0; bits <= 15; ++bits) hist2 = std::max(hist2, radix_scratch_elems(kNaMaxInstances, bits));
  take(B.views, sizeof(ViewDesc) * kNaMaxViews);
  take(B.images, sizeof(ViewImages) * kNaMaxViews);
  take(B.splats, sizeof(Splat) * kNaMaxSplats);
  take(B.rect, sizeof(int4) * kNaMaxSplats);
  take(B.ntiles, u4 * kNaMaxSplats);
  take(B.zkey, u4 * kNaMaxSplats);
  take(B.svals, u4 * kNaMaxSplats);
  take(B.zkey_alt, u4 * kNaMaxSplats);
  take(B.svals_alt, u4 * kNaMaxSplats);
  take(B.offsets, u4 * kNaMaxSplats);
  take(B.ikeys, u4 * kNaMaxInstances);
  take(B.ivals, u4 * kNaMaxInstances);
  take(B.ikeys_alt, u4 * kNaMaxInstances);
  take(B.ivals_alt, u4 * kNaMaxInstances);
  take(B.bkeys, u4 * kNaMaxInstances);
  take(B.bvals, u4 * kNaMaxInstances);
  take(B.btab, u4 * (size_t)kBlockTabWords);
  take(B.hist2, u4 * (size_t)hist2);
  take(B.block_rank, u4 * (size_t)emit_plan_elems(kNaMaxInstances));
  take(B.ranges, sizeof(uint2) * kNaMaxTiles);
  take(B.order, u4 * kNaMaxTiles);
  take(B.tile_last, u4 * kNaMaxTiles);
  take(B.tfinal, sizeof(float) * kNaMaxPixels);
  take(B.last, u4 * kNaMaxPixels);
  take(B.total, 64);
  // the scratch sizes of the depth sort and the scans grow with the splat
  // count up to this limit (one sort chunk size below 2^19 elements)
  take(B.hist, u4 * (size_t)radix_scratch_elems(kNaMaxSplats, 32));
  take(B.bins, u4 * (size_t)kNaMaxBinEntries);
  take(B.partials, 2 * u4 * (size_t)scan_partial_elems(std::max(kNaMaxSplats, kNaMaxBinEntries)));
  return ok;
}

}  // namespace

namespace gsr {

// Set-up of the allocation-free render for the current device (called by
// gsr_create): the device address of this device's `scratch` (looked up the
// first time a context is created on the device) and the buffers carved from
// it. On failure the context works as before and gsr_render_noalloc reports
// GSR_ERR_UNSUPPORTED.
int noalloc_attach(gsr_ctx* ctx) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return GSR_ERR_HIP;
  }
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return GSR_ERR_HIP;
      }
      g_ptr[dev] = p;
    }
    ptr = g_ptr[dev];
  }
  if (!carve(static_cast<unsigned char*>(ptr), ctx->na_bufs)) return GSR_ERR_UNSUPPORTED;
  ctx->na_device = dev;
  ctx->na_plan.views.reserve(kNaMaxViews);
  return GSR_OK;
}

}  // namespace gsr

namespace {

int render_noalloc_impl(gsr_ctx* ctx, const gsr_gaussians* g, int32_t nv, const gsr_camera* cams,
                        const gsr_image* out, hipStream_t st) {
  if (!ctx->na_bufs.total.p) return GSR_ERR_UNSUPPORTED;
  int dev = -1;
  HIP_TRY(ctx, hipGetDevice(&dev));
  if (dev != ctx->na_device) return GSR_ERR_INVALID;
  RET_IF(check_gaussians(g));
  RET_IF(check_cams(cams, nv));
  if (!out) return GSR_ERR_INVALID;
  if (nv > kNaMaxViews) return GSR_ERR_CAPACITY;
  for (int v = 0; v < nv; ++v)
    if (!out[v].rgb || !out[v].depth || !out[v].alpha) return GSR_ERR_INVALID;
  // the plan, without host allocation (its view array has room for every view)
  RenderPlan& P = ctx->na_plan;
  P.num = g->num;
  P.stride = g->stride;
  P.deg = g->sh_degree;
  P.nv = nv;
  P.total = g->num * nv;
  P.views.resize(nv);
  int64_t ntiles = 0, npix = 0;
  for (int v = 0; v < nv; ++v) {
    ViewDesc& d = P.views[v];
    fill_view(ctx, cams[v], ntiles, npix, d);
    ntiles += (int64_t)d.tiles_x * d.tiles_y;
    npix += (int64_t)cams[v].width * cams[v].height;
  }
  P.ntiles = ntiles;
  P.npix = npix;
  plan_blocks(ctx, P);
  if (P.total > kNaMaxSplats || P.npix > kNaMaxPixels || P.ntiles > kNaMaxTiles) return GSR_ERR_CAPACITY;
  P.capacity = kNaMaxInstances;
  P.forward_only = true;
  P.sorted_splats = P.inst_keys = P.inst_vals = nullptr;
  Buffers& B = ctx->na_bufs;
  ViewImages ims[kNaMaxViews];
  for (int v = 0; v < nv; ++v) ims[v] = ViewImages{out[v].rgb, out[v].depth, out[v].alpha};
  ctx->last_stream = st;
  // from here on the shared scratch is overwritten
  ctx->q_bufs = nullptr;
  ctx->q_plan = nullptr;
  RET_IF(upload(ctx, B.views.p, P.views.data(), sizeof(ViewDesc) * nv, st));
  RET_IF(upload(ctx, B.images.p, ims, sizeof(ViewImages) * nv, st));
  // the stage timers would create events: none in this call
  const uint32_t mask = ctx->profile_mask;
  ctx->profile_mask = 0;
  ClearList L{};
  front_clears(ctx, B, P, L);
  back_clears(B, P, L);
  launch_clear(L, st);
  int r = GSR_OK;
  if (hipGetLastError() != hipSuccess) r = GSR_ERR_HIP;
  if (r == GSR_OK) r = launch_front(ctx, B, P, g->params, st);
  if (r == GSR_OK) r = launch_back(ctx, B, P, st);
  ctx->profile_mask = mask;
  RET_IF(r);
  ctx->q_bufs = &B;
  ctx->q_plan = &P;
  ctx->q_params = g->params;
  return GSR_OK;
}

}  // namespace

extern "C" int gsr_render_noalloc(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views, const gsr_camera* cams,
                                  const gsr_image* out, void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  try {
    return render_noalloc_impl(ctx, g, num_views, cams, out, (hipStream_t)stream);
  } catch (...) {
    return GSR_ERR_INVALID;
  }
}
