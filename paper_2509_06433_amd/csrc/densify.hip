// Keyframe insertion: new Gaussians seeded from an RGB-D keyframe and
// appended to the map (gsr_densify).
//
// The mapping loop adds Gaussians where a new keyframe observes surface the
// map does not yet cover (paper Fig. "GS_SLAM": keyframe management feeds the
// map). On a grid of every step-th pixel, a pixel seeds one Gaussian when its
// observed depth is valid and the current map's rendered alpha there is below
// a threshold. The Gaussian sits at the pixel centre's back-projection to that
// depth, isotropic with a standard deviation proportional to the depth times
// the grid spacing over the focal length (the footprint of a grid cell),
// rotation identity, a given opacity logit, and the observed colour in its
// degree-0 spherical-harmonic coefficient (higher degrees zero). New
// Gaussians are appended in pixel order (row-major over the grid) after the
// existing ones, up to the buffer's capacity.

#include "context.h"

using namespace gsr;

namespace {

constexpr float kShC0 = 0.28209479177387814f;   // Y_00 = 1 / (2 sqrt(pi))

struct SeedArgs {
  const float* rgb;        // [3][H][W]
  const float* depth;      // [H][W]
  const float* coverage;   // [H][W] or null
  int width, height, step, gw, gh;
  float depth_min, depth_max, alpha_below;
};

__device__ __forceinline__ bool seeds(const SeedArgs& s, int m, int& px, int& py, float& d) {
  const int gx = m % s.gw, gy = m / s.gw;
  px = gx * s.step;
  py = gy * s.step;
  const int64_t p = (int64_t)py * s.width + px;
  d = s.depth[p];
  if (!(d >= s.depth_min) || !(d <= s.depth_max)) return false;       // false for NaN
  if (s.coverage && !(s.coverage[p] < s.alpha_below)) return false;
  return true;
}

__global__ void __launch_bounds__(256) seed_flags_kernel(SeedArgs s, uint32_t* __restrict__ flags, int64_t m_total) {
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < m_total; m += (int64_t)gridDim.x * blockDim.x) {
    int px, py;
    float d;
    flags[m] = seeds(s, (int)m, px, py, d) ? 1u : 0u;
  }
}

__global__ void __launch_bounds__(256) seed_write_kernel(SeedArgs s, const uint32_t* __restrict__ flags,
                                                         const uint32_t* __restrict__ offsets, int64_t m_total,
                                                         ViewDesc V, float* __restrict__ P, int64_t stride,
                                                         int64_t num, int64_t capacity, int deg, float scale_factor,
                                                         float logit) {
  const int K = (deg + 1) * (deg + 1);
  const float fmean = 0.5f * (V.fx + V.fy);
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < m_total; m += (int64_t)gridDim.x * blockDim.x) {
    if (!flags[m]) continue;
    const int64_t i = num + (int64_t)offsets[m];
    if (i >= capacity) continue;
    int px, py;
    float d;
    seeds(s, (int)m, px, py, d);
    // camera-space point on the pixel centre's ray at depth d, then to world:
    // x_world = R^T (x_cam - t)
    const float xc = ((float)px + 0.5f - V.cx) / V.fx * d;
    const float yc = ((float)py + 0.5f - V.cy) / V.fy * d;
    const float q[3] = {xc - V.t[0], yc - V.t[1], d - V.t[2]};
#pragma unroll
    for (int j = 0; j < 3; ++j) P[j * stride + i] = V.R[0 * 3 + j] * q[0] + V.R[1 * 3 + j] * q[1] + V.R[2 * 3 + j] * q[2];
    const float ls = logf(scale_factor * d * (float)s.step / fmean);
#pragma unroll
    for (int j = 0; j < 3; ++j) P[(3 + j) * stride + i] = ls;
    P[6 * stride + i] = 1.0f;
    P[7 * stride + i] = 0.0f;
    P[8 * stride + i] = 0.0f;
    P[9 * stride + i] = 0.0f;
    P[10 * stride + i] = logit;
    const int64_t HW = (int64_t)s.width * s.height;
    const int64_t p = (int64_t)py * s.width + px;
#pragma unroll
    for (int c = 0; c < 3; ++c) P[(11 + c) * stride + i] = (s.rgb[c * HW + p] - 0.5f) / kShC0;
    for (int k = 1; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) P[(11 + 3 * k + c) * stride + i] = 0.0f;
  }
}

int grid_blocks(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

int densify_impl(gsr_ctx* ctx, float* params, int64_t num, int64_t stride, int32_t deg, const gsr_camera* cam,
                 const float* rgb, const float* depth, const float* coverage, const gsr_densify_options* opt,
                 int64_t* appended, int64_t* wanted, hipStream_t st) {
  if (!params || !cam || !rgb || !depth || !opt || !appended) return GSR_ERR_INVALID;
  if (num < 0 || stride < num || stride > (int64_t(1) << 27) || deg < 0 || deg > 3) return GSR_ERR_INVALID;
  RET_IF(check_cams(cam, 1));
  if (opt->step < 1 || !(opt->scale_factor > 0.f) || !(opt->depth_max >= opt->depth_min)) return GSR_ERR_INVALID;
  SeedArgs s;
  s.rgb = rgb;
  s.depth = depth;
  s.coverage = coverage;
  s.width = cam->width;
  s.height = cam->height;
  s.step = opt->step;
  s.gw = (cam->width + opt->step - 1) / opt->step;
  s.gh = (cam->height + opt->step - 1) / opt->step;
  s.depth_min = opt->depth_min;
  s.depth_max = opt->depth_max;
  s.alpha_below = opt->alpha_below;
  const int64_t M = (int64_t)s.gw * s.gh;
  ctx->last_stream = st;
  RET_IF(ensure(ctx, ctx->seed_buf, sizeof(uint32_t) * (size_t)(2 * M + 2 * scan_partial_elems(M) + 8)));
  uint32_t* flags = as<uint32_t>(ctx->seed_buf);
  uint32_t* offs = flags + M;
  uint32_t* total = offs + M;
  uint32_t* scratch = total + 8;
  ViewDesc V;
  fill_view(ctx, *cam, 0, 0, V);
  ClearList L{};
  L.add(total, 8);
  L.add(scratch, 2 * scan_partial_elems(M));
  launch_clear(L, st);
  seed_flags_kernel<<<grid_blocks(M), 256, 0, st>>>(s, flags, M);
  CHECK_LAUNCH(ctx);
  scan_gather_exclusive(flags, nullptr, offs, M, nullptr, total, scratch, total + 1, false, st);
  CHECK_LAUNCH(ctx);
  seed_write_kernel<<<grid_blocks(M), 256, 0, st>>>(s, flags, offs, M, V, params, stride, num, stride, deg,
                                                    opt->scale_factor, opt->opacity_logit);
  CHECK_LAUNCH(ctx);
  uint32_t h[2] = {0, 0};
  HIP_TRY(ctx, hipMemcpyAsync(h, total, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (h[1]) return GSR_ERR_DEVICE;
  if (wanted) *wanted = (int64_t)h[0];
  *appended = std::min<int64_t>((int64_t)h[0], stride - num);
  return GSR_OK;
}

}  // namespace

extern "C" int gsr_densify(gsr_ctx* ctx, float* params, int64_t num, int64_t stride, int32_t sh_degree,
                           const gsr_camera* cam, const float* rgb, const float* depth, const float* coverage,
                           const gsr_densify_options* opt, int64_t* appended, int64_t* wanted, void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  try {
    return densify_impl(ctx, params, num, stride, sh_degree, cam, rgb, depth, coverage, opt, appended, wanted,
                        (hipStream_t)stream);
  } catch (...) {
    return GSR_ERR_INVALID;
  }
}
