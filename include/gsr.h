/*
 * gsr.h -- C ABI of the MI355X (gfx950) differentiable Gaussian rasterizer.
 *
 * The library renders a map of anisotropic 3D Gaussians (mean, covariance from
 * scale and rotation, opacity, spherical-harmonic colour; paper Sec. II-A) into
 * RGB, depth and alpha images, and back-propagates image gradients to the
 * Gaussian parameters, as the renderer that drives the continuous mapping
 * optimisation of a Gaussian-splatting SLAM system does (paper Sec. II-B,
 * Fig. "GS_SLAM", renderer I1). The paper gives no formula; the image
 * formation is EWA splatting with front-to-back alpha compositing: alpha is
 * clamped to 0.99, alphas below 1/255 are skipped and a pixel stops
 * (without compositing the Gaussian that would cross it) once its
 * transmittance would fall below 1e-4.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All pointers named "device" are HIP device memory on the current device;
 *   all others are host memory, read during the call only.
 * - `stream` is a hipStream_t (0 = legacy default stream). Every call is
 *   asynchronous on that stream unless stated otherwise; the context keeps
 *   device scratch that later calls on the same context reuse, so one context
 *   must not be used from two streams at the same time.
 * - Return value: GSR_OK (0) or a negative gsr_status. No C++ exception
 *   crosses this boundary. After GSR_ERR_HIP the HIP error code is available
 *   from gsr_last_hip_error().
 *
 * Parameter layout ("the map"), float32, planar structure-of-arrays [P][stride]:
 *   planes 0..2   mean x, y, z (world)
 *   planes 3..5   log-scale of the three local axes (scale = exp)
 *   planes 6..9   rotation quaternion (w, x, y, z), unnormalised
 *   plane  10     opacity logit (opacity = sigmoid)
 *   plane  11+3k+c  real spherical-harmonic coefficient k (k = l^2 + l + m,
 *                 Condon-Shortley phase), colour channel c
 *   P = 11 + 3 (sh_degree + 1)^2; colour = max(0, sum_k coef_k Y_k(dir) + 0.5)
 *   where dir is the unit vector from the camera centre to the mean.
 *
 * Cameras: world-to-camera rotation R (row-major) and translation t, OpenCV
 * axes (x right, y down, z forward), pinhole fx, fy, cx, cy; pixel (px, py)
 * is sampled at (px + 0.5, py + 0.5).
 *
 * Images: per view, planar float32 rgb [3][H][W], depth [H][W] (sum of
 * weights times camera-space z of each mean), alpha [H][W] (1 - final
 * transmittance); rgb includes final transmittance times the background.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GSR_OK = 0,
  GSR_ERR_INVALID = -1,      /* bad argument (null pointer, size, degree ...) */
  GSR_ERR_OOM = -2,          /* device allocation failed */
  GSR_ERR_HIP = -3,          /* a HIP runtime call failed */
  GSR_ERR_STATE = -4,        /* call order violated (backward without matching forward) */
  GSR_ERR_CAPACITY = -5,     /* fixed-capacity scratch too small (mapping iteration) */
  GSR_ERR_UNSUPPORTED = -6, /* option not supported by the library */
  GSR_ERR_DEVICE = -7        /* a bounded device-side wait expired; the call's results are invalid */
} gsr_status;

typedef struct gsr_ctx gsr_ctx;

typedef struct {
  int32_t tile_w, tile_h;   /* screen tile; 0 = 16 x 16. Supported: 16x16, 16x8, 8x8, 32x8 */
  int32_t batch_depth;      /* Gaussians staged in LDS per batch of the backward: 0 (default:
                               32 for workgroups of 256 threads, else 64), 16, 32 or 64
                               (capped at the workgroup's thread count). The forward stages
                               one Gaussian per thread. */
  float bg[3];              /* background colour; default 0 */
  float znear;              /* near-plane cull distance; <= 0 means 0.2 */
  int32_t pixels_per_thread; /* blend kernels: 0 = default (1), 1, or 2 (tiles of >= 128 pixels) */
  int32_t tile_order;       /* order in which blend workgroups take tiles: 0 = automatic (longest
                               list first when several views are rendered together, else
                               tile order), 1 = longest list first, 2 = tile order, 3 = balanced:
                               tiles sorted by weight (the walk length the previous render of
                               the same buffers recorded, else the list length) and dealt to
                               the CUs in snake order, so each CU starts with heavy and light
                               tiles (at most 8192 tiles, else as 1). Images are identical. */
  int32_t chunk_len;        /* work unit of the blend backward, in list positions: 0 = automatic
                               (chunks of 128 when a launch covers fewer than 4096 tiles, else
                               whole lists), -1 = whole tile lists, else a multiple of 16 up to
                               2^20. With chunks, the forward records each pixel's transmittance
                               and its colour and depth composited per chunk, so the chunks of
                               one tile are walked in reverse by independent workgroups. */
  int32_t max_chunks;       /* chunks per tile: 0 = default (4), else 1 .. 64; the last chunk
                               takes the rest of the list */
  int32_t fuse_blend;       /* mapping iteration: 0 = automatic (fused when the backward is
                               chunked, the batch depth is the default and the device holds
                               every tile's forward workgroup at once), 1 = fused whenever the
                               batch depth is the default, -1 = never. Fused, the blend forward
                               and backward are one launch: each tile's workgroup composites it
                               and walks its first chunk back, the later chunks' workgroups
                               wait for the tile's forward, so they fill the forward's tail.
                               Images and loss are identical to the two launches. */
  int32_t depth_sort;       /* 0 = automatic (per tile when the views hold at most 2^19 splats,
                               N x views, else once globally), 1 = each tile's list is sorted by
                               depth after binning (the splats are binned in index order),
                               2 = all visible splats are sorted by depth once before binning.
                               The lists are identical. */
  int32_t backward_schedule; /* blend backward: 0 = pixel-parallel (default: a thread per pixel
                               walks its list in reverse; per-Gaussian sums reduced over each
                               wavefront and workgroup before the atomics), 1 = splat-parallel
                               (a wavefront per tile, a Gaussian per lane, the tile's pixels
                               streamed through the lanes; one set of atomics per (tile,
                               Gaussian); the lists are walked whole, so chunk_len and
                               fuse_blend do not apply). Same gradient up to float summation
                               order. */
  int32_t binning;          /* grouping of the instances by tile: 0 = automatic (3 where it applies
                               with blocks of at least two tiles, else 2), 1 = by counting where each tile's list is sorted by
                               depth afterwards and every view has at most 8192 tiles
                               (per-workgroup tile counts in LDS, one scan, a scatter; equal
                               depths then ordered by index), else as 2; 2 = emission of one
                               instance per (splat, tile) in splat order and a radix sort of the
                               tile keys; 3 = by blocks of tiles where each tile's list is
                               sorted by depth afterwards and the views' tiles fit in 256
                               blocks of at most 8 x 8 tiles (one instance per (splat, block),
                               one 8-bit radix pass over the block ids, then each tile's
                               workgroup keeps the instances of its block that cover it and
                               sorts them by depth), else as 2. The lists are identical. */
} gsr_options;

typedef struct {
  float R[9];               /* world -> camera rotation, row-major */
  float t[3];               /* world -> camera translation */
  float fx, fy, cx, cy;     /* pinhole intrinsics, pixels */
  int32_t width, height;    /* image size, 1 .. 16384 each */
} gsr_camera;

typedef struct {
  const float* params;      /* device [P][stride] float32, layout above */
  int64_t num;              /* N Gaussians, 0 .. 2^27 */
  int64_t stride;           /* floats between planes, >= num */
  int32_t sh_degree;        /* 0 .. 3 */
} gsr_gaussians;

typedef struct {
  float* rgb;               /* device [3][H][W] */
  float* depth;             /* device [H][W] */
  float* alpha;             /* device [H][W] */
} gsr_image;

/* Create a context with the given options (NULL = defaults). *out receives
 * the handle. The context owns all device scratch (projected splats, sort
 * buffers, tile ranges, per-pixel backward state, screen-space gradient
 * accumulators); it grows on demand and is freed by gsr_destroy. */
int gsr_create(gsr_ctx** out, const gsr_options* opt);

/* Free the context and its device scratch (synchronises the device first).
 * NULL is ignored. */
void gsr_destroy(gsr_ctx* ctx);

/* Forward render of num_views views (>= 1) of the same map: EWA projection
 * of every Gaussian into every view, tile binning, depth-keyed radix sort of
 * the (tile, Gaussian) instances, front-to-back compositing per tile.
 * cams[num_views] host; out[num_views] host array of device image pointers.
 * Keeps what render_backward needs (per-pixel final transmittance and
 * last-composited index, the sorted instance lists) in the context.
 * Synchronises `stream` once to size the instance buffers. */
int gsr_render(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views,
               const gsr_camera* cams, const gsr_image* out, void* stream);

/* Single-view convenience form: gsr_render with num_views = 1. */
int gsr_render1(gsr_ctx* ctx, const gsr_gaussians* g, const gsr_camera* cam,
                const gsr_image* out, void* stream);

/* Allocation-free forward render, for callers that cannot allocate device
 * memory or wait on the device inside the call: code under HIP graph capture,
 * tight serving loops (a viewer rendering frames of a live map), harnesses
 * that forbid hipMalloc. Same arguments, kernels and images as gsr_render
 * (bit for bit), but every piece of device scratch comes from one static
 * array of 88 MiB in the library (a copy per GPU, held until the process
 * ends, set up by gsr_create), the instance storage has a fixed capacity, and
 * the call neither allocates (device or host) nor synchronises: it is
 * asynchronous on `stream` like the launches it makes.
 * Limits: num * num_views <= 2^18 splats, <= 2^20 pixels and <= 2^15 tiles
 * over all views, <= 16 views (else GSR_ERR_CAPACITY, nothing launched);
 * <= 2^21 (tile, Gaussian) instances, checked on the device: a render that
 * needs more leaves its images invalid, and gsr_query_status (which
 * synchronises) then returns GSR_ERR_CAPACITY with the required count.
 * The context must be used on the device it was created on (else
 * GSR_ERR_INVALID); GSR_ERR_UNSUPPORTED if its scratch could not be set up.
 * Every context on a GPU shares that GPU's scratch: two calls that overlap
 * in time on one GPU (other streams, other threads or contexts) race and
 * corrupt each other's images. It leaves gsr_render_backward referring to
 * the last gsr_render; the status, instance and work queries report on this
 * render until the next render call. */
int gsr_render_noalloc(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views,
                       const gsr_camera* cams, const gsr_image* out, void* stream);

/* Backward of the last gsr_render on this context: given dL/d(rgb, depth,
 * alpha) per view (grad_out[num_views], device pointers; a NULL plane means
 * zero), ADDS dL/dparams to grad_params (device [P][stride] float32, same
 * stride as g). g, num_views and cams must equal those of the last render
 * (else GSR_ERR_STATE). Per-pixel transmittance is recomputed in reverse
 * order from the stored final value; screen-space gradients are reduced
 * across each wavefront and workgroup before global atomics; gradients of
 * all views are summed. */
int gsr_render_backward(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views,
                        const gsr_camera* cams, const gsr_image* grad_out,
                        float* grad_params, void* stream);

/* Backward of the last gsr_render with respect to the cameras as well: the
 * gradient that tracking against a single map needs (paper Sec. II-B: SLAM
 * systems that track and map on the same Gaussian map). Same image gradients,
 * call order and GSR_ERR_STATE rule as gsr_render_backward.
 *   grad_params  device [P][stride] float32, += dL/dparams; NULL = not formed
 *   grad_cams    device [num_views][12] float64, += per view dL/dR (the nine
 *                entries of gsr_camera.R, row-major, each taken as free) and
 *                dL/dt (gsr_camera.t), for x_cam = R x + t. R acts through the
 *                camera-space means, the screen covariance J R Sigma R^T J^T
 *                and, for view-dependent colour (sh_degree >= 1), the camera
 *                centre -R^T t. Required.
 *   grad_twist   device [num_views][6] float64 or NULL: += the gradient with
 *                respect to a left perturbation of the pose, [R | t] <-
 *                exp(xi^) [R | t] with xi = (rho, phi) (rho translation, phi
 *                rotation vector): dL/drho = dL/dt, dL/dphi = (A21 - A12,
 *                A02 - A20, A10 - A01) with A = dL/dR R^T + dL/dt t^T.
 * Each view's sums are formed per workgroup in double and added with float64
 * atomics (the order of the additions varies from call to call). */
int gsr_render_backward_pose(gsr_ctx* ctx, const gsr_gaussians* g, int32_t num_views,
                             const gsr_camera* cams, const gsr_image* grad_out, float* grad_params,
                             double* grad_cams, double* grad_twist, void* stream);

/* Mapping loss of one or more rendered views against targets:
 *   L = sum_v [ mean|rgb_v - rgb*_v| + depth_weight * mean|depth_v - depth*_v| ]
 * (means over 3HW and HW; sign(0) = 0). Writes dL/drgb and dL/ddepth into
 * grad_out[v].rgb / .depth (device, overwritten; .alpha if non-NULL is set
 * to 0) and, if loss is not NULL, the scalar L into loss (device float,
 * overwritten). rendered/target/grad_out are host arrays of num_views
 * device-image descriptors (target alpha unused). */
int gsr_loss_l1(gsr_ctx* ctx, int32_t num_views, const gsr_camera* cams,
                const gsr_image* rendered, const gsr_image* target, float depth_weight,
                const gsr_image* grad_out, float* loss, void* stream);

/* One Adam step (bias-corrected, step >= 1) over P planes of `num` floats
 * with plane stride `stride` (device params, grads, m, v; params, m, v
 * updated in place):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr[plane] * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * lr_per_plane: host [num_planes]. */
int gsr_adam_step(gsr_ctx* ctx, float* params, const float* grads, float* m, float* v,
                  int64_t num, int64_t stride, int32_t num_planes, const float* lr_per_plane,
                  float beta1, float beta2, float eps, int32_t step, void* stream);

/* Optimiser of a mapping iteration: Adam over every parameter plane. */
typedef struct {
  float* m;                   /* device [P][stride] first moments, updated in place */
  float* v;                   /* device [P][stride] second moments, updated in place */
  const float* lr_per_plane;  /* host [P] learning rate of each parameter plane */
  float beta1, beta2, eps;
  int32_t step;               /* > 0: this call's update is Adam step `step` and the
                                 context's step count restarts there; 0: continue the
                                 count kept on the device (one per completed update) */
} gsr_adam;

/* One mapping iteration of the continuous map optimisation (paper Sec. II-B,
 * mapping thread): forward render of num_views views, the L1 loss of
 * gsr_loss_l1 against `targets`, the backward to the parameters and, if adam
 * is not NULL, one Adam update of params (in place) -- the whole iteration
 * enqueued on `stream` as one replay of a HIP graph, with no host
 * synchronisation.
 *   params       device [P][stride] (layout above; updated when adam != NULL)
 *   out          host [num_views] of device images: the rendered views (written)
 *   targets      host [num_views] of device images: rgb and depth targets
 *   grad_params  device [P][stride]: overwritten with dL/dparams
 *   loss         device float, overwritten with L (may be NULL)
 * The context captures the graph on the first call and again whenever a
 * pointer, size, num_views, image size, depth_weight, the Adam constants or
 * the profiling mask differ from the capture; camera poses and intrinsics,
 * target and output image pointers and learning rates may change between
 * calls without a new capture. Instance storage has a fixed capacity, set
 * from the instance count of a first pass (x1.25): an iteration whose count
 * exceeds it, or whose sort wait expired, is skipped on the device (params
 * and Adam state unchanged; its images, loss and gradients are not valid),
 * counted, and the next call captures again with a larger capacity. The
 * status and copy queries then report on this iteration's buffers. */
int gsr_mapping_iteration(gsr_ctx* ctx, float* params, int64_t num, int64_t stride, int32_t sh_degree,
                          int32_t num_views, const gsr_camera* cams, const gsr_image* out,
                          const gsr_image* targets, float depth_weight, float* grad_params,
                          float* loss, const gsr_adam* adam, void* stream);

/* Keyframe insertion (paper Fig. "GS_SLAM": keyframe management grows the
 * map): new Gaussians seeded from one RGB-D keyframe, appended to the map.
 * On the grid of every step-th pixel (pixels (gx*step, gy*step)), a pixel
 * seeds a Gaussian when its observed depth d lies in [depth_min, depth_max]
 * and, if coverage is given, the current map's rendered alpha there is below
 * alpha_below. The Gaussian: mean = the back-projection R^T (d ray - t) of
 * the pixel centre's ray ((px + 0.5 - cx)/fx, (py + 0.5 - cy)/fy, 1); three
 * equal log-scales log(scale_factor * d * step / ((fx + fy)/2)); quaternion
 * (1, 0, 0, 0); opacity logit opacity_logit; SH coefficient 0 of each channel
 * (rgb - 0.5) / Y_00 (so its colour is the observed one), the others 0. */
typedef struct {
  int32_t step;             /* grid spacing in pixels, >= 1 */
  float alpha_below;        /* seed only where coverage < alpha_below (ignored without coverage) */
  float depth_min, depth_max;
  float scale_factor;       /* > 0 */
  float opacity_logit;
} gsr_densify_options;

/* params: device [P][stride] float32 (P from sh_degree) holding num
 * Gaussians; the new ones are written at indices num, num + 1, ... in pixel
 * order (row-major over the grid), at most stride - num of them. rgb, depth:
 * device [3][H][W], [H][W] of the keyframe (cam's size); coverage: device
 * [H][W] (the alpha gsr_render gave for this view) or NULL. *appended (host)
 * receives the number written, *wanted (host, may be NULL) the number of
 * seeding pixels, so a caller whose buffer was too small can grow it (stride)
 * and call again with num + *appended. Synchronises `stream`. A mapping
 * iteration called with the new size captures its graph again. */
int gsr_densify(gsr_ctx* ctx, float* params, int64_t num, int64_t stride, int32_t sh_degree,
                const gsr_camera* cam, const float* rgb, const float* depth, const float* coverage,
                const gsr_densify_options* opt, int64_t* appended, int64_t* wanted, void* stream);

/* Counters of the context's mapping iterations (synchronises the stream of
 * the last iteration). Returns GSR_ERR_DEVICE if any iteration's sort wait
 * expired. */
typedef struct {
  int64_t iterations;       /* completed (not skipped) iterations */
  int64_t skipped;          /* iterations skipped for instance overflow or an expired wait */
  int64_t captures;         /* graphs captured */
  int64_t capacity;         /* instance slots of the current graph */
  int64_t last_instances;   /* instance count of the last iteration */
  int64_t adam_steps;       /* the device-side Adam step count */
} gsr_mapping_stats;
int gsr_mapping_status(gsr_ctx* ctx, gsr_mapping_stats* out);

/* Status of the last render (gsr_render or gsr_mapping_iteration) on this
 * context (synchronises the context's last stream). Any pointer may be NULL.
 *   num_instances     (tile, Gaussian) instances the render required over all
 *                     views; a mapping iteration whose count exceeds its
 *                     fixed capacity was skipped (gsr_mapping_status)
 *   num_visible       (view, Gaussian) splats with at least one tile
 *   num_tiles         tiles over all views
 *   nonfinite_culled  Gaussians culled for their values alone: a non-finite
 *                     mean, log-scale, rotation or opacity logit, or a
 *                     rotation quaternion of zero norm (counted once per
 *                     Gaussian, whatever the number of views). Such Gaussians
 *                     are not an error: they are drawn in no view and receive
 *                     no gradient. (A splat whose colour is non-finite is
 *                     culled in that view and not counted here.)
 * GSR_ERR_DEVICE if that render's sort wait expired; GSR_ERR_CAPACITY (with
 * the outputs filled) if it was a gsr_render_noalloc that needed more than
 * its 2^21 instance slots. */
int gsr_query_status(gsr_ctx* ctx, int64_t* num_instances, int64_t* num_visible,
                     int64_t* num_tiles, int64_t* nonfinite_culled);

/* Activations of the parameters as the projection computes them (paper
 * Sec. II-A: each Gaussian's covariance comes from its per-axis scales and
 * rotation, and it carries an opacity): scale[k][num] = exp(log-scale k) and
 * opacity[num] = 1 / (1 + exp(-logit)), in float, with exp correctly rounded
 * to float and the + and / of the sigmoid one correctly rounded float
 * operation each, exactly the values the projection uses. Reads planes 3..5
 * and 10 of g only. scale: device [3][g->num] (plane stride g->num) or NULL;
 * opacity: device [g->num] or NULL. Asynchronous on `stream`. */
int gsr_activations(gsr_ctx* ctx, const gsr_gaussians* g, float* scale, float* opacity, void* stream);

/* Copy the sorted instance list of the last render to host: tile[k] is the
 * global tile id (view tile offset + ty * tiles_x + tx, views in order),
 * gid[k] the Gaussian index, ordered by (tile, depth bits, Gaussian index).
 * Writes min(capacity, count) entries; *count receives the total. Synchronous. */
int gsr_copy_instances(gsr_ctx* ctx, uint32_t* tile, uint32_t* gid, int64_t capacity,
                       int64_t* count);

/* Copy the projected splats of view `view` of the last render to host:
 * out[num][16] = u, v, z, a, b, c (dilated 2D covariance), A, B, C (conic),
 * opacity, r, g, b, then px0, py0, px1, py1 (inclusive pixel rectangle,
 * stored as float) for visible Gaussians; culled rows are all zero with
 * px1 = py1 = -1. Synchronous. */
int gsr_copy_splats(gsr_ctx* ctx, int32_t view, float* out, int64_t num);

/* Work counters of the last render (synchronise the context's last stream):
 * pairs = sum over all pixels of the number of list entries up to and
 * including the last composited Gaussian (the pairs the backward walks);
 * visible[num_views] (may be NULL) = Gaussians with at least one tile per view. */
int gsr_count_work(gsr_ctx* ctx, int64_t* pairs, int64_t* visible, int32_t num_views);

/* ---- Sharing the live map with a viewer process on the same GPU ---------
 * The paper's viewer is a separate process that reads the map directly from
 * GPU memory through inter-process handles, so rendering for the operator
 * neither copies the map nor stalls the mapping loop (paper Sec. III,
 * Fig. "CUDA_IPC"). A handle is 64 opaque bytes to pass between processes
 * (a file, a pipe). None of these calls allocates device memory except the
 * event; all return GSR_ERR_HIP when the runtime refuses. */
typedef struct {
  unsigned char bytes[64];
} gsr_ipc_handle;

/* Export the device allocation holding dev_ptr: *out the handle of the whole
 * allocation, *offset the byte offset of dev_ptr inside it, *alloc_bytes (may
 * be NULL) its size. GSR_ERR_UNSUPPORTED for allocations above 1 GiB. */
int gsr_ipc_export_memory(const void* dev_ptr, gsr_ipc_handle* out, int64_t* offset, int64_t* alloc_bytes);
/* In another process: map the exported allocation; *dev_ptr = its base plus
 * offset (the exporter's pointer), *base the mapping to close. */
int gsr_ipc_open_memory(const gsr_ipc_handle* h, int64_t offset, void** dev_ptr, void** base);
int gsr_ipc_close_memory(void* base);
/* An inter-process event (no timing) and its handle; the other process
 * opens it, and gsr_ipc_event_wait makes a stream wait for its last record. */
int gsr_ipc_event_create(void** event, gsr_ipc_handle* out);
int gsr_ipc_event_open(const gsr_ipc_handle* h, void** event);
int gsr_ipc_event_record(void* event, void* stream);
int gsr_ipc_event_wait(void* event, void* stream);
int gsr_ipc_event_destroy(void* event);

/* Stages timed when profiling is on. */
typedef enum {
  GSR_STAGE_PROJECT = 0, GSR_STAGE_DEPTH_SORT, GSR_STAGE_SCAN, GSR_STAGE_EMIT,
  GSR_STAGE_TILE_SORT, GSR_STAGE_RANGES, GSR_STAGE_BLEND_FWD, GSR_STAGE_LOSS,
  GSR_STAGE_BLEND_BWD, GSR_STAGE_PROJECT_BWD, GSR_STAGE_ADAM, GSR_STAGE_ZERO,
  GSR_STAGE_BLEND,          /* fused blend forward and backward (mapping iteration) */
  GSR_STAGE_TILE_DEPTH,     /* per-tile depth sort */
  GSR_NUM_STAGES
} gsr_stage;

/* Per-stage timing: for every stage k with bit k set in stage_mask the
 * context records a pair of HIP events on the call's stream around the
 * stage's launches (0 turns timing off). */
int gsr_set_profiling(gsr_ctx* ctx, uint32_t stage_mask);

/* Accumulated time of one stage since the last reset, in ms, and the number
 * of timed launches (synchronises on the recorded events); reset != 0
 * clears the stage's record afterwards. */
int gsr_get_profile(gsr_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches, int32_t reset);

/* HIP error code recorded by the last GSR_ERR_HIP on this context; with ctx
 * NULL, that of the calling thread's last failed gsr_ipc_* call (0 if none). */
int gsr_last_hip_error(gsr_ctx* ctx);

/* Static description of a status code. */
const char* gsr_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
