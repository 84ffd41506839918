"""ctypes binding of libgsr.so (argument marshalling only).

Every function here has the name of the C entry point it calls (include/gsr.h)
and takes torch CUDA tensors for device buffers; all arithmetic happens in
the HIP kernels. There is no fallback: if libgsr.so is not built, loading
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

GSR_OK = 0
STATUS_NAMES = {0: "GSR_OK", -1: "GSR_ERR_INVALID", -2: "GSR_ERR_OOM", -3: "GSR_ERR_HIP",
                -4: "GSR_ERR_STATE", -5: "GSR_ERR_CAPACITY", -6: "GSR_ERR_UNSUPPORTED", -7: "GSR_ERR_DEVICE"}

EXPORTED = sorted(["gsr_create", "gsr_destroy", "gsr_render", "gsr_render1", "gsr_render_backward", "gsr_loss_l1",
                   "gsr_adam_step", "gsr_query_status", "gsr_copy_instances", "gsr_copy_splats",
                   "gsr_count_work", "gsr_set_profiling", "gsr_get_profile", "gsr_last_hip_error",
                   "gsr_status_string", "gsr_mapping_iteration", "gsr_mapping_status", "gsr_activations",
                   "gsr_render_noalloc", "gsr_render_backward_pose", "gsr_densify",
                   "gsr_ipc_export_memory", "gsr_ipc_open_memory", "gsr_ipc_close_memory", "gsr_ipc_event_create",
                   "gsr_ipc_event_open", "gsr_ipc_event_record", "gsr_ipc_event_wait", "gsr_ipc_event_destroy",
                   # achievable-peak probes (include/gsr_peaks.h)
                   "gsr_peak_copy", "gsr_peak_valu", "gsr_peak_exp", "gsr_peak_lds"])

STAGES = ["project", "depth_sort", "scan", "emit", "tile_sort", "ranges", "blend_fwd", "loss", "blend_bwd",
          "project_bwd", "adam", "zero", "blend", "tile_depth"]


class GsrError(RuntimeError):
    def __init__(self, fn, status, hip=0):
        self.status = status
        self.hip = hip
        msg = f"{fn} failed: {STATUS_NAMES.get(status, status)}"
        if hip:
            msg += f" (hipError {hip})"
        super().__init__(msg)


class gsr_options(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch_depth", ctypes.c_int32),
                ("bg", ctypes.c_float * 3), ("znear", ctypes.c_float), ("pixels_per_thread", ctypes.c_int32),
                ("tile_order", ctypes.c_int32), ("chunk_len", ctypes.c_int32), ("max_chunks", ctypes.c_int32),
                ("fuse_blend", ctypes.c_int32), ("depth_sort", ctypes.c_int32),
                ("backward_schedule", ctypes.c_int32), ("binning", ctypes.c_int32)]


class gsr_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class gsr_gaussians(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("num", ctypes.c_int64), ("stride", ctypes.c_int64),
                ("sh_degree", ctypes.c_int32)]


class gsr_image(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("alpha", ctypes.c_void_p)]


class gsr_adam(ctypes.Structure):
    _fields_ = [("m", ctypes.c_void_p), ("v", ctypes.c_void_p), ("lr_per_plane", ctypes.POINTER(ctypes.c_float)),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step", ctypes.c_int32)]


class gsr_densify_options(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int32), ("alpha_below", ctypes.c_float), ("depth_min", ctypes.c_float),
                ("depth_max", ctypes.c_float), ("scale_factor", ctypes.c_float), ("opacity_logit", ctypes.c_float)]


class gsr_ipc_handle(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_ubyte * 64)]


class gsr_mapping_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("skipped", ctypes.c_int64), ("captures", ctypes.c_int64),
                ("capacity", ctypes.c_int64), ("last_instances", ctypes.c_int64), ("adam_steps", ctypes.c_int64)]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2509_06433_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        sig = {
            "gsr_create": ([P(vp), P(gsr_options)], ctypes.c_int),
            "gsr_destroy": ([vp], None),
            "gsr_render": ([vp, P(gsr_gaussians), i32, P(gsr_camera), P(gsr_image), vp], ctypes.c_int),
            "gsr_render1": ([vp, P(gsr_gaussians), P(gsr_camera), P(gsr_image), vp], ctypes.c_int),
            "gsr_render_noalloc": ([vp, P(gsr_gaussians), i32, P(gsr_camera), P(gsr_image), vp], ctypes.c_int),
            "gsr_render_backward_pose": ([vp, P(gsr_gaussians), i32, P(gsr_camera), P(gsr_image), vp, vp, vp, vp],
                                         ctypes.c_int),
            "gsr_render_backward": ([vp, P(gsr_gaussians), i32, P(gsr_camera), P(gsr_image), vp, vp],
                                    ctypes.c_int),
            "gsr_loss_l1": ([vp, i32, P(gsr_camera), P(gsr_image), P(gsr_image), f32, P(gsr_image), vp, vp],
                            ctypes.c_int),
            "gsr_adam_step": ([vp, vp, vp, vp, vp, i64, i64, i32, P(f32), f32, f32, f32, i32, vp], ctypes.c_int),
            "gsr_query_status": ([vp, P(i64), P(i64), P(i64), P(i64)], ctypes.c_int),
            "gsr_activations": ([vp, P(gsr_gaussians), vp, vp, vp], ctypes.c_int),
            "gsr_copy_instances": ([vp, P(ctypes.c_uint32), P(ctypes.c_uint32), i64, P(i64)], ctypes.c_int),
            "gsr_copy_splats": ([vp, i32, P(f32), i64], ctypes.c_int),
            "gsr_count_work": ([vp, P(i64), P(i64), i32], ctypes.c_int),
            "gsr_set_profiling": ([vp, ctypes.c_uint32], ctypes.c_int),
            "gsr_get_profile": ([vp, i32, P(ctypes.c_double), P(i64), i32], ctypes.c_int),
            "gsr_last_hip_error": ([vp], ctypes.c_int),
            "gsr_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "gsr_mapping_iteration": ([vp, vp, i64, i64, i32, i32, P(gsr_camera), P(gsr_image), P(gsr_image), f32,
                                       vp, vp, P(gsr_adam), vp], ctypes.c_int),
            "gsr_mapping_status": ([vp, P(gsr_mapping_stats)], ctypes.c_int),
            "gsr_densify": ([vp, vp, i64, i64, i32, P(gsr_camera), vp, vp, vp, P(gsr_densify_options), P(i64),
                             P(i64), vp], ctypes.c_int),
            "gsr_ipc_export_memory": ([vp, P(gsr_ipc_handle), P(i64), P(i64)], ctypes.c_int),
            "gsr_ipc_open_memory": ([P(gsr_ipc_handle), i64, P(vp), P(vp)], ctypes.c_int),
            "gsr_ipc_close_memory": ([vp], ctypes.c_int),
            "gsr_ipc_event_create": ([P(vp), P(gsr_ipc_handle)], ctypes.c_int),
            "gsr_ipc_event_open": ([P(gsr_ipc_handle), P(vp)], ctypes.c_int),
            "gsr_ipc_event_record": ([vp, vp], ctypes.c_int),
            "gsr_ipc_event_wait": ([vp, vp], ctypes.c_int),
            "gsr_ipc_event_destroy": ([vp], ctypes.c_int),
            "gsr_peak_copy": ([i64, i32, vp, P(ctypes.c_double)], ctypes.c_int),
            "gsr_peak_valu": ([i32, vp, P(ctypes.c_double)], ctypes.c_int),
            "gsr_peak_exp": ([i32, vp, P(ctypes.c_double)], ctypes.c_int),
            "gsr_peak_lds": ([i32, vp, P(ctypes.c_double)], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def make_camera(cam) -> gsr_camera:
    """gsr_camera from any object with R (3x3), t (3), fx, fy, cx, cy, width, height."""
    c = gsr_camera()
    R = [float(x) for row in cam.R for x in row]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = float(cam.t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _cams(cams):
    arr = (gsr_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, gsr_camera) else make_camera(c)
    return arr


def _check_tensor(t, shape, name, device=None):
    """A device buffer handed to the library as a raw pointer: it must be a CUDA
    float32 tensor, contiguous, of exactly `shape` (and on `device` if given),
    or the kernels would read or write outside it."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _check_out(t, shape, name, device=None):
    if t is not None:
        _check_tensor(t, shape, name, device)


def _cam_hw(c):
    return (int(c.height), int(c.width))


def _images(imgs, cams, name, optional=(), device=None):
    """Descriptors of one (rgb [3,H,W], depth [H,W], alpha [H,W]) triple per camera;
    planes named in `optional` ("rgb", "depth", "alpha") may be None (NULL)."""
    imgs = list(imgs)
    if len(imgs) != len(cams):
        raise ValueError(f"{name}: {len(imgs)} images for {len(cams)} cameras")
    arr = (gsr_image * len(imgs))()
    for i, (im, cam) in enumerate(zip(imgs, cams)):
        if len(im) != 3:
            raise ValueError(f"{name}[{i}] must be (rgb, depth, alpha)")
        H, W = _cam_hw(cam)
        for plane, t, shape in zip(("rgb", "depth", "alpha"), im, ((3, H, W), (H, W), (H, W))):
            if t is None:
                if plane not in optional:
                    raise ValueError(f"{name}[{i}].{plane} is required")
                continue
            _check_tensor(t, shape, f"{name}[{i}].{plane}", device)
        arr[i] = gsr_image(_ptr(im[0]), _ptr(im[1]), _ptr(im[2]))
    return arr


def _check_like_params(t, params, name):
    """A gradient or optimiser-state tensor laid out like params (same shape and plane stride)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or t.device != params.device:
        raise ValueError(f"{name} must be a float32 tensor on {params.device}")
    if t.shape != params.shape or t.stride() != params.stride():
        raise ValueError(f"{name} must match params in shape and stride")


def _gauss(params: torch.Tensor, sh_degree: int, num=None, stride=None) -> gsr_gaussians:
    if not isinstance(params, torch.Tensor) or params.dtype != torch.float32 or not params.is_cuda \
            or params.dim() != 2:
        raise ValueError("params must be a CUDA float32 tensor [P, N]")
    if params.stride(1) != 1:
        raise ValueError("params planes must be contiguous")
    n = params.shape[1] if num is None else num
    st = params.stride(0) if stride is None else stride
    if params.shape[0] != 11 + 3 * (sh_degree + 1) ** 2:
        raise ValueError("params has the wrong number of planes for sh_degree")
    return gsr_gaussians(_ptr(params), n, st, sh_degree)


def _check(ctx, fn, rc):
    if rc != GSR_OK:
        hip = load().gsr_last_hip_error(ctx)
        raise GsrError(fn, rc, hip)


# --- one wrapper per C entry point ------------------------------------------

def gsr_create(tile_w=16, tile_h=16, batch_depth=0, bg=(0.0, 0.0, 0.0), znear=0.2, pixels_per_thread=0,
               tile_order=0, chunk_len=0, max_chunks=0, fuse_blend=0, depth_sort=0, backward_schedule=0, binning=0):
    opt = gsr_options(tile_w, tile_h, batch_depth, (ctypes.c_float * 3)(*bg), znear, pixels_per_thread, tile_order,
                      chunk_len, max_chunks, fuse_blend, depth_sort, backward_schedule, binning)
    h = ctypes.c_void_p()
    _check(None, "gsr_create", load().gsr_create(ctypes.byref(h), ctypes.byref(opt)))
    return h


def gsr_destroy(ctx):
    load().gsr_destroy(ctx)


def gsr_render(ctx, params, sh_degree, cams, outs, stream=None):
    """outs: list of (rgb [3,H,W], depth [H,W], alpha [H,W]) CUDA float32 tensors, written."""
    g = _gauss(params, sh_degree)
    ims = _images(outs, cams, "outs", device=params.device)
    _check(ctx, "gsr_render", load().gsr_render(ctx, ctypes.byref(g), len(cams), _cams(cams), ims, _stream(stream)))


def gsr_render_noalloc(ctx, params, sh_degree, cams, outs, stream=None):
    """gsr_render without device allocation or synchronisation (fixed-size scratch; see include/gsr.h)."""
    g = _gauss(params, sh_degree)
    ims = _images(outs, cams, "outs", device=params.device)
    _check(ctx, "gsr_render_noalloc",
           load().gsr_render_noalloc(ctx, ctypes.byref(g), len(cams), _cams(cams), ims, _stream(stream)))


def gsr_render1(ctx, params, sh_degree, cam, out, stream=None):
    g = _gauss(params, sh_degree)
    ims = _images([out], [cam], "out", device=params.device)
    _check(ctx, "gsr_render1", load().gsr_render1(ctx, ctypes.byref(g), _cams([cam]), ims, _stream(stream)))


def gsr_render_backward(ctx, params, sh_degree, cams, grads, grad_params, stream=None):
    """grads: list of (dL/drgb, dL/ddepth, dL/dalpha), entries may be None. grad_params += dL/dparams."""
    g = _gauss(params, sh_degree)
    _check_like_params(grad_params, params, "grad_params")
    ims = _images(grads, cams, "grads", optional=("rgb", "depth", "alpha"), device=params.device)
    _check(ctx, "gsr_render_backward",
           load().gsr_render_backward(ctx, ctypes.byref(g), len(cams), _cams(cams), ims, _ptr(grad_params),
                                      _stream(stream)))


def gsr_render_backward_pose(ctx, params, sh_degree, cams, grads, grad_cams, grad_params=None, grad_twist=None,
                             stream=None):
    """Backward with camera gradients: grad_cams [V, 12] (CUDA float64) += dL/dR (row-major), dL/dt per
    view; grad_twist [V, 6] (float64) or None += the left-perturbation gradient; grad_params like
    params or None."""
    g = _gauss(params, sh_degree)
    if grad_params is not None:
        _check_like_params(grad_params, params, "grad_params")
    nv = len(cams)
    for name, t, w in (("grad_cams", grad_cams, 12), ("grad_twist", grad_twist, 6)):
        if t is None and name == "grad_twist":
            continue
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != params.device \
                or not t.is_contiguous() or tuple(t.shape) != (nv, w):
            raise ValueError(f"{name} must be a contiguous float64 tensor [{nv}, {w}] on {params.device}")
    ims = _images(grads, cams, "grads", optional=("rgb", "depth", "alpha"), device=params.device)
    _check(ctx, "gsr_render_backward_pose",
           load().gsr_render_backward_pose(ctx, ctypes.byref(g), nv, _cams(cams), ims, _ptr(grad_params),
                                           _ptr(grad_cams), _ptr(grad_twist), _stream(stream)))


def gsr_loss_l1(ctx, cams, rendered, targets, grads, depth_weight=0.5, loss=None, stream=None):
    dev = rendered[0][0].device if len(rendered) and isinstance(rendered[0][0], torch.Tensor) else None
    r = _images(rendered, cams, "rendered", optional=("alpha",), device=dev)
    t = _images(targets, cams, "targets", optional=("alpha",), device=dev)
    gi = _images(grads, cams, "grads", optional=("alpha",), device=dev)
    _check_out(loss, (1,), "loss", dev)
    _check(ctx, "gsr_loss_l1",
           load().gsr_loss_l1(ctx, len(cams), _cams(cams), r, t, float(depth_weight), gi, _ptr(loss),
                              _stream(stream)))


def gsr_adam_step(ctx, params, grads, m, v, lr_per_plane, step, beta1=0.9, beta2=0.999, eps=1e-15,
                  stream=None):
    if not isinstance(params, torch.Tensor) or params.dtype != torch.float32 or not params.is_cuda \
            or params.dim() != 2 or params.stride(1) != 1:
        raise ValueError("params must be a CUDA float32 tensor [P, N] with contiguous planes")
    P, n = params.shape
    for name, t in (("grads", grads), ("m", m), ("v", v)):
        _check_like_params(t, params, name)
    if len(lr_per_plane) != P:
        raise ValueError("one learning rate per parameter plane")
    lr = (ctypes.c_float * P)(*[float(x) for x in lr_per_plane])
    _check(ctx, "gsr_adam_step",
           load().gsr_adam_step(ctx, _ptr(params), _ptr(grads), _ptr(m), _ptr(v), n, params.stride(0), P, lr,
                                beta1, beta2, eps, int(step), _stream(stream)))


def gsr_query_status(ctx):
    a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(ctx, "gsr_query_status", load().gsr_query_status(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                            ctypes.byref(d)))
    return {"instances": a.value, "visible": b.value, "tiles": c.value, "nonfinite_culled": d.value}


def gsr_activations(ctx, params, sh_degree, scale=None, opacity=None, stream=None):
    """scale [3, N] and opacity [N] (CUDA float32, contiguous; either may be None) = the activations
    the projection uses for params [P, N]."""
    g = _gauss(params, sh_degree)
    n = params.shape[1]
    _check_out(scale, (3, n), "scale")
    _check_out(opacity, (n,), "opacity")
    _check(ctx, "gsr_activations", load().gsr_activations(ctx, ctypes.byref(g), _ptr(scale), _ptr(opacity),
                                                          _stream(stream)))


def gsr_copy_instances(ctx):
    import numpy as np
    cnt = ctypes.c_int64()
    _check(ctx, "gsr_copy_instances", load().gsr_copy_instances(ctx, None, None, 0, ctypes.byref(cnt)))
    n = cnt.value
    tiles = np.empty(max(n, 1), np.uint32)
    gids = np.empty(max(n, 1), np.uint32)
    PU = ctypes.POINTER(ctypes.c_uint32)
    _check(ctx, "gsr_copy_instances",
           load().gsr_copy_instances(ctx, tiles.ctypes.data_as(PU), gids.ctypes.data_as(PU), n, ctypes.byref(cnt)))
    return tiles[:n], gids[:n]


def gsr_copy_splats(ctx, view, num):
    import numpy as np
    out = np.empty((num, 16), np.float32)
    _check(ctx, "gsr_copy_splats",
           load().gsr_copy_splats(ctx, int(view), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), num))
    return out


def gsr_count_work(ctx, num_views):
    pairs = ctypes.c_int64()
    vis = (ctypes.c_int64 * num_views)()
    _check(ctx, "gsr_count_work", load().gsr_count_work(ctx, ctypes.byref(pairs), vis, num_views))
    return pairs.value, list(vis)


def gsr_set_profiling(ctx, stages=None):
    """Time the named stages (None = all, [] = none)."""
    names = STAGES if stages is None else stages
    mask = 0
    for nm in names:
        mask |= 1 << STAGES.index(nm)
    _check(ctx, "gsr_set_profiling", load().gsr_set_profiling(ctx, mask))


def gsr_get_profile(ctx, reset=True):
    """{stage name: (total ms, launches)} accumulated since the last reset."""
    out = {}
    for k, name in enumerate(STAGES):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(ctx, "gsr_get_profile", load().gsr_get_profile(ctx, k, ctypes.byref(ms), ctypes.byref(n), int(reset)))
        out[name] = (ms.value, n.value)
    return out


def gsr_mapping_iteration(ctx, params, sh_degree, cams, outs, targets, depth_weight, grad_params, loss=None,
                          adam=None, stream=None):
    """One graph-replayed mapping iteration. targets: per view (rgb [3,H,W], depth [H,W]).
    adam: None or a dict with m, v (tensors like params), lr (per-plane list), beta1, beta2, eps,
    step (0 = continue the device count)."""
    g = _gauss(params, sh_degree)
    _check_like_params(grad_params, params, "grad_params")
    dev = params.device
    ims = _images(outs, cams, "outs", device=dev)
    tg = _images([(t[0], t[1], None) for t in targets], cams, "targets", optional=("alpha",), device=dev)
    _check_out(loss, (1,), "loss", dev)
    a = None
    if adam is not None:
        for name in ("m", "v"):
            _check_like_params(adam[name], params, "adam." + name)
        lr = adam["lr"]
        if len(lr) != params.shape[0]:
            raise ValueError("one learning rate per parameter plane")
        lr_arr = (ctypes.c_float * len(lr))(*[float(x) for x in lr])
        a = gsr_adam(_ptr(adam["m"]), _ptr(adam["v"]), lr_arr, float(adam.get("beta1", 0.9)),
                     float(adam.get("beta2", 0.999)), float(adam.get("eps", 1e-15)), int(adam.get("step", 0)))
    _check(ctx, "gsr_mapping_iteration",
           load().gsr_mapping_iteration(ctx, g.params, g.num, g.stride, sh_degree, len(cams), _cams(cams), ims, tg,
                                        float(depth_weight), _ptr(grad_params), _ptr(loss),
                                        ctypes.byref(a) if a is not None else None, _stream(stream)))


def gsr_densify(ctx, params, num, sh_degree, cam, rgb, depth, coverage=None, step=4, alpha_below=0.5,
                depth_min=0.2, depth_max=100.0, scale_factor=1.0, opacity_logit=0.0, stream=None):
    """Append Gaussians seeded from an RGB-D keyframe to the map buffer params [P, stride] (CUDA
    float32, contiguous; its first num Gaussians are the map) at indices num, num + 1, ...;
    returns (appended, wanted)."""
    if not isinstance(params, torch.Tensor) or params.dtype != torch.float32 or not params.is_cuda \
            or params.dim() != 2 or params.stride(1) != 1:
        raise ValueError("params must be a CUDA float32 tensor [P, stride] with contiguous planes")
    if params.shape[0] != 11 + 3 * (sh_degree + 1) ** 2:
        raise ValueError("params has the wrong number of planes for sh_degree")
    stride = params.stride(0)
    if params.shape[1] != stride:
        raise ValueError("params must be the whole [P, stride] buffer (new Gaussians go up to index stride - 1)")
    if not (0 <= num <= stride):
        raise ValueError("num must lie within params")
    H, W = int(cam.height), int(cam.width)
    _check_tensor(rgb, (3, H, W), "rgb", params.device)
    _check_tensor(depth, (H, W), "depth", params.device)
    _check_out(coverage, (H, W), "coverage", params.device)
    opt = gsr_densify_options(int(step), float(alpha_below), float(depth_min), float(depth_max), float(scale_factor),
                              float(opacity_logit))
    app, want = ctypes.c_int64(), ctypes.c_int64()
    _check(ctx, "gsr_densify",
           load().gsr_densify(ctx, _ptr(params), int(num), int(stride), int(sh_degree), _cams([cam]),
                              _ptr(rgb), _ptr(depth), _ptr(coverage), ctypes.byref(opt), ctypes.byref(app),
                              ctypes.byref(want), _stream(stream)))
    return app.value, want.value


def gsr_mapping_status(ctx):
    s = gsr_mapping_stats()
    _check(ctx, "gsr_mapping_status", load().gsr_mapping_status(ctx, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in gsr_mapping_stats._fields_}


def gsr_ipc_export_memory(t):
    """(handle bytes, offset, allocation bytes) of the CUDA tensor t's device allocation."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("a CUDA tensor is required")
    h, off, size = gsr_ipc_handle(), ctypes.c_int64(), ctypes.c_int64()
    _check(None, "gsr_ipc_export_memory",
           load().gsr_ipc_export_memory(_ptr(t), ctypes.byref(h), ctypes.byref(off), ctypes.byref(size)))
    return bytes(h.bytes), off.value, size.value


def gsr_ipc_open_memory(handle: bytes, offset: int):
    """(device address, base to close) of a buffer exported by another process."""
    if len(handle) != 64 or offset < 0:
        raise ValueError("a 64-byte handle and a non-negative offset are required")
    h = gsr_ipc_handle()
    ctypes.memmove(ctypes.addressof(h), handle, 64)
    ptr, base = ctypes.c_void_p(), ctypes.c_void_p()
    _check(None, "gsr_ipc_open_memory",
           load().gsr_ipc_open_memory(ctypes.byref(h), ctypes.c_int64(offset), ctypes.byref(ptr), ctypes.byref(base)))
    return ptr.value, base.value


def gsr_ipc_close_memory(base: int):
    _check(None, "gsr_ipc_close_memory", load().gsr_ipc_close_memory(ctypes.c_void_p(base)))


def gsr_ipc_event_open(handle: bytes):
    if len(handle) != 64:
        raise ValueError("a 64-byte handle is required")
    h, ev = gsr_ipc_handle(), ctypes.c_void_p()
    ctypes.memmove(ctypes.addressof(h), handle, 64)
    _check(None, "gsr_ipc_event_open", load().gsr_ipc_event_open(ctypes.byref(h), ctypes.byref(ev)))
    return ev.value


def gsr_ipc_event_wait(event, stream=None):
    _check(None, "gsr_ipc_event_wait", load().gsr_ipc_event_wait(ctypes.c_void_p(event), _stream(stream)))


def gsr_ipc_event_create():
    """(event handle as an int, its 64 handle bytes)."""
    ev, h = ctypes.c_void_p(), gsr_ipc_handle()
    _check(None, "gsr_ipc_event_create", load().gsr_ipc_event_create(ctypes.byref(ev), ctypes.byref(h)))
    return ev.value, bytes(h.bytes)


def gsr_ipc_event_record(event, stream=None):
    _check(None, "gsr_ipc_event_record", load().gsr_ipc_event_record(ctypes.c_void_p(event), _stream(stream)))


def gsr_ipc_event_destroy(event):
    _check(None, "gsr_ipc_event_destroy", load().gsr_ipc_event_destroy(ctypes.c_void_p(event)))


def gsr_status_string(status: int) -> str:
    return load().gsr_status_string(int(status)).decode()
