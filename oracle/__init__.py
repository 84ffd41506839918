"""CPU oracle for the differentiable Gaussian rasterizer (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the HIP library; it loads its own
C++ reference (oracle.cpp, built by oracle/build.py) and adds the parts that
are plain NumPy: the L1 mapping loss, Adam and keyframe insertion.

Parity status: every function here is pinned in tests/test_oracle_*.py by a
closed form, a library routine, an invariant, torch autograd or finite
differences; see the docstrings.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None

# Constants the oracle uses (repeated here only for the Python-side helpers).
ALPHA_MAX = np.float32(0.99)
ALPHA_MIN = np.float32(1.0) / np.float32(255.0)
TRANS_MIN = np.float32(1e-4)

F32P = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
I32P = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
U32P = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
I64P = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        c_i64, c_int, c_f = ctypes.c_int64, ctypes.c_int, ctypes.c_float
        L.orc_num_threads.argtypes = [c_int]
        L.orc_num_threads.restype = c_int
        L.orc_exp32.argtypes = [F32P, F32P, ctypes.c_void_p, c_i64]
        L.orc_exp32.restype = None
        L.orc_activations.argtypes = [F32P, F32P, F32P, F32P, c_i64]
        L.orc_activations.restype = None
        L.orc_sh_basis.argtypes = [c_int, F64P, c_i64, F64P, ctypes.c_void_p]
        L.orc_sh_basis.restype = None
        L.orc_project.argtypes = [c_int, F32P, c_i64, c_i64, c_int, F32P, c_int, c_int, c_f, F64P, I32P]
        L.orc_project.restype = c_int
        L.orc_tile_list.argtypes = [F32P, c_i64, c_i64, c_int, c_int, F32P, I32P, c_int, c_int, c_f,
                                    c_i64, U32P, U32P, ctypes.POINTER(c_i64)]
        L.orc_tile_list.restype = c_int
        L.orc_render.argtypes = [c_int, c_int, F32P, c_i64, c_i64, c_int, F32P, c_int, c_int, c_f, F32P,
                                 F64P, F64P, F64P, F64P, I32P, F64P, ctypes.c_void_p]
        L.orc_render.restype = c_int
        L.orc_backward.argtypes = [c_int, F32P, c_i64, c_i64, c_int, c_int, F32P, I32P, c_f, F32P,
                                   F32P, F32P, F32P, F64P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]
        L.orc_backward.restype = c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return lib().orc_num_threads(int(n))


def _cam_floats(cam) -> np.ndarray:
    return np.ascontiguousarray(cam.as_floats(), np.float32)


def exp32(x, with_tie=False):
    """The FP32 mode's exponential: exp(x) rounded to the nearest float (the
    library's double exp rounded to float, recomputed from its long double exp
    where the double result lies within 2^-50 of a rounding midpoint). With
    with_tie, also the relative distance of the long double exp from the
    nearest rounding midpoint, per element."""
    x = np.ascontiguousarray(x, np.float32).ravel()
    y = np.empty_like(x)
    tie = np.empty(x.size, np.float64) if with_tie else None
    lib().orc_exp32(x, y, tie.ctypes.data if with_tie else None, x.size)
    return (y, tie) if with_tie else y


def activations(logscale, logit):
    """The FP32 activations of O1, element by element: (exp(logscale),
    1 / (1 + exp(-logit))) in float with the exponential above."""
    ls = np.ascontiguousarray(logscale, np.float32).ravel()
    lg = np.ascontiguousarray(logit, np.float32).ravel()
    assert ls.size == lg.size
    s = np.empty_like(ls)
    o = np.empty_like(lg)
    lib().orc_activations(ls, lg, s, o, ls.size)
    return s, o


def sh_basis(deg: int, dirs, with_grad=False):
    """Real SH basis (Condon-Shortley phase) at unit directions [n, 3] -> [n, (deg+1)^2]."""
    d = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    K = (deg + 1) ** 2
    out = np.empty((d.shape[0], K), np.float64)
    grad = np.empty((d.shape[0], K, 3), np.float64) if with_grad else None
    lib().orc_sh_basis(deg, d, d.shape[0], out, grad.ctypes.data if with_grad else None)
    return (out, grad) if with_grad else out


PROJ_FIELDS = ["u", "v", "z", "a", "b", "c", "A", "B", "C", "o", "r", "g", "b_", "ex", "ey", "det", "vis"]


def project(params, sh_degree, cam, prec=32, znear=0.2):
    """Per-Gaussian projection (EWA): dict of arrays named PROJ_FIELDS plus
    'rect' [n, 4] = (px0, py0, px1, py1) inclusive, empty (0, 0, -1, -1) if culled."""
    p = np.ascontiguousarray(params, np.float32)
    n = p.shape[1]
    out = np.empty((n, 17), np.float64)
    rect = np.empty((n, 4), np.int32)
    rc = lib().orc_project(int(prec), p, n, n, int(sh_degree), _cam_floats(cam), cam.width, cam.height,
                           float(znear), out, rect)
    assert rc == 0
    d = {k: out[:, i] for i, k in enumerate(PROJ_FIELDS)}
    d["vis"] = out[:, 16] != 0
    d["rect"] = rect
    return d


def tile_list(params, sh_degree, cams, tile_w=16, tile_h=16, znear=0.2):
    """Sorted instance list over all views: (global tile id, Gaussian index), ordered
    by (global tile, FP32 depth bits, index). Global tile = view offset + ty*tiles_x + tx."""
    p = np.ascontiguousarray(params, np.float32)
    n = p.shape[1]
    camf = np.ascontiguousarray(np.stack([_cam_floats(c) for c in cams]), np.float32)
    wh = np.ascontiguousarray(np.array([[c.width, c.height] for c in cams], np.int32))
    cnt = ctypes.c_int64(0)
    empty = np.empty(1, np.uint32)
    lib().orc_tile_list(p, n, n, int(sh_degree), len(cams), camf, wh, tile_w, tile_h, float(znear), 0,
                        empty, empty, ctypes.byref(cnt))
    total = cnt.value
    tiles = np.empty(max(total, 1), np.uint32)
    gids = np.empty(max(total, 1), np.uint32)
    lib().orc_tile_list(p, n, n, int(sh_degree), len(cams), camf, wh, tile_w, tile_h, float(znear), total,
                        tiles, gids, ctypes.byref(cnt))
    return tiles[:total], gids[:total]


MODES = {"f32": 0, "f64pin": 1, "f64": 2}


def _window(window, cam):
    """(x0, y0, x1, y1, row_step) as int32, or None for the whole image."""
    if window is None:
        return None
    w = list(window) + [1] * (5 - len(window))
    return np.ascontiguousarray(w[:5], np.int32)


def render(params, sh_degree, cam, mode="f32", prefilter=True, bg=(0.0, 0.0, 0.0), znear=0.2, window=None):
    """Brute-force per-pixel render of one view. Returns dict with rgb [3,H,W],
    depth [H,W], alpha [H,W], tfinal [H,W], ncomp [H,W] (number of composited
    Gaussians) and margin [H,W] (smallest relative distance of any decision to
    its threshold, from the deciding precision). window = (x0, y0, x1, y1[,
    row_step]): only the pixels of [x0, x1) x [y0, y1) in every row_step-th
    row are composited (each pixel exactly as in the whole render); the others
    are left at 0 (margin +inf)."""
    p = np.ascontiguousarray(params, np.float32)
    n = p.shape[1]
    H, W = cam.height, cam.width
    rgb = np.zeros((3, H, W), np.float64)
    depth = np.zeros((H, W), np.float64)
    alpha = np.zeros((H, W), np.float64)
    tfin = np.zeros((H, W), np.float64)
    ncomp = np.zeros((H, W), np.int32)
    margin = np.full((H, W), np.inf, np.float64)
    win = _window(window, cam)
    rc = lib().orc_render(MODES[mode], int(bool(prefilter)), p, n, n, int(sh_degree), _cam_floats(cam), W, H,
                          float(znear), np.ascontiguousarray(bg, np.float32), rgb, depth, alpha, tfin, ncomp, margin,
                          win.ctypes.data if win is not None else None)
    assert rc == 0
    return dict(rgb=rgb, depth=depth, alpha=alpha, tfinal=tfin, ncomp=ncomp, margin=margin)


def backward(params, sh_degree, cams, grads, pinned=True, bg=(0.0, 0.0, 0.0), znear=0.2, want_2d=False,
             windows=None, want_cam=False, want_abs=False):
    """FP64 analytic gradient of sum_v <grads_v, (rgb_v, depth_v, alpha_v)> with respect
    to the parameters [P, N]. grads: list of (g_rgb [3,H,W], g_depth [H,W], g_alpha [H,W]).
    pinned: False = FP64 decisions; True = decisions from the FP32 recurrence;
    "splats32" = FP32 decisions and FP32-rounded screen-space splat values
    (u, v, conic, opacity, colour, depth), FP64 arithmetic. windows: per view a
    window as render's (or None): only its pixels are walked, which equals the
    gradient with the upstream gradient zeroed outside it. want_cam: also
    return each view's camera gradient [V, 12] (dL/dR row-major, then dL/dt)
    for x_cam = R x + t. want_abs: also return [P, N], per parameter, the sum of
    the magnitudes of the terms the gradient adds up (screen-space terms in
    absolute value through the projection's Jacobian in absolute value):
    |grad| <= abs, and abs / |grad| measures how much the sum cancels."""
    p = np.ascontiguousarray(params, np.float32)
    P, n = p.shape
    camf = np.ascontiguousarray(np.stack([_cam_floats(c) for c in cams]), np.float32)
    wh = np.ascontiguousarray(np.array([[c.width, c.height] for c in cams], np.int32))
    # per-view [3][HW] blocks laid out back to back
    grgb = np.ascontiguousarray(np.concatenate([np.asarray(g[0], np.float32).ravel() for g in grads]))
    gdep = np.ascontiguousarray(np.concatenate([np.asarray(g[1], np.float32).ravel() for g in grads]))
    galp = np.ascontiguousarray(np.concatenate([np.asarray(g[2], np.float32).ravel() for g in grads]))
    grad = np.empty((P, n), np.float64)
    g2 = np.empty((len(cams), n, 10), np.float64) if want_2d else None
    win = None
    if windows is not None:
        win = np.ascontiguousarray(np.stack([_window(w, c) if w is not None else
                                             np.array([0, 0, c.width, c.height, 1], np.int32)
                                             for w, c in zip(windows, cams)]), np.int32)
    mode = 2 if pinned == "splats32" else int(bool(pinned))
    gcam = np.zeros((len(cams), 12), np.float64) if want_cam else None
    gabs = np.zeros((P, n), np.float64) if want_abs else None
    rc = lib().orc_backward(mode, p, n, n, int(sh_degree), len(cams), camf, wh, float(znear),
                            np.ascontiguousarray(bg, np.float32), grgb, gdep, galp, grad,
                            g2.ctypes.data if want_2d else None, win.ctypes.data if win is not None else None,
                            gcam.ctypes.data if want_cam else None, gabs.ctypes.data if want_abs else None)
    assert rc == 0
    out = (grad,)
    if want_2d:
        out += (g2,)
    if want_cam:
        out += (gcam,)
    if want_abs:
        out += (gabs,)
    return out if len(out) > 1 else grad


# ---------------------------------------------------------------------------
# Mapping loss and optimiser (plain NumPy, float64)
# ---------------------------------------------------------------------------

def l1_loss_and_grad(rgb, depth, target_rgb, target_depth, depth_weight=0.5):
    """L = mean|rgb - rgb*| + depth_weight * mean|depth - depth*| for one view
    (means over 3HW and HW); sign(0) = 0. Returns (L, dL/drgb, dL/ddepth)."""
    rgb = np.asarray(rgb, np.float64)
    depth = np.asarray(depth, np.float64)
    dr = rgb - np.asarray(target_rgb, np.float64)
    dd = depth - np.asarray(target_depth, np.float64)
    L = np.abs(dr).mean() + depth_weight * np.abs(dd).mean()
    return L, np.sign(dr) / dr.size, depth_weight * np.sign(dd) / dd.size


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step with bias correction (step counts from 1); lr may be a scalar or
    broadcast per row. Returns (param, m, v) in float64."""
    param = np.asarray(param, np.float64)
    grad = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    lr = np.asarray(lr, np.float64)
    if lr.ndim == 1:
        lr = lr[:, None]
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# Keyframe insertion (plain NumPy, float64)
# ---------------------------------------------------------------------------

Y00 = 0.5 / np.sqrt(np.pi)      # the constant real spherical harmonic


def densify(sh_degree, cam, rgb, depth, coverage=None, step=4, alpha_below=0.5, depth_min=0.2, depth_max=100.0,
            scale_factor=1.0, opacity_logit=0.0):
    """New Gaussians seeded from one RGB-D keyframe, in seeding order, as
    (params [P, M] float64, pixel coordinates [M, 2]). A grid pixel (gx*step,
    gy*step), taken in row-major order, seeds one Gaussian when its depth d
    lies in [depth_min, depth_max] and (with coverage) coverage < alpha_below:
    mean = R^T (d * ray - t) for the ray ((px + 0.5 - cx)/fx, (py + 0.5 - cy)/fy,
    1) through the pixel centre; log-scales log(scale_factor d step / ((fx +
    fy)/2)); quaternion (1, 0, 0, 0); the given opacity logit; SH coefficient
    0 = (rgb - 0.5) / Y_00 per channel, the rest 0."""
    H, W = cam.height, cam.width
    depth = np.asarray(depth, np.float64)
    rgb = np.asarray(rgb, np.float64)
    ys = np.arange(0, H, step)
    xs = np.arange(0, W, step)
    py, px = [a.ravel() for a in np.meshgrid(ys, xs, indexing="ij")]      # row-major over the grid
    d = depth[py, px]
    keep = (d >= depth_min) & (d <= depth_max)
    if coverage is not None:
        keep &= np.asarray(coverage, np.float64)[py, px] < alpha_below
    px, py, d = px[keep], py[keep], d[keep]
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    xcam = np.stack([(px + 0.5 - cam.cx) / cam.fx * d, (py + 0.5 - cam.cy) / cam.fy * d, d], axis=1)
    mean = (xcam - t) @ R                      # rows: R^T (x - t)
    m = len(d)
    P = 11 + 3 * (sh_degree + 1) ** 2
    out = np.zeros((P, m), np.float64)
    out[0:3] = mean.T
    out[3:6] = np.log(scale_factor * d * step / (0.5 * (cam.fx + cam.fy)))[None, :]
    out[6] = 1.0
    out[10] = opacity_logit
    out[11:14] = (rgb[:, py, px] - 0.5) / Y00
    return out, np.stack([px, py], axis=1)
