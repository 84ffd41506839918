"""CPU oracle for the differentiable Gaussian rasterizer (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the HIP library; it loads its own
C++ reference (oracle.cpp, built by oracle/build.py) and adds the parts that
are plain NumPy: the L1 mapping loss and Adam.

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
        L.orc_exp32.argtypes = [F32P, F32P, c_i64]
        L.orc_exp32.restype = None
        L.orc_sh_basis.argtypes = [c_int, F64P, c_i64, F64P, ctypes.c_void_p]
        L.orc_sh_basis.restype = None
        L.orc_project.argtypes = [c_int, F32P, c_i64, c_i64, c_int, F32P, c_int, c_int, c_f, F64P, I32P]
        L.orc_project.restype = c_int
        L.orc_tile_list.argtypes = [F32P, c_i64, c_i64, c_int, c_int, F32P, I32P, c_int, c_int, c_f,
                                    c_i64, U32P, U32P, ctypes.POINTER(c_i64)]
        L.orc_tile_list.restype = c_int
        L.orc_render.argtypes = [c_int, c_int, F32P, c_i64, c_i64, c_int, F32P, c_int, c_int, c_f, F32P,
                                 F64P, F64P, F64P, F64P, I32P, F64P]
        L.orc_render.restype = c_int
        L.orc_backward.argtypes = [c_int, F32P, c_i64, c_i64, c_int, c_int, F32P, I32P, c_f, F32P,
                                   F32P, F32P, F32P, F64P, ctypes.c_void_p]
        L.orc_backward.restype = c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return lib().orc_num_threads(int(n))


def _cam_floats(cam) -> np.ndarray:
    return np.ascontiguousarray(cam.as_floats(), np.float32)


def exp32(x) -> np.ndarray:
    """The oracle's own FP32 exponential (Cody-Waite reduction + degree-7 polynomial)."""
    x = np.ascontiguousarray(x, np.float32).ravel()
    y = np.empty_like(x)
    lib().orc_exp32(x, y, x.size)
    return y


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


def render(params, sh_degree, cam, mode="f32", prefilter=True, bg=(0.0, 0.0, 0.0), znear=0.2):
    """Brute-force per-pixel render of one view. Returns dict with rgb [3,H,W],
    depth [H,W], alpha [H,W], tfinal [H,W], ncomp [H,W] (number of composited
    Gaussians) and margin [H,W] (smallest relative distance of any decision to
    its threshold, from the deciding precision)."""
    p = np.ascontiguousarray(params, np.float32)
    n = p.shape[1]
    H, W = cam.height, cam.width
    rgb = np.empty((3, H, W), np.float64)
    depth = np.empty((H, W), np.float64)
    alpha = np.empty((H, W), np.float64)
    tfin = np.empty((H, W), np.float64)
    ncomp = np.empty((H, W), np.int32)
    margin = np.empty((H, W), np.float64)
    rc = lib().orc_render(MODES[mode], int(bool(prefilter)), p, n, n, int(sh_degree), _cam_floats(cam), W, H,
                          float(znear), np.ascontiguousarray(bg, np.float32), rgb, depth, alpha, tfin, ncomp, margin)
    assert rc == 0
    return dict(rgb=rgb, depth=depth, alpha=alpha, tfinal=tfin, ncomp=ncomp, margin=margin)


def backward(params, sh_degree, cams, grads, pinned=True, bg=(0.0, 0.0, 0.0), znear=0.2, want_2d=False):
    """FP64 analytic gradient of sum_v <grads_v, (rgb_v, depth_v, alpha_v)> with respect
    to the parameters [P, N]. grads: list of (g_rgb [3,H,W], g_depth [H,W], g_alpha [H,W]).
    pinned: False = FP64 decisions; True = decisions from the FP32 recurrence;
    "splats32" = FP32 decisions and FP32-rounded screen-space splat values
    (u, v, conic, opacity, colour, depth), FP64 arithmetic."""
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
    mode = 2 if pinned == "splats32" else int(bool(pinned))
    rc = lib().orc_backward(mode, p, n, n, int(sh_degree), len(cams), camf, wh, float(znear),
                            np.ascontiguousarray(bg, np.float32), grgb, gdep, galp, grad,
                            g2.ctypes.data if want_2d else None)
    assert rc == 0
    return (grad, g2) if want_2d else grad


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
