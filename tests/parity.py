"""Tolerance metrics shared by the GPU parity tests.

Images (colour, depth): |x - ref| <= 1e-5 * max(|ref|, 0.01 * max|ref| of that
plane), evaluated on pixels whose compositing decisions are not ambiguous.
A pixel is ambiguous when some decision it took (alpha >= 1/255, alpha clamp
at 0.99, T (1 - alpha) >= 1e-4, exponent <= 0) lies within 1e-5 relative of
its threshold in the FP32 oracle: there the GPU's FP32 exponential (a few ulp
from the oracle's) may take the other branch.

Gradients: per parameter group, |g - ref| <= 1e-3 * max(|ref|, 0.01 * rms(ref_group),
1e-6 * rms(ref_all)); the last floor only matters for groups whose exact
gradient vanishes (rotations of isotropic Gaussians). The reference is the
oracle's FP64 backward at the FP32 projection's splat values (the values the
method composites). Against the FP64 backward at FP64 splat values the same
bar holds per element after adding that element's own sensitivity to the FP32
rounding of the splats, |ref_splats32 - ref_fp64|, which the oracle measures
without the GPU (grad_violations_conditioned).

Where a gradient element is a sum that cancels heavily (an L1 loss's sign
targets give upstream gradients of both signs and equal size everywhere), no
FP32 summation reaches 1e-3 of the result: its error scales with the sum of
the magnitudes of the terms, not with the sum. The oracle reports that
magnitude sum A per element (|grad| <= A); the full-size checks add
ACCUM_ULPS * 2^-24 * A to the tolerance. 64 units: each term is formed in a
handful of FP32 operations, summed in a six-level tree inside a wavefront,
then across wavefronts and tiles by atomic adds, whose rounding errors add up
like a random walk rather than in the worst case ((n - 1) units for n terms).
"""
import numpy as np

IMG_RTOL = 1e-5
GRAD_RTOL = 1e-3
AMBIGUOUS_MARGIN = 1e-5
ACCUM_ULPS = 64

GROUPS = {"mean": slice(0, 3), "logscale": slice(3, 6), "quat": slice(6, 10), "logit": slice(10, 11)}


def image_violations(x, ref, mask=None, rtol=IMG_RTOL):
    """(number of pixels outside tolerance, worst |x - ref| / tolerance) over `mask`."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = 0.01 * np.abs(ref).max() if ref.size else 0.0
    tol = rtol * np.maximum(np.abs(ref), floor)
    tol = np.where(tol > 0, tol, 1e-30)
    ratio = np.abs(x - ref) / tol
    if mask is not None:
        ratio = np.where(mask, ratio, 0.0)
    return int((ratio > 1.0).sum()), float(ratio.max(initial=0.0))


def grad_groups(P):
    g = dict(GROUPS)
    g["sh"] = slice(11, P)
    return g


def _accum(gabs, sl):
    if gabs is None:
        return 0.0
    return ACCUM_ULPS * 2.0 ** -24 * np.asarray(gabs[sl], np.float64).ravel()


def grad_violations(g, ref, rtol=GRAD_RTOL, gabs=None):
    """Returns {group: (violations, worst relative error, relative L2)}; with
    gabs (the oracle's summand magnitudes), the summation allowance is added
    to each element's tolerance and the worst error is reported relative to
    that tolerance."""
    out = {}
    P = ref.shape[0]
    ref = np.asarray(ref, np.float64)
    rms_all = np.sqrt(np.mean(ref * ref)) if ref.size else 0.0
    for name, sl in grad_groups(P).items():
        a = np.asarray(g[sl], np.float64).ravel()
        b = np.asarray(ref[sl], np.float64).ravel()
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        scale = np.maximum(np.abs(b), max(0.01 * rms, 1e-6 * rms_all))
        scale = np.where(scale > 0, scale, 1e-30)
        rel = np.abs(a - b) / (scale + _accum(gabs, sl) / rtol)
        l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-6 * rms_all * np.sqrt(b.size), 1e-300)
        out[name] = (int((rel > rtol).sum()), float(rel.max(initial=0.0)), float(l2))
    return out


def grad_violations_conditioned(g, ref64, ref32, rtol=GRAD_RTOL, gabs=None):
    """Per-element check against the FP64 backward at FP64 splat values:
    |g - ref64| <= rtol * max(|ref64|, floors) + |ref32 - ref64|, where ref32 is
    the oracle's FP64 backward at the FP32-rounded splat values. The added
    term is how far rounding the screen-space values (u, v, conic, opacity,
    colour, depth) to float moves this element's exact gradient: any method
    that composites FP32 splats carries it. Returns {group: (violations, worst
    |g - ref64| / tolerance, relative L2 vs ref64, elements that pass only
    with the added term)}. With gabs, the summation allowance is added too
    and counts as part of the added term."""
    out = {}
    P = ref64.shape[0]
    ref64 = np.asarray(ref64, np.float64)
    ref32 = np.asarray(ref32, np.float64)
    rms_all = np.sqrt(np.mean(ref64 * ref64)) if ref64.size else 0.0
    for name, sl in grad_groups(P).items():
        a = np.asarray(g[sl], np.float64).ravel()
        b = ref64[sl].ravel()
        c = ref32[sl].ravel()
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        base = rtol * np.maximum(np.abs(b), max(0.01 * rms, 1e-6 * rms_all))
        cond = np.abs(c - b) + _accum(gabs, sl)
        err = np.abs(a - b)
        tol = np.where(base + cond > 0, base + cond, 1e-300)
        l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-6 * rms_all * np.sqrt(b.size), 1e-300)
        widened = int(((err > base) & (err <= tol)).sum())
        out[name] = (int((err > tol).sum()), float((err / tol).max(initial=0.0)), float(l2), widened)
    return out
