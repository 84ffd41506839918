"""Pins of the oracle's analytic backward (FP64), loss and Adam: central finite
differences, an independent torch float64 autograd renderer, torch's L1 loss
and torch.optim.Adam. CPU only."""
import numpy as np
import pytest
import torch

import scenes
from scenes import identity_camera

import torch_ref


def _masked_grads(orc, s, seed, margin_floor=1e-3):
    """Seeded upstream gradients with pixels near a decision threshold zeroed,
    so that a small parameter step cannot move a contributing decision."""
    grads = scenes.random_image_grads(seed, s.cameras)
    out = []
    for cam, (gr, gd, ga) in zip(s.cameras, grads):
        r = orc.render(s.params, s.sh_degree, cam, mode="f64")
        keep = (r["margin"] > margin_floor).astype(np.float32)
        out.append((gr * keep[None], gd * keep, ga * keep))
    return out


def _objective(orc, params, s, grads):
    total = 0.0
    for cam, (gr, gd, ga) in zip(s.cameras, grads):
        r = orc.render(params, s.sh_degree, cam, mode="f64")
        total += (gr * r["rgb"]).sum() + (gd * r["depth"]).sum() + (ga * r["alpha"]).sum()
    return total


@pytest.mark.parametrize("k,deg,two_views", [(0, 0, False), (1, 3, False), (2, 1, True)])
def test_backward_matches_central_differences(orc, k, deg, two_views):
    s = scenes.tiny_random(k, n=10, width=28, height=24, sh_degree=deg)
    if two_views:
        s.cameras.append(scenes.look_at_camera([0.4, -0.3, -0.2], [0.0, 0.0, 2.0], 26, 22, 24.0))
    grads = _masked_grads(orc, s, k)
    g = orc.backward(s.params, s.sh_degree, s.cameras, grads, pinned=False)
    rng = np.random.default_rng(k)
    P, n = s.params.shape
    # the parameters are float32; perturb them in float32 with a step that
    # is exactly representable relative to each value
    checked = bad = 0
    for _ in range(60):
        pl, i = int(rng.integers(0, P)), int(rng.integers(0, n))
        theta = float(s.params[pl, i])
        h = 2.0 ** (np.floor(np.log2(max(abs(theta), 0.25))) - 12)
        vals = []
        for sgn in (+1, -1, +2, -2):
            p = s.params.copy()
            p[pl, i] = np.float32(theta + sgn * h)
            vals.append(_objective(orc, p, s, grads))
        fd1 = (vals[0] - vals[1]) / (2 * h)
        fd2 = (vals[2] - vals[3]) / (4 * h)
        if abs(fd1 - fd2) > 1e-3 * max(abs(fd1), 1e-3):
            continue                                # non-smooth here (kink), skip
        checked += 1
        scale = max(abs(fd1), 1e-2 * np.abs(g[pl]).max(), 1e-8)
        if abs(g[pl, i] - fd1) > 2e-3 * scale:
            bad += 1
    assert checked >= 45
    assert bad == 0


@pytest.mark.parametrize("k,deg", [(5, 0), (6, 3), (7, 2)])
def test_backward_matches_torch_autograd(orc, k, deg):
    s = scenes.tiny_random(k, n=14, width=30, height=26, sh_degree=deg)
    grads = scenes.random_image_grads(k, s.cameras)
    g = orc.backward(s.params, deg, s.cameras, grads, pinned=False)
    p = torch.tensor(s.params, dtype=torch.float64, requires_grad=True)
    rgb, depth, alpha = torch_ref.render(p, deg, s.cameras[0])
    gr, gd, ga = grads[0]
    L = (torch.tensor(gr, dtype=torch.float64) * rgb).sum() + (torch.tensor(gd, dtype=torch.float64) * depth).sum() \
        + (torch.tensor(ga, dtype=torch.float64) * alpha).sum()
    L.backward()
    ref = p.grad.numpy()
    # forward values agree too
    r = orc.render(s.params, deg, s.cameras[0], mode="f64")
    assert np.allclose(r["rgb"], rgb.detach().numpy(), rtol=1e-12, atol=1e-13)
    assert np.allclose(g, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


def test_pinned_equals_unpinned_away_from_thresholds(orc):
    s = scenes.tiny_random(8, n=16, width=32, height=32)
    grads = _masked_grads(orc, s, 8, margin_floor=1e-4)
    a = orc.backward(s.params, 0, s.cameras, grads, pinned=True)
    b = orc.backward(s.params, 0, s.cameras, grads, pinned=False)
    assert np.allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(b).max())


def test_screen_space_gradients_sum_over_views(orc):
    s = scenes.tiny_random(9, n=12, width=24, height=20)
    cams = [s.cameras[0], identity_camera(24, 20, 22.0, cx=11.0, cy=9.0)]
    grads = scenes.random_image_grads(9, cams)
    both = orc.backward(s.params, 0, cams, grads, pinned=True)
    one = orc.backward(s.params, 0, cams[:1], grads[:1], pinned=True)
    two = orc.backward(s.params, 0, cams[1:], grads[1:], pinned=True)
    assert np.allclose(both, one + two, rtol=1e-12, atol=1e-15)


def test_l1_loss_matches_torch(orc):
    rng = np.random.default_rng(0)
    rgb, trgb = rng.random((3, 7, 9)), rng.random((3, 7, 9))
    dep, tdep = rng.random((7, 9)) * 4, rng.random((7, 9)) * 4
    dep[0, 0] = tdep[0, 0]                       # sign(0) = 0
    L, gr, gd = orc.l1_loss_and_grad(rgb, dep, trgb, tdep)
    a = torch.tensor(rgb, requires_grad=True)
    b = torch.tensor(dep, requires_grad=True)
    T = torch.nn.functional.l1_loss(a, torch.tensor(trgb)) + 0.5 * torch.nn.functional.l1_loss(b, torch.tensor(tdep))
    T.backward()
    assert np.isclose(L, T.item(), rtol=1e-14)
    assert np.allclose(gr, a.grad.numpy(), rtol=1e-14)
    assert np.allclose(gd, b.grad.numpy(), rtol=1e-14)


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(1)
    P, n = 6, 50
    x0 = rng.normal(size=(P, n))
    lrs = np.array([1e-3, 2e-3, 5e-3, 1e-2, 3e-2, 1e-1])
    params = [torch.tensor(x0[i].copy(), requires_grad=True) for i in range(P)]
    opt = torch.optim.Adam([{"params": [params[i]], "lr": lrs[i]} for i in range(P)], betas=(0.9, 0.999), eps=1e-15)
    x, m, v = x0.copy(), np.zeros_like(x0), np.zeros_like(x0)
    for step in range(1, 6):
        g = rng.normal(size=(P, n))
        for i in range(P):
            params[i].grad = torch.tensor(g[i].copy())
        opt.step()
        x, m, v = orc.adam_step(x, g, m, v, step, lrs)
    ref = np.stack([p.detach().numpy() for p in params])
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-14)


def test_fp32_splat_rounding_changes_gradients_only_at_rounding_level(orc):
    # the FP32-splat reference differs from the FP64 one only by the rounding
    # of u, v, conic, opacity, colour and depth to float: per element by up to
    # about 1e-3 where the gradient is ill-conditioned (measured 1.2e-3 on this
    # scene), in relative L2 by about 1e-6
    from parity import grad_violations
    s = scenes.small_128x96()
    grads = _masked_grads(orc, s, 1, margin_floor=1e-5)
    a = orc.backward(s.params, 0, s.cameras, grads, pinned=True)
    b = orc.backward(s.params, 0, s.cameras, grads, pinned="splats32")
    for grp, (nbad, worst, l2) in grad_violations(b, a, rtol=3e-3).items():
        assert nbad == 0 and l2 < 1e-5, grp


@pytest.mark.parametrize("k,deg", [(5, 0), (6, 3)])
def test_splats32_matches_torch_at_fp32_splats(orc, k, deg):
    """The oracle's "splats32" gradient is the FP64 derivative of the
    compositing evaluated at the FP32 projection's splat values, chained
    through the FP64 projection: here torch autograd forms the same thing
    independently (the compositing of the FP32 splat values as float64 leaf
    tensors, its gradient pushed back through the float64 torch projection),
    on pixels away from every decision threshold."""
    s = scenes.tiny_random(k, n=14, width=30, height=26, sh_degree=deg)
    cam = s.cameras[0]
    grads = _masked_grads(orc, s, k, margin_floor=1e-3)
    g = orc.backward(s.params, deg, s.cameras, grads, pinned="splats32")
    p = torch.tensor(s.params, dtype=torch.float64, requires_grad=True)
    sp64 = torch_ref.project(p, deg, cam)
    pr = orc.project(s.params, deg, cam, prec=32)
    leaf = {}
    for key, src in (("u", "u"), ("v", "v"), ("A", "A"), ("B", "B"), ("C", "C"), ("o", "o"), ("z", "z")):
        leaf[key] = torch.tensor(np.where(pr["vis"], pr[src], sp64[key].detach().numpy()), requires_grad=True)
    col32 = np.stack([pr["r"], pr["g"], pr["b_"]], 1)
    leaf["col"] = torch.tensor(np.where(pr["vis"][:, None], col32, sp64["col"].detach().numpy()),
                               requires_grad=True)
    leaf["tz"], leaf["det"] = sp64["tz"].detach(), sp64["det"].detach()
    rgb, depth, alpha = torch_ref.composite(leaf, cam)
    gr, gd, ga = grads[0]
    L = (torch.tensor(gr, dtype=torch.float64) * rgb).sum() + (torch.tensor(gd, dtype=torch.float64) * depth).sum() \
        + (torch.tensor(ga, dtype=torch.float64) * alpha).sum()
    keys = ["u", "v", "A", "B", "C", "o", "col", "z"]
    dsp = torch.autograd.grad(L, [leaf[k2] for k2 in keys], allow_unused=True)
    outs = [sp64[k2] for k2 in keys]
    gsp = [d if d is not None else torch.zeros_like(o) for d, o in zip(dsp, outs)]
    torch.autograd.backward(outs, gsp)
    ref = p.grad.numpy()
    assert np.abs(ref).max() > 0
    assert np.allclose(g, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("k,deg", [(15, 0), (16, 3)])
def test_camera_gradient_matches_torch_autograd(orc, k, deg):
    """The oracle's camera gradient (dL/dR, dL/dt of x_cam = R x + t) against
    torch float64 autograd through the independent renderer."""
    s = scenes.tiny_random(k, n=14, width=30, height=26, sh_degree=deg)
    s.cameras = [scenes.look_at_camera([0.2, -0.1, -0.3], [0.05, 0.0, 2.0], 30, 26, 28.0)]
    cam = s.cameras[0]
    grads = _masked_grads(orc, s, k, margin_floor=1e-3)
    _, gcam = orc.backward(s.params, deg, s.cameras, grads, pinned=False, want_cam=True)
    p = torch.tensor(s.params, dtype=torch.float64)
    Rt = torch.tensor(np.asarray(cam.R, np.float32).astype(np.float64), requires_grad=True)
    tt = torch.tensor(np.asarray(cam.t, np.float32).astype(np.float64), requires_grad=True)
    rgb, depth, alpha = torch_ref.render(p, deg, cam, pose_R=Rt, pose_t=tt)
    gr, gd, ga = grads[0]
    L = (torch.tensor(gr, dtype=torch.float64) * rgb).sum() + (torch.tensor(gd, dtype=torch.float64) * depth).sum() \
        + (torch.tensor(ga, dtype=torch.float64) * alpha).sum()
    L.backward()
    ref = np.concatenate([Rt.grad.numpy().ravel(), tt.grad.numpy()])
    assert np.abs(ref).max() > 0
    assert np.allclose(gcam[0], ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max()), (gcam[0], ref)


def test_camera_gradient_matches_central_differences(orc):
    """Each of the 12 camera entries (the rotation's nine entries taken as
    free, as the forward uses them) against central differences of the FP64
    oracle's render."""
    from scenes import Camera
    s = scenes.tiny_random(17, n=12, width=28, height=24, sh_degree=1)
    cam = scenes.look_at_camera([0.15, 0.1, -0.25], [0.0, 0.05, 2.0], 28, 24, 26.0)
    s.cameras = [cam]
    grads = _masked_grads(orc, s, 17, margin_floor=1e-3)
    _, gcam = orc.backward(s.params, 1, s.cameras, grads, pinned=False, want_cam=True)
    base = np.concatenate([np.asarray(cam.R, np.float32).ravel(), np.asarray(cam.t, np.float32)])
    checked = 0
    for k in range(12):
        # a camera step moves every splat: 2^-16 (exact in float for entries
        # below 1) keeps every pixel's decisions where they are
        h = 2.0 ** -16
        vals = []
        for sgn in (+1, -1, +2, -2):
            x = base.astype(np.float64).copy()
            x[k] += sgn * h
            x = x.astype(np.float32)
            c = Camera(x[:9].reshape(3, 3), x[9:], cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height)
            r = orc.render(s.params, 1, c, mode="f64")
            gr, gd, ga = grads[0]
            vals.append((gr * r["rgb"]).sum() + (gd * r["depth"]).sum() + (ga * r["alpha"]).sum())
        fd1 = (vals[0] - vals[1]) / (2 * h)
        fd2 = (vals[2] - vals[3]) / (4 * h)
        if abs(fd1 - fd2) > 1e-3 * max(abs(fd1), 1e-6):
            continue
        checked += 1
        scale = max(abs(fd1), 1e-2 * np.abs(gcam[0]).max())
        assert abs(gcam[0, k] - fd1) <= 1e-3 * scale, (k, gcam[0, k], fd1)
    assert checked >= 11


@pytest.mark.parametrize("k,deg", [(21, 0), (22, 3)])
def test_summand_magnitudes_bound_the_gradient(orc, k, deg):
    """The summand-magnitude output is, per parameter, the sum of the absolute
    values of the terms whose signed sum is the gradient, so by the triangle
    inequality it is never below |gradient|; on a generic scene with signed
    upstream gradients it exceeds it somewhere (the sums cancel)."""
    s = scenes.tiny_random(k, n=20, width=40, height=34, sh_degree=deg)
    grads = scenes.random_image_grads(k, s.cameras)
    g, a = orc.backward(s.params, deg, s.cameras, grads, pinned=True, want_abs=True)
    assert a.shape == g.shape and np.all(a >= 0)
    # up to rounding residues where the exact gradient is zero
    assert np.all(np.abs(g) <= a * (1 + 1e-12) + 1e-12 * a.max())
    assert np.any(a > 2 * np.abs(g))
    # odd in the upstream gradient for g, even for a
    neg = [(-gr, -gd, -ga) for gr, gd, ga in grads]
    g2, a2 = orc.backward(s.params, deg, s.cameras, neg, pinned=True, want_abs=True)
    assert np.allclose(g2, -g, rtol=1e-12, atol=0) and np.allclose(a2, a, rtol=1e-12, atol=0)


def test_summand_magnitudes_equal_gradient_without_cancellation(orc):
    """With a positive colour gradient only, every term of the degree-0
    colour coefficients' gradient (blend weight x upstream gradient x Y00,
    where the colour is not clamped) is non-negative: there the bound is the
    gradient itself. A missing or doubled term on either side breaks this."""
    s = scenes.tiny_random(23, n=20, width=40, height=34, sh_degree=0)
    cam = s.cameras[0]
    rng = np.random.default_rng(23)
    gr = rng.uniform(0.5, 1.5, (3, cam.height, cam.width)).astype(np.float32)
    z = np.zeros((cam.height, cam.width), np.float32)
    g, a = orc.backward(s.params, 0, s.cameras, [(gr, z, z)], pinned=True, want_abs=True)
    sh0 = slice(11, 14)
    assert np.all(g[sh0] >= 0) and np.count_nonzero(g[sh0]) > 10
    assert np.allclose(a[sh0], g[sh0], rtol=1e-12, atol=0)
    # the means do cancel: their terms have both signs
    assert np.any(a[0:3] > 1.5 * np.abs(g[0:3]))
