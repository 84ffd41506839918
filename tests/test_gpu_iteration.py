"""GPU tests of the graph-replayed mapping iteration (gsr_mapping_iteration).

Every replay is checked against the eager entry points run on the same
parameters (render, loss, backward, Adam) with the program's own eager work
and synchronisations between replays: images bit-exact (same kernels, same
inputs), loss to float rounding, gradients to the order of their float
atomics, parameters after Adam to a few ulp. The first replay's images are
also checked against the FP32 oracle.
"""
import sys

import numpy as np
import pytest
import torch

import scenes
from parity import AMBIGUOUS_MARGIN, grad_violations, image_violations

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2509_06433_amd import rasterize
    return rasterize


def to_dev(p):
    return torch.from_numpy(np.ascontiguousarray(p)).cuda()


def lrs_for(P):
    return [1.6e-4] * 3 + [5e-3] * 3 + [1e-3] * 4 + [5e-2] + [2.5e-3] * 3 + [1.25e-4] * (P - 14)


def two_view_scene(sh_degree=1):
    s = scenes.tiny_random(11, n=300, width=70, height=45, sh_degree=sh_degree)
    s.cameras = [s.cameras[0], scenes.look_at_camera([0.25, -0.1, -0.4], [0, 0, 2], 53, 38, 45.0)]
    rng = np.random.default_rng(scenes.SEED_BASE + 515)
    s.target_params = scenes.perturb(rng, s.params, s.sh_degree)
    return s


def targets_for(gpu, s):
    E = gpu.Rasterizer()
    outs = E.render(to_dev(s.target_params), s.sh_degree, s.cameras)
    torch.cuda.synchronize()
    return [(o[0].clone(), o[1].clone()) for o in outs]


def eager_iteration(gpu, E, p, deg, cams, targets):
    outs = E.render(p, deg, cams)
    loss, gimgs = E.loss_l1(cams, outs, [(t[0], t[1], None) for t in targets], 0.5)
    g = E.render_backward(p, deg, cams, gimgs)
    return outs, loss, g


def check_grad_close(g, ref, label):
    res = grad_violations(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-4)
    say(label, res)
    for grp, (nbad, worst, l2) in res.items():
        assert nbad == 0, (label, grp, worst)


# (chunk_len, max_chunks, fuse_blend[, tile_order]): automatic (chunked and
# fused at this size), explicit chunks fused, whole lists fused, two
# launches, and the balanced tile order (weights from the previous replay)
@pytest.mark.parametrize("chunk", [(0, 0, 0), (16, 5, 0), (-1, 0, 1), (0, 0, -1), (0, 0, 0, 3)])
def test_replays_match_eager(gpu, orc, chunk):
    s = two_view_scene()
    deg, cams = s.sh_degree, s.cameras
    targets = targets_for(gpu, s)
    say("backward chunks, fused, tile order", chunk)
    opts = dict(chunk_len=chunk[0], max_chunks=chunk[1])
    order = chunk[3] if len(chunk) > 3 else 0
    R, E = gpu.Rasterizer(fuse_blend=chunk[2], tile_order=order, **opts), gpu.Rasterizer(**opts)
    p = to_dev(s.params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    grad = torch.full_like(p, 7.0)
    loss = torch.zeros(1, device="cuda")
    outs = R.alloc_images(cams)
    lrs = lrs_for(p.shape[0])
    for k in range(4):
        say("replay", k)
        p0, m0, v0 = p.clone(), m.clone(), v.clone()
        R.mapping_iteration(p, deg, cams, outs, targets, grad, 0.5, loss,
                            adam=dict(m=m, v=v, lr=lrs, step=1 if k == 0 else 0))
        torch.cuda.synchronize()
        eo, el, eg = eager_iteration(gpu, E, p0, deg, cams, targets)
        torch.cuda.synchronize()
        for view in range(len(cams)):
            for a, b in zip(outs[view], eo[view]):
                assert torch.equal(a, b), (k, view)
        assert abs(loss.item() - el.item()) <= 1e-6 * abs(el.item()) + 1e-9, (loss.item(), el.item())
        check_grad_close(grad, eg, f"replay {k}")
        # Adam on the replay's own gradient: step k + 1
        E.adam_step(p0, grad, m0, v0, lrs, k + 1)
        torch.cuda.synchronize()
        # the bias corrections differ in rounding only (float powf on the device)
        ulp = torch.abs(p0).clamp_min(1e-30) * 2.0 ** -23
        lr_t = torch.tensor(lrs, device="cuda")[:, None]
        assert torch.all(torch.abs(p - p0) <= 4 * ulp + 1e-6 * lr_t), k
        assert torch.equal(m, m0) and torch.equal(v, v0)
        if k == 0:
            for view, cam in enumerate(cams):
                ref = orc.render(s.params, deg, cam, mode="f32")
                mask = ref["margin"] >= AMBIGUOUS_MARGIN
                rgb = eo[view][0].cpu().numpy()
                for ch in range(3):
                    nbad, worst = image_violations(rgb[ch], ref["rgb"][ch], mask)
                    assert nbad == 0, (view, ch, worst)
    st = R.mapping_status()
    say(st)
    assert st["iterations"] == 4 and st["skipped"] == 0 and st["captures"] == 1 and st["adam_steps"] == 4
    assert st["last_instances"] == R.status()["instances"]


def test_pose_change_without_recapture(gpu):
    s = two_view_scene(sh_degree=0)
    deg = s.sh_degree
    targets = targets_for(gpu, s)
    R, E = gpu.Rasterizer(), gpu.Rasterizer()
    p = to_dev(s.params)
    grad = torch.zeros_like(p)
    outs = R.alloc_images(s.cameras)
    R.mapping_iteration(p, deg, s.cameras, outs, targets, grad)
    moved = [s.cameras[0], scenes.look_at_camera([0.2, 0.05, -0.45], [0.05, 0, 2], 53, 38, 47.0)]
    R.mapping_iteration(p, deg, moved, outs, targets, grad)
    torch.cuda.synchronize()
    eo, el, eg = eager_iteration(gpu, E, p, deg, moved, targets)
    torch.cuda.synchronize()
    for view in range(2):
        for a, b in zip(outs[view], eo[view]):
            assert torch.equal(a, b), view
    check_grad_close(grad, eg, "moved camera")
    st = R.mapping_status()
    assert st["captures"] == 1 and st["iterations"] == 2


def test_no_adam_overwrites_gradient(gpu):
    s = two_view_scene(sh_degree=0)
    targets = targets_for(gpu, s)
    R, E = gpu.Rasterizer(), gpu.Rasterizer()
    p = to_dev(s.params)
    grad = torch.full_like(p, -3.0)
    p_copy = p.clone()
    R.mapping_iteration(p, 0, s.cameras, R.alloc_images(s.cameras), targets, grad)
    torch.cuda.synchronize()
    assert torch.equal(p, p_copy)
    _, _, eg = eager_iteration(gpu, E, p, 0, s.cameras, targets)
    check_grad_close(grad, eg, "no adam")


def test_overflow_skips_then_recaptures(gpu):
    # small Gaussians first, then (same buffer) scaled up so every Gaussian
    # covers many tiles: the instance count outgrows the captured capacity
    s = scenes.tiny_random(12, n=3000, width=128, height=96, sh_degree=0, anisotropic=False)
    s.params[3:6] = np.float32(-6.0)
    s.target_params = s.params.copy()
    targets = targets_for(gpu, s)
    R, E = gpu.Rasterizer(), gpu.Rasterizer()
    p = to_dev(s.params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    grad = torch.zeros_like(p)
    outs = R.alloc_images(s.cameras)
    lrs = lrs_for(p.shape[0])
    R.mapping_iteration(p, 0, s.cameras, outs, targets, grad, adam=dict(m=m, v=v, lr=lrs, step=1))
    st = R.mapping_status()
    say("before", st)
    assert st["skipped"] == 0 and st["iterations"] == 1
    cap = st["capacity"]
    p[3:6] = -1.0
    p_before, m_before, v_before = p.clone(), m.clone(), v.clone()
    R.mapping_iteration(p, 0, s.cameras, outs, targets, grad, adam=dict(m=m, v=v, lr=lrs))
    st = R.mapping_status()
    say("overflow", st)
    assert st["last_instances"] > cap
    assert st["skipped"] == 1 and st["iterations"] == 1 and st["adam_steps"] == 1
    assert torch.equal(p, p_before) and torch.equal(m, m_before) and torch.equal(v, v_before)
    # next call sees the skip and captures a larger graph
    R.mapping_iteration(p, 0, s.cameras, outs, targets, grad, adam=dict(m=m, v=v, lr=lrs))
    st = R.mapping_status()
    say("recaptured", st)
    assert st["captures"] == 2 and st["capacity"] >= st["last_instances"] and st["iterations"] == 2
    assert st["adam_steps"] == 2
    eo, _, eg = eager_iteration(gpu, E, p_before, 0, s.cameras, targets)
    torch.cuda.synchronize()
    for a, b in zip(outs[0], eo[0]):
        assert torch.equal(a, b)
    check_grad_close(grad, eg, "after recapture")


@pytest.mark.parametrize("fuse", [0, -1])
def test_profiled_replays(gpu, fuse):
    # with the fused blend launch (automatic at this size) its time is the
    # "blend" stage, else "blend_bwd"
    s = two_view_scene(sh_degree=0)
    targets = targets_for(gpu, s)
    R = gpu.Rasterizer(fuse_blend=fuse)
    p = to_dev(s.params)
    grad = torch.zeros_like(p)
    outs = R.alloc_images(s.cameras)
    blend = "blend" if fuse == 0 else "blend_bwd"
    R.set_profiling([blend, "project"])
    R.profile(reset=True)
    for _ in range(3):
        R.mapping_iteration(p, 0, s.cameras, outs, targets, grad)
    torch.cuda.synchronize()
    prof = R.profile(reset=True)
    say(prof)
    assert prof[blend][1] == 3 and prof["project"][1] == 3
    assert prof[blend][0] > 0 and prof["project"][0] > 0
    assert prof["blend_fwd"][1] == 0


def test_eager_after_iteration_uses_own_buffers(gpu, orc):
    s = two_view_scene(sh_degree=0)
    targets = targets_for(gpu, s)
    R = gpu.Rasterizer()
    p = to_dev(s.params)
    grad = torch.zeros_like(p)
    R.mapping_iteration(p, 0, s.cameras, R.alloc_images(s.cameras), targets, grad)
    one = [s.cameras[1]]
    R.render(p, 0, one)
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(s.params, 0, one, 16, 16)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)
    # and the next replay is unaffected by the eager render in between
    outs = R.alloc_images(s.cameras)
    R.mapping_iteration(p, 0, s.cameras, outs, targets, grad)
    torch.cuda.synchronize()
    E = gpu.Rasterizer()
    eo = E.render(p, 0, s.cameras)
    for view in range(2):
        for a, b in zip(outs[view], eo[view]):
            assert torch.equal(a, b)


def test_autotuner_picks_a_timed_candidate(gpu, tmp_path, monkeypatch):
    monkeypatch.setenv("GSR_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2509_06433_amd import autotune
    s = two_view_scene(sh_degree=0)
    targets = targets_for(gpu, s)
    p = to_dev(s.params)
    p0 = p.clone()
    cands = [(16, 16, 1, 0, 0, 0), (16, 8, 2, 32, -1, 0), (8, 8, 1, 64, 16, 8)]
    res = autotune.tune(p, 0, s.cameras, targets, candidates=cands, warmup=1, steps=2)
    say(res)
    assert not res["cached"] and len(res["table"]) == 3
    assert tuple(res[f] for f in autotune.FIELDS) in cands
    assert res["ms"] == min(r[-1] for r in res["table"]) and res["ms"] > 0
    assert torch.equal(p, p0)
    again = autotune.tune(p, 0, s.cameras, targets, candidates=cands)
    assert again["cached"] and again["tile_w"] == res["tile_w"]


@pytest.mark.parametrize("chunk_len", [0, -1])
def test_queue_fused_launch_matches_eager(gpu, orc, chunk_len):
    """The fused blend launch over a work queue: 8 views of 320x240 (2400
    tiles, more than the workgroups the device holds at once), chunked and
    whole lists. Images bit-exact and gradients to float order against the
    eager entry points, over three replays; the first replay's images against
    the FP32 oracle."""
    s = scenes.tiny_random(31, n=4000, width=320, height=240, sh_degree=1)
    rng = np.random.default_rng(scenes.SEED_BASE + 531)
    cams = [s.cameras[0]]
    for k in range(7):
        eye = [0.3 * np.cos(k), 0.15 * np.sin(2 * k), -0.5 + 0.05 * k]
        cams.append(scenes.look_at_camera(eye, [0.0, 0.0, 2.5], 320, 240, 260.0))
    s.cameras = cams
    s.target_params = scenes.perturb(rng, s.params, s.sh_degree)
    deg = s.sh_degree
    targets = targets_for(gpu, s)
    R = gpu.Rasterizer(fuse_blend=1, chunk_len=chunk_len)
    E = gpu.Rasterizer(chunk_len=chunk_len)
    p = to_dev(s.params)
    grad = torch.zeros_like(p)
    loss = torch.zeros(1, device="cuda")
    outs = R.alloc_images(cams)
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    say("queue fused launch: tiles", tiles, "chunk_len", chunk_len)
    assert tiles == 2400
    for k in range(3):
        R.mapping_iteration(p, deg, cams, outs, targets, grad, 0.5, loss)
        torch.cuda.synchronize()
        eo, el, eg = eager_iteration(gpu, E, p, deg, cams, targets)
        torch.cuda.synchronize()
        for view in range(len(cams)):
            for a, b in zip(outs[view], eo[view]):
                assert torch.equal(a, b), (k, view)
        # the loss is a float sum over 614k pixels in both launches, added
        # up in different orders (workgroup atomics in different numbers)
        assert abs(loss.item() - el.item()) <= 1e-5 * abs(el.item()) + 1e-9, (loss.item(), el.item())
        check_grad_close(grad, eg, f"queue replay {k}")
        if k == 0:
            for view in (0, 5):
                ref = orc.render(s.params, deg, cams[view], mode="f32")
                mask = ref["margin"] >= AMBIGUOUS_MARGIN
                rgb = eo[view][0].cpu().numpy()
                for ch in range(3):
                    nbad, worst = image_violations(rgb[ch], ref["rgb"][ch], mask)
                    assert nbad == 0, (view, ch, worst)
    st = R.mapping_status()
    say(st)
    assert st["iterations"] == 3 and st["skipped"] == 0
