"""Keyframe insertion (gsr_densify) through the C ABI against the oracle's
definition, its capacity rule, and a mapping iteration on the grown map."""
import sys

import numpy as np
import pytest
import torch

import scenes
from parity import AMBIGUOUS_MARGIN, image_violations

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2509_06433_amd import _lib, rasterize
    return _lib, rasterize


def keyframe_case(seed=41):
    """A map covering part of the view, and an RGB-D observation of the view."""
    rng = np.random.default_rng(seed)
    s = scenes.tiny_random(seed, n=80, width=96, height=72)
    cam = s.cameras[0]
    depth = rng.uniform(1.0, 4.0, (72, 96)).astype(np.float32)
    depth[rng.random((72, 96)) < 0.05] = np.nan           # holes in the depth image
    rgb = rng.uniform(0.0, 1.0, (3, 72, 96)).astype(np.float32)
    return s, cam, rgb, depth


def check_new(got, ref, label):
    assert got.shape == ref.shape, (label, got.shape, ref.shape)
    for planes, rtol, atol in ((slice(0, 3), 1e-6, 1e-6), (slice(3, 6), 0, 2e-6), (slice(6, 11), 0, 0),
                               (slice(11, None), 1e-6, 1e-6)):
        a, b = got[planes].astype(np.float64), ref[planes]
        assert np.allclose(a, b, rtol=rtol, atol=atol), (label, planes, np.abs(a - b).max())


def test_densify_matches_oracle(gpu, orc):
    _lib, rasterize = gpu
    s, cam, rgb, depth = keyframe_case()
    R = rasterize.Rasterizer()
    p = torch.from_numpy(s.params).cuda()
    cov = R.render(p, 0, [cam])[0][2]
    cap = s.num + 3000
    buf = torch.zeros(s.params.shape[0], cap, device="cuda")
    buf[:, :s.num] = p
    opts = dict(step=3, alpha_below=0.9, depth_min=1.2, depth_max=3.8, scale_factor=0.8, opacity_logit=-0.5)
    added, wanted = _lib.gsr_densify(R.handle, buf, s.num, 0, cam, torch.from_numpy(rgb).cuda(),
                                     torch.from_numpy(depth).cuda(), cov, **opts)
    ref, pix = orc.densify(0, cam, rgb, depth, coverage=cov.cpu().numpy(), **opts)
    say("seeded", added, "of", wanted, "oracle", ref.shape[1])
    assert added == wanted == ref.shape[1] > 20
    got = buf[:, s.num:s.num + added].cpu().numpy()
    check_new(got, ref, "densify")
    assert torch.equal(buf[:, :s.num], p)                      # the map itself is untouched
    assert (buf[:, s.num + added:] == 0).all()                 # nothing past the new ones
    # a buffer too small: the first ones in pixel order, and the count wanted
    room = wanted // 2
    small = torch.zeros(s.params.shape[0], s.num + room, device="cuda")
    small[:, :s.num] = p
    a2, w2 = _lib.gsr_densify(R.handle, small, s.num, 0, cam, torch.from_numpy(rgb).cuda(),
                              torch.from_numpy(depth).cuda(), cov, **opts)
    assert (a2, w2) == (room, wanted)
    check_new(small[:, s.num:].cpu().numpy(), ref[:, :room], "densify, full buffer")


def test_map_grows_and_mapping_iteration_recaptures(gpu, orc):
    """GaussianMap.insert_keyframe grows its buffers; the next mapping
    iteration (with Adam) runs on the grown map with a new capture, and its
    images equal the oracle's render of the grown map."""
    _lib, rasterize = gpu
    s, cam, rgb, depth = keyframe_case(43)
    R = rasterize.Rasterizer()
    M = rasterize.GaussianMap(torch.from_numpy(s.params).cuda(), 0, capacity=s.num + 10)
    targets = [(torch.from_numpy(rgb).cuda(), torch.nan_to_num(torch.from_numpy(depth), nan=0.0).cuda())]
    lrs = [1e-3] * 14
    outs = R.alloc_images([cam])

    def iterate(step):
        grad = M.zeros()
        R.mapping_iteration(M.params, 0, [cam], outs, targets, grad, 0.5, None,
                            dict(m=M.m, v=M.v, lr=lrs, step=step))
        torch.cuda.synchronize()
        return R.mapping_status()

    st = iterate(1)
    assert st["captures"] == 1
    cov = outs[0][2].clone()
    n0 = M.num
    added = M.insert_keyframe(R, cam, targets[0][0], targets[0][1], cov, step=4, alpha_below=0.6,
                              depth_min=1.0, depth_max=4.0)
    say("added", added, "capacity", M.capacity)
    assert added > 10 and M.num == n0 + added and M.capacity >= M.num
    assert (M.m[:, n0:] == 0).all() and (M.v[:, n0:] == 0).all()
    st = iterate(0)
    assert st["captures"] == 2 and st["skipped"] == 0 and st["iterations"] == 2
    # the images the replay rendered are those of the grown map before its Adam step:
    # render the same map eagerly and against the oracle
    E = rasterize.Rasterizer()
    grown = M.params.clone()
    ref_outs = E.render(grown, 0, [cam])
    r = orc.render(grown.cpu().numpy(), 0, cam, mode="f32")
    mask = r["margin"] >= AMBIGUOUS_MARGIN
    for ch in range(3):
        assert image_violations(ref_outs[0][0][ch].cpu().numpy(), r["rgb"][ch], mask)[0] == 0
    assert torch.isfinite(M.params).all()
