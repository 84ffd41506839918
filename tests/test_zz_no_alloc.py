"""gsr_render_noalloc through the C ABI: the same images and sorted instance
list as gsr_render (bit for bit) on two calls in a row, the second with a
smaller input, and its limits refused up front."""
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


def render_both(_lib, rasterize, s, noalloc_ctx):
    p = torch.from_numpy(s.params).cuda()
    E = rasterize.Rasterizer()
    ref = E.render(p, s.sh_degree, s.cameras)
    t_ref, g_ref = E.instances()
    outs = rasterize.Rasterizer.alloc_images(s.cameras)
    for o in outs:
        for t in o:
            t.fill_(-7.0)
    _lib.gsr_render_noalloc(noalloc_ctx.handle, p, s.sh_degree, s.cameras, outs)
    torch.cuda.synchronize()
    st = noalloc_ctx.status()
    t_na, g_na = noalloc_ctx.instances()
    E.close()
    return ref, outs, st, (t_ref, g_ref), (t_na, g_na)


def test_noalloc_matches_render_on_two_calls(gpu, orc):
    _lib, rasterize = gpu
    R = rasterize.Rasterizer()
    # first a 640x480 view of 200k Gaussians, then a smaller scene and image
    for label, s in (("keyframe", scenes.keyframe_640x480()),
                     ("small", scenes.tiny_random(11, n=900, width=83, height=61))):
        say("noalloc case", label, s.num, s.cameras[0].width, s.cameras[0].height)
        ref, outs, st, (t_ref, g_ref), (t_na, g_na) = render_both(_lib, rasterize, s, R)
        say(label, "status", st)
        assert st["instances"] == len(t_ref)
        assert np.array_equal(t_na, t_ref) and np.array_equal(g_na, g_ref)
        for a, b in zip(outs[0], ref[0]):
            assert torch.equal(a, b), label
        # and, like gsr_render, within 1e-5 of the FP32 oracle off ambiguous pixels
        r = orc.render(s.params, s.sh_degree, s.cameras[0], mode="f32")
        mask = r["margin"] >= AMBIGUOUS_MARGIN
        rgb = outs[0][0].cpu().numpy()
        for ch in range(3):
            assert image_violations(rgb[ch], r["rgb"][ch], mask)[0] == 0
        assert image_violations(outs[0][1].cpu().numpy(), r["depth"], mask)[0] == 0
    R.close()


def test_noalloc_limits_refused(gpu):
    _lib, rasterize = gpu
    R = rasterize.Rasterizer()
    cam = scenes.identity_camera(64, 48, 50.0)
    big = torch.zeros(14, (1 << 18) + 1, device="cuda")
    outs = rasterize.Rasterizer.alloc_images([cam])
    with pytest.raises(_lib.GsrError) as e:
        _lib.gsr_render_noalloc(R.handle, big, 0, [cam], outs)
    assert e.value.status == -5
    wide = scenes.identity_camera(2048, 1024, 500.0)           # 2^21 pixels
    outs = rasterize.Rasterizer.alloc_images([wide])
    with pytest.raises(_lib.GsrError) as e:
        _lib.gsr_render_noalloc(R.handle, torch.zeros(14, 10, device="cuda"), 0, [wide], outs)
    assert e.value.status == -5
    R.close()
