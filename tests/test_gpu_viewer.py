"""The viewer process (gsr_viewer) on the live map of a mapping process,
through the inter-process handles of the C ABI: a frame it renders equals the
mapping process's own render of the same view (bit for bit) and the FP32
oracle; at the paper's viewer resolution (672x376) and 30 frames per second it
runs beside the mapping loop, whose rate is measured with and without it."""
import os
import sys
import time

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
    from paper_2509_06433_amd import rasterize, viewer
    return rasterize, viewer


def viewer_camera(cam):
    """The keyframe's pose at 672x376 (the paper's viewer resolution), same field of view."""
    f = cam.fx * 672 / cam.width
    return scenes.Camera(cam.R, cam.t, f, f, 336.0, 188.0, 672, 376)


def test_viewer_frame_equals_render_and_oracle(gpu, orc, tmp_path):
    rasterize, viewer = gpu
    s = scenes.keyframe_640x480()
    p = torch.from_numpy(s.params).cuda()
    shared = viewer.SharedMap(p, 0, with_event=False)
    say("exported", shared.alloc_bytes, "bytes at offset", shared.offset)
    cam = viewer_camera(s.cameras[0])
    dump = str(tmp_path / "frame.bin")
    v = viewer.ViewerProcess(shared, cam, frames=3, dump=dump)
    rep = v.wait()
    say("viewer", rep)
    assert rep["frames"] == 3 and rep["status"] == 0
    rgb, depth, alpha, camf, (W, H) = viewer.read_dump(dump)
    assert (W, H) == (672, 376)
    assert np.array_equal(camf, np.asarray(cam.as_floats(), np.float32))
    R = rasterize.Rasterizer()
    own = R.render(p, 0, [cam])[0]
    assert np.array_equal(rgb, own[0].cpu().numpy())
    assert np.array_equal(depth, own[1].cpu().numpy()) and np.array_equal(alpha, own[2].cpu().numpy())
    ref = orc.render(s.params, 0, cam, mode="f32")
    mask = ref["margin"] >= AMBIGUOUS_MARGIN
    for ch in range(3):
        assert image_violations(rgb[ch], ref["rgb"][ch], mask)[0] == 0
    assert image_violations(depth, ref["depth"], mask)[0] == 0
    shared.close()


def test_viewer_alongside_mapping(gpu):
    """The mapping loop (640x480, 200k Gaussians, with Adam, recording the
    inter-process event after each iteration) with and without the viewer
    rendering 672x376 frames at 30 per second, panning, each frame ordered
    after the mapper's last finished iteration (where the driver offers
    inter-process events; else the frames read the live buffer unordered).
    The loop issues each iteration from Python, so its rate is set by the
    host as much as by the GPU: the rate with the viewer is compared with
    the mean of the rates measured without it before and after, which
    brackets a drift of the host's speed over the test."""
    rasterize, viewer = gpu
    s = scenes.keyframe_640x480()
    p = torch.from_numpy(s.params).cuda()
    shared = viewer.SharedMap(p, 0)
    say("inter-process event:", "yes" if shared.event is not None else shared.event_error)
    R = rasterize.Rasterizer()
    E = rasterize.Rasterizer()
    targets = [(o[0].clone(), o[1].clone()) for o in E.render(torch.from_numpy(s.target_params).cuda(), 0, s.cameras)]
    outs = R.alloc_images(s.cameras)
    grad = torch.zeros_like(p)
    adam = dict(m=torch.zeros_like(p), v=torch.zeros_like(p), lr=[1e-4] * 14, step=1)

    def mapping(seconds):
        n = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            for _ in range(20):
                R.mapping_iteration(p, 0, s.cameras, outs, targets, grad, 0.5, None, adam)
                adam["step"] = 0
                shared.record()
            n += 20
            torch.cuda.synchronize()
        return n / (time.perf_counter() - t0)

    mapping(0.5)
    alone = mapping(2.0)
    v = viewer.ViewerProcess(shared, viewer_camera(s.cameras[0]), seconds=3.0, fps=30.0, pan_deg=4.0,
                             wait_event=shared.event is not None)
    v.wait_ready()
    together = mapping(2.5)
    rep = v.wait()
    after = mapping(1.0)
    say("mapping iters/s alone", round(alone, 1), "with the viewer", round(together, 1), "after", round(after, 1))
    say("viewer", rep)
    assert R.mapping_status()["skipped"] == 0
    assert rep["fps"] >= 28.0, rep
    assert together >= 0.85 * 0.5 * (alone + after), (alone, together, after)
    shared.close()
