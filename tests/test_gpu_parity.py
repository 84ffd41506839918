"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Bit-exact: projected geometry (u, v, z, screen covariance, conic, opacity,
pixel rectangle) and the sorted instance list. Colour/depth/alpha within
1e-5 relative of the FP32 oracle off ambiguous pixels; parameter gradients
within 1e-3 relative of the FP64 oracle with FP32-pinned decisions.
"""
import sys

import numpy as np
import pytest
import torch

import scenes
from scenes import identity_camera
from parity import AMBIGUOUS_MARGIN, grad_violations, grad_violations_conditioned, image_violations

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


def make(gpu, **kw):
    return gpu.Rasterizer(**kw)


def to_dev(p):
    return torch.from_numpy(np.ascontiguousarray(p)).cuda()


def scene_cases():
    s_small = scenes.small_128x96()
    s_tiny = scenes.tiny_random(3, n=40, width=45, height=37)
    s_sh3 = scenes.tiny_random(6, n=60, width=50, height=42, sh_degree=3)
    return {"small": s_small, "tiny_ragged": s_tiny, "tiny_sh3": s_sh3}


CASES = scene_cases()


# ---------------------------------------------------------------------------
# projection and binning: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
def test_projection_bit_exact(gpu, orc, name):
    s = CASES[name]
    say("case", name)
    R = make(gpu)
    p = to_dev(s.params)
    R.render(p, s.sh_degree, s.cameras)
    sp = R.splats(0, s.num)
    ref = orc.project(s.params, s.sh_degree, s.cameras[0], prec=32)
    vis = ref["vis"]
    assert np.array_equal(sp[:, 15] >= 0, vis)
    f32 = lambda x: np.asarray(x, np.float32)
    for col, key in [(0, "u"), (1, "v"), (2, "z"), (3, "a"), (4, "b"), (5, "c"), (6, "A"), (7, "B"), (8, "C"),
                     (9, "o")]:
        assert np.array_equal(sp[vis, col], f32(ref[key][vis])), key
    assert np.array_equal(sp[vis, 13:16].astype(np.int32), ref["rect"][vis, :3])
    for col, key in [(10, "r"), (11, "g"), (12, "b_")]:
        assert np.allclose(sp[vis, col], ref[key][vis], rtol=2e-6, atol=1e-7), key


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 8)])
@pytest.mark.parametrize("name", list(CASES))
def test_tile_list_bit_exact(gpu, orc, name, tile):
    s = CASES[name]
    say("case", name, tile)
    R = make(gpu, tile_w=tile[0], tile_h=tile[1])
    R.render(to_dev(s.params), s.sh_degree, s.cameras)
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(s.params, s.sh_degree, s.cameras, tile[0], tile[1])
    assert len(t_gpu) == len(t_ref)
    assert np.array_equal(t_gpu, t_ref)
    assert np.array_equal(g_gpu, g_ref)


def depth_case(big):
    """(scene, params) of the depth-order tests (see below)."""
    if big == "all":
        s = scenes.tiny_random(23, n=5000, width=40, height=24)
        p = s.params.copy()
        p[3:6] = np.log(0.6)
        p[0:3, 1:10] = p[0:3, 0:1]
    elif big == "mixed":
        s = scenes.tiny_random(25, n=4000, width=96, height=32)
        p = s.params.copy()
        cam = s.cameras[0]
        rng = np.random.default_rng(scenes.SEED_BASE + 25)
        k = 2000
        z = 2.0 + rng.uniform(-0.2, 0.2, k)
        u, v = 16 + rng.uniform(-4, 4, k), 16 + rng.uniform(-4, 4, k)
        p[0, :k] = (u - cam.cx) / cam.fx * z
        p[1, :k] = (v - cam.cy) / cam.fy * z
        p[2, :k] = z
        p[3:6, :k] = np.log(0.09)
        p[3:6, k:] = np.log(0.03)
    else:
        s = scenes.tiny_random(24, n=300, width=70, height=45)
        p = s.params
    return s, p


@pytest.mark.parametrize("depth_sort", [1, 2])
@pytest.mark.parametrize("big", ["none", "all", "mixed"])
def test_tile_list_depth_sort_modes(gpu, orc, depth_sort, big):
    """Both depth orders (per tile after binning; once over all splats before
    binning) against the oracle's list, bit-exact. all: 5000 Gaussians large
    enough to cover every tile of a 40x24 view, so every list is longer than
    the 1536 entries a tile sorts in LDS; ten of them share one depth, so the
    index breaks their tie. mixed: on a 96x32 view 2000 Gaussians crowd the
    four left tiles (over 2000 entries each) while 2000 small ones spread over
    the rest (under 700), so both paths meet in one launch."""
    s, p = depth_case(big)
    R = make(gpu, depth_sort=depth_sort)
    outs = R.render(to_dev(p), s.sh_degree, s.cameras)
    torch.cuda.synchronize()
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(p, s.sh_degree, s.cameras, 16, 16)
    say("depth sort", depth_sort, "big", big, "instances", len(t_gpu), "lists",
        np.bincount(t_ref.astype(np.int64)).tolist())
    counts = np.bincount(t_ref.astype(np.int64))
    if big == "all":
        assert counts.min() > 1536
    elif big == "mixed":
        assert counts.max() > 1536 and counts[counts > 0].min() <= 1536
    assert len(t_gpu) == len(t_ref)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)
    # the other order gives bit-identical images
    O = make(gpu, depth_sort=3 - depth_sort)
    other = O.render(to_dev(p), s.sh_degree, s.cameras)
    torch.cuda.synchronize()
    for a, b in zip(outs[0], other[0]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("depth_sort", [1, 2])
def test_tile_list_bit_exact_large_sorts(gpu, orc, depth_sort):
    """600k Gaussians at 640x480, 4.5M instances: the tile sort takes
    reduce-then-scan passes (more than 2^19 keys) in both modes, the global
    depth sort its look-back passes over 600k keys, and lists of up to 4265
    entries reach the per-tile sort's path through global memory. Lists
    bit-exact against the oracle."""
    s = scenes.keyframe_640x480(n=600_000, seed_offset=7)
    say("large sorts, depth sort", depth_sort)
    R = make(gpu, depth_sort=depth_sort)
    R.render(to_dev(s.params), s.sh_degree, s.cameras)
    torch.cuda.synchronize()
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(s.params, s.sh_degree, s.cameras, 16, 16)
    assert s.num > 2**19 and len(t_ref) > 2**19
    assert len(t_gpu) == len(t_ref)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)


@pytest.mark.parametrize("case", ["none", "all", "mixed", "multiview", "tile8x8"])
def test_tile_list_counting_binning(gpu, orc, case):
    """The binning by counting (option binning = 1: per-workgroup tile counts,
    one scan, a scatter in LDS-atomic order, equal depths put in index order
    by the per-tile sort): lists bit-exact against the oracle, including ten
    Gaussians of one depth ("all") and lists past the per-tile sort's LDS
    capacity; images bit-identical to the radix binning's."""
    tw = th = 16
    if case == "multiview":
        s = scenes.tiny_random(4, n=80, width=45, height=37)
        cams = [s.cameras[0], identity_camera(29, 21, 25.0),
                scenes.look_at_camera([0.3, 0.1, -0.5], [0, 0, 2], 64, 33, 40.0)]
        p = s.params
    elif case == "tile8x8":
        s, p = depth_case("none")
        cams = s.cameras
        tw = th = 8
    else:
        s, p = depth_case(case)
        cams = s.cameras
    say("counting binning", case)
    R = make(gpu, binning=1, depth_sort=1, tile_w=tw, tile_h=th)
    outs = R.render(to_dev(p), s.sh_degree, cams)
    torch.cuda.synchronize()
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(p, s.sh_degree, cams, tw, th)
    assert len(t_gpu) == len(t_ref)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)
    assert R.status()["visible"] == int(sum(orc.project(p, s.sh_degree, c)["vis"].sum() for c in cams))
    O = make(gpu, depth_sort=1, tile_w=tw, tile_h=th)
    other = O.render(to_dev(p), s.sh_degree, cams)
    torch.cuda.synchronize()
    for v in range(len(cams)):
        for a, b in zip(outs[v], other[v]):
            assert torch.equal(a, b)


def block_case(case):
    """(scene, params, cameras, tile size) of the block-binning tests."""
    if case == "huge":
        # 9000 Gaussians over a 64x48 view: twelve 1x1-tile blocks whose lists
        # (about 9000 entries) take two rounds of keep masks, and every tile
        # list passes the per-tile sort's LDS capacity
        s = scenes.tiny_random(41, n=9000, width=64, height=48)
        p = s.params.copy()
        p[3:6] = np.log(0.5)
        return s, p, s.cameras, 16
    if case == "ragged8x8":
        # 8x8 tiles on 200x150: 475 tiles, so blocks of 2x1 tiles, the last
        # block column and tile row ragged
        s = scenes.tiny_random(42, n=2500, width=200, height=150)
        return s, s.params, s.cameras, 8
    if case == "multiview8x8":
        # three 160x120 views at 8x8 (900 tiles): 2x2-tile blocks, ragged
        # rows, one view looking away from the scene
        s = scenes.tiny_random(43, n=1500, width=160, height=120)
        cams = [s.cameras[0], scenes.look_at_camera([0.2, -0.1, -0.3], [0.1, 0.0, 2.0], 160, 120, 140.0),
                scenes.look_at_camera([0.0, 0.0, 0.0], [0.0, 0.0, -5.0], 160, 120, 140.0)]
        return s, s.params, cams, 8
    s, p = depth_case(case)
    return s, p, s.cameras, 16


@pytest.mark.parametrize("case", ["none", "all", "mixed", "huge", "ragged8x8", "multiview8x8"])
def test_tile_list_block_binning(gpu, orc, case):
    """Binning by blocks of tiles (option binning = 3; what the automatic
    choice takes for the per-tile depth order): one instance per (splat,
    block), one pass over the block ids, each tile's list filtered from its
    block's and sorted by depth. Lists bit-exact against the oracle, with
    block lists long enough for two rounds of keep masks ("huge"), lists past
    the LDS capacity, ragged blocks and several views; images bit-identical
    to the radix binning's (option 2)."""
    s, p, cams, t = block_case(case)
    say("block binning", case)
    R = make(gpu, binning=3, depth_sort=1, tile_w=t, tile_h=t)
    outs = R.render(to_dev(p), s.sh_degree, cams)
    torch.cuda.synchronize()
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(p, s.sh_degree, cams, t, t)
    counts = np.bincount(t_ref.astype(np.int64))
    say("instances", len(t_ref), "longest list", int(counts.max()) if len(counts) else 0)
    if case == "huge":
        assert counts.max() > 8192 and counts.min() > 1536
    assert len(t_gpu) == len(t_ref)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)
    assert R.status()["instances"] == len(t_ref)
    O = make(gpu, binning=2, depth_sort=1, tile_w=t, tile_h=t)
    other = O.render(to_dev(p), s.sh_degree, cams)
    torch.cuda.synchronize()
    for v in range(len(cams)):
        for a, b in zip(outs[v], other[v]):
            assert torch.equal(a, b)


def depth_range_case(case):
    """Scene whose depths span a chosen key range: "flat" puts every
    Gaussian at one depth (equal keys: the index decides the whole order),
    "one_digit" within 300 float ulps of 2.0 (one 9-bit digit), "two_digits"
    within 2e-3 of 2.0 (about 13 bits)."""
    s = scenes.tiny_random(44, n=3000, width=96, height=64)
    p = s.params.copy()
    cam = s.cameras[0]
    rng = np.random.default_rng(scenes.SEED_BASE + 44)
    n = p.shape[1]
    if case == "flat":
        z = np.full(n, 2.0, np.float32)
    elif case == "one_digit":
        z = (np.float32(2.0) + np.float32(np.spacing(np.float32(2.0))) *
             rng.integers(0, 300, n).astype(np.float32)).astype(np.float32)
    else:
        z = (2.0 + rng.uniform(0.0, 2e-3, n)).astype(np.float32)
    u, v = rng.uniform(0, cam.width, n), rng.uniform(0, cam.height, n)
    p[0] = ((u - cam.cx) / cam.fx * z).astype(np.float32)
    p[1] = ((v - cam.cy) / cam.fy * z).astype(np.float32)
    p[2] = z
    p[3:6] = np.log(0.02)
    return s, p


@pytest.mark.parametrize("binning", [2, 3])
@pytest.mark.parametrize("case", ["flat", "one_digit", "two_digits"])
def test_tile_list_depth_ranges(gpu, orc, case, binning):
    """The per-tile depth sort takes as many 9-bit passes as the range of a
    list's keys needs: none for equal depths, one or two for narrow ranges.
    Lists bit-exact against the oracle's (tile, depth, index) order with both
    the radix and the block binning."""
    s, p = depth_range_case(case)
    say("depth range", case, "binning", binning)
    R = make(gpu, binning=binning, depth_sort=1)
    R.render(to_dev(p), s.sh_degree, s.cameras)
    torch.cuda.synchronize()
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(p, s.sh_degree, s.cameras, 16, 16)
    zk = orc.project(p, s.sh_degree, s.cameras[0], prec=32)["z"]
    vis = orc.project(p, s.sh_degree, s.cameras[0], prec=32)["vis"]
    zs = np.unique(np.asarray(zk, np.float32)[vis])
    say("instances", len(t_ref), "distinct depths", len(zs))
    if case == "flat":
        assert len(zs) == 1
    assert len(t_gpu) == len(t_ref)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)


def ring_cameras(count, seed):
    """`count` small cameras on a ring around the tiny scenes' volume (z in
    [1, 3]); every seventh looks away from it, so that it culls everything."""
    rng = np.random.default_rng(seed)
    cams = []
    for k in range(count):
        t = 2.0 * np.pi * k / count
        eye = [0.5 * np.cos(t), 0.4 * np.sin(t), -0.4 + 0.3 * np.sin(3.0 * t)]
        target = [0.0, 0.0, -6.0] if k % 7 == 6 else [0.5 * rng.normal(), 0.5 * rng.normal(), 2.0]
        w, h = [(40, 30), (33, 27), (48, 20)][k % 3]
        cams.append(scenes.look_at_camera(eye, target, w, h, 1.6 * w))
    return cams


# several views: the lock-step cull, the colour coefficients staged once per
# Gaussian (degree > 0) and the views taken in chunks of 64 (70 views)
@pytest.mark.parametrize("deg,count", [(3, 5), (1, 70), (2, 17)])
def test_projection_multiview_bit_exact(gpu, orc, deg, count):
    s = scenes.tiny_random(7, n=90, width=40, height=30, sh_degree=deg)
    cams = ring_cameras(count, deg)
    say("degree", deg, "views", count)
    R = make(gpu)
    R.render(to_dev(s.params), deg, cams)
    f32 = lambda x: np.asarray(x, np.float32)
    seen = 0
    for v, cam in enumerate(cams):
        sp = R.splats(v, s.num)
        ref = orc.project(s.params, deg, cam, prec=32)
        vis = ref["vis"]
        seen += int(vis.sum())
        assert np.array_equal(sp[:, 15] >= 0, vis), v
        for col, key in [(0, "u"), (1, "v"), (2, "z"), (6, "A"), (7, "B"), (8, "C"), (9, "o")]:
            assert np.array_equal(sp[vis, col], f32(ref[key][vis])), (v, key)
        for col, key in [(10, "r"), (11, "g"), (12, "b_")]:
            assert np.allclose(sp[vis, col], ref[key][vis], rtol=2e-6, atol=1e-7), (v, key)
    assert seen > 2 * count
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(s.params, deg, cams, 16, 16)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)


def test_tile_list_multiview_bit_exact(gpu, orc):
    s = scenes.tiny_random(4, n=80, width=45, height=37)
    cams = [s.cameras[0], identity_camera(29, 21, 25.0), scenes.look_at_camera([0.3, 0.1, -0.5], [0, 0, 2], 64, 33, 40.0)]
    R = make(gpu)
    R.render(to_dev(s.params), 0, cams)
    t_gpu, g_gpu = R.instances()
    t_ref, g_ref = orc.tile_list(s.params, 0, cams, 16, 16)
    assert np.array_equal(t_gpu, t_ref) and np.array_equal(g_gpu, g_ref)


# ---------------------------------------------------------------------------
# forward images: 1e-5 relative off ambiguous pixels
# ---------------------------------------------------------------------------

def check_images(outs, ref, label):
    rgb, depth, alpha = [o.cpu().numpy() for o in outs]
    mask = ref["margin"] >= AMBIGUOUS_MARGIN
    amb = int((~mask).sum())
    say(label, "ambiguous pixels", amb, "of", mask.size)
    assert amb <= max(2, 1e-3 * mask.size)
    worst = {}
    for ch in range(3):
        nbad, worst[f"rgb{ch}"] = image_violations(rgb[ch], ref["rgb"][ch], mask)
        assert nbad == 0, (label, "rgb", ch, worst)
    nbad, worst["depth"] = image_violations(depth, ref["depth"], mask)
    assert nbad == 0, (label, "depth", worst)
    nbad, worst["alpha"] = image_violations(alpha, ref["alpha"], mask)
    assert nbad == 0, (label, "alpha", worst)
    say(label, "worst ratio to tolerance", worst)


@pytest.mark.parametrize("ppt", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_forward_matches_fp32_oracle(gpu, orc, name, ppt):
    s = CASES[name]
    say("case", name, "pixels per thread", ppt)
    R = make(gpu, pixels_per_thread=ppt)
    outs = R.render(to_dev(s.params), s.sh_degree, s.cameras)
    ref = orc.render(s.params, s.sh_degree, s.cameras[0], mode="f32")
    check_images(outs[0], ref, name)


def test_forward_background(gpu, orc):
    s = CASES["tiny_ragged"]
    bg = (0.25, 0.5, 0.75)
    R = make(gpu, bg=bg)
    outs = R.render(to_dev(s.params), 0, s.cameras)
    ref = orc.render(s.params, 0, s.cameras[0], mode="f32", bg=bg)
    check_images(outs[0], ref, "bg")


# ---------------------------------------------------------------------------
# backward: 1e-3 relative against the FP64 oracle (FP32-pinned decisions)
# ---------------------------------------------------------------------------

def masked_grads(orc, s, seed):
    grads = scenes.random_image_grads(seed, s.cameras)
    out = []
    for cam, (gr, gd, ga) in zip(s.cameras, grads):
        r = orc.render(s.params, s.sh_degree, cam, mode="f32")
        keep = (r["margin"] >= AMBIGUOUS_MARGIN).astype(np.float32)
        out.append((gr * keep[None], gd * keep, ga * keep))
    return out


def check_grads(g, ref, label, ref64=None, gabs=None):
    """Per element against the FP64 backward at the FP32 splats (1e-3); per
    element against the FP64 backward at FP64 splats (1e-3 plus the element's
    own sensitivity to the FP32 rounding of the splats, measured by the
    oracle), and relative L2 within 1e-4 there. With gabs (the oracle's
    summand magnitudes) both bars also allow for FP32 summation."""
    res = grad_violations(g, ref, gabs=gabs)
    say(label, "vs FP64 at FP32 splats", res)
    for grp, (nbad, worst, l2) in res.items():
        assert nbad == 0, (label, grp, nbad, worst, l2)
    if ref64 is not None:
        res = grad_violations_conditioned(g, ref64, ref, gabs=gabs)
        say(label, "vs FP64", res)
        for grp, (nbad, worst, l2, widened) in res.items():
            assert nbad == 0 and l2 <= 1e-4, (label, grp, nbad, worst, l2)


def oracle_grads(orc, s, cams, grads):
    return (orc.backward(s.params, s.sh_degree, cams, grads, pinned="splats32"),
            orc.backward(s.params, s.sh_degree, cams, grads, pinned=True))


@pytest.mark.parametrize("ppt", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_backward_matches_fp64_oracle(gpu, orc, name, ppt):
    s = CASES[name]
    say("case", name, "pixels per thread", ppt)
    grads = masked_grads(orc, s, 1)
    R = make(gpu, pixels_per_thread=ppt)
    p = to_dev(s.params)
    R.render(p, s.sh_degree, s.cameras)
    dgr = [tuple(to_dev(x) for x in gv) for gv in grads]
    g = R.render_backward(p, s.sh_degree, s.cameras, dgr).cpu().numpy()
    ref32, ref64 = oracle_grads(orc, s, s.cameras, grads)
    check_grads(g, ref32, name, ref64)


@pytest.mark.parametrize("depth", [16, 32, 64])
def test_backward_batch_depth(gpu, orc, depth):
    s = CASES["small"]
    say("batch depth", depth)
    grads = masked_grads(orc, s, 4)
    R = make(gpu, batch_depth=depth)
    p = to_dev(s.params)
    R.render(p, s.sh_degree, s.cameras)
    g = R.render_backward(p, s.sh_degree, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32, ref64 = oracle_grads(orc, s, s.cameras, grads)
    check_grads(g, ref32, f"depth {depth}", ref64)


@pytest.mark.parametrize("chunk,nchunks,ppt", [(16, 4, 1), (16, 64, 1), (32, 3, 2), (16, 1, 1), (-1, 0, 1)])
def test_backward_chunked(gpu, orc, chunk, nchunks, ppt):
    """The backward split into chunks of the tile lists (each chunk's reverse
    walk starts from the state the forward recorded at its end) against the
    FP64 oracle; -1 walks whole tile lists."""
    s = CASES["small"]
    say("chunk", chunk, "chunks", nchunks, "pixels per thread", ppt)
    grads = masked_grads(orc, s, 6)
    R = make(gpu, chunk_len=chunk, max_chunks=nchunks, pixels_per_thread=ppt)
    p = to_dev(s.params)
    R.render(p, s.sh_degree, s.cameras)
    g = R.render_backward(p, s.sh_degree, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32, ref64 = oracle_grads(orc, s, s.cameras, grads)
    check_grads(g, ref32, f"chunk {chunk}x{nchunks}", ref64)


def test_backward_chunked_background_multiview(gpu, orc):
    s = scenes.tiny_random(4, n=50, width=40, height=30)
    s.cameras = [s.cameras[0], scenes.look_at_camera([0.3, 0.1, -0.5], [0, 0, 2], 36, 28, 30.0)]
    bg = (0.2, 0.5, 0.8)
    grads = masked_grads(orc, s, 7)
    R = make(gpu, chunk_len=16, max_chunks=3, bg=bg)
    p = to_dev(s.params)
    R.render(p, 0, s.cameras)
    g = R.render_backward(p, 0, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32 = orc.backward(s.params, 0, s.cameras, grads, pinned="splats32", bg=bg)
    ref64 = orc.backward(s.params, 0, s.cameras, grads, pinned=True, bg=bg)
    check_grads(g, ref32, "chunked, background, two views", ref64)


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 8)])
@pytest.mark.parametrize("name", list(CASES))
def test_backward_splat_parallel_matches_fp64_oracle(gpu, orc, name, tile):
    """The splat-parallel schedule (a wavefront per tile, a Gaussian per lane,
    the pixels pipelined through the lanes) against the FP64 oracle."""
    s = CASES[name]
    say("splat-parallel backward", name, tile)
    grads = masked_grads(orc, s, 12)
    R = make(gpu, tile_w=tile[0], tile_h=tile[1], backward_schedule=1)
    p = to_dev(s.params)
    R.render(p, s.sh_degree, s.cameras)
    g = R.render_backward(p, s.sh_degree, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32, ref64 = oracle_grads(orc, s, s.cameras, grads)
    check_grads(g, ref32, f"splat-parallel {name} {tile}", ref64)


def test_backward_splat_parallel_background_multiview_alpha(gpu, orc):
    """Splat-parallel: two views, a background colour and an alpha-image gradient."""
    s = scenes.tiny_random(4, n=50, width=40, height=30)
    s.cameras = [s.cameras[0], scenes.look_at_camera([0.3, 0.1, -0.5], [0, 0, 2], 36, 28, 30.0)]
    bg = (0.2, 0.5, 0.8)
    grads = masked_grads(orc, s, 13)
    R = make(gpu, bg=bg, backward_schedule=1)
    p = to_dev(s.params)
    R.render(p, 0, s.cameras)
    g = R.render_backward(p, 0, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32 = orc.backward(s.params, 0, s.cameras, grads, pinned="splats32", bg=bg)
    ref64 = orc.backward(s.params, 0, s.cameras, grads, pinned=True, bg=bg)
    check_grads(g, ref32, "splat-parallel, background, two views", ref64)


def test_backward_splat_parallel_long_lists(gpu, orc):
    """Splat-parallel with tile lists of several hundred Gaussians (many
    64-entry batches, pixels whose walks end in different batches)."""
    rng = np.random.default_rng(21)
    cam = identity_camera(64, 48, 60.0)
    n = 3000
    mean = scenes.volume_uniform_in_frustum(rng, n, cam, 1.0, 4.0)
    p = scenes._assemble(mean, rng.normal(-3.2, 0.5, (n, 3)), rng.normal(size=(n, 4)), rng.normal(-1.5, 1.0, n),
                         rng.uniform(-0.5, 0.5, (n, 1, 3)))
    s = scenes.Scene("long_lists", p, 0, [cam])
    grads = masked_grads(orc, s, 14)
    R = make(gpu, backward_schedule=1)
    dp = to_dev(p)
    R.render(dp, 0, s.cameras)
    lens = np.bincount(R.instances()[0])
    say("list lengths: max", int(lens.max()), "mean", float(lens.mean()))
    assert lens.max() > 300
    g = R.render_backward(dp, 0, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32 = orc.backward(s.params, 0, s.cameras, grads, pinned="splats32")
    ref64, gabs = orc.backward(s.params, 0, s.cameras, grads, pinned=True, want_abs=True)
    check_grads(g, ref32, "splat-parallel long lists", ref64, gabs)


def test_chunking_leaves_forward_unchanged(gpu):
    s = CASES["small"]
    p = to_dev(s.params)
    a = make(gpu, chunk_len=-1).render(p, s.sh_degree, s.cameras)[0]
    b = make(gpu, chunk_len=16, max_chunks=8).render(p, s.sh_degree, s.cameras)[0]
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_backward_multiview_sums(gpu, orc):
    s = scenes.tiny_random(4, n=50, width=40, height=30)
    s.cameras = [s.cameras[0], scenes.look_at_camera([0.3, 0.1, -0.5], [0, 0, 2], 36, 28, 30.0)]
    grads = masked_grads(orc, s, 2)
    R = make(gpu)
    p = to_dev(s.params)
    R.render(p, 0, s.cameras)
    g = R.render_backward(p, 0, s.cameras, [tuple(to_dev(x) for x in gv) for gv in grads]).cpu().numpy()
    ref32, ref64 = oracle_grads(orc, s, s.cameras, grads)
    check_grads(g, ref32, "multiview", ref64)


def test_autograd_function(gpu, orc):
    s = CASES["tiny_ragged"]
    R = make(gpu)
    p = to_dev(s.params).requires_grad_(True)
    (rgb, depth, alpha), = gpu.rasterize(p, 0, s.cameras, R)
    grads = masked_grads(orc, s, 3)
    gr, gd, ga = [to_dev(x) for x in grads[0]]
    L = (rgb * gr).sum() + (depth * gd).sum() + (alpha * ga).sum()
    L.backward()
    ref32, ref64 = oracle_grads(orc, s, s.cameras, grads)
    check_grads(p.grad.cpu().numpy(), ref32, "autograd", ref64)


# ---------------------------------------------------------------------------
# loss and Adam
# ---------------------------------------------------------------------------

def test_loss_matches_oracle(gpu, orc):
    s = CASES["small"]
    R = make(gpu)
    outs = R.render(to_dev(s.params), 0, s.cameras)
    rng = np.random.default_rng(0)
    trgb = rng.random((3, 96, 128)).astype(np.float32)
    tdep = (rng.random((96, 128)) * 4).astype(np.float32)
    tgt = [(to_dev(trgb), to_dev(tdep), None)]
    loss, grads = R.loss_l1(s.cameras, outs, tgt)
    L, gr, gd = orc.l1_loss_and_grad(outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy(), trgb, tdep)
    assert np.isclose(loss.item(), L, rtol=1e-5)
    assert np.allclose(grads[0][0].cpu().numpy(), gr, rtol=1e-6, atol=0)
    assert np.allclose(grads[0][1].cpu().numpy(), gd, rtol=1e-6, atol=0)
    assert (grads[0][2].cpu().numpy() == 0).all()


@pytest.mark.parametrize("n,pad", [(1000, 0), (1003, 0), (1003, 5)])
def test_adam_matches_oracle(gpu, orc, n, pad):
    """Adam against the oracle's float64 step; planes of 1000 (four scalars
    per load), 1003 with pitch 1003 (one by one) and with pitch 1008 (four
    per load and a tail of three)."""
    rng = np.random.default_rng(2)
    P = 14
    x0 = rng.normal(size=(P, n)).astype(np.float32)
    lrs = np.linspace(1e-3, 1e-2, P).astype(np.float32)
    R = make(gpu)

    def padded(a):
        t = torch.zeros(P, n + pad, device="cuda")
        t[:, :n] = torch.from_numpy(np.ascontiguousarray(a)).cuda()
        return t[:, :n]

    x = padded(x0)
    m = padded(np.zeros((P, n), np.float32))
    v = padded(np.zeros((P, n), np.float32))
    xr, mr, vr = x0.astype(np.float64), np.zeros((P, n)), np.zeros((P, n))
    for step in range(1, 4):
        g = rng.normal(size=(P, n)).astype(np.float32)
        R.adam_step(x, padded(g), m, v, lrs, step)
        xr, mr, vr = orc.adam_step(xr, g, mr, vr, step, lrs.astype(np.float64))
    # float32 arithmetic: a few ulp of the parameter plus 1e-5 of the total update
    upd = np.abs(xr - x0)
    ulp = np.spacing(np.abs(xr).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(x.cpu().numpy() - xr) <= 1e-5 * upd + 4 * ulp)


# ---------------------------------------------------------------------------
# invariants of the tiled method
# ---------------------------------------------------------------------------

def test_tile_size_invariance(gpu):
    s = CASES["small"]
    p = to_dev(s.params)
    ref = None
    # (tile_w, tile_h, pixels per thread, tile order; 3 = balanced over the CUs)
    for tile in [(16, 16, 1, 0), (16, 16, 2, 1), (16, 8, 1, 2), (16, 8, 2, 1), (8, 8, 1, 1), (32, 8, 1, 2),
                 (32, 8, 2, 1), (16, 16, 1, 3), (8, 8, 1, 3)]:
        outs = make(gpu, tile_w=tile[0], tile_h=tile[1], pixels_per_thread=tile[2],
                    tile_order=tile[3]).render(p, 0, s.cameras)
        cur = [o.cpu().numpy() for o in outs[0]]
        if ref is None:
            ref = cur
        else:
            for a, b in zip(cur, ref):
                assert np.array_equal(a, b), tile


def test_batched_equals_single(gpu):
    s = scenes.tiny_random(4, n=200, width=45, height=37)
    cams = [s.cameras[0], identity_camera(29, 21, 25.0), scenes.look_at_camera([0.3, 0.1, -0.5], [0, 0, 2], 64, 33, 40.0)]
    p = to_dev(s.params)
    R = make(gpu)
    both = R.render(p, 0, cams)
    for v, cam in enumerate(cams):
        one = make(gpu).render(p, 0, [cam])
        for a, b in zip(both[v], one[0]):
            assert torch.equal(a, b)


def test_forward_deterministic_and_permutation_invariant(gpu):
    s = CASES["small"]
    R = make(gpu)
    a = [o.clone() for o in R.render(to_dev(s.params), 0, s.cameras)[0]]
    b = R.render(to_dev(s.params), 0, s.cameras)[0]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    perm = np.random.default_rng(7).permutation(s.num)
    c = R.render(to_dev(s.params[:, perm]), 0, s.cameras)[0]
    for x, y in zip(a, c):
        assert torch.equal(x, y)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_and_culled(gpu, orc):
    R = make(gpu, bg=(0.1, 0.2, 0.3))
    cam = identity_camera(33, 17, 20.0)
    p = torch.zeros(14, 0, device="cuda")
    outs = R.render(p, 0, [cam])
    assert torch.allclose(outs[0][0][2], torch.full((17, 33), 0.3, device="cuda"))
    assert (outs[0][2] == 0).all()
    assert R.status()["instances"] == 0
    g = R.render_backward(p, 0, [cam], [(torch.ones(3, 17, 33, device="cuda"), None, None)])
    assert g.shape == (14, 0)
    # everything behind the camera
    q = np.zeros((14, 5), np.float32)
    q[2] = -3.0
    q[6] = 1.0
    outs = R.render(to_dev(q), 0, [cam])
    assert (outs[0][2] == 0).all()
    assert R.status()["instances"] == 0


def test_nonfinite_gaussians_culled_and_counted(gpu, orc):
    """Gaussians with a NaN or infinite parameter or a zero quaternion, placed
    in view, are culled (the images equal the oracle's, which culls them and
    draws the rest), counted once each by gsr_query_status in every render,
    and get zero gradient; a non-finite SH coefficient culls the splat but is
    not counted."""
    s = scenes.tiny_random(5, n=60, width=48, height=40)
    p = s.params.copy()
    planted = {0: (1, np.nan), 1: (4, np.inf), 2: (10, -np.inf), 3: (8, np.nan), 5: (0, -np.inf)}
    for i, (plane, val) in planted.items():
        p[plane, i] = val
    p[6:10, 4] = 0.0                                 # zero quaternion
    p[12, 6] = np.inf                                # SH coefficient: culled, not counted
    counted = len(planted) + 1
    for nv in (1, 2):
        cams = s.cameras * nv
        R = make(gpu)
        dp = to_dev(p)
        outs = R.render(dp, 0, cams)
        st = R.status()
        say("status", nv, st)
        assert st["nonfinite_culled"] == counted
        ref = orc.render(p, 0, s.cameras[0], mode="f32")
        for v in range(nv):
            check_images(outs[v], ref, f"nonfinite view {v}")
        pr = orc.project(p, 0, s.cameras[0])
        assert not pr["vis"][[0, 1, 2, 3, 4, 5, 6]].any()
        gimg = [(torch.ones(3, 40, 48, device="cuda"), torch.ones(40, 48, device="cuda"), None)] * nv
        g = R.render_backward(dp, 0, cams, gimg).cpu().numpy()
        assert np.isfinite(g).all()
        assert (g[:, :7] == 0).all()
        R.close()


def test_one_pixel_and_huge_gaussian(gpu, orc):
    cam1 = identity_camera(1, 1, 1.0)
    big = np.zeros((14, 1), np.float32)
    big[2], big[3:6], big[6], big[10] = 2.0, np.log(5.0), 1.0, 3.0
    R = make(gpu)
    outs = R.render(to_dev(big), 0, [cam1])
    ref = orc.render(big, 0, cam1, mode="f32")
    assert np.allclose(outs[0][2].cpu().numpy(), ref["alpha"], rtol=1e-6)
    cam = identity_camera(200, 150, 100.0)
    outs = R.render(to_dev(big), 0, [cam])
    assert R.status()["instances"] == 13 * 10        # covers every tile
    ref = orc.render(big, 0, cam, mode="f32")
    check_images(outs[0], ref, "huge")


def test_backward_without_forward_is_state_error(gpu):
    from paper_2509_06433_amd._lib import GsrError
    R = make(gpu)
    s = CASES["tiny_ragged"]
    p = to_dev(s.params)
    with pytest.raises(GsrError) as e:
        R.render_backward(p, 0, s.cameras, [(None, None, None)])
    assert e.value.status == -4
    R.render(p, 0, s.cameras)
    other = [identity_camera(45, 37, 30.0)]
    with pytest.raises(GsrError) as e:
        R.render_backward(p, 0, other, [(None, None, None)])
    assert e.value.status == -4


def test_invalid_arguments(gpu):
    from paper_2509_06433_amd import _lib
    with pytest.raises(_lib.GsrError) as e:
        _lib.gsr_create(tile_w=12, tile_h=12)
    assert e.value.status == -6
    for kw in (dict(chunk_len=24), dict(chunk_len=-2), dict(chunk_len=64, max_chunks=65), dict(max_chunks=-1),
               dict(fuse_blend=2), dict(depth_sort=3), dict(depth_sort=-1)):
        with pytest.raises(_lib.GsrError) as e:
            _lib.gsr_create(**kw)
        assert e.value.status == -6, kw
    R = make(gpu)
    bad = identity_camera(0, 10, 10.0)
    with pytest.raises(_lib.GsrError) as e:
        # image buffers of the camera's own (empty) shape pass the binding's
        # checks; the library rejects the zero-width camera
        R.render(torch.zeros(14, 3, device="cuda"), 0, [bad],
                 outs=[(torch.empty(3, 10, 0, device="cuda"), torch.empty(10, 0, device="cuda"),
                        torch.empty(10, 0, device="cuda"))])
    assert e.value.status == -1
