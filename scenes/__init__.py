"""Seeded synthetic scenes shaped like indoor RGB-D mapping workloads.

This module only draws random numbers and arranges them into the parameter
layout; it holds none of the rasterizer's arithmetic (no projection, no
spherical harmonics, no compositing). Both the HIP path and the CPU oracle
take their inputs from here, so that neither ever feeds the other.

Parameter layout ("the map"), float32, planar structure-of-arrays [P][N]:
    plane 0..2   mean x, y, z (world, metres)
    plane 3..5   log-scale along the three local axes
    plane 6..9   rotation quaternion (w, x, y, z), unnormalised
    plane 10     opacity logit
    plane 11+3k+c  spherical-harmonic coefficient k in [0, (deg+1)^2), colour channel c
P = 11 + 3 (deg + 1)^2  (14 for degree 0, 59 for degree 3).

Cameras are world-to-camera rigid transforms with OpenCV axes (x right, y down,
z forward) and pinhole intrinsics.

The paper (Sec. IV) evaluates on a dedicated recorded RGB-D dataset from a ZED 2i
at 672x376 that is not available; these seeded scenes stand in for it, with the
shapes, sizes and value distributions of the five workloads below. No dataset
item is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2509064330

PLANE_MEAN = 0
PLANE_LOGSCALE = 3
PLANE_QUAT = 6
PLANE_LOGIT = 10
PLANE_SH = 11


def num_planes(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


@dataclasses.dataclass
class Camera:
    R: np.ndarray          # (3, 3) float32, world -> camera rotation, row-major
    t: np.ndarray          # (3,) float32, world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_floats(self) -> np.ndarray:
        """The 16 floats R[9], t[3], fx, fy, cx, cy in the C-ABI's order."""
        return np.concatenate([
            np.asarray(self.R, np.float32).reshape(9),
            np.asarray(self.t, np.float32).reshape(3),
            np.array([self.fx, self.fy, self.cx, self.cy], np.float32)])


@dataclasses.dataclass
class Scene:
    name: str
    params: np.ndarray            # (P, N) float32
    sh_degree: int
    cameras: list                 # list[Camera]
    target_params: np.ndarray | None = None   # perturbed map whose render is the target
    notes: str = ""

    @property
    def num(self) -> int:
        return self.params.shape[1]


def identity_camera(width, height, fx, fy=None, cx=None, cy=None) -> Camera:
    fy = fx if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32),
                  float(fx), float(fy), float(cx), float(cy), int(width), int(height))


def look_at_camera(eye, target, width, height, fx, up=(0.0, 0.0, 1.0)) -> Camera:
    """Camera at `eye` whose +z axis points at `target`; +y (image down) is -up."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, np.float64)
    right = np.cross(fwd, up)
    if np.linalg.norm(right) < 1e-6:
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)      # rows: camera axes in world
    t = (-R.astype(np.float64) @ eye).astype(np.float32)
    return Camera(R, t, float(fx), float(fx), width / 2.0, height / 2.0, int(width), int(height))


def _cam_to_world(cam: Camera, pc: np.ndarray) -> np.ndarray:
    R = cam.R.astype(np.float64)
    return (pc - cam.t.astype(np.float64)[None, :]) @ R        # R^T (p - t), row-vector form


def volume_uniform_in_frustum(rng, n, cam: Camera, z0, z1) -> np.ndarray:
    """Points uniform in volume inside the view frustum between depths z0 and z1."""
    U = rng.random(n)
    z = np.cbrt(z0 ** 3 + U * (z1 ** 3 - z0 ** 3))
    u = rng.random(n) * cam.width
    v = rng.random(n) * cam.height
    pc = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], axis=1)
    return _cam_to_world(cam, pc)


def _assemble(mean, logscale, quat, logit, sh) -> np.ndarray:
    n = mean.shape[0]
    planes = [mean.T, logscale.T, quat.T, logit[None, :], sh.reshape(n, -1).T]
    return np.ascontiguousarray(np.concatenate(planes, axis=0).astype(np.float32))


def _sh_block(rng, n, deg, dc_uniform: bool, sigma=0.2):
    """SH coefficients [n, (deg+1)^2, 3]. With dc_uniform the degree-0 term is drawn
    uniform on [-sqrt(pi), sqrt(pi)], the range that degree-0 colour maps onto
    RGB in [0, 1]; otherwise every coefficient is N(0, sigma)."""
    k = (deg + 1) ** 2
    sh = rng.normal(0.0, sigma, size=(n, k, 3))
    if dc_uniform:
        sh[:, 0, :] = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), size=(n, 3))
    return sh


def perturb(rng, params: np.ndarray, sh_degree: int) -> np.ndarray:
    """Perturbed copy of a map: mean +N(0, 1 cm), log-scale +N(0, 0.1),
    quaternion +N(0, 0.05), logit +N(0, 0.2), SH +N(0, 0.1)."""
    p = params.astype(np.float64).copy()
    n = p.shape[1]
    p[0:3] += rng.normal(0, 0.01, (3, n))
    p[3:6] += rng.normal(0, 0.1, (3, n))
    p[6:10] += rng.normal(0, 0.05, (4, n))
    p[10] += rng.normal(0, 0.2, n)
    p[11:] += rng.normal(0, 0.1, p[11:].shape)
    return np.ascontiguousarray(p.astype(np.float32))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def small_128x96(seed_offset=0) -> Scene:
    """Single view 128x96, 2,000 isotropic Gaussians, SH degree 0, forward only."""
    rng = np.random.default_rng(SEED_BASE + 0 + seed_offset)
    cam = identity_camera(128, 96, 100.0, 100.0, 64.0, 48.0)
    n = 2000
    mean = volume_uniform_in_frustum(rng, n, cam, 1.0, 5.0)
    ls = rng.normal(-3.0, 0.5, n)
    logscale = np.stack([ls, ls, ls], axis=1)
    quat = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    logit = rng.normal(0.0, 1.0, n)
    sh = _sh_block(rng, n, 0, dc_uniform=True)
    return Scene("small_128x96_2k_iso", _assemble(mean, logscale, quat, logit, sh), 0, [cam])


def keyframe_640x480(n=200_000, seed_offset=0) -> Scene:
    """Single RGB-D keyframe 640x480, 200k anisotropic Gaussians, SH degree 0.
    Intrinsics f = 525, principal point at the image centre (a reading)."""
    rng = np.random.default_rng(SEED_BASE + 1 + seed_offset)
    cam = identity_camera(640, 480, 525.0)
    mean = volume_uniform_in_frustum(rng, n, cam, 1.0, 5.0)
    logscale = rng.normal(-4.0, 0.7, (n, 3))
    quat = rng.normal(0.0, 1.0, (n, 4))
    logit = rng.normal(0.0, 1.0, n)
    sh = _sh_block(rng, n, 0, dc_uniform=True)
    params = _assemble(mean, logscale, quat, logit, sh)
    target = perturb(rng, params, 0)
    return Scene("keyframe_640x480_200k", params, 0, [cam], target)


def _random_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def surfaces_1200x680(n=1_000_000, n_patches=20, seed_offset=0) -> Scene:
    """Single view 1200x680, 1M Gaussians, SH degree 3; 90% on 20 random planar
    patches (sides U[1, 4] m, 5 mm normal jitter), 10% uniform clutter."""
    rng = np.random.default_rng(SEED_BASE + 2 + seed_offset)
    cam = identity_camera(1200, 680, 600.0, 600.0, 600.0, 340.0)
    n_surf = int(round(0.9 * n))
    centres = volume_uniform_in_frustum(rng, n_patches, cam, 1.0, 5.0)
    normals = _random_unit(rng, n_patches)
    a1 = np.cross(normals, _random_unit(rng, n_patches))
    a1 /= np.linalg.norm(a1, axis=1, keepdims=True)
    a2 = np.cross(normals, a1)
    sides = rng.uniform(1.0, 4.0, (n_patches, 2))
    which = rng.integers(0, n_patches, n_surf)
    s1 = (rng.random(n_surf) - 0.5) * sides[which, 0]
    s2 = (rng.random(n_surf) - 0.5) * sides[which, 1]
    off = rng.normal(0.0, 0.005, n_surf)
    surf = centres[which] + s1[:, None] * a1[which] + s2[:, None] * a2[which] + off[:, None] * normals[which]
    clutter = volume_uniform_in_frustum(rng, n - n_surf, cam, 1.0, 5.0)
    mean = np.concatenate([surf, clutter], axis=0)
    logscale = rng.normal(-4.0, 0.7, (n, 3))
    quat = rng.normal(0.0, 1.0, (n, 4))
    logit = rng.normal(0.0, 1.0, n)
    sh = _sh_block(rng, n, 3, dc_uniform=False, sigma=0.2)
    params = _assemble(mean, logscale, quat, logit, sh)
    target = perturb(rng, params, 3)
    return Scene("surfaces_1200x680_1M_sh3", params, 3, [cam], target)


def _room_points(rng, n, size, frac_walls):
    """Points on the 5 visible surfaces of an axis-aligned room (floor + 4 walls)
    spanning [0, sx] x [0, sy] x [0, sz], plus uniform clutter inside."""
    sx, sy, sz = size
    n_w = int(round(frac_walls * n))
    face = rng.integers(0, 5, n_w)
    u = rng.random(n_w)
    v = rng.random(n_w)
    p = np.zeros((n_w, 3))
    f0 = face == 0                                             # floor z = 0
    p[f0] = np.stack([u[f0] * sx, v[f0] * sy, np.zeros(f0.sum())], 1)
    for k, (axis, val) in enumerate([(0, 0.0), (0, sx), (1, 0.0), (1, sy)], start=1):
        fk = face == k
        q = np.zeros((fk.sum(), 3))
        q[:, axis] = val
        other = 1 - axis
        q[:, other] = u[fk] * (sx if other == 0 else sy)
        q[:, 2] = v[fk] * sz
        p[fk] = q
    p += rng.normal(0.0, 0.005, p.shape)
    clutter = rng.random((n - n_w, 3)) * np.array([sx, sy, sz])
    return np.concatenate([p, clutter], axis=0)


BATCH8_TRAJ_SEED = 3     # per-view visibility 32% .. 83% (seeded search over 0..7)


def _room_trajectory(rng, n_views, size, step=0.1, turn_deg=5.0, stride=1):
    """Smooth random walk of camera poses inside the room: position steps of
    `step` metres and heading turns of `turn_deg` degrees between consecutive
    poses; every `stride`-th pose becomes a keyframe."""
    sx, sy, sz = size
    pos = np.array([sx * 0.5, sy * 0.5, 1.4])
    yaw = rng.uniform(0, 2 * math.pi)
    pitch = -0.2
    poses = []
    for i in range(n_views * stride):
        yaw += math.radians(turn_deg) * rng.choice([-1.0, 1.0, 1.0])
        pitch = float(np.clip(pitch + math.radians(turn_deg) * rng.normal(0, 0.5), -0.6, 0.2))
        d = np.array([math.cos(yaw), math.sin(yaw), 0.0])
        nxt = pos + step * d
        margin = 1.0
        if not (margin < nxt[0] < sx - margin and margin < nxt[1] < sy - margin):
            yaw += math.pi / 2
            d = np.array([math.cos(yaw), math.sin(yaw), 0.0])
            nxt = pos + step * d
            nxt[0] = np.clip(nxt[0], margin, sx - margin)
            nxt[1] = np.clip(nxt[1], margin, sy - margin)
        pos = nxt
        if i % stride == 0:
            fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
            poses.append((pos.copy(), pos + fwd))
    return poses


def _corner_exit_trajectory(rng, n_views, start, stride, step=0.1, turn_deg=5.0):
    """Smooth random trajectory that backs out of a room through its (+x, +y)
    corner while looking across the room: position steps of `step` metres along
    a fixed diagonal, heading and pitch turns of at most `turn_deg` degrees per
    step (heading kept within 20 degrees of the room's diagonal). Every
    `stride`-th pose is a keyframe. Seen from inside the corner a view holds
    about a third of the room; backing out, most of it."""
    pos = np.array(start, np.float64)
    walk = np.array([1.0, 1.0, 0.12])
    walk /= np.linalg.norm(walk)
    yaw_c = math.radians(225.0)
    yaw, pitch = yaw_c, -0.35
    poses = []
    for i in range(n_views * stride):
        if i % stride == 0:
            fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
            poses.append((pos.copy(), pos + fwd))
        dyaw = math.radians(turn_deg) * rng.choice([-1.0, 0.0, 1.0])
        if abs(yaw + dyaw - yaw_c) > math.radians(20.0):
            dyaw = -dyaw
        yaw += dyaw
        pitch = float(np.clip(pitch + math.radians(turn_deg) * rng.normal(0.0, 0.4), -0.55, -0.15))
        pos = pos + step * walk
    return poses


def batch8_640x480(n=500_000, seed_offset=0, traj_seed=BATCH8_TRAJ_SEED) -> Scene:
    """8 keyframes at 640x480 over a shared 500k-Gaussian room (6x6x3 m, 85% on
    walls/floor, 15% clutter); poses on a smooth trajectory (0.1 m / 5 deg steps)
    that backs out through a corner, so that the fraction of Gaussians each view
    sees is uneven, from about 30% to about 90%."""
    rng = np.random.default_rng(SEED_BASE + 3 + seed_offset)
    size = (6.0, 6.0, 3.0)
    mean = _room_points(rng, n, size, 0.85)
    logscale = rng.normal(-4.0, 0.7, (n, 3))
    quat = rng.normal(0.0, 1.0, (n, 4))
    logit = rng.normal(0.0, 1.0, n)
    sh = _sh_block(rng, n, 0, dc_uniform=True)
    params = _assemble(mean, logscale, quat, logit, sh)
    trng = np.random.default_rng(SEED_BASE + 3 + 1000 + traj_seed)
    poses = _corner_exit_trajectory(trng, 8, (5.1, 5.1, 1.7), stride=5)
    cams = [look_at_camera(e, t, 640, 480, 525.0) for e, t in poses]
    target = perturb(rng, params, 0)
    return Scene("batch8_640x480_500k", params, 0, cams, target)


MIXED16_RESOLUTIONS = [(320, 240)] * 5 + [(640, 480)] * 6 + [(1280, 720)] * 5


def mixed16_2m(n=2_000_000, seed_offset=0, traj_seed=0, res_div=1, logscale_mean=-4.0) -> Scene:
    """16 views at mixed resolutions (5x 320x240, 6x 640x480, 5x 1280x720, seeded
    order) over a 2M-Gaussian SH-degree-3 room scaled to 10 m (depths 0.5-10 m).
    res_div divides every resolution (and so the focal length)."""
    rng = np.random.default_rng(SEED_BASE + 4 + seed_offset)
    size = (10.0, 10.0, 4.0)
    mean = _room_points(rng, n, size, 0.85)
    logscale = rng.normal(logscale_mean, 0.7, (n, 3))
    quat = rng.normal(0.0, 1.0, (n, 4))
    logit = rng.normal(0.0, 1.0, n)
    sh = _sh_block(rng, n, 3, dc_uniform=False, sigma=0.2)
    params = _assemble(mean, logscale, quat, logit, sh)
    trng = np.random.default_rng(SEED_BASE + 4 + 1000 + traj_seed)
    res = [(w // res_div, h // res_div) for w, h in MIXED16_RESOLUTIONS]
    trng.shuffle(res)
    poses = _room_trajectory(trng, 16, size, stride=3)
    cams = [look_at_camera(e, t, w, h, 0.8203 * w) for (e, t), (w, h) in zip(poses, res)]
    target = perturb(rng, params, 3)
    name = "mixed16_2M_sh3" if (n, res_div) == (2_000_000, 1) else f"mixed16_{n}_div{res_div}_sh3"
    return Scene(name, params, 3, cams, target)


def mixed16_small() -> Scene:
    """The 16-view mixed-resolution room at 1/8 of every resolution with 20k
    Gaussians ten times larger (the same image coverage), for checks against
    the CPU oracle that need many renders."""
    return mixed16_2m(n=20_000, res_div=8, logscale_mean=-4.0 + np.log(10.0))


def tiny_random(k: int, n=12, width=32, height=32, sh_degree=0, anisotropic=True) -> Scene:
    """Tiny seeded scene (n Gaussians, width x height) for brute-force checks."""
    rng = np.random.default_rng(SEED_BASE + 100 * (k + 1))
    f = 0.9 * width
    cam = identity_camera(width, height, f)
    mean = volume_uniform_in_frustum(rng, n, cam, 1.0, 3.0)
    if anisotropic:
        logscale = rng.normal(-1.9, 0.4, (n, 3))
        quat = rng.normal(0.0, 1.0, (n, 4))
    else:
        ls = rng.normal(-1.9, 0.4, n)
        logscale = np.stack([ls, ls, ls], 1)
        quat = np.tile(np.array([1.0, 0, 0, 0]), (n, 1))
    logit = rng.normal(0.5, 1.0, n)
    sh = _sh_block(rng, n, sh_degree, dc_uniform=(sh_degree == 0), sigma=0.3)
    params = _assemble(mean, logscale, quat, logit, sh)
    target = perturb(rng, params, sh_degree)
    return Scene(f"tiny_{k}", params, sh_degree, [cam], target)


WORKLOADS = {
    "small_128x96_2k_iso": small_128x96,
    "keyframe_640x480_200k": keyframe_640x480,
    "surfaces_1200x680_1M_sh3": surfaces_1200x680,
    "batch8_640x480_500k": batch8_640x480,
    "mixed16_2M_sh3": mixed16_2m,
}


def random_image_grads(seed, cams, scale=1.0):
    """Seeded upstream gradients dL/d(rgb, depth, alpha) per view, for parity tests."""
    rng = np.random.default_rng(SEED_BASE + 7777 + seed)
    out = []
    for c in cams:
        hw = (c.height, c.width)
        out.append((rng.normal(0, scale, (3,) + hw).astype(np.float32),
                    rng.normal(0, scale, hw).astype(np.float32),
                    rng.normal(0, scale, hw).astype(np.float32)))
    return out
