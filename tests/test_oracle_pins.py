"""Pins of the CPU oracle against facts fixed outside it: closed forms, library
routines (scipy rotations and spherical harmonics, torch), invariants,
hand-computed special cases and brute force. CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes
from scenes import Camera, identity_camera

F32 = np.float32


def one_gaussian(mean, logscale, quat=(1, 0, 0, 0), logit=2.0, sh=None, deg=0):
    K = (deg + 1) ** 2
    p = np.zeros((scenes.num_planes(deg), 1), np.float32)
    p[0:3, 0] = mean
    p[3:6, 0] = logscale
    p[6:10, 0] = quat
    p[10, 0] = logit
    if sh is not None:
        p[11:, 0] = np.asarray(sh, np.float32).reshape(K * 3)
    return p


def stack(*ps):
    return np.ascontiguousarray(np.concatenate(ps, axis=1))


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def f32(x):
    """The double value of x rounded to float32 (inputs and constants are float32)."""
    return float(np.float32(x))


DIL = f32(0.3)                 # dilation constant, float32 promoted
AMIN = f32(np.float32(1) / np.float32(255))
AMAX = f32(0.99)


Y00 = 1.0 / math.sqrt(4.0 * math.pi)          # constant real spherical harmonic


# --------------------------------------------------------------------------
# FP32 exponential: exp(x) correctly rounded to float
# --------------------------------------------------------------------------

def exp_rounded_to_float(x):
    """exp(x) rounded to the nearest float32 from a 60-digit decimal exp
    (Python's decimal module: an arbitrary-precision library routine), by
    comparing the exact value with the midpoints between neighbouring floats."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 60
        e = Decimal(float(x)).exp()
        c = np.float32(float(e))
        for _ in range(3):
            up = np.nextafter(c, np.float32(np.inf))
            dn = np.nextafter(c, np.float32(0))
            if e > (Decimal(float(c)) + Decimal(float(up))) / 2:
                c = up
            elif c > 0 and e < (Decimal(float(c)) + Decimal(float(dn))) / 2:
                c = dn
            else:
                break
        return c


def near_tie_inputs(lo_bits, hi_bits, below=2.0 ** -50):
    """Floats (bit patterns in [lo_bits, hi_bits)) whose double-precision exp
    lies within `below` (relative) of a midpoint between two floats."""
    x = np.arange(lo_bits, hi_bits, dtype=np.uint32).view(np.float32)
    y = np.exp(x.astype(np.float64))
    f = y.astype(np.float32)
    nb = np.where(y >= f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf)))
    d = np.abs(y - 0.5 * (f.astype(np.float64) + nb)) / y
    return x[d < below]


def test_exp32_correctly_rounded(orc):
    """The oracle's FP32 exp equals exp(x) correctly rounded to float on random
    inputs across the whole finite range, on the activation ranges, at special
    values, and on inputs whose double exp sits within 2^-50 of a rounding
    midpoint (where the oracle falls back to the long double exp)."""
    rng = np.random.default_rng(1)
    ties = np.concatenate([near_tie_inputs(0x40000000, 0x40800000),     # [2, 4)
                           near_tie_inputs(0xC0000000, 0xC0800000),     # [-4, -2)
                           near_tie_inputs(0xB3000000, 0xB3400000)])    # around -2^-25
    assert ties.size >= 2, ties
    special = np.array([0.0, -0.0, 1.0, -1.0, 2.0 ** -25, -(2.0 ** -25), 2.0 ** -24, -(2.0 ** -24), 88.0, 88.72,
                        -87.0, -103.0, -104.5, 1e-30, -1e-30], np.float32)
    x = np.concatenate([rng.uniform(-104, 88.7, 4000), rng.uniform(-9, 7, 4000), rng.normal(-4, 0.7, 2000),
                        rng.normal(0, 1, 2000)]).astype(np.float32)
    x = np.concatenate([x, special, ties])
    y, tie = orc.exp32(x, with_tie=True)
    ref = np.array([exp_rounded_to_float(v) for v in x], np.float32)
    bad = np.flatnonzero(y.view(np.uint32) != ref.view(np.uint32))
    assert bad.size == 0, list(zip(x[bad], y[bad], ref[bad]))
    # the long double exp decides every one of these far from a midpoint
    assert np.all(tie[np.isfinite(tie)] > 2.0 ** -60)
    assert orc.exp32(np.array([0.0], np.float32))[0] == 1.0


def test_activations_are_exp_and_sigmoid_in_float(orc):
    """orc.activations: scale = exp32(log-scale) and opacity = 1 / (1 + exp32(-logit))
    with one correctly rounded float operation per step (numpy float32 + and /)."""
    rng = np.random.default_rng(2)
    ls = rng.normal(-4, 0.7, 5000).astype(np.float32)
    lg = rng.normal(0, 1, 5000).astype(np.float32)
    s, o = orc.activations(ls, lg)
    assert np.array_equal(s.view(np.uint32), orc.exp32(ls).view(np.uint32))
    e = orc.exp32(-lg)
    ref = np.float32(1.0) / (np.float32(1.0) + e)
    assert ref.dtype == np.float32
    assert np.array_equal(o.view(np.uint32), ref.view(np.uint32))
    assert np.all((o > 0) & (o < 1))


# --------------------------------------------------------------------------
# Spherical harmonics: scipy's complex SH (Condon-Shortley phase included)
# --------------------------------------------------------------------------

def _scipy_real_sh(deg, d):
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(d[:, 2], -1, 1))          # polar
    phi = np.arctan2(d[:, 1], d[:, 0])                  # azimuth
    cols = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                cols.append(Y.real)
            elif m > 0:
                cols.append(math.sqrt(2) * Y.real)
            else:
                cols.append(math.sqrt(2) * Y.imag)
    return np.stack(cols, 1)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 5])
def test_sh_basis_matches_scipy(orc, deg):
    rng = np.random.default_rng(deg)
    d = rng.normal(size=(2000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ours = orc.sh_basis(deg, d)
    assert np.allclose(ours, _scipy_real_sh(deg, d), atol=1e-12, rtol=1e-10)


def test_sh_band1_convention(orc):
    # band 1 is (-c y, c z, -c x) with c = sqrt(3/(4 pi)) for m = -1, 0, 1
    d = np.array([[0.36, 0.48, 0.8]])
    Y = orc.sh_basis(1, d)[0]
    c = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y, [1 / math.sqrt(4 * math.pi), -c * 0.48, c * 0.8, -c * 0.36], rtol=1e-14)


def test_sh_orthonormal_by_quadrature(orc):
    # Gauss-Legendre in cos(theta) x uniform in phi integrates products of degree <= 6 exactly
    deg = 3
    xs, ws = np.polynomial.legendre.leggauss(12)
    nphi = 16
    phis = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xs, phis, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (ws[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = orc.sh_basis(deg, d)
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(3)
    d = rng.normal(size=(50, 3))
    Y, dY = orc.sh_basis(3, d / np.linalg.norm(d, axis=1, keepdims=True), with_grad=True)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        # the basis is a polynomial in (x, y, z): differentiate it off the sphere
        fd = (orc.sh_basis(3, d / np.linalg.norm(d, axis=1, keepdims=True) + e)
              - orc.sh_basis(3, d / np.linalg.norm(d, axis=1, keepdims=True) - e)) / (2 * h)
        assert np.allclose(fd, dY[:, :, j], atol=1e-8)


# --------------------------------------------------------------------------
# P1: single isotropic Gaussian on the optical axis -- closed form
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["f64", "f64pin", "f32"])
def test_p1_isotropic_on_axis_closed_form(orc, mode):
    W, H, f = 40, 30, 50.0
    cam = identity_camera(W, H, f)          # cx = 20, cy = 15
    z, s, logit = 2.5, 0.08, 1.3
    col = np.array([0.9, 0.4, 0.15])
    p = one_gaussian([0, 0, z], [math.log(s)] * 3, logit=logit, sh=(col - 0.5) / Y00)
    bg = (0.1, 0.2, 0.3)
    out = orc.render(p, 0, cam, mode=mode, bg=[f32(b) for b in bg])
    bg = [f32(b) for b in bg]
    o = sigmoid(f32(logit))
    s = math.exp(f32(math.log(s)))
    col = p[11:14, 0].astype(np.float64) * Y00 + 0.5
    var = (f * s / z) ** 2 + DIL
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    r2 = (xs - 20.0) ** 2 + (ys - 15.0) ** 2
    alpha = np.minimum(AMAX, o * np.exp(-0.5 * r2 / var))
    alpha = np.where(alpha < AMIN, 0.0, alpha)
    tol = dict(rtol=1e-12, atol=1e-13) if mode != "f32" else dict(rtol=2e-6, atol=2e-7)
    for ch in range(3):
        assert np.allclose(out["rgb"][ch], alpha * col[ch] + (1 - alpha) * bg[ch], **tol)
    assert np.allclose(out["depth"], alpha * z, **tol)
    assert np.allclose(out["alpha"], alpha, **tol)
    assert (out["ncomp"] == (alpha > 0)).all()


def test_p1_projection_and_extent(orc):
    W, H, f = 64, 48, 80.0
    cam = identity_camera(W, H, f)
    z, s = 3.0, 0.05
    p = one_gaussian([0, 0, z], [math.log(s)] * 3)
    pr = orc.project(p, 0, cam, prec=64)
    s = math.exp(f32(math.log(s)))
    var = (f * s / z) ** 2 + DIL
    assert np.allclose([pr["a"][0], pr["b"][0], pr["c"][0]], [var, 0, var], rtol=1e-13, atol=1e-15)
    assert np.allclose([pr["A"][0], pr["C"][0]], [1 / var, 1 / var], rtol=1e-13)
    assert pr["u"][0] == 32.0 and pr["v"][0] == 24.0 and pr["z"][0] == 3.0
    e = math.sqrt(f32(11.2) * var)
    assert np.isclose(pr["ex"][0], e, rtol=1e-13)
    x0 = max(0, math.ceil(32 - e - 0.5))
    x1 = min(W - 1, math.floor(32 + e - 0.5))
    assert tuple(pr["rect"][0]) == (x0, max(0, math.ceil(24 - e - 0.5)), x1, min(H - 1, math.floor(24 + e - 0.5)))


# --------------------------------------------------------------------------
# P2: anisotropic, rotated, off-axis Gaussian seen by a rotated camera.
# Reference: scipy rotations and the numerical Jacobian of the pinhole map.
# --------------------------------------------------------------------------

def _pinhole(cam, pc):
    return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])


def _num_jacobian(cam, pc, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pinhole(cam, pc + e) - _pinhole(cam, pc - e)) / (2 * h)
    return J


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_p2_anisotropic_projection_reference(orc, seed):
    rng = np.random.default_rng(100 + seed)
    Wc = Rotation.random(random_state=seed).as_matrix()
    cam = Camera(Wc.astype(np.float32), rng.normal(0, 0.5, 3).astype(np.float32), 70.0, 65.0, 31.0, 23.5, 64, 48)
    Wc = cam.R.astype(np.float64)
    tc = cam.t.astype(np.float64)
    # mean at a chosen camera-space point, well inside the frustum
    pc = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2), 1.0]) * rng.uniform(1.5, 3.0)
    mean = (Wc.T @ (pc - tc)).astype(np.float32)
    q = rng.normal(size=4).astype(np.float32)
    ls = rng.normal(-2.5, 0.5, 3).astype(np.float32)
    p = one_gaussian(mean, ls, q)
    pr = orc.project(p, 0, cam, prec=64)
    qd = q.astype(np.float64)
    Rq = Rotation.from_quat([qd[1], qd[2], qd[3], qd[0]]).as_matrix()        # scipy is scalar-last
    S = Rq @ np.diag(np.exp(2 * ls.astype(np.float64))) @ Rq.T
    pcam = Wc @ mean.astype(np.float64) + tc
    J = _num_jacobian(cam, pcam)
    S2 = J @ (Wc @ S @ Wc.T) @ J.T + DIL * np.eye(2)
    assert np.allclose([pr["a"][0], pr["b"][0], pr["c"][0]], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)
    assert np.allclose([pr["u"][0], pr["v"][0]], _pinhole(cam, pcam), rtol=1e-12)
    assert np.isclose(pr["z"][0], pcam[2], rtol=1e-12)
    Ci = np.linalg.inv(S2)
    assert np.allclose([pr["A"][0], pr["B"][0], pr["C"][0]], [Ci[0, 0], Ci[0, 1], Ci[1, 1]], rtol=1e-6)


def test_p2_jacobian_clamp(orc):
    # A large Gaussian whose mean lies beyond 1.3x the half-FoV tangent: the
    # Jacobian is taken at the clamped direction (lim * z, y, z).
    W, H, f = 64, 48, 60.0
    cam = identity_camera(W, H, f)
    lim = 1.3 * (0.5 * W / f)
    z = 2.0
    pc = np.array([1.8 * lim * z, 0.1, z])
    p = one_gaussian(pc, [math.log(0.9), math.log(0.3), math.log(0.5)], [0.9, 0.2, -0.3, 0.1])
    pr = orc.project(p, 0, cam, prec=64)
    assert pr["vis"][0]
    q = p[6:10, 0].astype(np.float64)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    S = Rq @ np.diag(np.exp(2 * p[3:6, 0].astype(np.float64))) @ Rq.T
    J = _num_jacobian(cam, np.array([f32(lim) * z, f32(0.1), z]))
    S2 = J @ S @ J.T + DIL * np.eye(2)
    assert np.allclose([pr["a"][0], pr["b"][0], pr["c"][0]], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)
    # the projected mean itself is not clamped
    assert np.isclose(pr["u"][0], f * f32(pc[0]) / z + cam.cx, rtol=1e-12)


def test_world_to_camera_convention(orc):
    # A camera looking along world +x from (-2, 0, 0): a point on the world
    # x axis projects to the principal point at depth 2 + x.
    cam = scenes.look_at_camera([-2.0, 0.0, 0.0], [0.0, 0.0, 0.0], 64, 48, 50.0)
    p = stack(one_gaussian([0.5, 0, 0], [-3] * 3), one_gaussian([0.5, 0.0, 0.2], [-3] * 3))
    pr = orc.project(p, 0, cam, prec=64)
    assert np.allclose([pr["u"][0], pr["v"][0], pr["z"][0]], [32.0, 24.0, 2.5], atol=1e-6)
    # world +z is image up (-v)
    assert pr["v"][1] < 24.0 and np.isclose(pr["u"][1], 32.0, atol=1e-6)


# --------------------------------------------------------------------------
# P3: two Gaussians -- closed form, and storage order independence
# --------------------------------------------------------------------------

def test_p3_two_gaussians_closed_form(orc):
    W, H, f = 32, 32, 40.0
    cam = identity_camera(W, H, f)
    c1, c2 = np.array([0.8, 0.1, 0.3]), np.array([0.2, 0.7, 0.9])
    g1 = one_gaussian([0.05, 0, 1.5], [math.log(0.06)] * 3, logit=0.5, sh=(c1 - 0.5) / Y00)
    g2 = one_gaussian([-0.05, 0.02, 2.5], [math.log(0.1)] * 3, logit=1.5, sh=(c2 - 0.5) / Y00)
    ys, xs = np.mgrid[0:H, 0:W] + 0.5

    def alpha_of(mu, s, logit):
        mu = np.array([f32(m) for m in mu])
        s = math.exp(f32(math.log(s)))
        u, v = _pinhole(cam, mu)
        J = _num_jacobian(cam, mu)               # off-axis: the projection is anisotropic
        S2 = s * s * (J @ J.T) + DIL * np.eye(2)
        Q = np.linalg.inv(S2)
        dx, dy = xs - u, ys - v
        q = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        a = np.minimum(AMAX, sigmoid(f32(logit)) * np.exp(-0.5 * q))
        return np.where(a < AMIN, 0.0, a)

    c1 = g1[11:14, 0].astype(np.float64) * Y00 + 0.5
    c2 = g2[11:14, 0].astype(np.float64) * Y00 + 0.5

    a1 = alpha_of([0.05, 0, 1.5], 0.06, 0.5)
    a2 = alpha_of([-0.05, 0.02, 2.5], 0.1, 1.5)
    for order in [(g1, g2), (g2, g1)]:
        out = orc.render(stack(*order), 0, cam, mode="f64")
        for ch in range(3):
            assert np.allclose(out["rgb"][ch], a1 * c1[ch] + (1 - a1) * a2 * c2[ch], rtol=1e-8, atol=1e-10)
        assert np.allclose(out["alpha"], 1 - (1 - a1) * (1 - a2), rtol=1e-8, atol=1e-10)
        assert np.allclose(out["depth"], a1 * 1.5 + (1 - a1) * a2 * 2.5, rtol=1e-8, atol=1e-10)
    o1 = orc.render(stack(g1, g2), 0, cam, mode="f32")
    o2 = orc.render(stack(g2, g1), 0, cam, mode="f32")
    for k in ("rgb", "depth", "alpha"):
        assert np.array_equal(o1[k], o2[k])


# --------------------------------------------------------------------------
# P4: worked stop example (exclusive stop, FP32 thresholds)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["f32", "f64pin", "f64"])
def test_p4_exclusive_stop(orc, mode):
    W, H, f = 16, 16, 20.0
    cam = identity_camera(W, H, f)
    cols = [np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])]
    gs = [one_gaussian([0, 0, z], [math.log(5.0)] * 3, logit=12.0, sh=(c - 0.5) / Y00) for z, c in
          zip([2.0, 2.1, 2.2], cols)]
    out = orc.render(stack(*gs), 0, cam, mode=mode)
    # at the pixel next to the principal point o * G > 0.99, so alpha = 0.99f;
    # T after one = 1 - 0.99f = 0.0099999904632568359375 and
    # T * (1 - alpha) = 9.99998e-5 < 1e-4f, so the second is not composited
    py, px = 8, 8
    assert out["ncomp"][py, px] == 1
    a = float(np.float32(0.99))
    assert np.isclose(out["rgb"][0, py, px], a, rtol=1e-7)
    assert out["rgb"][1, py, px] == 0.0 and out["rgb"][2, py, px] == 0.0
    expect_alpha = float(np.float32(1) - (np.float32(1) - np.float32(0.99)))
    assert np.isclose(out["alpha"][py, px], expect_alpha, rtol=1e-7)
    assert out["tfinal"][py, px] >= 1e-4 * (1 - 1e-7)


# --------------------------------------------------------------------------
# P5, P6: invariants on random scenes
# --------------------------------------------------------------------------

def test_p5_transmittance_invariants(orc):
    s = scenes.small_128x96()
    out = orc.render(s.params, 0, s.cameras[0], mode="f64pin")
    assert (out["tfinal"] >= float(np.float32(1e-4)) * (1 - 1e-9)).all()
    assert (out["tfinal"] <= 1.0).all()
    assert np.allclose(out["alpha"], 1 - out["tfinal"])
    # all colours 1, background 0 => rgb = sum of weights = 1 - T
    p = s.params.copy()
    p[11:14] = (1.0 - 0.5) / Y00
    out = orc.render(p, 0, s.cameras[0], mode="f64pin")
    for ch in range(3):
        assert np.allclose(out["rgb"][ch], out["alpha"], atol=1e-12)
    # monotone: adding a Gaussian far behind can only lower T
    far = one_gaussian([0, 0, 4.9], [math.log(2.0)] * 3, logit=3.0)
    out2 = orc.render(stack(s.params, far), 0, s.cameras[0], mode="f64pin")
    assert (out2["tfinal"] <= out["tfinal"] + 1e-15).all()


def test_p6_order_independence(orc):
    s = scenes.small_128x96()
    rng = np.random.default_rng(5)
    perm = rng.permutation(s.num)
    a = orc.render(s.params, 0, s.cameras[0], mode="f32")
    b = orc.render(s.params[:, perm], 0, s.cameras[0], mode="f32")
    z = orc.project(s.params, 0, s.cameras[0], prec=32)["z"]
    assert len(np.unique(z[z > 0])) == (z > 0).sum()    # distinct depths
    for k in ("rgb", "depth", "alpha", "ncomp"):
        assert np.array_equal(a[k], b[k])


# --------------------------------------------------------------------------
# P7: containment -- binning never drops a contributing pair
# --------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["small", "tiny_aniso", "near"])
def test_p7_prefilter_equals_brute_force(orc, which):
    if which == "small":
        s = scenes.small_128x96()
    elif which == "tiny_aniso":
        s = scenes.tiny_random(3, n=40, width=48, height=40)
    else:
        # large, opaque, elongated Gaussians close to the camera
        rng = np.random.default_rng(11)
        cam = identity_camera(96, 64, 80.0)
        n = 60
        mean = scenes.volume_uniform_in_frustum(rng, n, cam, 0.3, 1.2)
        p = scenes._assemble(mean, rng.normal(-2.5, 1.0, (n, 3)), rng.normal(size=(n, 4)),
                             rng.normal(4.0, 1.0, n), rng.normal(0, 1, (n, 1, 3)))
        s = scenes.Scene("near", p, 0, [cam])
    a = orc.render(s.params, s.sh_degree, s.cameras[0], mode="f32", prefilter=True)
    b = orc.render(s.params, s.sh_degree, s.cameras[0], mode="f32", prefilter=False)
    for k in ("rgb", "depth", "alpha", "ncomp"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("mode", ["f32", "f64pin", "f64"])
def test_window_render_equals_whole_render(orc, mode):
    """A window (and a row subset of it) renders exactly the pixels of the
    whole render: every pixel is composited on its own."""
    s = scenes.tiny_random(6, n=40, width=45, height=37)
    full = orc.render(s.params, 0, s.cameras[0], mode=mode)
    for win in [(5, 3, 40, 30), (0, 0, 45, 37, 4), (7, 2, 19, 37, 3)]:
        part = orc.render(s.params, 0, s.cameras[0], mode=mode, window=win)
        x0, y0, x1, y1 = win[:4]
        step = win[4] if len(win) > 4 else 1
        sel = np.zeros((37, 45), bool)
        sel[y0:y1:step, x0:x1] = True
        for k in ("depth", "alpha", "tfinal", "ncomp", "margin"):
            assert np.array_equal(part[k][sel], full[k][sel]), (k, win)
        assert np.array_equal(part["rgb"][:, sel], full["rgb"][:, sel])
        assert (part["alpha"][~sel] == 0).all() and np.isinf(part["margin"][~sel]).all()


def test_window_backward_equals_zeroed_upstream(orc):
    """Walking only a window's pixels equals the whole backward with the
    upstream gradient zeroed outside the window (same terms, other order)."""
    s = scenes.tiny_random(7, n=30, width=40, height=30)
    cams = [s.cameras[0], identity_camera(40, 30, 28.0, cx=19.0, cy=14.0)]
    grads = scenes.random_image_grads(3, cams)
    wins = [(4, 2, 33, 29, 3), (10, 0, 40, 20)]
    zeroed = []
    for (gr, gd, ga), w in zip(grads, wins):
        sel = np.zeros((30, 40), bool)
        sel[w[1]:w[3]:(w[4] if len(w) > 4 else 1), w[0]:w[2]] = True
        zeroed.append((gr * sel[None], gd * sel, ga * sel))
    for pinned in (True, "splats32", False):
        a = orc.backward(s.params, 0, cams, grads, pinned=pinned, windows=wins)
        b = orc.backward(s.params, 0, cams, zeroed, pinned=pinned)
        assert np.abs(b).max() > 0
        assert np.allclose(a, b, rtol=1e-12, atol=1e-15 * np.abs(b).max()), pinned


def test_tile_list_brute_force(orc):
    s = scenes.tiny_random(4, n=30, width=45, height=37)
    cams = [s.cameras[0], identity_camera(29, 21, 25.0)]
    tw, th = 8, 4
    tiles, gids = orc.tile_list(s.params, 0, cams, tw, th)
    expect = []
    off = 0
    for cam in cams:
        pr = orc.project(s.params, 0, cam, prec=32)
        tx_n = -(-cam.width // tw)
        ty_n = -(-cam.height // th)
        for i in range(s.num):
            if not pr["vis"][i]:
                continue
            x0, y0, x1, y1 = pr["rect"][i]
            zb = np.float32(pr["z"][i]).view(np.uint32)
            for ty in range(ty_n):
                for tx in range(tx_n):
                    # tile overlaps the pixel rectangle
                    if tx * tw <= x1 and (tx + 1) * tw - 1 >= x0 and ty * th <= y1 and (ty + 1) * th - 1 >= y0:
                        expect.append((off + ty * tx_n + tx, int(zb), i))
        off += tx_n * ty_n
    expect.sort()
    assert [(int(t), int(g)) for t, g in zip(tiles, gids)] == [(t, g) for t, _, g in expect]


# --------------------------------------------------------------------------
# Culling and degenerate inputs
# --------------------------------------------------------------------------

def test_culling_rules(orc):
    cam = identity_camera(32, 32, 30.0)
    ok = one_gaussian([0, 0, 2], [-2] * 3)
    behind = one_gaussian([0, 0, -2], [-2] * 3)
    near = one_gaussian([0, 0, 0.1], [-2] * 3)
    nanp = one_gaussian([0, np.nan, 2], [-2] * 3)
    zeroq = one_gaussian([0, 0, 2], [-2] * 3, quat=(0, 0, 0, 0))
    infs = one_gaussian([0, 0, 2], [np.inf, -2, -2])
    offscreen = one_gaussian([50, 0, 2], [-3] * 3)
    p = stack(ok, behind, near, nanp, zeroq, infs, offscreen)
    for prec in (32, 64):
        pr = orc.project(p, 0, cam, prec=prec)
        assert pr["vis"].tolist() == [True, False, False, False, False, False, False]
    out = orc.render(p, 0, cam, mode="f32")
    ref = orc.render(ok, 0, cam, mode="f32")
    for k in ("rgb", "depth", "alpha"):
        assert np.array_equal(out[k], ref[k])


def test_empty_scene(orc):
    cam = identity_camera(8, 8, 10.0)
    p = np.zeros((14, 0), np.float32)
    out = orc.render(p, 0, cam, mode="f32", bg=(0.2, 0.3, 0.4))
    assert np.allclose(out["rgb"][1], 0.3) and (out["alpha"] == 0).all() and (out["ncomp"] == 0).all()
    t, g = orc.tile_list(p, 0, [cam])
    assert len(t) == 0


def test_fp32_close_to_fp64(orc):
    s = scenes.small_128x96()
    a = orc.render(s.params, 0, s.cameras[0], mode="f32")
    b = orc.render(s.params, 0, s.cameras[0], mode="f64pin")
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-4
    assert np.abs(a["depth"] - b["depth"]).max() < 5e-4


# --------------------------------------------------------------------------
# Keyframe insertion
# --------------------------------------------------------------------------

def test_densify_seeds_reproject_to_their_pixels(orc):
    """Every seeded Gaussian projects back to its pixel centre at the
    observed depth, has the observed colour, and a scale of scale_factor grid
    cells at that depth (the FP64 projection)."""
    rng = np.random.default_rng(31)
    cam = scenes.look_at_camera([0.3, -0.2, -0.4], [0.1, 0.0, 2.5], 50, 40, 45.0)
    depth = rng.uniform(1.0, 4.0, (40, 50)).astype(np.float32)
    rgb = rng.uniform(0.0, 1.0, (3, 40, 50)).astype(np.float32)
    new, pix = orc.densify(1, cam, rgb, depth, step=3, scale_factor=0.7)
    assert new.shape[1] == len(range(0, 40, 3)) * len(range(0, 50, 3))
    pr = orc.project(new.astype(np.float32), 1, cam, prec=64)
    # the means go through float32 here: reprojection to 1e-5 px
    assert np.allclose(pr["u"], pix[:, 0] + 0.5, atol=1e-4) and np.allclose(pr["v"], pix[:, 1] + 0.5, atol=1e-4)
    assert np.allclose(pr["z"], depth[pix[:, 1], pix[:, 0]], rtol=1e-6)
    col = np.stack([pr["r"], pr["g"], pr["b_"]])
    assert np.allclose(col, rgb[:, pix[:, 1], pix[:, 0]], atol=1e-6)
    s = np.exp(new[3])
    assert np.allclose(s * 0.5 * (cam.fx + cam.fy) / depth[pix[:, 1], pix[:, 0]], 0.7 * 3)
    assert (new[6] == 1).all() and (new[7:10] == 0).all() and (new[14:] == 0).all()


def test_densify_selection_rule(orc):
    """Seeding pixels: valid depth (NaN, too near and too far excluded) and,
    with coverage, coverage below the threshold; in row-major grid order."""
    cam = identity_camera(8, 6, 10.0)
    depth = np.full((6, 8), 2.0, np.float32)
    depth[0, 0] = np.nan
    depth[0, 2] = 0.1
    depth[2, 4] = 50.0
    cov = np.zeros((6, 8), np.float32)
    cov[4, 0] = 0.5
    cov[4, 2] = 0.49
    rgb = np.full((3, 6, 8), 0.5, np.float32)
    new, pix = orc.densify(0, cam, rgb, depth, coverage=cov, step=2, depth_min=0.2, depth_max=10.0, alpha_below=0.5)
    expect = [(x, y) for y in (0, 2, 4) for x in (0, 2, 4, 6)
              if not ((x, y) in [(0, 0), (2, 0), (4, 2), (0, 4)])]
    assert [tuple(p) for p in pix] == expect
    assert np.allclose(new[11:14], 0.0)
