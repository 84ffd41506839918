"""Independent float64 torch renderer used only to pin the oracle's analytic
backward with autograd on tiny scenes. Written separately from the oracle
(different formulation: rotation via explicit matrix products, spherical
harmonics as explicit Cartesian polynomials up to degree 3, compositing
vectorised over pixels) so that agreement is evidence, not repetition.
"""
import math

import torch

ALPHA_MAX = float(torch.tensor(0.99, dtype=torch.float32))
ALPHA_MIN = float(torch.tensor(1.0, dtype=torch.float32) / 255.0)
TRANS_MIN = float(torch.tensor(1e-4, dtype=torch.float32))
DILATION = float(torch.tensor(0.3, dtype=torch.float32))
CLAMP_FOV = float(torch.tensor(1.3, dtype=torch.float32))


def sh_poly(deg, d):
    """Real SH with the Condon-Shortley phase as Cartesian polynomials, [n, (deg+1)^2]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [torch.full_like(x, math.sqrt(1 / (4 * pi)))]
    if deg >= 1:
        c1 = math.sqrt(3 / (4 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if deg >= 2:
        a = math.sqrt(15 / (4 * pi))
        b = math.sqrt(5 / (16 * pi))
        c = math.sqrt(15 / (16 * pi))
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if deg >= 3:
        k0 = math.sqrt(35 / (32 * pi))
        k1 = math.sqrt(105 / (4 * pi))
        k2 = math.sqrt(21 / (32 * pi))
        k3 = math.sqrt(7 / (16 * pi))
        k5 = math.sqrt(105 / (16 * pi))
        r2 = x * x + y * y
        out += [-k0 * y * (3 * x * x - y * y), k1 * x * y * z, -k2 * y * (4 * z * z - r2),
                k3 * z * (2 * z * z - 3 * r2), -k2 * x * (4 * z * z - r2), k5 * z * (x * x - y * y),
                -k0 * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=1)


def quat_to_rot(q):
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    R = torch.stack([
        torch.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], 1)], 1)
    return R


def project(params, deg, cam, pose_R=None, pose_t=None):
    """Screen-space splats of every Gaussian, float64 and differentiable:
    dict with u, v, A, B, C (conic), o (opacity), col [n, 3], z, and the
    culling inputs tz and det. pose_R [3, 3] and pose_t [3] (float64 tensors,
    may require grad) replace the camera's pose."""
    P, n = params.shape
    mean = params[0:3].T
    scale = torch.exp(params[3:6].T)
    R = quat_to_rot(params[6:10].T)
    opac = torch.sigmoid(params[10])
    K = (deg + 1) ** 2
    sh = params[11:].T.reshape(n, K, 3)
    W = torch.tensor(cam.R, dtype=torch.float64) if pose_R is None else pose_R
    t = torch.tensor(cam.t, dtype=torch.float64) if pose_t is None else pose_t
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy
    Wd, Hd = cam.width, cam.height
    pc = mean @ W.T + t
    Sigma = R @ torch.diag_embed(scale * scale) @ R.transpose(1, 2)
    Scam = W @ Sigma @ W.T
    tz = pc[:, 2]
    limx = CLAMP_FOV * (0.5 * Wd / fx)
    limy = CLAMP_FOV * (0.5 * Hd / fy)
    xi = torch.clamp(pc[:, 0] / tz, -limx, limx)
    yi = torch.clamp(pc[:, 1] / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * xi / tz], 1),
                     torch.stack([zero, fy / tz, -fy * yi / tz], 1)], 1)
    S2 = J @ Scam @ J.transpose(1, 2)
    a = S2[:, 0, 0] + DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    A, B, C = c / det, -b / det, a / det
    u = fx * pc[:, 0] / tz + cx
    v = fy * pc[:, 1] / tz + cy
    campos = -(W.T @ t)
    dvec = mean - campos
    d = dvec / dvec.norm(dim=1, keepdim=True)
    Y = sh_poly(deg, d)
    col = torch.clamp((Y[:, :, None] * sh).sum(1) + 0.5, min=0.0)
    return dict(u=u, v=v, A=A, B=B, C=C, o=opac, col=col, z=tz, tz=tz, det=det)


def composite(sp, cam, bg=(0.0, 0.0, 0.0), znear=0.2):
    """Front-to-back compositing of given splat values (dict as project returns),
    vectorised over the pixels. Returns rgb [3,H,W], depth, alpha."""
    u, v, A, B, C, opac, col, z = (sp[k] for k in ("u", "v", "A", "B", "C", "o", "col", "z"))
    tz, det = sp["tz"], sp["det"]
    Wd, Hd = cam.width, cam.height
    order = torch.argsort(z.detach())
    ys, xs = torch.meshgrid(torch.arange(Hd, dtype=torch.float64) + 0.5,
                            torch.arange(Wd, dtype=torch.float64) + 0.5, indexing="ij")
    T = torch.ones(Hd, Wd, dtype=torch.float64)
    done = torch.zeros(Hd, Wd, dtype=torch.bool)
    Cacc = torch.zeros(3, Hd, Wd, dtype=torch.float64)
    D = torch.zeros(Hd, Wd, dtype=torch.float64)
    for i in order.tolist():
        if not (float(tz[i].detach()) >= znear) or not (float(det[i].detach()) > 0):
            continue
        dx = u[i] - xs
        dy = v[i] - ys
        power = -0.5 * (A[i] * dx * dx + C[i] * dy * dy) - B[i] * dx * dy
        araw = opac[i] * torch.exp(power)
        alpha = torch.where(araw > ALPHA_MAX, torch.full_like(araw, ALPHA_MAX), araw)
        use = (~done) & (power <= 0) & (alpha >= ALPHA_MIN)
        Tn = T * (1 - alpha)
        stop = use & (Tn < TRANS_MIN)
        use = use & ~stop
        done = done | stop
        w = torch.where(use, alpha * T, torch.zeros_like(T))
        Cacc = Cacc + w[None] * col[i][:, None, None]
        D = D + w * z[i]
        T = torch.where(use, Tn, T)
    bgt = torch.tensor(bg, dtype=torch.float64)[:, None, None]
    return Cacc + T[None] * bgt, D, 1 - T


def render(params, deg, cam, bg=(0.0, 0.0, 0.0), znear=0.2, pose_R=None, pose_t=None):
    """params: float64 tensor [P, N] (may require grad). Returns rgb [3,H,W], depth, alpha.
    pose_R, pose_t: optional pose tensors (may require grad) in place of the camera's."""
    return composite(project(params, deg, cam, pose_R, pose_t), cam, bg, znear)
