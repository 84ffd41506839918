"""Differentiable rasterization for torch: a context object and an
autograd Function whose forward and backward are the library's HIP kernels.

The backward saves nothing per Gaussian: it calls gsr_render_backward, which
recomputes each pixel's transmittance in reverse order from the final value
the forward stored in the context.
"""
from __future__ import annotations

import torch

from . import _lib


class Rasterizer:
    """Owns one gsr context (device scratch) and its options."""

    def __init__(self, tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0), znear=0.2, pixels_per_thread=0, batch_depth=0,
                 tile_order=0, chunk_len=0, max_chunks=0, fuse_blend=0, depth_sort=0, backward_schedule=0, binning=0):
        self.tile_w, self.tile_h = tile_w, tile_h
        self.pixels_per_thread, self.batch_depth, self.tile_order = pixels_per_thread, batch_depth, tile_order
        self.chunk_len, self.max_chunks, self.fuse_blend = chunk_len, max_chunks, fuse_blend
        self.depth_sort, self.backward_schedule, self.binning = depth_sort, backward_schedule, binning
        self.bg = tuple(float(x) for x in bg)
        self.znear = znear
        self.handle = _lib.gsr_create(tile_w, tile_h, batch_depth, self.bg, znear, pixels_per_thread, tile_order,
                                      chunk_len, max_chunks, fuse_blend, depth_sort, backward_schedule, binning)

    def close(self):
        if self.handle is not None:
            _lib.gsr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def alloc_images(cams, device="cuda"):
        return [(torch.empty(3, c.height, c.width, device=device),
                 torch.empty(c.height, c.width, device=device),
                 torch.empty(c.height, c.width, device=device)) for c in cams]

    def render(self, params, sh_degree, cams, outs=None):
        if outs is None:
            outs = self.alloc_images(cams, params.device)
        _lib.gsr_render(self.handle, params, sh_degree, cams, outs)
        return outs

    def render_backward(self, params, sh_degree, cams, grads, grad_params=None):
        if grad_params is None:
            grad_params = torch.zeros_like(params)
        _lib.gsr_render_backward(self.handle, params, sh_degree, cams, grads, grad_params)
        return grad_params

    def render_backward_pose(self, params, sh_degree, cams, grads, grad_params=None, twist=True):
        """Camera gradients of the last render: (dL/d(R, t) [V, 12] float64, twist [V, 6] or None); with
        grad_params (a tensor like params) the parameter gradient is added there as well."""
        nv = len(cams)
        gc = torch.zeros(nv, 12, dtype=torch.float64, device=params.device)
        tw = torch.zeros(nv, 6, dtype=torch.float64, device=params.device) if twist else None
        _lib.gsr_render_backward_pose(self.handle, params, sh_degree, cams, grads, gc, grad_params, tw)
        return gc, tw

    def loss_l1(self, cams, rendered, targets, depth_weight=0.5):
        grads = [(torch.empty_like(r[0]), torch.empty_like(r[1]), torch.empty_like(r[2])) for r in rendered]
        loss = torch.empty(1, device=rendered[0][0].device)
        _lib.gsr_loss_l1(self.handle, cams, rendered, targets, grads, depth_weight, loss)
        return loss, grads

    def adam_step(self, params, grads, m, v, lr_per_plane, step, beta1=0.9, beta2=0.999, eps=1e-15):
        _lib.gsr_adam_step(self.handle, params, grads, m, v, lr_per_plane, step, beta1, beta2, eps)

    def mapping_iteration(self, params, sh_degree, cams, outs, targets, grad_params, depth_weight=0.5, loss=None,
                          adam=None):
        """Render, L1 loss, backward and (optionally) Adam of one mapping iteration, replayed as one HIP
        graph; grad_params is overwritten, params updated in place when adam is given."""
        _lib.gsr_mapping_iteration(self.handle, params, sh_degree, cams, outs, targets, depth_weight, grad_params,
                                   loss, adam)

    def mapping_status(self):
        return _lib.gsr_mapping_status(self.handle)

    def status(self):
        return _lib.gsr_query_status(self.handle)

    def set_profiling(self, stages=None):
        _lib.gsr_set_profiling(self.handle, stages)

    def profile(self, reset=True):
        return _lib.gsr_get_profile(self.handle, reset)

    def count_work(self, num_views):
        return _lib.gsr_count_work(self.handle, num_views)

    def instances(self):
        return _lib.gsr_copy_instances(self.handle)

    def splats(self, view, num):
        return _lib.gsr_copy_splats(self.handle, view, num)


class Rasterize(torch.autograd.Function):
    """rgb_0, depth_0, alpha_0, rgb_1, ... = Rasterize.apply(params, sh_degree, cams, rasterizer)."""

    @staticmethod
    def forward(ctx, params, sh_degree, cams, rasterizer):
        outs = rasterizer.render(params.detach(), sh_degree, cams)
        ctx.save_for_backward(params)
        ctx.sh_degree, ctx.cams, ctx.rasterizer = sh_degree, cams, rasterizer
        return tuple(t for o in outs for t in o)

    @staticmethod
    def backward(ctx, *grads):
        (params,) = ctx.saved_tensors
        per_view = [tuple(g.contiguous() if g is not None else None for g in grads[3 * v:3 * v + 3])
                    for v in range(len(ctx.cams))]
        gp = ctx.rasterizer.render_backward(params.detach(), ctx.sh_degree, ctx.cams, per_view)
        return gp, None, None, None


def rasterize(params, sh_degree, cams, rasterizer):
    """List of (rgb, depth, alpha) per view, differentiable with respect to params."""
    flat = Rasterize.apply(params, sh_degree, cams, rasterizer)
    return [tuple(flat[3 * v:3 * v + 3]) for v in range(len(cams))]


class GaussianMap:
    """A map that grows by keyframe insertion: parameters and Adam moments in
    buffers [P, capacity] with spare room, the first `num` Gaussians being the
    map. params/m/v are [P, num] views with the buffers' plane stride, which
    every entry point accepts. Growing moves the buffers, so the next mapping
    iteration captures its graph again."""

    def __init__(self, params, sh_degree, capacity=None, growth=1.5):
        P, n = params.shape
        self.sh_degree, self.growth, self.num = sh_degree, growth, n
        cap = max(int(capacity or n), n, 1)
        self._p = torch.zeros(P, cap, dtype=torch.float32, device=params.device)
        self._p[:, :n] = params
        self._m = torch.zeros_like(self._p)
        self._v = torch.zeros_like(self._p)

    @property
    def capacity(self):
        return self._p.shape[1]

    @property
    def params(self):
        return self._p[:, :self.num]

    @property
    def m(self):
        return self._m[:, :self.num]

    @property
    def v(self):
        return self._v[:, :self.num]

    def zeros(self):
        """A zero tensor laid out like params (same plane stride), e.g. for the gradient."""
        return torch.zeros(self._p.shape[0], self.capacity, dtype=torch.float32, device=self._p.device)[:, :self.num]

    def reserve(self, n):
        if n <= self.capacity:
            return
        cap = max(n, int(self.capacity * self.growth) + 1)
        for name in ("_p", "_m", "_v"):
            old = getattr(self, name)
            new = torch.zeros(old.shape[0], cap, dtype=old.dtype, device=old.device)
            new[:, :self.num] = old[:, :self.num]
            setattr(self, name, new)

    def insert_keyframe(self, rasterizer, cam, rgb, depth, coverage=None, **options):
        """Seed Gaussians from an RGB-D keyframe (gsr_densify) and append them,
        growing the buffers when they are full. Returns the number added."""
        added, wanted = _lib.gsr_densify(rasterizer.handle, self._p, self.num, self.sh_degree, cam, rgb, depth,
                                         coverage, **options)
        if wanted > added:
            self.reserve(self.num + wanted)
            added, wanted = _lib.gsr_densify(rasterizer.handle, self._p, self.num, self.sh_degree, cam, rgb, depth,
                                             coverage, **options)
        assert added == wanted
        self.num += added
        return added
