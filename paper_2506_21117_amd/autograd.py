"""torch.autograd wrapper of the renderer (differentiation as a system form).

``render(params..., cameras, bg, mode)`` returns images [V, 3, H, W] and differentiates
with respect to the five raw parameter tensors.  In ``"recompute"`` mode the forward
keeps only its inputs; the backward re-runs preprocess, binning and the forward render
to rebuild the per-pixel compositing state (final transmittance, contributor count and
the per-chunk state of the tile lists) and then runs the backward kernels — nothing of size pixels x views or pairs survives
between the two passes.  ``"stored"`` keeps that state instead.

All kernels run through the C-ABI on the current stream.
"""
from __future__ import annotations

import torch

from . import api


class _Renderer:
    """Buffers reused across calls of one (N, views, resolution)."""

    def __init__(self):
        self._key = None
        self.proj = None
        self.bins = None

    def render(self, g, cams, bg, state):
        """Preprocess, depth-sliced binning and forward; grows the pair buffers and
        renders again if they were too small."""
        dev = g.means.device
        key = (g.n, len(cams), cams[0].width, cams[0].height, str(dev))
        if key != self._key:
            self._key = key
            self.proj = api.ProjectedBuffers.alloc(g.n, len(cams), dev)
            self.bins = None
        api.project_preprocess(g, cams, self.proj)
        while True:
            if self.bins is None:
                cap = max(1 << 20, 4 * g.n * len(cams))
                self.bins = api.BinBuffers.alloc(g.n, len(cams), cams[0].width, cams[0].height, cap, dev)
            api.bin_and_sort(self.proj, cams, None, False, self.bins)
            out = api.render_forward(self.proj, self.bins, cams, bg, state=state)
            c = self.bins.read_counters()
            if not c["overflow"]:
                return self.proj, self.bins, out
            cap = int(c["pairs"] * 1.25) + 1024
            self.bins = api.BinBuffers.alloc(g.n, len(cams), cams[0].width, cams[0].height, cap, dev)


_RENDERER = _Renderer()


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logit, sh, cams, bg, sh_degree, mode):
        if mode not in ("recompute", "stored"):
            raise ValueError("mode must be 'recompute' or 'stored'")
        g = api.GaussianTensors(means.detach().contiguous(), log_scales.detach().contiguous(),
                                quats.detach().contiguous(), opacity_logit.detach().contiguous(),
                                sh.detach().contiguous(), sh_degree)
        state = api.render_state(cams, g.means.device) if mode == "stored" else None
        proj, bins, (image, T, nc) = _RENDERER.render(g, cams, bg, state)
        ctx.cams, ctx.bg, ctx.sh_degree, ctx.mode = cams, bg, sh_degree, mode
        if mode == "stored":
            # keep private copies of the compositing state and the depth lists
            ctx.state = (api.ProjectedBuffers(proj.splat.clone(), proj.depth.clone(), proj.rect.clone(),
                                              proj.flags.clone(), proj.n, proj.views),
                         api.BinBuffers(bins.values.clone(), bins.keys.clone(), bins.ranges.clone(),
                                        bins.ranges2.clone(), bins.tile_mask.clone(), bins.alive_mask.clone(),
                                        bins.tile_list.clone(), bins.counters.clone(), bins.ws[:1], bins.capacity,
                                        bins.n, bins.views, bins.width, bins.height, bins.mode),
                         T, nc, state)
        else:
            ctx.state = None
        ctx.save_for_backward(*g.tensors())
        return image

    @staticmethod
    def backward(ctx, grad_image):
        tensors = ctx.saved_tensors
        g = api.GaussianTensors(*tensors, ctx.sh_degree)
        cams = ctx.cams
        if ctx.state is None:
            state = api.render_state(cams, g.means.device)
            proj, bins, (_, T, nc) = _RENDERER.render(g, cams, ctx.bg, state)
        else:
            proj, bins, T, nc, state = ctx.state
        grads = g.zeros_like()
        api.render_backward(g, proj, bins, cams, ctx.bg, None, T, nc, state, grad_image.contiguous(), grads)
        ctx.state = None
        return (grads.means, grads.log_scales, grads.quats, grads.opacity_logit, grads.sh, None, None, None, None)


def render(means, log_scales, quats, opacity_logit, sh, cams, bg=(0.0, 0.0, 0.0), mode="recompute"):
    """Differentiable render of all views in ``cams`` (equal sizes).  Parameter tensors
    are float32 CUDA tensors in the C-ABI layout; ``sh`` is [K, 3, N]."""
    K = sh.shape[0]
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[K]
    return RenderFunction.apply(means, log_scales, quats, opacity_logit, sh, list(cams), tuple(bg), deg, mode)
