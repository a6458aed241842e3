"""torch.autograd.Function over the C-ABI: image = render(offset grid, variance, lengthscale,
albedo); the backward pass is the library's path-replay adjoint (gpss_render_adjoint)."""
from __future__ import annotations

import torch

from .gpss import GpssScene


class GPSSRender(torch.autograd.Function):
    """forward: gpss_scene_set_params + gpss_render; backward: gpss_scene_set_params (to the
    parameters of this forward) + gpss_render_adjoint.  The gradient is that of the
    frozen-sampling estimator: the same random numbers and sampling decisions as the
    forward image."""

    @staticmethod
    def forward(ctx, offset, variance, lengthscale, albedo, scene: GpssScene, s0: int, s1: int):
        params = (offset.detach() if offset is not None else None, float(variance), float(lengthscale),
                  float(albedo))
        scene.set_params(*params)
        img = scene.render(s0, s1)
        ctx.scene = scene
        ctx.params = params
        ctx.range = (s0, s1)
        ctx.like = [(t.device, t.dtype) if torch.is_tensor(t) else None
                    for t in (offset, variance, lengthscale, albedo)]
        return img

    @staticmethod
    def backward(ctx, grad_img):
        scene = ctx.scene
        scene.set_params(*ctx.params)
        g_off, g_sc = scene.render_adjoint(grad_img.contiguous(), *ctx.range)
        grads = [g_off, g_sc[0], g_sc[1], g_sc[2]]
        out = []
        for g, like in zip(grads, ctx.like):
            out.append(None if (g is None or like is None) else g.to(device=like[0], dtype=like[1]))
        return (*out, None, None, None)


def render(scene: GpssScene, offset, variance, lengthscale, albedo, s0: int = 0, s1=None):
    """Differentiable image of `scene` (mean over samples [s0, s1), default all)."""
    s1 = scene.scene.spp if s1 is None else s1
    return GPSSRender.apply(offset, variance, lengthscale, albedo, scene, s0, s1)
