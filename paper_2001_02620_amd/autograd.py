"""Differentiable rendering with respect to per-face albedo.

``RenderAlbedo.apply(albedo, scene, cams, settings, opts)`` renders the packed
image with the given albedo and, on backward, runs the library's path-replay
adjoint kernel: every path is replayed from its random-number counters (so the
hits are the forward pass's hits) and the derivative of each pixel with respect
to the albedo of every face on its paths is accumulated, with hit points and
visibility held fixed.
"""
from __future__ import annotations

import torch

from . import render, render_backward


class RenderAlbedo(torch.autograd.Function):
    @staticmethod
    def forward(ctx, albedo, scene, cams, settings, opts=None):
        opts = dict(opts or {})
        a = albedo.detach().contiguous().float()
        scene.set_albedo(a)
        img = render(scene, cams, settings, **opts)
        ctx.scene = scene
        ctx.cams = cams
        ctx.settings = settings
        ctx.opts = opts
        ctx.save_for_backward(a)
        return img

    @staticmethod
    def backward(ctx, grad_img):
        (a,) = ctx.saved_tensors
        ctx.scene.set_albedo(a)  # the adjoint reads the forward albedo
        opts = {k: v for k, v in ctx.opts.items() if k not in ("counters", "view_done", "start_tick")}
        g = render_backward(ctx.scene, ctx.cams, ctx.settings, grad_img.contiguous(), **opts)
        return g, None, None, None, None
