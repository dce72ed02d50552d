"""torch.autograd.Function around the library's forward and backward raster.

    images = rasterize(means, log_scales, quats, opacity_logits, sh, cameras, sh_degree=3)
    loss(images).backward()   # gradients land in the five parameter tensors

Each call owns its workspace (the frame state lives there until the backward);
the optional `stats` dict (see raster.new_stats) accumulates the opacity-gradient
statistic of Sec. 3.3 during the backward.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .raster import Rasterizer, SceneTensors, Workspace

_default = {}


def default_rasterizer(device=None) -> Rasterizer:
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    key = dev.index if dev.index is not None else torch.cuda.current_device()
    if key not in _default:
        _default[key] = Rasterizer(key)
    return _default[key]


class GaussianRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, cameras, sh_degree, rasterizer, precision,
                cluster_cull, stats, deterministic):
        st = SceneTensors(means.detach().contiguous(), log_scales.detach().contiguous(),
                          quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                          sh.detach().contiguous(), int(sh_degree))
        frame = rasterizer.forward(st, cameras, precision=precision, cluster_cull=cluster_cull,
                                   stats=stats is not None, workspace=Workspace(rasterizer.device),
                                   deterministic=deterministic)
        ctx.frame = frame
        ctx.rasterizer = rasterizer
        ctx.stats = stats
        return tuple(frame.images)

    @staticmethod
    def backward(ctx, *grad_images):
        frame = ctx.frame
        dl = []
        for g, cam in zip(grad_images, frame.cameras):
            if g is None:
                g = torch.zeros((3, cam.height, cam.width), dtype=torch.float32, device=ctx.rasterizer.device)
            dl.append(g.float().contiguous())
        grads = ctx.rasterizer.backward(frame, dl, stats=ctx.stats)
        ctx.frame = None
        return (grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"],
                None, None, None, None, None, None, None)


def rasterize(means, log_scales, quats, opacity_logits, sh, cameras, sh_degree, rasterizer=None,
              precision=L.GSR_FP32, cluster_cull=True, stats=None, deterministic=False):
    """Differentiable render of `cameras` (a list); returns a list of [3, H, W] images.
    deterministic: bitwise reproducible gradients (fixed-point per-tile sums)."""
    rz = rasterizer or default_rasterizer(means.device)
    out = GaussianRasterize.apply(means, log_scales, quats, opacity_logits, sh, list(cameras), sh_degree, rz,
                                  precision, cluster_cull, stats, bool(deterministic))
    return list(out)
