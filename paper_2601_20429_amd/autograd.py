"""torch.autograd.Function around the HIP forward and backward kernels.

    rgb, depth, opacity = GRTXRender.apply(means, scales, quats, opacities, sh, origins, dirs, settings)

`settings` is a RenderSettings. The forward builds the acceleration structure from the
current parameters (as a training step would) and traces with a hit-id list; the
backward replays each ray's blended hits in the HIP backward kernel. Gradients flow to
means, scales, quats, opacities and sh; rays receive none.
"""
from __future__ import annotations

import warnings
from dataclasses import dataclass

import torch

from . import grtx


@dataclass(frozen=True)
class RenderSettings:
    sh_degree: int = 3
    k: int = 16
    T_min: float = 1e-3
    alpha_min: float = 1.0 / 255.0
    mode: int = grtx.CHECKPOINT
    kind: int = grtx.SPHERE_INSTANCE
    bg: tuple = (0.0, 0.0, 0.0)
    hit_capacity: int = 512
    # > 0: the rays are a row-major image of this width (8x8 tile scheduling; results are
    # unaffected)
    image_width: int = 0
    # after each backward, read the number of rays whose blended hits overflowed the list
    # (a device-to-host read) and warn: their gradients miss the hits past the list
    check_truncation: bool = True


class GRTXRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, origins, dirs, settings: RenderSettings):
        scene = grtx.SceneTensors(means.detach().contiguous(), scales.detach().contiguous(),
                                  quats.detach().contiguous(), opacities.detach().contiguous(),
                                  sh.detach().contiguous(), settings.sh_degree)
        bvh = grtx.build(scene, kind=settings.kind, alpha_min=settings.alpha_min)
        o = origins.detach().contiguous()
        d = dirs.detach().contiguous()
        out = grtx.trace(bvh, o, d, k=settings.k, T_min=settings.T_min, mode=settings.mode, bg=settings.bg,
                         hit_capacity=settings.hit_capacity, image_width=settings.image_width)
        ctx.bvh = bvh
        ctx.settings = settings
        ctx.save_for_backward(o, d, out["rgb"], out["depth"], out["opacity"], out["hit_ids"], out["hit_counts"])
        return out["rgb"], out["depth"], out["opacity"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_opac):
        o, d, rgb, depth, opacity, hit_ids, hit_counts = ctx.saved_tensors
        s = ctx.settings
        fwd = dict(rgb=rgb, depth=depth, opacity=opacity, hit_ids=hit_ids, hit_counts=hit_counts)
        grads, truncated = grtx.trace_backward(
            ctx.bvh, o, d, fwd,
            grad_rgb=None if g_rgb is None else g_rgb.contiguous(),
            grad_depth=None if g_depth is None else g_depth.contiguous(),
            grad_opacity=None if g_opac is None else g_opac.contiguous(),
            k=s.k, T_min=s.T_min, mode=s.mode, bg=s.bg)
        ctx.truncated = truncated
        if s.check_truncation:
            n = int(truncated.item())
            if n > 0:
                warnings.warn(f"GRTXRender.backward: {n} rays blended more hits than hit_capacity="
                              f"{s.hit_capacity}; their gradients cover only the first {s.hit_capacity} hits",
                              RuntimeWarning)
        return grads["means"], grads["scales"], grads["quats"], grads["opacities"], grads["sh"], None, None, None


def render(means, scales, quats, opacities, sh, origins, dirs, settings: RenderSettings = RenderSettings()):
    return GRTXRender.apply(means, scales, quats, opacities, sh, origins, dirs, settings)
