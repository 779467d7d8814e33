"""The training objective of Eq. 9 with the denoiser of Eq. 11, as torch autograd
Functions over the C ABI (every step runs in the library's kernels):

    loss = mean_i | D(R(I_p^i, theta)) - I_c^i |  +  lambda_reg * sum_m L(m)

D is the cross-bilateral filter steered by guide features of the scene (first-hit
albedo, normal, distance and coverage through each pixel centre, which do not depend
on theta's differentiated parameters); L(m) is the total variation of each BRDF map.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import dpcs


@dataclass
class DenoiseConfig:
    """Window radius and the 1 / (2 sigma^2) factors of D's weights.  The defaults suit
    the guide of gbuffer(): albedo (sigma 0.1), normal (0.3), distance (0.05 scene
    units), coverage (0.1); spatial sigma 2 pixels."""
    radius: int = 3
    spatial: float = 0.125
    guide: tuple = field(default_factory=lambda: (50.0, 50.0, 50.0, 5.56, 5.56, 5.56, 200.0, 50.0))

    def params(self, width: int, height: int, channels: int) -> dpcs.DenoiseParams:
        if channels != len(self.guide):
            raise ValueError(f"guide has {channels} channels, config gives {len(self.guide)} factors")
        return dpcs.denoise_params(width, height, self.radius, self.spatial, self.guide)


def _f32(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError("expected a float32 CUDA tensor")
    return t.contiguous()


def gbuffer(ctx: dpcs.Context, scene: dpcs.Scene, params: dpcs.RenderParams) -> torch.Tensor:
    """Hc x Wc x 8 guide features (albedo rgb, normal xyz, distance, coverage)."""
    out = torch.empty((params.camera.height, params.camera.width, 8), dtype=torch.float32, device="cuda")
    dpcs.dpcs_render_gbuffer(ctx, scene, params, out)
    return out


class Denoise(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx, cfg, image, guide):
        image, guide = _f32(image), _f32(guide)
        H, W = image.shape[:2]
        p = cfg.params(W, H, guide.shape[2])
        out = torch.empty_like(image)
        dpcs.dpcs_denoise(ctx, p, image, guide, out)
        fctx.dctx, fctx.p = ctx, p
        fctx.save_for_backward(guide)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        (guide,) = fctx.saved_tensors
        g = torch.empty(grad_out.shape, dtype=torch.float32, device=grad_out.device)
        dpcs.dpcs_denoise_vjp(fctx.dctx, fctx.p, _f32(grad_out), guide, g)
        return None, None, g, None


class TV(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx, m):
        m = _f32(m)
        loss = torch.empty((), dtype=torch.float32, device=m.device)
        dpcs.dpcs_tv_loss(ctx, m, loss)
        fctx.dctx = ctx
        fctx.save_for_backward(m)
        return loss

    @staticmethod
    def backward(fctx, grad_loss):
        (m,) = fctx.saved_tensors
        g = torch.empty_like(m)
        dpcs.dpcs_tv_vjp(fctx.dctx, m, _f32(grad_loss.reshape(())), g)
        return None, g


class L1(torch.autograd.Function):
    """mean |a - b|; b is a constant (the capture)."""
    @staticmethod
    def forward(fctx, ctx, a, b):
        a, b = _f32(a), _f32(b)
        if a.shape != b.shape:
            raise ValueError("a and b must have the same shape")
        loss = torch.empty((), dtype=torch.float32, device=a.device)
        dpcs.dpcs_l1_loss(ctx, a, b, loss)
        fctx.dctx = ctx
        fctx.save_for_backward(a, b)
        return loss

    @staticmethod
    def backward(fctx, grad_loss):
        a, b = fctx.saved_tensors
        g = torch.empty_like(a)
        dpcs.dpcs_l1_vjp(fctx.dctx, a, b, _f32(grad_loss.reshape(())), g)
        return None, g, None


def denoise(ctx, image, guide, cfg: DenoiseConfig | None = None):
    return Denoise.apply(ctx, cfg or DenoiseConfig(), image, guide)


def tv(ctx, m):
    return TV.apply(ctx, m)


def l1(ctx, a, b):
    return L1.apply(ctx, a, b)
