"""torch.autograd.Function over the C ABI: forward = psm_forward, backward =
psm_backward (the hand-written adjoint kernels).  Parameters are activated
values (opacity in (0,1], positive scales); quaternions (w,x,y,z) need not be
unit length."""
from __future__ import annotations

import torch

from . import psm


class RasterizeSurfels(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, rgb, feat, camera, k, tile_mode, blend):
        cam = camera if isinstance(camera, psm.Camera) else psm.camera_struct(camera)
        out, ws = psm.forward(means, scales, quats, opacity, rgb, feat, cam, k, tile_mode, blend)
        ctx.save_for_backward(means, scales, quats, opacity, rgb, feat)
        ctx.ws, ctx.cam, ctx.k, ctx.tile_mode, ctx.blend = ws, cam, k, tile_mode, blend
        f = out["feat"]
        if f is None:
            f = torch.zeros(cam.height, cam.width, 0, device=means.device)
        return out["rgb"], out["depth"], out["normal"], out["alpha"], f

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_normal, g_alpha, g_feat):
        means, scales, quats, opacity, rgb, feat = ctx.saved_tensors
        gout = {"rgb": g_rgb, "depth": g_depth, "normal": g_normal, "alpha": g_alpha,
                "feat": g_feat if feat is not None else None}
        g = psm.backward(means, scales, quats, opacity, rgb, feat, ctx.cam, ctx.ws, gout, ctx.k,
                         ctx.tile_mode, ctx.blend)
        ctx.ws = None
        gf = None if feat is None else g["feat"].to(feat.dtype)
        return g["means"], g["scales"], g["quats"], g["opacity"], g["rgb"], gf, None, None, None, None


def render(means, scales, quats, opacity, rgb, feat, camera, k: int = 16, tile_mode: str = "ellipse",
           blend: str = "topk"):
    """Render RGB [H,W,3], depth [H,W], normal [H,W,3], alpha [H,W] and the
    feature map [H,W,C] of 2D Gaussian surfels seen by `camera`; features are
    blended over the K largest weights per pixel (blend="topk") or over every
    contributor (blend="full")."""
    return RasterizeSurfels.apply(means, scales, quats, opacity, rgb, feat, camera, k, tile_mode, blend)
