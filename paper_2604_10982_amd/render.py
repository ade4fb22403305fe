"""torch.autograd.Function over the C ABI: forward = psm_forward, backward =
psm_backward (the hand-written adjoint kernels).  Parameters are activated
values (opacity in (0,1], positive scales); quaternions (w,x,y,z) need not be
unit length."""
from __future__ import annotations

import torch

from . import psm


class RasterizeSurfels(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, rgb, feat, camera, k, tile_mode, blend, flags=0, feat_ext=None):
        if flags & psm.FLAG_FEATURE_ONLY:
            raise ValueError("render() returns every map; use psm.forward for feature-only rendering")
        cam = camera if isinstance(camera, psm.Camera) else psm.camera_struct(camera)
        out, ws = psm.forward(means, scales, quats, opacity, rgb, feat, cam, k, tile_mode, blend, flags=flags,
                              feat_ext=feat_ext)
        ctx.save_for_backward(means, scales, quats, opacity, rgb, feat, feat_ext)
        ctx.ws, ctx.cam, ctx.k, ctx.tile_mode, ctx.blend, ctx.flags = ws, cam, k, tile_mode, blend, flags
        f = out["feat"]
        if f is None:
            f = torch.zeros(cam.height, cam.width, 0, device=means.device)
        return out["rgb"], out["depth"], out["normal"], out["alpha"], f

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_normal, g_alpha, g_feat):
        means, scales, quats, opacity, rgb, feat, feat_ext = ctx.saved_tensors
        gout = {"rgb": g_rgb, "depth": g_depth, "normal": g_normal, "alpha": g_alpha,
                "feat": g_feat if feat is not None or feat_ext is not None else None}
        g = psm.backward(means, scales, quats, opacity, rgb, feat, ctx.cam, ctx.ws, gout, ctx.k,
                         ctx.tile_mode, ctx.blend, flags=ctx.flags, feat_ext=feat_ext)
        ctx.ws = None
        gf = None if feat is None else g["feat"].to(feat.dtype)
        ge = None if feat_ext is None else g["feat_ext"]
        return g["means"], g["scales"], g["quats"], g["opacity"], g["rgb"], gf, None, None, None, None, None, ge


def render(means, scales, quats, opacity, rgb, feat, camera, k: int = 16, tile_mode: str = "ellipse",
           blend: str = "topk", flags: int = 0, feat_ext=None):
    """Render RGB [H,W,3], depth [H,W], normal [H,W,3], alpha [H,W] and the
    feature map [H,W,C] of 2D Gaussian surfels seen by `camera`; features are
    blended over the K largest weights per pixel (blend="topk") or over every
    contributor (blend="full").  `flags`: psm.FLAG_OPACITY_FOOTPRINT,
    FLAG_TOPK_RENORM, FLAG_LOWPASS (FLAG_FEATURE_ONLY is refused: every map is
    returned).  `feat_ext`: optional FP32 [N, C_ext] features gathered by the
    same walk after feat's channels (the map then has C + C_ext channels)."""
    return RasterizeSurfels.apply(means, scales, quats, opacity, rgb, feat, camera, k, tile_mode, blend, flags,
                                  feat_ext)


class InstanceLabels(torch.autograd.Function):
    """Labels of surfels from localized queries (Sec. 4.1, eqs. (4)-(7)); the
    forward and the backward run in the library's kernels.  Returns the
    (n, label_width(n_q)) array whose columns >= n_q are zero."""

    @staticmethod
    def forward(ctx, means, f_ins, q_feat, q_mean, q_prec):
        lab = psm.instance_labels(means, f_ins, q_feat, q_mean, q_prec)
        ctx.save_for_backward(means, f_ins, q_feat, q_mean, q_prec)
        return lab

    @staticmethod
    def backward(ctx, g):
        means, f_ins, q_feat, q_mean, q_prec = ctx.saved_tensors
        nq = q_feat.shape[0]
        gl = g.float().contiguous().clone()
        gl[:, nq:] = 0.0  # the padding columns are constants
        out = psm.instance_labels_backward(means, f_ins, q_feat, q_mean, q_prec, gl, gl.shape[1])
        return out["means"], out["f_ins"].to(f_ins.dtype), out["q_feat"], out["q_mean"], out["q_prec"]


def instance_labels(means, f_ins, q_feat, q_mean, q_prec):
    """(n, n_q) labels: softmax over the queries of sigmoid(f_q . f_g) times the
    query Gaussian's density ratio at the surfel centre."""
    return InstanceLabels.apply(means, f_ins, q_feat, q_mean, q_prec)[:, :q_feat.shape[0]]


def render_panoptic(means, scales, quats, opacity, rgb, f_sem, f_ins, q_feat, q_mean, q_prec, camera, k: int = 16,
                    tile_mode: str = "ellipse", blend: str = "topk"):
    """One walk and one Top-K selection render the semantic features and the
    instance labels (eq. (8)): the blend gathers each selected surfel's row
    from both arrays -- the semantic features in their own storage dtype, the
    FP32 labels (padded to a multiple of 8 columns with zeros) after them --
    so no concatenated copy is made.  Returns (rgb, depth, normal, alpha,
    semantic map [H,W,C_s], instance map [H,W,n_q])."""
    labels = InstanceLabels.apply(means, f_ins, q_feat, q_mean, q_prec)
    nq, cs = q_feat.shape[0], f_sem.shape[1]
    rgb_o, depth, normal, alpha, f = render(means, scales, quats, opacity, rgb, f_sem, camera, k, tile_mode, blend,
                                            feat_ext=labels)
    return rgb_o, depth, normal, alpha, f[..., :cs], f[..., cs:cs + nq]
