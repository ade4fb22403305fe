"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the
CPU oracle)."""
import numpy as np
import torch

from paper_2604_10982_amd import psm

DEV = torch.device("cuda:0")
TORCH_DTYPES = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
OUTPUTS = ("rgb", "depth", "normal", "alpha", "feat")


# Relative decision margins below which the HIP path and the FP64 oracle may
# legitimately decide differently ("several results correct"): the hit test is
# FP64 on both sides; alpha, transmittance and the blend weights are FP32 on
# the GPU (the transmittance product accumulates about n * 6e-8 relative).
# Order: rho vs 9, alpha vs 1/255 and 0.99, T' vs 1e-4, Top-K gap.
MARGIN_TOL = (1e-9, 1e-5, 5e-5, 5e-5)


def decided(ref, tol=MARGIN_TOL):
    """Pixels whose every decision is farther than `tol` from its threshold."""
    return np.all(ref["margins"] > np.asarray(tol), axis=-1)


def require_gpu():
    assert torch.cuda.is_available(), "GPU parity tests need a HIP device"


def to_dev(sc, feat_dtype="f32"):
    t = {k: torch.tensor(np.ascontiguousarray(getattr(sc, k)), device=DEV)
         for k in ("means", "scales", "quats", "opacity", "rgb")}
    t["feat"] = torch.tensor(sc.feat, device=DEV).to(TORCH_DTYPES[feat_dtype]).contiguous()
    return t


def stored_feat(t):
    """Feature values as stored on the device (after bf16/fp16 rounding), FP64."""
    return t["feat"].float().cpu().numpy().astype(np.float64)


def render(t, cam, K, tile_mode="ellipse", blend="topk", capacity=None):
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K,
                          tile_mode, blend, capacity=capacity)
    torch.cuda.synchronize()
    return out, ws


def np_out(out):
    return {k: (None if v is None else v.cpu().numpy().astype(np.float64)) for k, v in out.items()}


def image_errors(gpu, ref, ref_absfeat, ok, tol):
    """Max of |gpu - ref| / (tol * scale) over pixels with ok margin, where the
    scale is sum_j w_j |x_j| (the conditioning of the blend sum) per channel."""
    scales = {"rgb": ref["rgb"], "depth": ref["depth"][..., None],
              "normal": np.repeat(ref["alpha"][..., None], 3, -1), "alpha": np.ones_like(ref["alpha"])[..., None],
              "feat": ref_absfeat}
    worst = {}
    for k in OUTPUTS:
        g = gpu[k].reshape(*ok.shape, -1)
        r = ref[k].reshape(*ok.shape, -1)
        s = scales[k].reshape(*ok.shape, -1)
        ratio = np.abs(g - r) / (tol * s + 1e-7)
        worst[k] = float(ratio[ok].max()) if ok.any() else 0.0
    return worst
