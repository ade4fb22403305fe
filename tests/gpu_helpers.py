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


# Launch choices (schedule, bwd_schedule, blend_pass, bwd_pass).  BENCH_LAUNCH
# is what the autotuner picks for the 1080p benchmark steps (persistent
# longest-first forward and backward, Top-K blend pass 32, feature-adjoint
# pass 16); GRID_LAUNCH takes every other choice (grid schedules, pass 16 /
# 32), so a test that renders both covers each kernel's variants.
BENCH_LAUNCH = (1, 1, 32, 16)
GRID_LAUNCH = (0, 0, 16, 32)


def render(t, cam, K, tile_mode="ellipse", blend="topk", capacity=None, launch=None):
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K,
                          tile_mode, blend, capacity=capacity, launch=launch)
    torch.cuda.synchronize()
    return out, ws


def tile_pixels(tiles, cam):
    """Flat pixel indices of the listed 16x16 tiles, ascending."""
    ntx = (cam.width + 15) // 16
    pix = []
    for tt in tiles:
        ty, tx = divmod(int(tt), ntx)
        ys, xs = np.mgrid[ty * 16:min(ty * 16 + 16, cam.height), tx * 16:min(tx * 16 + 16, cam.width)]
        pix.append((ys * cam.width + xs).ravel())
    return np.unique(np.concatenate(pix)).astype(np.int64) if pix else np.zeros(0, np.int64)


def stratified_picks(count, rng, per=16, cap=None):
    """Surfels drawn across the whole distribution of pairs per surfel: `per`
    each from the lightest (1-2 pairs), the middle (between the median and the
    90th percentile), the heavy (90th-99th), the heaviest 1% and those with
    more than 64 pairs (longer than one 64-pair batch of the reductions);
    `cap` bounds the pairs of a pick (the oracle renders its tiles)."""
    nz = count[count > 0]
    q50, q90, q99 = np.percentile(nz, [50, 90, 99])
    top = count <= (cap if cap is not None else count.max())
    bands = [(count > 0) & (count <= 2), (count > q50) & (count <= q90), (count > q90) & (count <= q99),
             (count > q99) & top, (count > 64) & top]
    picks = []
    for b in bands:
        cand = np.nonzero(b)[0]
        if cand.size:
            picks.append(rng.choice(cand, min(per, cand.size), replace=False))
    return np.unique(np.concatenate(picks))


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
