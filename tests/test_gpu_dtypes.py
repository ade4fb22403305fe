"""bf16 / fp16 feature storage with FP32 accumulation.

Against the oracle run on the rounded features: pure accumulation error,
within 1e-5 of sum_j w_j |f_j| per channel.  Against the unrounded FP32
features: the worst case is bounded by the storage format's unit roundoff
(bf16 2^-8 = 3.9e-3, fp16 2^-11), and the RMS relative error over pixels and
channels must stay below 2e-3."""
import numpy as np
import pytest

from gpu_helpers import decided, image_errors, np_out, render, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_half_features(orc, dtype, blend):
    require_gpu()
    sc = scenes.street40(30_000, 64, seed=8)
    cam = scenes.pinhole(320, 180)
    t = to_dev(sc, dtype)
    out, _ = render(t, cam, 16, "ellipse", blend)
    b = orc.TOPK if blend == "topk" else orc.FULL
    rounded = stored_feat(t)
    ref = orc.render(sc, cam, 16, b, feat=rounded)
    ok = decided(ref)
    absf = orc.render(sc, cam, 16, b, feat=np.abs(rounded))["feat"]
    g = np_out(out)
    worst = image_errors(g, ref, absf, ok, 1e-5)
    assert max(worst.values()) <= 1.0, worst
    ref32 = orc.render(sc, cam, 16, b)
    absf32 = orc.render(sc, cam, 16, b, feat=np.abs(sc.feat.astype(np.float64)))["feat"]
    unit = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}[dtype]
    diff = np.abs(g["feat"] - ref32["feat"])
    bound = unit * absf32 + 1e-5 * absf + 1e-7
    assert (diff / bound)[ok].max() <= 1.0
    rel = diff[ok] / (absf32[ok] + 1e-12)
    live = absf32[ok] > 1e-3
    rms = float(np.sqrt(np.mean(rel[live] ** 2)))
    assert rms < 2e-3, rms
    per_channel = np.sqrt(np.mean(rel ** 2, axis=0))
    assert per_channel.shape == (64,) and per_channel.max() < 2e-3
