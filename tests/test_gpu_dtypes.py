"""bf16 / fp16 feature storage with FP32 accumulation: against the oracle run
on the rounded features (pure accumulation error, 1e-5) and on the unrounded
FP32 features (2e-3 of sum_j w_j |f_j|), per output channel."""
import numpy as np
import pytest

from gpu_helpers import image_errors, np_out, render, require_gpu, stored_feat, to_dev
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
    ok = ref["margin"] > 1e-4
    absf = orc.render(sc, cam, 16, b, feat=np.abs(rounded))["feat"]
    g = np_out(out)
    worst = image_errors(g, ref, absf, ok, 1e-5)
    assert max(worst.values()) <= 1.0, worst
    ref32 = orc.render(sc, cam, 16, b)
    err = np.abs(g["feat"] - ref32["feat"]) / (2e-3 * absf + 1e-7)
    assert err[ok].max() <= 1.0
    per_channel = np.abs(g["feat"] - ref32["feat"])[ok].max(0)
    assert per_channel.shape == (64,)
