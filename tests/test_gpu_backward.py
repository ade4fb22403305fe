"""Backward parity: the hand-written adjoint kernels against the FP64 oracle
(|g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 rms(group))).  Pixels whose forward
decisions sit within the rounding margin get a zero upstream gradient on both
sides, so both differentiate the same piecewise-smooth function."""
import numpy as np
import pytest
import torch

from gpu_helpers import decided, DEV, render, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes

pytestmark = pytest.mark.gpu

GROUPS = ("means", "scales", "quats", "opacity", "rgb", "feat")


def grad_errors(got, ref):
    worst = {}
    for k in GROUPS:
        r = ref[k]
        g = got[k]
        rms = np.sqrt(np.mean(r ** 2)) if r.size else 0.0
        scale = np.maximum(np.abs(r), 1e-2 * rms) + 1e-30
        worst[k] = float((np.abs(g - r) / scale).max()) if r.size else 0.0
    return worst


CASES = {
    "box300": lambda: (scenes.uniform_box(300, 16, seed=4, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12)),
                       scenes.pinhole(64, 48, f=56.0), 4),
    "c1_box2k": lambda: scenes.config("c1_box2k")[:3],
    "planes20k": lambda: (scenes.planes7(20_000, 16, seed=5), scenes.pinhole(328, 200), 8),
}


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("case", list(CASES))
def test_gradients_match_oracle(orc, case, blend):
    require_gpu()
    sc, cam, K = CASES[case]()
    t = to_dev(sc)
    out, ws = render(t, cam, K, "ellipse", blend)
    feat = stored_feat(t)
    b = orc.TOPK if blend == "topk" else orc.FULL
    ref_f = orc.render(sc, cam, K, b, feat=feat)
    ok = decided(ref_f)
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
    for k in g:
        g[k][~ok] = 0.0
    ref = orc.backward(sc, cam, g, K=K, blend=b, feat=feat)
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    got = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                       "ellipse", blend)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got, ref)
    assert max(worst.values()) <= 1e-3, worst
