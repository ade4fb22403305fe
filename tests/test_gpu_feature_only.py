"""Feature-only rendering (an exact work reduction of the forward walk): the
Top-K selection and the feature map equal the full walk's bit for bit with
fewer contributor evaluations, and the backward of a feature loss matches the
FP64 oracle (|g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 rms(group)))."""
import numpy as np
import pytest
import torch

from gpu_helpers import decided, DEV, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from test_gpu_backward import grad_errors

pytestmark = pytest.mark.gpu

FO = psm.FLAG_FEATURE_ONLY

CASES = {
    "box3k_dense": lambda: (scenes.uniform_box(3000, 16, seed=11, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12),
                                               scale_sigma=0.4), scenes.pinhole(64, 48, f=56.0), 4),
    "planes20k": lambda: (scenes.planes7(20_000, 16, seed=5), scenes.pinhole(328, 200), 8),
    "street60k_ragged": lambda: (scenes.street40(60_000, 8, seed=4), scenes.pinhole(801, 449), 16),
}


def _fwd(t, cam, K, flags):
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K, "ellipse",
                          "topk", flags=flags)
    torch.cuda.synchronize()
    cfg = psm.config_struct(K, "ellipse", "topk", flags)
    sel = psm.read_selection(ws, psm.camera_struct(cam), cfg)
    st = psm.read_stats(ws, t["means"].shape[0], psm.camera_struct(cam), cfg, t["feat"].shape[1], ws.capacity)
    return out, ws, sel, st


@pytest.mark.parametrize("case", list(CASES))
def test_feature_only_selection_and_features_bitwise(case):
    require_gpu()
    sc, cam, K = CASES[case]()
    t = to_dev(sc)
    out0, _, sel0, st0 = _fwd(t, cam, K, 0)
    out1, _, sel1, st1 = _fwd(t, cam, K, FO)
    assert out1["rgb"] is None and out1["alpha"] is None
    assert torch.equal(out0["feat"], out1["feat"])
    assert torch.equal(sel0["sel_id"], sel1["sel_id"])
    assert torch.equal(sel0["sel_w"], sel1["sel_w"])
    assert st1.contributors <= st0.contributors
    assert st1.pairs_walked <= st0.pairs_walked
    if case == "box3k_dense":  # ~40 contributors per pixel: the stop removes work
        assert st1.contributors < 0.7 * st0.contributors


@pytest.mark.parametrize("case", list(CASES))
def test_feature_only_gradients_match_oracle(orc, case):
    require_gpu()
    sc, cam, K = CASES[case]()
    t = to_dev(sc)
    _, ws, _, _ = _fwd(t, cam, K, FO)
    feat = stored_feat(t)
    ref_f = orc.render(sc, cam, K, orc.TOPK, feat=feat)
    ok = decided(ref_f)
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
    for k in ("rgb", "depth", "normal", "alpha"):
        g[k] = np.zeros_like(g[k])
    g["feat"][~ok] = 0.0
    ref = orc.backward(sc, cam, g, K=K, blend=orc.TOPK_FEATURE_ONLY, feat=feat)
    gt = {"feat": torch.tensor(g["feat"], device=DEV)}
    got = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                       "ellipse", "topk", flags=FO)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got, ref)
    assert max(worst.values()) <= 1e-3, worst


def test_feature_only_rejects_other_maps():
    require_gpu()
    sc, cam, K = CASES["box3k_dense"]()
    t = to_dev(sc)
    ctx = psm.context(0)
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    c = psm.camera_struct(cam)
    cfg = psm.config_struct(K, "ellipse", "topk", FO)
    ws = psm.alloc_workspace(s.n, c, cfg, s.c, psm.capacity_guess(s.n, c), DEV)
    with pytest.raises(Exception, match="FEATURE_ONLY"):
        psm.forward_into(ctx, s, c, cfg, ws, psm.alloc_images(c, s.c, DEV))   # rgb etc. allocated
    with pytest.raises(Exception, match="FEATURE_ONLY"):
        full = psm.config_struct(K, "ellipse", "full", FO)
        psm.forward_into(ctx, s, c, full, ws, psm.alloc_images(c, s.c, DEV, feature_only=True))
