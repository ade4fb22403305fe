"""Renormalised Top-K (the selected weights rescaled to sum 1): the HIP feature
map against the FP64 oracle on the stored feature values (|F - F_ref| <=
1e-5 sum_sel w |f| / W per channel), the selection and the geometry maps unchanged
by the flag, and the backward of the quotient against the oracle's
(|g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 rms(group)))."""
import numpy as np
import pytest
import torch

from gpu_helpers import decided, DEV, image_errors, np_out, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from test_gpu_backward import grad_errors

pytestmark = pytest.mark.gpu

RN = psm.FLAG_TOPK_RENORM

CASES = {
    "box3k_dense": lambda: (scenes.uniform_box(3000, 16, seed=11, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12),
                                               scale_sigma=0.4), scenes.pinhole(64, 48, f=56.0), 4, "f32"),
    "planes20k": lambda: (scenes.planes7(20_000, 16, seed=5), scenes.pinhole(328, 200), 8, "f32"),
    "street60k_ragged_bf16": lambda: (scenes.street40(60_000, 8, seed=4), scenes.pinhole(801, 449), 16, "bf16"),
}


def _fwd(t, cam, K, flags):
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K, "ellipse",
                          "topk", flags=flags)
    torch.cuda.synchronize()
    cfg = psm.config_struct(K, "ellipse", "topk", flags)
    sel = psm.read_selection(ws, psm.camera_struct(cam), cfg)
    return out, ws, sel


@pytest.mark.parametrize("case", list(CASES))
def test_renorm_features_match_oracle(orc, case):
    require_gpu()
    sc, cam, K, dt = CASES[case]()
    t = to_dev(sc, dt)
    out0, _, sel0 = _fwd(t, cam, K, 0)
    out1, _, sel1 = _fwd(t, cam, K, RN)
    # the flag changes only the feature map
    assert torch.equal(sel0["sel_id"], sel1["sel_id"]) and torch.equal(sel0["sel_w"], sel1["sel_w"])
    for k in ("rgb", "depth", "normal", "alpha"):
        assert torch.equal(out0[k], out1[k]), k
    feat = stored_feat(t)
    ref = orc.render(sc, cam, K, orc.TOPK_RENORM, feat=feat)
    absf = orc.render(sc, cam, K, orc.TOPK_RENORM, feat=np.abs(feat))["feat"]
    ok = decided(ref)
    assert ok.mean() > 0.9
    got = np_out(out1)
    worst = image_errors(got, ref, absf, ok, 1e-5)
    assert worst["feat"] <= 1.0, worst
    # pixels with nothing selected report zero features
    empty = (sel1["sel_w"].sum(-1) == 0).cpu().numpy().reshape(ok.shape)
    assert np.all(got["feat"].reshape(*ok.shape, -1)[empty] == 0.0)


@pytest.mark.parametrize("case", list(CASES))
def test_renorm_gradients_match_oracle(orc, case):
    require_gpu()
    sc, cam, K, dt = CASES[case]()
    t = to_dev(sc, dt)
    _, ws, _ = _fwd(t, cam, K, RN)
    feat = stored_feat(t)
    ref_f = orc.render(sc, cam, K, orc.TOPK_RENORM, feat=feat)
    ok = decided(ref_f)
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
    for k in g:
        g[k][~ok] = 0.0
    ref = orc.backward(sc, cam, g, K=K, blend=orc.TOPK_RENORM, feat=feat)
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    got = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                       "ellipse", "topk", flags=RN)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got, ref)
    assert max(worst.values()) <= 1e-3, worst


def test_renorm_rejects_dense_blend():
    require_gpu()
    sc, cam, K, _ = CASES["box3k_dense"]()
    t = to_dev(sc)
    ctx = psm.context(0)
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    c = psm.camera_struct(cam)
    with pytest.raises(Exception, match="TOPK_RENORM"):  # refused already when sizing the workspace
        cfg = psm.config_struct(K, "ellipse", "full", RN)
        psm.alloc_workspace(s.n, c, cfg, s.c, psm.capacity_guess(s.n, c), DEV)
    cfg = psm.config_struct(K, "ellipse", "topk", 0)
    ws = psm.alloc_workspace(s.n, c, cfg, s.c, psm.capacity_guess(s.n, c), DEV)
    with pytest.raises(Exception, match="TOPK_RENORM"):
        psm.forward_into(ctx, s, c, psm.config_struct(K, "ellipse", "full", RN), ws, psm.alloc_images(c, s.c, DEV))
