"""The feature-gradient reduction's heavy path.  A surfel whose flagged rows
(its (tile, surfel) pairs with a selection) outnumber what one compaction
list holds (1792 rows a drain) is summed by the block-per-surfel pass over
several drains.  Here one faint, wide surfel in front of a 1280 x 720 camera
is selected in about 3000 of its 3600 tiles:

* every gradient, that surfel's included, matches the FP64 oracle;
* with the opacity-aware footprint (which drops the tiles of the surfel's
  outer ring, where no pixel reaches alpha 1/255, so none selects it) every
  gradient is bit-identical: the heavy path's order of addition depends only
  on the flagged rows.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, decided, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from test_gpu_backward import grad_errors

pytestmark = pytest.mark.gpu


def _scene():
    small = scenes.uniform_box(60, 16, seed=12, xy=1.5, z=(3.0, 6.0), scale_mu=np.log(0.15))
    rng = np.random.default_rng(13)
    # fronto-parallel (identity rotation), 240 px per unit of its tangent
    # frame at this depth and focal length, opacity 0.06: alpha reaches 1/255
    # at rho = 2 ln(255 * 0.06), about 2.34 units (560 px) from its centre,
    # while the 3-unit cutoff reaches 720 px, past the image's corners
    big = scenes.Scene(np.array([[0.02, -0.01, 2.0]], np.float32), np.array([[0.5, 0.5]], np.float32),
                       np.array([[1.0, 0.0, 0.0, 0.0]], np.float32), np.array([0.06], np.float32),
                       np.array([[0.8, 0.3, 0.1]], np.float32),
                       rng.standard_normal((1, 16)).astype(np.float32))
    cat = lambda a, b: np.ascontiguousarray(np.concatenate([a, b], 0))
    return scenes.Scene(cat(small.means, big.means), cat(small.scales, big.scales), cat(small.quats, big.quats),
                        cat(small.opacity, big.opacity), cat(small.rgb, big.rgb), cat(small.feat, big.feat))


def _backward(t, cam, K, ws, gt, flags):
    g = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                     "ellipse", "topk", flags=flags)
    torch.cuda.synchronize()
    return g


def test_heavy_surfel_gradients_match_oracle_and_ignore_unflagged_pairs(orc):
    require_gpu()
    sc = _scene()
    cam = scenes.pinhole(1280, 720, f=960.0)
    K = 4
    t = to_dev(sc)
    print("[heavy] render 1280x720, one surfel over the whole image", flush=True)
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K,
                          "ellipse", "topk")
    torch.cuda.synchronize()
    # precondition: the wide surfel is selected in more tiles than one drain holds
    cs = psm.camera_struct(cam)
    sel = psm.read_selection(ws, cs, psm.config_struct(K))["sel_id"].cpu().numpy()
    H, W = sel.shape[:2]
    tile = (np.arange(H)[:, None] // 16) * ((W + 15) // 16) + np.arange(W)[None, :] // 16
    big = sc.n - 1
    tiles_big = np.unique(np.broadcast_to(tile[:, :, None], sel.shape)[sel == big]).size
    assert tiles_big > 1792, tiles_big

    feat = stored_feat(t)
    ref_f = orc.render(sc, cam, K, orc.TOPK, feat=feat)
    ok = decided(ref_f)
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=3)
    for k in g:
        g[k][~ok] = 0.0
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    got = _backward(t, cam, K, ws, gt, 0)
    ref = orc.backward(sc, cam, g, K=K, blend=orc.TOPK, feat=feat)
    got64 = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got64, ref)
    assert max(worst.values()) <= 1e-3, worst

    # the opacity-aware footprint drops only pairs that carry no row
    out2, ws2 = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K,
                            "ellipse", "topk", flags=psm.FLAG_OPACITY_FOOTPRINT)
    torch.cuda.synchronize()
    st1 = psm.read_stats(ws, sc.n, cs, psm.config_struct(K), sc.c, ws.capacity)
    st2 = psm.read_stats(ws2, sc.n, cs, psm.config_struct(K, flags=psm.FLAG_OPACITY_FOOTPRINT), sc.c, ws2.capacity)
    assert st2.pairs < st1.pairs, (st2.pairs, st1.pairs)
    assert st2.selected_pairs == st1.selected_pairs
    for k in out:
        assert torch.equal(out[k], out2[k]), k
    got2 = _backward(t, cam, K, ws2, gt, psm.FLAG_OPACITY_FOOTPRINT)
    for k in got:
        assert torch.equal(got[k], got2[k]), k
