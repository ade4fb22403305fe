"""Crowded tiles: tens of thousands of small surfels over a few tiles, so a
tile's list spans several ranking windows (more than 16384 list positions)
and its pixels select hundreds of distinct surfels (more slots than one
staged chunk holds).  The Top-K feature blend and the feature adjoint take
their windowed paths there; images, selections and gradients are checked
against the FP64 oracle as in the other parity tests."""
import numpy as np
import pytest
import torch

from gpu_helpers import decided, DEV, image_errors, np_out, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from paper_2604_10982_amd.scenes import Scene
from test_gpu_backward import grad_errors

pytestmark = pytest.mark.gpu


def crowded(n=60_000, c=16, seed=7):
    """n surfels of about 1 px radius over the central 40x24 px of a 64x48 image."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(2.0, 6.0, n)
    f = 48.0
    px = rng.uniform(12.0, 52.0, n)
    py = rng.uniform(12.0, 36.0, n)
    means = np.stack([(px - 32.0) * z / f, (py - 24.0) * z / f, z], -1)
    q = rng.standard_normal((n, 4))
    scales = np.exp(rng.normal(np.log(0.45 / f), 0.3, (n, 2))) * z[:, None]
    sc = Scene(means.astype(np.float32), scales.astype(np.float32), q.astype(np.float32),
               rng.uniform(0.05, 0.3, n).astype(np.float32), rng.uniform(0, 1, (n, 3)).astype(np.float32),
               rng.standard_normal((n, c)).astype(np.float32))
    return sc, scenes.pinhole(64, 48, f=f)


@pytest.mark.parametrize("K", [16, 32])
def test_crowded_tiles_match_oracle(orc, K):
    require_gpu()
    sc, cam = crowded()
    t = to_dev(sc)
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K)
    torch.cuda.synchronize()
    cfg = psm.config_struct(K)
    pairs = psm.read_pairs(ws, psm.camera_struct(cam), cfg)
    tiles = pairs["tile"].numpy()
    assert np.bincount(tiles).max() > 16384  # a list longer than one ranking window
    feat = stored_feat(t)
    ref = orc.render(sc, cam, K, orc.TOPK, feat=feat)
    sel_ids = ref["sel_id"].reshape(3, 16, 4, 16, K).transpose(0, 2, 1, 3, 4).reshape(12, -1)
    assert max(len(np.unique(s[s >= 0])) for s in sel_ids) > 128  # more slots than one chunk
    absf = orc.render(sc, cam, K, orc.TOPK, feat=np.abs(feat))["feat"]
    ok = decided(ref)
    assert ok.mean() > 0.99
    worst = image_errors(np_out(out), ref, absf, ok, 1e-5)
    assert max(worst.values()) <= 1.0, worst
    sel = psm.read_selection(ws, psm.camera_struct(cam), cfg)
    np.testing.assert_array_equal(sel["sel_id"].cpu().numpy()[ok], ref["sel_id"][ok])
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=2)
    for k in g:
        g[k][~ok] = 0.0
    gref = orc.backward(sc, cam, g, K=K, blend=orc.TOPK, feat=feat)
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    got = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got, gref)
    assert max(worst.values()) <= 1e-3, worst
