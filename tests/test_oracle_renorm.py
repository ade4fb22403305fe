"""Pins of the oracle's renormalised Top-K blend (a described variant): the
selected weights are rescaled to sum 1, F = sum_sel w f / sum_sel w.  Pinned
against the plain Top-K render (same selection, divided by the selected
weights' sum), by constant features (a partition of unity reproduces them),
and its gradients by central differences (tests/test_oracle_grad.py)."""
import numpy as np

from paper_2604_10982_amd import scenes


def _case():
    sc = scenes.uniform_box(800, 6, seed=21, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12), scale_sigma=0.4)
    return sc, scenes.pinhole(48, 40, f=48.0)


def test_renorm_is_topk_over_selected_weight(orc):
    sc, cam = _case()
    K = 4
    top = orc.render(sc, cam, K, orc.TOPK)
    ren = orc.render(sc, cam, K, orc.TOPK_RENORM)
    np.testing.assert_array_equal(ren["sel_id"], top["sel_id"])
    W = top["sel_w"].sum(-1)
    has = W > 0
    assert has.mean() > 0.5
    np.testing.assert_allclose(ren["feat"][has], top["feat"][has] / W[has][:, None], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(ren["feat"][~has], 0.0)
    # geometry outputs do not depend on the feature blend
    for k in ("rgb", "depth", "alpha"):
        np.testing.assert_array_equal(ren[k], top[k])


def test_renorm_reproduces_constant_features(orc):
    sc, cam = _case()
    v = np.array([0.3, -1.2, 2.0, 0.0, 5.5, -0.7])
    feat = np.tile(v, (sc.n, 1))
    ren = orc.render(sc, cam, 4, orc.TOPK_RENORM, feat=feat)
    has = ren["sel_w"].sum(-1) > 0
    np.testing.assert_allclose(ren["feat"][has], np.broadcast_to(v, ren["feat"][has].shape), rtol=1e-13, atol=1e-14)
