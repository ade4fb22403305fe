"""Pins of the oracle's feature-only early stop (an exact work reduction):
a pixel's walk ends once it holds K weights and 0.99 T is at most the
smallest, since no later weight alpha T' (alpha <= 0.99, T' <= T) can then
enter the K largest.  The Top-K selection, its weights and the feature map
must equal those of the full walk exactly; the feature-only gradients must
equal the full walk's gradients of the same feature loss."""
import numpy as np
import pytest

from paper_2604_10982_amd import scenes
from paper_2604_10982_amd.scenes import upstream


@pytest.fixture(scope="module")
def dense_case():
    # about 40 contributors per pixel, so the stop triggers often
    sc = scenes.uniform_box(3000, 6, seed=11, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12), scale_sigma=0.4)
    return sc, scenes.pinhole(64, 48, f=56.0)


@pytest.mark.parametrize("K", [1, 4, 8])
def test_selection_and_features_unchanged(orc, dense_case, K):
    sc, cam = dense_case
    full = orc.render(sc, cam, K, orc.TOPK)
    fo = orc.render(sc, cam, K, orc.TOPK_FEATURE_ONLY)
    np.testing.assert_array_equal(fo["sel_id"], full["sel_id"])
    np.testing.assert_array_equal(fo["sel_w"], full["sel_w"])
    np.testing.assert_array_equal(fo["feat"], full["feat"])
    assert (fo["ncontrib"] <= full["ncontrib"]).all()
    # the stop removes work: contributors walked fall
    assert fo["ncontrib"].sum() < 0.7 * full["ncontrib"].sum()
    # where it stopped early, the full walk's later contributors are never selected
    stopped = fo["ncontrib"] < full["ncontrib"]
    assert stopped.sum() > 100


def test_stop_rule_by_hand():
    """One pixel, K = 1: weights 0.5, then 0.99 * 0.5 * ... -- after the first
    surfel T = 0.5 and 0.99 T = 0.495 < 0.5, so nothing later can be selected."""
    T, w1 = 1.0, 0.5
    T *= 1 - 0.5
    assert 0.99 * T <= w1
    # a later surfel with the largest possible alpha would weigh 0.99 * T < w1
    assert 0.99 * T < w1


def test_gradients_of_a_feature_loss_unchanged(orc, dense_case):
    sc, cam = dense_case
    K = 4
    g = upstream(cam.height, cam.width, sc.c, seed=3)
    for k in ("rgb", "depth", "normal", "alpha"):
        g[k] = np.zeros_like(g[k])
    full = orc.backward(sc, cam, g, K=K, blend=orc.TOPK)
    fo = orc.backward(sc, cam, g, K=K, blend=orc.TOPK_FEATURE_ONLY)
    for key in full:
        a, b = np.asarray(fo[key]), np.asarray(full[key])
        scale = max(np.abs(b).max(), 1e-30)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * scale, err_msg=key)
