"""Degenerate and boundary cases of the HIP path through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_helpers import decided, DEV, OUTPUTS, image_errors, np_out, render, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from paper_2604_10982_amd.scenes import Scene

pytestmark = pytest.mark.gpu


def _empty(n=0, c=8):
    f = lambda *s: np.zeros(s, np.float32)
    return Scene(f(n, 3), f(n, 2) + 0.1, f(n, 4) + 0.5, f(n) + 0.5, f(n, 3), f(n, c))


def test_no_surfels():
    require_gpu()
    cam = scenes.pinhole(70, 45)
    t = to_dev(_empty())
    out, ws = render(t, cam, 4)
    for k in OUTPUTS:
        assert torch.count_nonzero(out[k]) == 0, k
    g = {k: torch.ones_like(out[k]) for k in OUTPUTS}
    gr = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, g, 4)
    assert gr["means"].shape == (0, 3)


def test_everything_culled():
    require_gpu()
    cam = scenes.pinhole(64, 64)
    sc = scenes.uniform_box(500, 8, seed=1)
    sc.means[:, 2] *= -1.0                       # behind the camera
    t = to_dev(sc)
    out, ws = render(t, cam, 4)
    for k in OUTPUTS:
        assert torch.count_nonzero(out[k]) == 0, k
    st = psm.read_stats(ws, sc.n, psm.camera_struct(cam), psm.config_struct(4), sc.c, ws.capacity)
    assert st.visible == 0 and st.culled[2] == 500 and st.pairs == 0
    g = {k: torch.randn_like(out[k]) for k in OUTPUTS}
    gr = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, g, 4)
    for k, v in gr.items():
        assert torch.count_nonzero(v) == 0, k


def test_single_pixel_and_single_tile_images(orc):
    require_gpu()
    sc = scenes.uniform_box(300, 8, seed=2, xy=0.3, z=(2.0, 4.0))
    for w, h in ((1, 1), (16, 16), (17, 1), (3, 33)):
        cam = scenes.pinhole(w, h, f=20.0)
        t = to_dev(sc)
        out, _ = render(t, cam, 4)
        ref = orc.render(sc, cam, 4, orc.TOPK)
        absf = orc.render(sc, cam, 4, orc.TOPK, feat=np.abs(sc.feat.astype(np.float64)))["feat"]
        ok = decided(ref)
        worst = image_errors(np_out(out), ref, absf, ok, 1e-5)
        assert max(worst.values()) <= 1.0, (w, h, worst)


def test_capacity_overflow_is_reported_and_retried():
    require_gpu()
    sc, cam, K, _ = scenes.config("c1_box2k")
    t = to_dev(sc)
    cs = psm.camera_struct(cam)
    cfg = psm.config_struct(K)
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    ws = psm.alloc_workspace(sc.n, cs, cfg, sc.c, 100, DEV)
    out = psm.alloc_images(cs, sc.c, DEV)
    with pytest.raises(psm.CapacityError):
        psm.forward_into(psm.context(0), s, cs, cfg, ws, out)
    st = psm.read_stats(ws, sc.n, cs, cfg, sc.c, 100)
    assert st.pairs_required > 100 and st.pairs == 100
    full, ws2 = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K,
                            capacity=100)
    ref, _ = render(t, cam, K)
    for k in OUTPUTS:
        assert torch.equal(full[k], ref[k]), k
    assert ws2.capacity >= st.pairs_required


def test_invalid_arguments_raise():
    require_gpu()
    sc = scenes.uniform_box(10, 12, seed=0)
    t = to_dev(sc)
    cam = scenes.pinhole(32, 32)
    with pytest.raises(psm.PsmError) as e:
        render(t, cam, 4)
    assert e.value.status == psm.ERR_UNSUPPORTED
    sc = scenes.uniform_box(10, 8, seed=0)
    t = to_dev(sc)
    for k in (0, 33):
        with pytest.raises(psm.PsmError) as e:
            render(t, cam, k)
        assert e.value.status == psm.ERR_INVALID_ARG
    with pytest.raises(ValueError):
        psm.forward(t["means"].cpu(), t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, 4)


def test_near_plane_straddling_and_degenerate_surfels(orc):
    require_gpu()
    cam = scenes.pinhole(96, 64)
    sc = scenes.uniform_box(800, 8, seed=9, xy=1.5, z=(0.1, 3.0), scale_mu=np.log(0.2))
    sc.scales[:50, 1] = 1e-6                      # nearly a line
    t = to_dev(sc)
    out, ws = render(t, cam, 8)
    got = psm.read_pairs(ws, psm.camera_struct(cam), psm.config_struct(8))
    ref = orc.keystage(sc, cam, "ellipse")
    np.testing.assert_array_equal(got["cull"].numpy(), ref["cull"])
    assert (ref["cull"] == 3).sum() > 10
    np.testing.assert_array_equal(got["id"].numpy(), ref["id"])
    r = orc.render(sc, cam, 8, orc.TOPK)
    absf = orc.render(sc, cam, 8, orc.TOPK, feat=np.abs(sc.feat.astype(np.float64)))["feat"]
    ok = decided(r)
    worst = image_errors(np_out(out), r, absf, ok, 1e-5)
    assert max(worst.values()) <= 1.0, worst
