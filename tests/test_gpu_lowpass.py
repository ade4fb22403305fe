"""Screen-space low-pass filter (PSM_FLAG_LOWPASS, the 2DGS variant of the
surfel kernel): the GPU's (tile, surfel) lists equal the oracle's bit for bit
in every footprint mode (alone and with the opacity-aware footprint); images
within 1e-5 of sum_j w_j |x_j| per channel and the Top-K selection equal to
the FP64 oracle's; gradients within |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2
rms(group)).  Scenes mix sub-pixel surfels (the filter term decides) with
wide ones (the ray-splat term decides)."""
import numpy as np
import pytest
import torch

from gpu_helpers import decided, DEV, image_errors, np_out, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from test_gpu_backward import grad_errors

pytestmark = pytest.mark.gpu

LP = psm.FLAG_LOWPASS


def _cases():
    return {
        "tiny400": lambda: (scenes.uniform_box(400, 8, seed=9, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.004),
                                               scale_sigma=0.3), scenes.pinhole(64, 48, f=48.0), 8),
        "mixed3k_ragged": lambda: (scenes.uniform_box(3000, 16, seed=12, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.01),
                                                      scale_sigma=0.9), scenes.pinhole(133, 97, f=96.0), 8),
        "street60k": lambda: (scenes.street40(60_000, 8, seed=4, scale_mu=np.log(0.01)), scenes.pinhole(800, 450),
                              16),
    }


def _fwd(t, cam, K, mode, blend, flags):
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K, mode,
                          blend, flags=flags)
    torch.cuda.synchronize()
    return out, ws


@pytest.mark.parametrize("mode", ["sphere", "aabb", "ellipse"])
@pytest.mark.parametrize("case", list(_cases()))
def test_lowpass_lists_bit_exact(orc, case, mode):
    require_gpu()
    sc, cam, K = _cases()[case]()
    t = to_dev(sc)
    flag_sets = [(LP, False)] + ([(LP | psm.FLAG_OPACITY_FOOTPRINT, True)] if mode == "ellipse" else [])
    for flags, opa in flag_sets:
        _, ws = _fwd(t, cam, K, mode, "topk", flags)
        got = psm.read_pairs(ws, psm.camera_struct(cam), psm.config_struct(K, mode, "topk", flags))
        ref = orc.keystage(sc, cam, mode, opacity_footprint=opa, lowpass=True)
        np.testing.assert_array_equal(got["cull"].numpy(), ref["cull"])
        np.testing.assert_array_equal(got["count"].numpy(), ref["count"])
        assert got["P"] == ref["P"]
        np.testing.assert_array_equal(got["tile"].numpy(), ref["tile"])
        np.testing.assert_array_equal(got["id"].numpy(), ref["id"])
    assert ref["P"] >= orc.keystage(sc, cam, mode, pairs=False, opacity_footprint=opa)["P"]


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("case", list(_cases()))
def test_lowpass_images_match_oracle(orc, case, blend):
    require_gpu()
    sc, cam, K = _cases()[case]()
    t = to_dev(sc)
    out, ws = _fwd(t, cam, K, "ellipse", blend, LP)
    b = orc.TOPK if blend == "topk" else orc.FULL
    feat = stored_feat(t)
    ref = orc.render(sc, cam, K, b, feat=feat, lowpass=True)
    absf = orc.render(sc, cam, K, b, feat=np.abs(feat), lowpass=True)["feat"]
    ok = decided(ref)
    assert (~ok).mean() < 1e-3, f"{(~ok).sum()} pixels within the decision margin"
    worst = image_errors(np_out(out), ref, absf, ok, 1e-5)
    assert max(worst.values()) <= 1.0, worst
    # the filter changes the images of these scenes
    plain = orc.render(sc, cam, K, b, feat=feat)
    assert np.abs(plain["alpha"] - ref["alpha"]).max() > 0.05
    if blend == "topk":
        sel = psm.read_selection(ws, psm.camera_struct(cam), psm.config_struct(K, "ellipse", "topk", LP))
        np.testing.assert_array_equal(sel["sel_id"].cpu().numpy()[ok], ref["sel_id"][ok])


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("case", list(_cases()))
def test_lowpass_gradients_match_oracle(orc, case, blend):
    require_gpu()
    sc, cam, K = _cases()[case]()
    t = to_dev(sc)
    _, ws = _fwd(t, cam, K, "ellipse", blend, LP)
    b = orc.TOPK if blend == "topk" else orc.FULL
    feat = stored_feat(t)
    ok = decided(orc.render(sc, cam, K, b, feat=feat, lowpass=True))
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
    for k in g:
        g[k][~ok] = 0.0
    ref = orc.backward(sc, cam, g, K=K, blend=b, feat=feat, lowpass=True)
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    got = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                       "ellipse", blend, flags=LP)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got, ref)
    assert max(worst.values()) <= 1e-3, worst


def test_lowpass_batch_equals_single_renders():
    require_gpu()
    sc = scenes.street40(40_000, 16, seed=3, scale_mu=np.log(0.01))
    cams = scenes.street_cameras(((200, 150), (96, 64), (333, 211)))
    t = to_dev(sc, "f16")
    K = 8
    cfg = psm.config_struct(K, "ellipse", "topk", LP)
    out, ws, carr = psm.forward_batch(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cams,
                                      K, cfg=cfg)
    torch.cuda.synchronize()
    per = psm.split_images(out, carr)
    sel = psm.read_selection_batch(ws, carr, cfg)
    p0 = 0
    for b, cam in enumerate(cams):
        single, ws1 = _fwd(t, cam, K, "ellipse", "topk", LP)
        for k in ("rgb", "depth", "normal", "alpha", "feat"):
            assert torch.equal(per[b][k], single[k]), (b, k)
        s1 = psm.read_selection(ws1, psm.camera_struct(cam), cfg)
        hw = cam.height * cam.width
        assert torch.equal(sel["sel_id"][p0:p0 + hw].reshape(cam.height, cam.width, K), s1["sel_id"])
        p0 += hw


def test_lowpass_with_feature_variants(orc):
    """The filter composes with the feature-only stop (selection and features
    bit-identical to the filtered full walk) and with the renormalised Top-K
    (features vs the oracle)."""
    require_gpu()
    sc, cam, K = _cases()["mixed3k_ragged"]()
    t = to_dev(sc)
    out0, ws0 = _fwd(t, cam, K, "ellipse", "topk", LP)
    out1, ws1 = _fwd(t, cam, K, "ellipse", "topk", LP | psm.FLAG_FEATURE_ONLY)
    assert torch.equal(out0["feat"], out1["feat"])
    c0 = psm.config_struct(K, "ellipse", "topk", LP)
    s0 = psm.read_selection(ws0, psm.camera_struct(cam), c0)
    s1 = psm.read_selection(ws1, psm.camera_struct(cam), psm.config_struct(K, "ellipse", "topk",
                                                                          LP | psm.FLAG_FEATURE_ONLY))
    assert torch.equal(s0["sel_id"], s1["sel_id"]) and torch.equal(s0["sel_w"], s1["sel_w"])
    out2, _ = _fwd(t, cam, K, "ellipse", "topk", LP | psm.FLAG_TOPK_RENORM)
    feat = stored_feat(t)
    ref = orc.render(sc, cam, K, orc.TOPK_RENORM, feat=feat, lowpass=True)
    absf = orc.render(sc, cam, K, orc.TOPK_RENORM, feat=np.abs(feat), lowpass=True)["feat"]
    ok = decided(ref)
    worst = image_errors(np_out(out2), ref, absf, ok, 1e-5)
    assert max(worst.values()) <= 1.0, worst


def test_autograd_render_takes_the_flags():
    """render() (torch autograd over the C ABI) passes its flags to both
    directions: outputs and gradients equal the direct calls bit for bit."""
    require_gpu()
    from paper_2604_10982_amd import render as R
    sc, cam, K = _cases()["mixed3k_ragged"]()
    t = to_dev(sc)
    flags = LP | psm.FLAG_TOPK_RENORM
    params = {k: t[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "rgb", "feat")}
    maps = R.render(*(params[k] for k in ("means", "scales", "quats", "opacity", "rgb", "feat")), cam, K,
                    "ellipse", "topk", flags)
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=3)
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    names = ("rgb", "depth", "normal", "alpha", "feat")
    loss = sum((m * gt[k]).sum() for m, k in zip(maps, names))
    loss.backward()
    out, ws = _fwd(t, cam, K, "ellipse", "topk", flags)
    for m, k in zip(maps, names):
        assert torch.equal(m.detach(), out[k]), k
    ref = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                       "ellipse", "topk", flags=flags)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(params[k].grad, ref[k].to(params[k].grad.dtype)), k
    with pytest.raises(ValueError):
        R.render(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K, "ellipse", "topk",
                 psm.FLAG_FEATURE_ONLY)
