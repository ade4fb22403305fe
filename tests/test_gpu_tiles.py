"""Tile shapes (a launch choice of the tile-based rasteriser, Sec. 5): tiles of
tw x (256 / tw) pixels, tw in {8, 16, 32, 64}, one 256-thread block per tile.

* The key stage's lists for each shape are bit-exact to the oracle's FP32 key
  stage with that shape, in all three footprint modes.
* A pixel's contributors and their depth order do not depend on the tile that
  holds it, so every image and the Top-K selection are bit-identical to the
  16 x 16 render.
* The backward groups its sums per (tile, surfel), so gradients differ from
  the 16 x 16 ones only by rounding: they are checked against the FP64 oracle.
* Several cameras in one call with a non-square shape equal the single renders.
* The autotuner times the shapes and the step it picks renders the same images.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, OUTPUTS, decided, render, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from test_gpu_backward import grad_errors
from test_oracle_footprint import varied_scene

pytestmark = pytest.mark.gpu

SHAPES = (8, 32, 64)


def _launch(tw, persistent=False):
    s = 1 if persistent else 0
    return (s, s, 0, 0, tw)


def _cases():
    return {
        "varied300": lambda: (varied_scene(), scenes.pinhole(96, 80, f=80.0), 8),
        "planes40k_ragged": lambda: (scenes.planes7(40_000, 16, seed=3), scenes.pinhole(641, 359), 16),
    }


@pytest.mark.parametrize("mode", ["sphere", "aabb", "ellipse"])
@pytest.mark.parametrize("tw", SHAPES)
@pytest.mark.parametrize("case", list(_cases()))
def test_lists_bit_exact_per_shape(orc, case, tw, mode):
    require_gpu()
    sc, cam, K = _cases()[case]()
    print(f"[tiles] lists {case} tw={tw} {mode}", flush=True)
    t = to_dev(sc)
    _, ws = render(t, cam, K, mode, "topk", launch=_launch(tw))
    got = psm.read_pairs(ws, psm.camera_struct(cam), psm.config_struct(K, mode, "topk", tile_w=tw))
    ref = orc.keystage(sc, cam, mode, tile=(tw, 256 // tw))
    np.testing.assert_array_equal(got["count"].numpy(), ref["count"])
    assert got["P"] == ref["P"]
    np.testing.assert_array_equal(got["tile"].numpy(), ref["tile"])
    np.testing.assert_array_equal(got["id"].numpy(), ref["id"])


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("case", list(_cases()))
def test_images_and_selection_independent_of_shape(case, blend):
    require_gpu()
    sc, cam, K = _cases()[case]()
    t = to_dev(sc)
    ref, ws0 = render(t, cam, K, "ellipse", blend)
    cfg0 = psm.config_struct(K, "ellipse", blend)
    sel0 = psm.read_selection(ws0, psm.camera_struct(cam), cfg0) if blend == "topk" else None
    for tw in SHAPES:
        for persistent in (False, True):
            print(f"[tiles] images {case} {blend} tw={tw} persistent={persistent}", flush=True)
            out, ws = render(t, cam, K, "ellipse", blend, launch=_launch(tw, persistent))
            for k in OUTPUTS:
                assert torch.equal(out[k], ref[k]), (tw, persistent, k)
            if sel0 is not None:
                cfg = psm.config_struct(K, "ellipse", blend, tile_w=tw)
                sel = psm.read_selection(ws, psm.camera_struct(cam), cfg)
                for k in ("sel_id", "sel_w", "T_final"):  # n_last is a position in the tile's list
                    assert torch.equal(sel[k], sel0[k]), (tw, k)


GRAD_CASES = {
    "box300": lambda: (scenes.uniform_box(300, 16, seed=4, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12)),
                       scenes.pinhole(64, 48, f=56.0), 4),
    "planes20k": lambda: (scenes.planes7(20_000, 16, seed=5), scenes.pinhole(328, 200), 8),
}


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("tw", SHAPES)
@pytest.mark.parametrize("case", list(GRAD_CASES))
def test_gradients_per_shape_match_oracle(orc, case, tw, blend):
    require_gpu()
    sc, cam, K = GRAD_CASES[case]()
    print(f"[tiles] gradients {case} tw={tw} {blend}", flush=True)
    t = to_dev(sc)
    launch = _launch(tw, persistent=True)
    _, ws = render(t, cam, K, "ellipse", blend, launch=launch)
    feat = stored_feat(t)
    b = orc.TOPK if blend == "topk" else orc.FULL
    ok = decided(orc.render(sc, cam, K, b, feat=feat))
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
    for k in g:
        g[k][~ok] = 0.0
    ref = orc.backward(sc, cam, g, K=K, blend=b, feat=feat)
    gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    got = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gt, K,
                       "ellipse", blend, launch=launch)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    worst = grad_errors(got, ref)
    assert max(worst.values()) <= 1e-3, worst


def test_batch_with_wide_tiles_equals_single_renders():
    require_gpu()
    sc = scenes.street40(60_000, 16, 3)
    cams = scenes.street_cameras(((200, 150), (96, 64), (333, 211)))
    t = to_dev(sc, "f16")
    K = 8
    args = (t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    for tw in (32, 8):
        cfg = psm.config_struct(K, "ellipse", "topk", tile_w=tw)
        out, ws, carr = psm.forward_batch(*args, cams, K, cfg=cfg)
        torch.cuda.synchronize()
        per = psm.split_images(out, carr)
        for b, cam in enumerate(cams):
            single, _ = render(t, cam, K, "ellipse", "topk")
            for k in OUTPUTS:
                assert torch.equal(per[b][k], single[k]), (tw, b, k)


def test_autotuner_picks_a_shape_with_the_same_images():
    require_gpu()
    sc, cam, K = _cases()["planes40k_ragged"]()
    t = to_dev(sc)
    ref, _ = render(t, cam, K, "ellipse", "topk")
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    cs = psm.camera_struct(cam)
    need = 0
    for tw in (8, 16, 32, 64):
        c0 = psm.config_struct(K, tile_w=tw)
        _, w0 = render(t, cam, K, "ellipse", "topk", launch=_launch(tw))
        need = max(need, int(psm.read_stats(w0, s.n, cs, c0, s.c, w0.capacity).pairs_required))
    cfg = psm.config_struct(K, "ellipse", "topk")
    ws = psm.alloc_workspace_shapes(s.n, [cs], cfg, s.c, need + 1024, DEV)
    out = psm.alloc_images(cs, s.c, DEV)
    ms = psm.autotune(psm.context(0), s, psm.camera_array([cs]), cfg, ws, out, cache=False)
    assert ms is not None and ms > 0
    assert cfg.tile_w in (8, 16, 32, 64)
    psm.forward_into(psm.context(0), s, cs, cfg, ws, out)
    torch.cuda.synchronize()
    for k in OUTPUTS:
        assert torch.equal(out[k], ref[k]), (cfg.tile_w, k)
