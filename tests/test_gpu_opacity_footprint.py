"""Opacity-aware footprint (an exact work reduction of the key stage): the
GPU's (tile, surfel) list equals the oracle's bit for bit, and images, the
Top-K selection and every gradient equal the standard footprint's bit for
bit, with fewer pairs."""
import numpy as np
import pytest
import torch

from gpu_helpers import require_gpu, to_dev
from paper_2604_10982_amd import psm, scenes
from paper_2604_10982_amd.scenes import Scene
from test_oracle_footprint import faint_scene

pytestmark = pytest.mark.gpu

OPA = psm.FLAG_OPACITY_FOOTPRINT


def _faint(sc, seed):
    rng = np.random.default_rng(seed)
    op = np.clip(rng.beta(0.6, 3.0, sc.n), 0.002, 0.99).astype(np.float32)
    return Scene(sc.means, sc.scales, sc.quats, op, sc.rgb, sc.feat)


def _cases():
    return {
        "faint300": lambda: (faint_scene(), scenes.pinhole(96, 80, f=80.0)),
        "planes40k_faint_ragged": lambda: (_faint(scenes.planes7(40_000, 8, seed=3), 1), scenes.pinhole(641, 359)),
        "street60k_faint": lambda: (_faint(scenes.street40(60_000, 8, seed=4), 2), scenes.pinhole(800, 450)),
    }


def _fwd(t, cam, K, mode, flags):
    out, ws = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K, mode,
                          "topk", flags=flags)
    torch.cuda.synchronize()
    return out, ws


@pytest.mark.parametrize("mode", ["aabb", "ellipse"])
@pytest.mark.parametrize("case", list(_cases()))
def test_opacity_footprint_lists_bit_exact(orc, case, mode):
    require_gpu()
    sc, cam = _cases()[case]()
    t = to_dev(sc)
    _, ws = _fwd(t, cam, 8, mode, OPA)
    got = psm.read_pairs(ws, psm.camera_struct(cam), psm.config_struct(8, mode, "topk", OPA))
    ref = orc.keystage(sc, cam, mode, opacity_footprint=True)
    np.testing.assert_array_equal(got["cull"].numpy(), ref["cull"])
    np.testing.assert_array_equal(got["count"].numpy(), ref["count"])
    assert got["P"] == ref["P"]
    np.testing.assert_array_equal(got["tile"].numpy(), ref["tile"])
    np.testing.assert_array_equal(got["id"].numpy(), ref["id"])
    assert ref["P"] < orc.keystage(sc, cam, mode, pairs=False)["P"]


@pytest.mark.parametrize("case", list(_cases()))
def test_opacity_footprint_changes_no_output_bit(case):
    require_gpu()
    sc, cam = _cases()[case]()
    t = to_dev(sc)
    K = 8
    outs, grads = [], []
    rng = np.random.default_rng(5)
    H, W = cam.height, cam.width
    gout = {"rgb": torch.tensor(rng.standard_normal((H, W, 3)), dtype=torch.float32, device="cuda"),
            "depth": torch.tensor(rng.standard_normal((H, W)), dtype=torch.float32, device="cuda"),
            "normal": torch.tensor(rng.standard_normal((H, W, 3)), dtype=torch.float32, device="cuda"),
            "alpha": torch.tensor(rng.standard_normal((H, W)), dtype=torch.float32, device="cuda"),
            "feat": torch.tensor(rng.standard_normal((H, W, sc.c)), dtype=torch.float32, device="cuda")}
    pairs = []
    for flags in (0, OPA):
        out, ws = _fwd(t, cam, K, "ellipse", flags)
        g = psm.backward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, ws, gout, K,
                         "ellipse", "topk", flags=flags)
        torch.cuda.synchronize()
        sel = psm.read_selection(ws, psm.camera_struct(cam), psm.config_struct(K, "ellipse", "topk", flags))
        outs.append(({k: v.clone() for k, v in out.items() if v is not None}, sel))
        grads.append({k: v.clone() for k, v in g.items() if v is not None})
        pairs.append(psm.read_stats(ws, sc.n, psm.camera_struct(cam), psm.config_struct(K, "ellipse", "topk", flags),
                                    sc.c, ws.capacity).pairs)
    assert pairs[1] < pairs[0]
    for k in outs[0][0]:
        assert torch.equal(outs[0][0][k], outs[1][0][k]), k
    # selected surfel ids, weights and final transmittance (n_last is a list
    # position, which the shorter lists renumber)
    for k in ("sel_id", "sel_w", "T_final"):
        assert torch.equal(outs[0][1][k], outs[1][1][k]), k
    for k in grads[0]:
        assert torch.equal(grads[0][k], grads[1][k]), k
