"""Two feature sources in one render (psm_surfels.feat_ext): the blend gathers
channels [0, c) from the features in their storage dtype and channels
[c, c + c_ext) from an FP32 array, as the panoptic render of eq. (8) does
with semantic features and instance labels.

Every kernel sees the same feature values in the same order as with the two
arrays concatenated into one FP32 array (bf16/fp16 values widen to FP32
exactly), so the images, the selection and the gradients are bit-identical
to the concatenated render, whose own parity with the oracle is tested
elsewhere; the gradient comes back split into the two sources.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, OUTPUTS, require_gpu, to_dev
from paper_2604_10982_amd import psm, scenes

pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "bf16": torch.bfloat16}


def _inputs(dtype, c_ext, seed=3):
    sc = scenes.planes7(20_000, 16, seed=seed)
    t = to_dev(sc, dtype)
    rng = np.random.default_rng(seed + 1)
    ext = torch.tensor(rng.standard_normal((sc.n, c_ext)).astype(np.float32), device=DEV)
    cat = torch.cat([t["feat"].float(), ext], 1).contiguous()
    return sc, t, ext, cat


@pytest.mark.parametrize("blend", ["topk", "full"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_two_sources_equal_the_concatenated_render(blend, dtype):
    require_gpu()
    sc, t, ext, cat = _inputs(dtype, 24)
    cam = scenes.pinhole(328, 200)
    K = 8
    base = (t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"])
    print(f"[feat_ext] {blend} {dtype}", flush=True)
    out2, ws2 = psm.forward(*base, t["feat"], cam, K, "ellipse", blend, feat_ext=ext)
    out1, ws1 = psm.forward(*base, cat, cam, K, "ellipse", blend)
    torch.cuda.synchronize()
    for k in OUTPUTS:
        assert torch.equal(out2[k], out1[k]), k
    assert out2["feat"].shape[-1] == 16 + 24
    if blend == "topk":
        cs = psm.camera_struct(cam)
        s1 = psm.read_selection(ws1, cs, psm.config_struct(K, "ellipse", blend))
        s2 = psm.read_selection(ws2, cs, psm.config_struct(K, "ellipse", blend))
        for k in ("sel_id", "sel_w", "n_last", "T_final"):
            assert torch.equal(s1[k], s2[k]), k
    g = scenes.upstream(cam.height, cam.width, 16 + 24, seed=2)
    gout = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    g2 = psm.backward(*base, t["feat"], cam, ws2, gout, K, "ellipse", blend, feat_ext=ext)
    g1 = psm.backward(*base, cat, cam, ws1, gout, K, "ellipse", blend)
    torch.cuda.synchronize()
    for k in ("means", "scales", "quats", "opacity", "rgb"):
        assert torch.equal(g2[k], g1[k]), k
    assert torch.equal(g2["feat"], g1["feat"][:, :16])
    assert torch.equal(g2["feat_ext"], g1["feat"][:, 16:])


def test_only_the_second_source():
    """c = 0: every channel from the FP32 array."""
    require_gpu()
    sc, t, ext, _ = _inputs("f32", 16, seed=5)
    cam = scenes.pinhole(200, 136)
    base = (t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"])
    out2, ws2 = psm.forward(*base, None, cam, 8, "ellipse", "topk", feat_ext=ext)
    out1, ws1 = psm.forward(*base, ext, cam, 8, "ellipse", "topk")
    torch.cuda.synchronize()
    for k in OUTPUTS:
        assert torch.equal(out2[k], out1[k]), k
    g = scenes.upstream(cam.height, cam.width, 16, seed=4)
    gout = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
    g2 = psm.backward(*base, None, cam, ws2, gout, 8, "ellipse", "topk", feat_ext=ext)
    g1 = psm.backward(*base, ext, cam, ws1, gout, 8, "ellipse", "topk")
    torch.cuda.synchronize()
    assert g2["feat"] is None
    assert torch.equal(g2["feat_ext"], g1["feat"])
    assert torch.equal(g2["means"], g1["means"])


def test_batch_with_two_sources():
    require_gpu()
    sc = scenes.street40(40_000, 16, 3)
    cams = scenes.street_cameras(((200, 150), (96, 64), (333, 211)))
    t = to_dev(sc, "f16")
    rng = np.random.default_rng(8)
    ext = torch.tensor(rng.standard_normal((sc.n, 8)).astype(np.float32), device=DEV)
    cat = torch.cat([t["feat"].float(), ext], 1).contiguous()
    base = (t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"])
    cfg = psm.config_struct(8, "ellipse", "topk")
    out2, ws2, carr = psm.forward_batch(*base, t["feat"], cams, 8, cfg=cfg, feat_ext=ext)
    out1, ws1, _ = psm.forward_batch(*base, cat, cams, 8, cfg=psm.config_struct(8, "ellipse", "topk"))
    torch.cuda.synchronize()
    for k in OUTPUTS:
        assert torch.equal(out2[k], out1[k]), k
    gout = {"feat": torch.tensor(rng.standard_normal(tuple(out1["feat"].shape)).astype(np.float32), device=DEV)}
    g2 = psm.backward_batch(*base, t["feat"], carr, ws2, gout, cfg, feat_ext=ext)
    g1 = psm.backward_batch(*base, cat, carr, ws1, gout, psm.config_struct(8, "ellipse", "topk"))
    torch.cuda.synchronize()
    assert torch.equal(g2["feat"], g1["feat"][:, :16])
    assert torch.equal(g2["feat_ext"], g1["feat"][:, 16:])


def test_second_source_validation():
    require_gpu()
    sc, t, ext, _ = _inputs("f32", 16, seed=6)
    cam = scenes.pinhole(96, 64)
    base = (t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"])
    with pytest.raises(psm.PsmError) as e:  # c_ext not a multiple of 8
        psm.forward(*base, t["feat"], cam, 8, feat_ext=ext[:, :12].contiguous())
    assert e.value.status == psm.ERR_UNSUPPORTED
    s = psm._surfels(*base, t["feat"], ext)
    s.feat_ext = None  # c_ext > 0 with no array
    cs = psm.camera_struct(cam)
    cfg = psm.config_struct(8)
    ws = psm.alloc_workspace(s.n, cs, cfg, s.width, 200_000, DEV)
    out = psm.alloc_images(cs, s.width, DEV)
    with pytest.raises(psm.PsmError) as e:
        psm.forward_into(psm.context(0), s, cs, cfg, ws, out)
    assert e.value.status == psm.ERR_INVALID_ARG
