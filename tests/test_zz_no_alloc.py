"""The forward on the library's static device workspace (psm_forward_static,
for callers that cannot allocate device memory) against psm_forward on a
caller workspace: the same kernels on the same inputs, so every output bit
must agree.  Two calls in a row, the second on a smaller input, so the second
result would show any state the first left in the shared array."""
import numpy as np
import pytest
import torch

from gpu_helpers import BENCH_LAUNCH, DEV, GRID_LAUNCH, OUTPUTS, require_gpu, to_dev
from paper_2604_10982_amd import psm, scenes

pytestmark = pytest.mark.gpu


def _small_camera():
    # 100 x 72: ragged tiles in both directions
    return scenes.pinhole(100, 72, 90.0)


def _inputs(name, n=None, cam=None):
    sc, cam0, K, _ = scenes.config(name, n=n)
    return sc, (cam if cam is not None else cam0), K


def _bits(x):
    return x.contiguous().view(torch.int32).cpu().numpy()


def _static_vs_caller(sc, cam, K, launch, blend="topk"):
    t = to_dev(sc)
    ref, _ = psm.forward(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"], cam, K,
                         "ellipse", blend, launch=launch)
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    cs = psm.camera_struct(cam)
    cfg = psm.launch_config(K, "ellipse", blend, 0, launch)
    out = psm.alloc_images(cs, s.c, DEV)
    for v in out.values():
        v.fill_(float("nan"))  # a pixel the static forward did not write shows
    psm.forward_static_into(psm.context(0), s, cs, cfg, out)
    torch.cuda.synchronize()
    for k in OUTPUTS:
        assert np.array_equal(_bits(out[k]), _bits(ref[k])), k


@pytest.mark.parametrize("launch", [GRID_LAUNCH, BENCH_LAUNCH], ids=["grid", "bench"])
def test_static_forward_equals_caller_workspace_twice(launch):
    require_gpu()
    print(f"[no-alloc] c1_box2k 128x128 launch={launch}", flush=True)
    sc, cam, K = _inputs("c1_box2k")
    _static_vs_caller(sc, cam, K, launch)
    print(f"[no-alloc] c1_box2k n=700 100x72 launch={launch}", flush=True)
    sc2, cam2, K2 = _inputs("c1_box2k", n=700, cam=_small_camera())
    _static_vs_caller(sc2, cam2, K2, launch)


def test_static_forward_dense_blend():
    require_gpu()
    sc, cam, K = _inputs("c1_box2k", n=1200)
    _static_vs_caller(sc, cam, K, None, blend="full")


def test_static_forward_rejects_sizes_beyond_the_array():
    require_gpu()
    # 1080p, C = 128, K = 16: the per-pixel saved state alone exceeds 64 MiB
    sc, cam, K = _inputs("c1_box2k", n=64, cam=scenes.pinhole(1920, 1080, 1440.0))
    t = to_dev(sc)
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    cs = psm.camera_struct(cam)
    cfg = psm.launch_config(16, "ellipse", "topk", 0, None)
    out = psm.alloc_images(cs, s.c, DEV)
    with pytest.raises(psm.PsmError) as ei:
        psm.forward_static_into(psm.context(0), s, cs, cfg, out)
    assert ei.value.status == psm.ERR_INVALID_ARG and "static workspace" in str(ei.value)
    # an explicit capacity beyond the array is rejected the same way
    sc2, cam2, K2 = _inputs("c1_box2k")
    t2 = to_dev(sc2)
    s2 = psm._surfels(t2["means"], t2["scales"], t2["quats"], t2["opacity"], t2["rgb"], t2["feat"])
    cs2 = psm.camera_struct(cam2)
    cfg2 = psm.launch_config(K2, "ellipse", "topk", 0, None)
    out2 = psm.alloc_images(cs2, s2.c, DEV)
    with pytest.raises(psm.PsmError) as ei:
        psm.forward_static_into(psm.context(0), s2, cs2, cfg2, out2, pair_capacity=1 << 30)
    assert ei.value.status == psm.ERR_INVALID_ARG


def test_static_forward_reports_capacity():
    require_gpu()
    sc, cam, K = _inputs("c1_box2k")
    t = to_dev(sc)
    s = psm._surfels(t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"])
    cs = psm.camera_struct(cam)
    cfg = psm.launch_config(K, "ellipse", "topk", 0, None)
    out = psm.alloc_images(cs, s.c, DEV)
    with pytest.raises(psm.CapacityError):
        psm.forward_static_into(psm.context(0), s, cs, cfg, out, pair_capacity=16)
    # the next call with room for every pair is exact again
    _static_vs_caller(sc, cam, K, None)
