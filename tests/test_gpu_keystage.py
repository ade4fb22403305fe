"""Key stage on the GPU is bit-exact to the oracle's FP32 key stage: cull
codes, depth-key bits, per-surfel pair counts, and the (tile, surfel) list in
(tile, depth, id) order, for all three footprint modes (Sec. 5)."""
import numpy as np
import pytest

from gpu_helpers import render, require_gpu, to_dev
from paper_2604_10982_amd import psm, scenes
from test_oracle_footprint import varied_scene

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "c1_box2k": lambda: scenes.config("c1_box2k")[:2],
        "varied300": lambda: (varied_scene(), scenes.pinhole(96, 80, f=80.0)),
        "planes40k_ragged": lambda: (scenes.planes7(40_000, 8, seed=3), scenes.pinhole(641, 359)),
        "street60k": lambda: (scenes.street40(60_000, 8, seed=4), scenes.pinhole(800, 450)),
    }


@pytest.mark.parametrize("mode", ["sphere", "aabb", "ellipse"])
@pytest.mark.parametrize("case", list(_cases()))
def test_keystage_bit_exact(orc, case, mode):
    require_gpu()
    sc, cam = _cases()[case]()
    t = to_dev(sc)
    out, ws = render(t, cam, 8, mode, "topk")
    got = psm.read_pairs(ws, psm.camera_struct(cam), psm.config_struct(8, mode, "topk"))
    ref = orc.keystage(sc, cam, mode)
    np.testing.assert_array_equal(got["cull"].numpy(), ref["cull"])
    vis = ref["cull"] == 0
    np.testing.assert_array_equal(got["depth_bits"].numpy().view(np.uint32)[vis], ref["depth_bits"][vis])
    np.testing.assert_array_equal(got["count"].numpy(), ref["count"])
    assert got["P"] == ref["P"]
    np.testing.assert_array_equal(got["tile"].numpy(), ref["tile"])
    np.testing.assert_array_equal(got["id"].numpy(), ref["id"])
    st = got["stats"]
    assert st.visible == int(vis.sum())
    assert [st.culled[i] for i in range(1, 5)] == [int((ref["cull"] == i).sum()) for i in range(1, 5)]
