"""SOGMM geometric loss (eq. (3), eq. (13), L_iso) on the GPU against the
FP64 oracle: the MAP component of every surfel bit for bit where the oracle's
two best FP32 scores differ by more than 1e-5 (relative; both sides evaluate
the same FP32 operations, only the FP32 records may differ in the last bit),
the loss totals and per-surfel gradients within FP32 rounding, run-to-run
bit-identical."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, require_gpu
from oracle import geometry as GE
from paper_2604_10982_amd import psm, scenes

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.ascontiguousarray(a, np.float32), device=DEV)


def _run(sc, gm, lam):
    out = psm.geometry_loss(T(sc.means), T(sc.scales), T(sc.quats), T(gm[0]), T(gm[1]), T(gm[2]), lam,
                            return_assign=True)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in out.items()}


def _clear(x, comp, idx=None):
    s = GE.scores_f32(x if idx is None else x[idx], comp).astype(np.float64)
    srt = np.sort(s, 1)
    return (srt[:, 1] - srt[:, 0]) > 1e-5 * np.maximum(1.0, np.abs(srt[:, 0]))


CASES = {
    "planes20k_K64": lambda: (scenes.planes7(20_000, 4, seed=5), 64),
    "street60k_K300": lambda: (scenes.street40(60_000, 4, seed=4), 300),
    "box5k_K1500": lambda: (scenes.uniform_box(5000, 4, seed=2, xy=3.0, z=(1.0, 8.0)), 1500),  # > one LDS chunk
}


@pytest.mark.parametrize("case", list(CASES))
def test_geometry_loss_matches_oracle(case):
    require_gpu()
    sc, K = CASES[case]()
    gm = scenes.plane_gmm(sc, K, 1)
    lam = 0.4
    got = _run(sc, gm, lam)
    comp = GE.prepare(*gm)
    ref = GE.loss(sc.means, sc.scales, sc.quats, comp, lam)
    clear = _clear(sc.means, comp)
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(got["assign"][clear], ref["assign"][clear])
    # totals: terms of order 1, summed in FP64 over FP32 terms
    tot_geo = np.abs(ref["geo_i"]).sum()
    assert abs(float(got["geo"]) - ref["geo"]) <= 1e-5 * tot_geo + 1e-3 * (~clear).sum()
    assert abs(float(got["iso"]) - ref["iso"]) <= 1e-5 * ref["iso"] + 1e-12
    c = clear & (np.abs(ref["delta"]) > 1e-5) & (np.abs(ref["dot"]) > 1e-5)
    np.testing.assert_allclose(got["d_means"][c], ref["d_means"][c], atol=2e-6)
    np.testing.assert_allclose(got["d_scales"], ref["d_scales"], rtol=1e-5, atol=1e-7)
    scale = np.abs(ref["d_quats"][c]).max(1, keepdims=True) + 1e-6
    assert float((np.abs(got["d_quats"][c] - ref["d_quats"][c]) / scale).max()) <= 1e-4


def test_geometry_loss_deterministic_and_edges():
    require_gpu()
    sc, K = CASES["street60k_K300"]()
    gm = scenes.plane_gmm(sc, K, 2)
    a, b = _run(sc, gm, 0.4), _run(sc, gm, 0.4)
    for k in ("d_means", "d_quats", "d_scales", "assign"):
        np.testing.assert_array_equal(a[k], b[k])
    assert float(a["geo"]) == float(b["geo"]) and float(a["iso"]) == float(b["iso"])
    # one component: every surfel takes it
    one = _run(sc, (gm[0][:1], gm[1][:1], gm[2][:1] * 0 + 1), 0.4)
    assert (one["assign"] == 0).all()
    # no surfels: zero losses
    out = psm.geometry_loss(torch.zeros(0, 3, device=DEV), torch.zeros(0, 2, device=DEV), torch.zeros(0, 4, device=DEV),
                            T(gm[0]), T(gm[1]), T(gm[2]), 0.4)
    torch.cuda.synchronize()
    assert float(out["geo"]) == 0.0 and float(out["iso"]) == 0.0


def test_geometry_loss_full_size_planes1m():
    """The benchmark's shape: the 1M-surfel plane scene and 512 plane
    components.  The oracle assigns every surfel itself (its two best FP32
    scores kept, to tell clear surfels from near ties); L_geo and L_iso are
    compared in total, d_means, d_quats and d_scales per clear surfel."""
    require_gpu()
    sc, _, _, _ = scenes.config("planes1m_1080p")
    gm = scenes.plane_gmm(sc, 512, 3)
    got = _run(sc, gm, 0.4)
    comp = GE.prepare(*gm)
    n = sc.n
    k1, k2 = np.empty(n, np.int64), np.empty(n, np.int64)
    clear = np.empty(n, bool)
    for a in range(0, n, 8192):
        s = GE.scores_f32(sc.means[a:a + 8192], comp).astype(np.float64)
        two = np.argpartition(s, 1, axis=1)[:, :2]
        sv = np.take_along_axis(s, two, 1)
        order = np.argsort(sv, 1, kind="stable")
        two, sv = np.take_along_axis(two, order, 1), np.take_along_axis(sv, order, 1)
        # ties in score go to the lower index, as the MAP rule states
        tie = sv[:, 0] == sv[:, 1]
        two[tie] = np.sort(two[tie], 1)
        k1[a:a + 8192], k2[a:a + 8192] = two[:, 0], two[:, 1]
        clear[a:a + 8192] = (sv[:, 1] - sv[:, 0]) > 1e-5 * np.maximum(1.0, np.abs(sv[:, 0]))
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(got["assign"][clear], k1[clear])
    lam = 0.4
    ref = GE.loss(sc.means, sc.scales, sc.quats, comp, lam, k=k1)
    alt = GE.loss(sc.means[~clear], sc.scales[~clear], sc.quats[~clear], comp, lam, k=k2[~clear])
    # a near tie may go either way: its term may be either component's
    slack = np.abs(ref["geo_i"][~clear] - alt["geo_i"]).sum()
    tot_geo = np.abs(ref["geo_i"]).sum()
    assert abs(float(got["geo"]) - ref["geo"]) <= 1e-5 * tot_geo + slack
    assert abs(float(got["iso"]) - ref["iso"]) <= 1e-5 * ref["iso"]
    c = clear & (np.abs(ref["delta"]) > 1e-5) & (np.abs(ref["dot"]) > 1e-5)
    assert c.mean() > 0.98
    np.testing.assert_allclose(got["d_means"][c], ref["d_means"][c], atol=2e-6)
    np.testing.assert_allclose(got["d_scales"], ref["d_scales"], rtol=1e-5, atol=1e-7)
    scale = np.abs(ref["d_quats"][c]).max(1, keepdims=True) + 1e-6
    assert float((np.abs(got["d_quats"][c] - ref["d_quats"][c]) / scale).max()) <= 1e-4
