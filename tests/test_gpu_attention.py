"""Frustum-local cross-attention (Sec. 4.1, eqs. (9)-(11)) on the matrix
cores against the FP64 oracle: the active set bit for bit (an FP32 decision
taken in the same operation order on both sides), the attended queries
within 1e-4 of sum_j p_ij |(V W_V)_j| (FP32 products and sums over up to
millions of keys), run-to-run bit-identical, and the edge cases."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, TORCH_DTYPES, require_gpu
from oracle import attention as AT
from paper_2604_10982_amd import psm, scenes

pytestmark = pytest.mark.gpu


def _weights(C, d, nq, seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((nq, C)).astype(np.float32)
    wq, wk, wv = ((rng.standard_normal((C, d)) / np.sqrt(C)).astype(np.float32) for _ in range(3))
    return q, wq, wk, wv


def _feat(n, C, seed):
    return (np.random.default_rng(seed).standard_normal((n, C)) * 0.8).astype(np.float32)


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _run(sc, feat, cam, q, wq, wk, wv, L, dtype="f32"):
    tf = T(feat).to(TORCH_DTYPES[dtype]).contiguous()
    out, act = psm.frustum_attention(T(sc.means), T(sc.scales), tf, T(q), T(wq), T(wk), T(wv), cam, L,
                                     return_active=True)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), act.cpu().numpy().astype(bool), tf.float().cpu().numpy()


def _check(got, ref):
    scale = ref["P"] @ np.abs(ref["Vp"]) if ref["idx"].size else np.zeros_like(got)
    err = np.abs(got - ref["out"]) / (1e-4 * scale + 1e-7)
    assert float(err.max()) <= 1.0, float(err.max())


CASES = {
    "planes40k_ragged": lambda: (scenes.planes7(40_000, 8, seed=3), scenes.pinhole(641, 359)),
    "street60k": lambda: (scenes.street40(60_000, 8, seed=4), scenes.pinhole(800, 450)),
    "box5k": lambda: (scenes.uniform_box(5000, 8, seed=2, xy=3.0, z=(-1.0, 8.0)), scenes.pinhole(96, 80, f=80.0)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_active_set_bit_exact(case):
    require_gpu()
    sc, cam = CASES[case]()
    q, wq, wk, wv = _weights(32, 32, 8, 1)
    _, act, _ = _run(sc, _feat(sc.n, 32, 2), cam, q, wq, wk, wv, 16.0)
    ref = AT.frustum_active(sc.means, sc.scales, cam)
    np.testing.assert_array_equal(act, ref)
    assert 0 < ref.sum() < sc.n


@pytest.mark.parametrize("C,d", [(16, 16), (32, 32), (64, 32), (64, 64)])
@pytest.mark.parametrize("nq", [1, 17, 64, 256])
def test_attention_matches_oracle(C, d, nq):
    require_gpu()
    sc, cam = CASES["planes40k_ragged"]()
    feat = _feat(sc.n, C, 5)
    q, wq, wk, wv = _weights(C, d, nq, 6)
    got, _, _ = _run(sc, feat, cam, q, wq, wk, wv, 16.0)
    ref = AT.attention(sc.means, sc.scales, feat, cam, q, wq, wk, wv, 16.0)
    _check(got, ref)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_attention_half_features(dtype):
    require_gpu()
    sc, cam = CASES["street60k"]()
    feat = _feat(sc.n, 32, 7)
    q, wq, wk, wv = _weights(32, 32, 64, 8)
    got, _, stored = _run(sc, feat, cam, q, wq, wk, wv, 16.0, dtype)
    ref = AT.attention(sc.means, sc.scales, stored, cam, q, wq, wk, wv, 16.0)   # oracle on the stored values
    _check(got, ref)


def test_attention_deterministic():
    require_gpu()
    sc, cam = CASES["street60k"]()
    feat = _feat(sc.n, 32, 9)
    q, wq, wk, wv = _weights(32, 32, 64, 10)
    a = _run(sc, feat, cam, q, wq, wk, wv, 16.0)[0]
    b = _run(sc, feat, cam, q, wq, wk, wv, 16.0)[0]
    np.testing.assert_array_equal(a, b)


def test_attention_edge_cases():
    require_gpu()
    cam = scenes.pinhole(96, 80, f=80.0)
    q, wq, wk, wv = _weights(16, 16, 5, 11)
    sc = scenes.uniform_box(300, 8, seed=12, xy=1.0, z=(2.0, 5.0))
    feat = _feat(sc.n, 16, 13)
    # nothing in front of the camera: zero
    far = scenes.Scene(sc.means - np.array([0, 0, 20.0], np.float32), sc.scales, sc.quats, sc.opacity, sc.rgb,
                       sc.feat)
    got, act, _ = _run(far, feat, cam, q, wq, wk, wv, 4.0)
    assert not act.any()
    np.testing.assert_array_equal(got, 0.0)
    # one surfel: every query gets its projected value row
    one = scenes.Scene(sc.means[:1], sc.scales[:1], sc.quats[:1], sc.opacity[:1], sc.rgb[:1], sc.feat[:1])
    got, act, _ = _run(one, feat[:1], cam, q, wq, wk, wv, 4.0)
    assert act.all()
    np.testing.assert_allclose(got, np.repeat(feat[:1].astype(np.float64) @ wv, 5, 0), rtol=1e-5, atol=1e-6)
    # fewer active surfels than one staged step, and no surfels at all
    few = scenes.Scene(sc.means[:37], sc.scales[:37], sc.quats[:37], sc.opacity[:37], sc.rgb[:37], sc.feat[:37])
    got, _, _ = _run(few, feat[:37], cam, q, wq, wk, wv, 4.0)
    _check(got, AT.attention(few.means, few.scales, feat[:37], cam, q, wq, wk, wv, 4.0))
    out = psm.frustum_attention(torch.zeros(0, 3, device=DEV), torch.zeros(0, 2, device=DEV),
                                torch.zeros(0, 16, device=DEV), T(q), T(wq), T(wk), T(wv), cam, 4.0)
    torch.cuda.synchronize()
    assert (out == 0).all()


def test_attention_full_size_street2m():
    """The benchmark's shape: 2M surfels, a 1920x1080 camera, 64 queries,
    32-d features and projections."""
    require_gpu()
    sc = scenes.street40(2_000_000, 8, seed=1)
    cam = scenes.street_cameras()[-1]
    feat = _feat(sc.n, 32, 14)
    q, wq, wk, wv = _weights(32, 32, 64, 15)
    got, act, _ = _run(sc, feat, cam, q, wq, wk, wv, 16.0)
    np.testing.assert_array_equal(act, AT.frustum_active(sc.means, sc.scales, cam))
    _check(got, AT.attention(sc.means, sc.scales, feat, cam, q, wq, wk, wv, 16.0))
