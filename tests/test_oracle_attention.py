"""Pins of the oracle's frustum-local cross-attention (Sec. 4.1, eqs. (9)-(11)).

The active set is pinned by hand-placed surfels and by sampling points of
each surfel's 99% disk (any sample inside the frustum forces the surfel
active); the attention by torch's own float64 scaled-dot-product attention
on a separate transcription, and by special cases (one active surfel, equal
scores, permutation of the surfels, no active surfel)."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import attention as AT
from paper_2604_10982_amd.scenes import pinhole


def _cam():
    return pinhole(64, 48, f=50.0, near=0.2)


def _problem(n=400, C=16, d=16, nq=12, seed=0):
    rng = np.random.default_rng(seed)
    means = np.c_[rng.uniform(-4, 4, n), rng.uniform(-3, 3, n), rng.uniform(-2, 9, n)].astype(np.float32)
    scales = np.exp(rng.normal(np.log(0.1), 0.6, (n, 2))).astype(np.float32)
    feat = rng.standard_normal((n, C)).astype(np.float32)
    q = rng.standard_normal((nq, C))
    wq, wk, wv = (rng.standard_normal((C, d)) / np.sqrt(C) for _ in range(3))
    return means, scales, feat, q, wq, wk, wv


def test_frustum_by_hand():
    cam = _cam()   # fx = fy = 50, cx = 32, cy = 24: half-angles atan(32/50), atan(24/50)
    s = 0.1
    r = float(AT.R99_F32) * s
    z = 5.0
    xedge = 32.0 / 50.0 * z        # the left/right planes meet z = 5 at x = -+3.2
    cases = [([0.0, 0.0, z], True), ([0.0, 0.0, -1.0], False), ([0.0, 0.0, 0.2 - 0.5 * r], True),
             ([0.0, 0.0, 0.2 - 2.0 * r], False)]
    # just outside the left plane: inside iff the plane distance is at most r
    nl = math.hypot(50.0, 32.0)
    for dist, want in ((0.9 * r, True), (1.1 * r, False)):
        # point at signed distance -dist from the left plane, at depth z
        x = (-32.0 * z - dist * nl) / 50.0
        cases.append(([x, 0.0, z], want))
    for dist, want in ((0.9 * r, True), (1.1 * r, False)):
        nb = math.hypot(50.0, 48.0 - 24.0)
        y = ((48.0 - 24.0) * z + dist * nb) / 50.0   # below the bottom plane
        cases.append(([0.0, y, z], want))
    means = np.array([c[0] for c in cases], np.float32)
    scales = np.full((len(cases), 2), s, np.float32)
    got = AT.frustum_active(means, scales, cam)
    assert got.tolist() == [c[1] for c in cases]
    assert xedge > 0


def test_frustum_has_no_false_negatives_by_sampling():
    cam = _cam()
    rng = np.random.default_rng(3)
    n = 3000
    means = np.c_[rng.uniform(-6, 6, n), rng.uniform(-5, 5, n), rng.uniform(-1, 8, n)].astype(np.float32)
    scales = np.exp(rng.normal(np.log(0.3), 0.5, (n, 2))).astype(np.float32)
    quats = rng.standard_normal((n, 4))
    act = AT.frustum_active(means, scales, cam)
    Rq = Rotation.from_quat(quats[:, [1, 2, 3, 0]]).as_matrix()
    ang = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    rad = np.linspace(0, 1, 6)
    uv = np.array([(r * np.cos(a), r * np.sin(a)) for r in rad for a in ang])
    r99 = math.sqrt(AT.R99_SQ)
    inside_any = np.zeros(n, bool)
    for j in range(n):
        pts = means[j] + r99 * (uv[:, :1] * scales[j, 0] * Rq[j][:, 0] + uv[:, 1:] * scales[j, 1] * Rq[j][:, 1])
        z = pts[:, 2]
        ok = z > cam.near
        x = cam.fx * pts[:, 0] / np.where(ok, z, 1) + cam.cx
        y = cam.fy * pts[:, 1] / np.where(ok, z, 1) + cam.cy
        inside_any[j] = np.any(ok & (x >= 0) & (x <= cam.width) & (y >= 0) & (y <= cam.height))
    assert inside_any.sum() > 200
    assert not np.any(inside_any & ~act)
    assert (~act).sum() > 500


def test_posenc_values():
    mu = np.array([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5]])
    psi = AT.posenc(mu, 13, 4.0)
    assert np.allclose(psi[0], [0, 0, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1, 0])
    # channel 7: axis 1, band 1, sin -> sin(2 pi * (-2) / 4) = sin(-pi) = 0 ; channel 9: axis 0, band 1, cos
    assert abs(psi[1, 7] - math.sin(2 * math.pi * -2.0 / 4.0)) < 1e-15
    assert abs(psi[1, 9] - math.cos(2 * math.pi * 1.0 / 4.0)) < 1e-15
    assert abs(psi[1, 2] - math.sin(math.pi * 0.5 / 4.0)) < 1e-15


def test_attention_matches_torch_sdpa():
    means, scales, feat, q, wq, wk, wv = _problem()
    cam = _cam()
    L = 8.0
    o = AT.attention(means, scales, feat, cam, q, wq, wk, wv, L)
    idx = o["idx"]
    assert 20 < idx.size < len(means)
    T = lambda a: torch.tensor(np.asarray(a, np.float64))
    mu = T(means[idx])
    c = torch.arange(feat.shape[1])
    arg = torch.pow(2.0, (c // 6).double()) * math.pi * mu[:, c % 3] / L
    psi = torch.where((c // 3) % 2 == 0, torch.sin(arg), torch.cos(arg))
    K = (T(feat[idx]) + psi) @ T(wk)
    V = T(feat[idx]) @ T(wv)
    Q = T(q) @ T(wq)
    ref = torch.nn.functional.scaled_dot_product_attention(Q[None], K[None], V[None])[0]
    np.testing.assert_allclose(o["out"], ref.numpy(), rtol=1e-12, atol=1e-13)


def test_special_cases():
    means, scales, feat, q, wq, wk, wv = _problem(n=50, seed=2)
    cam = _cam()
    act = AT.frustum_active(means, scales, cam)
    j = int(np.nonzero(act)[0][0])
    # one active surfel: every query gets its projected value row
    one = AT.attention(means[j:j + 1], scales[j:j + 1], feat[j:j + 1], cam, q, wq, wk, wv, 8.0)
    np.testing.assert_allclose(one["out"], np.repeat(feat[j:j + 1].astype(np.float64) @ wv, len(q), 0), rtol=1e-13)
    # equal keys (W_K = 0): uniform attention, the mean of the value rows
    o = AT.attention(means, scales, feat, cam, q, wq, np.zeros_like(wk), wv, 8.0)
    np.testing.assert_allclose(o["out"], np.repeat((feat[act].astype(np.float64) @ wv).mean(0, keepdims=True),
                                                   len(q), 0), rtol=1e-12)
    # permuting the surfels changes nothing but rounding
    p = np.random.default_rng(5).permutation(len(means))
    a = AT.attention(means, scales, feat, cam, q, wq, wk, wv, 8.0)["out"]
    b = AT.attention(means[p], scales[p], feat[p], cam, q, wq, wk, wv, 8.0)["out"]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    # no active surfel: zero
    far = means.copy()
    far[:, 2] = -10.0
    np.testing.assert_array_equal(AT.attention(far, scales, feat, cam, q, wq, wk, wv, 8.0)["out"], 0.0)
