"""Pins of the oracle's SOGMM geometric loss (eq. (3), eq. (13), L_iso).

Pinned by a hand-computed one-plane case, the reference normal of a flat
covariance built from a known rotation, the assignment against scipy's
Gaussian log-density (where the best two differ by a clear margin), and the
gradients by central differences and by torch float64 autograd of a separate
transcription (rotation matrix from the quaternion, then its third column)."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

from oracle import geometry as GE


def _components(K=24, seed=0):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-5, 5, (K, 3))
    R = Rotation.random(K, random_state=seed).as_matrix()
    sd = np.c_[rng.uniform(0.5, 2.0, K), rng.uniform(0.5, 2.0, K), rng.uniform(0.01, 0.05, K)]
    S = np.einsum("kij,kj,klj->kil", R, sd ** 2, R)
    cov6 = np.stack([S[:, i, j] for i, j in GE.SYM], 1)
    w = rng.dirichlet(np.ones(K))
    return mean, cov6, w, R


def _surfels(n=300, seed=1):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-6, 6, (n, 3)).astype(np.float32)
    scales = np.exp(rng.normal(np.log(0.1), 0.5, (n, 2))).astype(np.float32)
    quats = rng.standard_normal((n, 4)).astype(np.float32)
    return means, scales, quats


def test_one_plane_by_hand():
    comp = GE.prepare(np.zeros((1, 3)), [[1, 0, 0, 1, 0, 1e-4]], [1.0])
    th = 0.4
    q = np.array([[math.cos(th / 2), math.sin(th / 2), 0, 0]])
    out = GE.loss(np.array([[1.0, 2.0, 0.3]]), np.array([[0.2, 0.05]]), q, comp, 0.5)
    assert abs(out["geo"] - (0.3 + 0.5 * (1 - math.cos(th)))) < 1e-12
    assert abs(out["iso"] - 0.15 ** 2) < 1e-15
    np.testing.assert_allclose(np.abs(out["d_means"][0]), [0, 0, 1], atol=1e-12)


def test_reference_normal_is_the_flat_axis():
    mean, cov6, w, R = _components()
    comp = GE.prepare(mean, cov6, w)
    np.testing.assert_allclose(np.abs(np.einsum("ki,ki->k", comp["normal"], R[:, :, 2])), 1.0, atol=1e-9)


def test_assignment_is_the_map_component():
    mean, cov6, w, _ = _components()
    comp = GE.prepare(mean, cov6, w)
    x = _surfels(2000)[0]
    k = GE.assign(x, comp)
    S = GE.cov_matrix(cov6)
    lp = np.stack([np.log(w[j]) + multivariate_normal(mean[j], S[j]).logpdf(x.astype(np.float64))
                   for j in range(len(w))], 1)
    srt = np.sort(lp, 1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-3 * np.maximum(1.0, np.abs(srt[:, -1]))
    assert clear.sum() > 1900
    np.testing.assert_array_equal(k[clear], np.argmax(lp, 1)[clear])


def test_gradients_by_central_differences():
    mean, cov6, w, _ = _components(K=8, seed=2)
    comp = GE.prepare(mean, cov6, w)
    means, scales, quats = (a.astype(np.float64) for a in _surfels(20, seed=3))
    lam = 0.7
    ref = GE.loss(means, scales, quats, comp, lam)
    k = ref["assign"]
    tot = lambda m, s, q: (lambda o: o["geo"] + o["iso"])(GE.loss(m, s, q, comp, lam, k=k))
    for name, arr, g in (("means", means, ref["d_means"]), ("scales", scales, ref["d_scales"]),
                         ("quats", quats, ref["d_quats"])):
        num = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            h = 1e-6
            a, b = arr.copy(), arr.copy()
            a[idx] += h
            b[idx] -= h
            args = {"means": means, "scales": scales, "quats": quats}
            args[name] = a
            fp = tot(args["means"], args["scales"], args["quats"])
            args[name] = b
            fm = tot(args["means"], args["scales"], args["quats"])
            num[idx] = (fp - fm) / (2 * h)
        np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-7, err_msg=name)


def test_gradients_against_torch():
    mean, cov6, w, _ = _components(K=8, seed=4)
    comp = GE.prepare(mean, cov6, w)
    means, scales, quats = (a.astype(np.float64) for a in _surfels(50, seed=5))
    lam = 1.3
    ref = GE.loss(means, scales, quats, comp, lam)
    k = ref["assign"]
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    tm, ts, tq = T(means), T(scales), T(quats)
    qn = tq / tq.norm(dim=1, keepdim=True)
    w_, x, y, z = qn.unbind(1)
    Rm = torch.stack([torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w_ * z), 2 * (x * z + w_ * y)], 1),
                      torch.stack([2 * (x * y + w_ * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w_ * x)], 1),
                      torch.stack([2 * (x * z - w_ * y), 2 * (y * z + w_ * x), 1 - 2 * (x * x + y * y)], 1)], 1)
    n = Rm[:, :, 2]
    nk = torch.tensor(comp["normal"][k])
    mk = torch.tensor(comp["mean"][k].astype(np.float64))
    L = ((tm - mk) * nk).sum(1).abs().sum() + lam * (1 - (n * nk).sum(1).abs()).sum() + \
        ((ts[:, 0] - ts[:, 1]) ** 2).sum()
    L.backward()
    assert abs(L.item() - (ref["geo"] + ref["iso"])) < 1e-9
    np.testing.assert_allclose(ref["d_means"], tm.grad.numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ref["d_scales"], ts.grad.numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ref["d_quats"], tq.grad.numpy(), rtol=1e-10, atol=1e-12)
