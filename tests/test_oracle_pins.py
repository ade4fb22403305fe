"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle's forward model (Sec. 3.1: surfel kernel, alpha,
eq. (1) blending; Sec. 5: eq. (18) Top-K) against a closed form, an
independent library routine (scipy rotations, ray-plane intersection), an
invariant, or brute force on tiny inputs.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2604_10982_amd import scenes
from paper_2604_10982_amd.scenes import Scene, pinhole


def make_scene(means, scales, quats, opacity, rgb=None, feat=None, c=4):
    n = len(means)
    rgb = np.ones((n, 3)) if rgb is None else rgb
    feat = np.zeros((n, c)) if feat is None else feat
    f = lambda a: np.ascontiguousarray(a, np.float32)
    return Scene(f(means), f(scales), f(quats), f(opacity), f(rgb), f(feat))


def z_rot_quat(theta):
    return [math.cos(theta / 2), 0.0, 0.0, math.sin(theta / 2)]


def closed_form_alpha(x, y, cam, X0, Y0, z0, theta, su, sv, o):
    """Fronto-parallel surfel at depth z0 rotated by theta about the optical
    axis: the ray through (x, y) meets its plane at d = ((x-xc) z0/fx, (y-yc) z0/fy)
    relative to the centre; tangent coordinates are R(theta)^T d / s.
    Parameters are taken at their float32 values, as the renderer stores them."""
    f = lambda v: float(np.float32(v))
    X0, Y0, z0, su, sv, o = map(f, (X0, Y0, z0, su, sv, o))
    qw, qz = (np.float32(v) for v in (math.cos(theta / 2), math.sin(theta / 2)))
    theta = 2.0 * math.atan2(float(qz), float(qw))
    xc = cam.fx * X0 / z0 + cam.cx
    yc = cam.fy * Y0 / z0 + cam.cy
    dx = (x - xc) * z0 / cam.fx
    dy = (y - yc) * z0 / cam.fy
    u = (math.cos(theta) * dx + math.sin(theta) * dy) / su
    v = (-math.sin(theta) * dx + math.cos(theta) * dy) / sv
    rho = u * u + v * v
    return np.where(rho <= 9.0, o * np.exp(-0.5 * rho), 0.0), rho


def pixel_grid(cam):
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    return xs + 0.5, ys + 0.5


def test_single_fronto_parallel_closed_form(orc):
    cam = pinhole(64, 48, f=60.0)
    X0, Y0, z0, th, su, sv, o = 0.3, -0.2, 4.0, 0.6, 0.5, 0.25, 0.8
    sc = make_scene([[X0, Y0, z0]], [[su, sv]], [z_rot_quat(th)], [o])
    r = orc.render(sc, cam, K=4, blend=orc.FULL)
    x, y = pixel_grid(cam)
    a, rho = closed_form_alpha(x, y, cam, X0, Y0, z0, th, su, sv, o)
    a = np.where(a >= 1 / 255, a, 0.0)
    assert (a > 0).sum() > 100
    np.testing.assert_allclose(r["rgb"][..., 0], a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["alpha"], a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["depth"], a * z0, rtol=1e-12, atol=1e-14)
    # n = +z faces away from the camera at the origin, so it is flipped to -z
    np.testing.assert_allclose(r["normal"][..., 2], -a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["normal"][..., :2], 0.0, atol=1e-15)


def _ray_plane_rho(sc, cam, x, y):
    """Independent (u, v): scipy rotation + ray/plane intersection."""
    out_rho, out_z = [], []
    for i in range(sc.n):
        w, qx, qy, qz = sc.quats[i].astype(np.float64)
        Rq = Rotation.from_quat([qx, qy, qz, w]).as_matrix()      # scalar-last
        mu = sc.means[i].astype(np.float64)
        tu, tv, n = Rq[:, 0], Rq[:, 1], Rq[:, 2]
        d = np.stack([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, np.ones_like(x)], -1)
        t = (mu @ n) / (d @ n)
        X = d * t[..., None]
        u = ((X - mu) @ tu) / sc.scales[i, 0]
        v = ((X - mu) @ tv) / sc.scales[i, 1]
        out_rho.append(u * u + v * v)
        out_z.append(X[..., 2])
    return np.array(out_rho), np.array(out_z)


def test_tilted_surfels_match_ray_plane_intersection(orc):
    rng = np.random.default_rng(5)
    n = 20
    cam = pinhole(48, 40, f=50.0)
    q = rng.standard_normal((n, 4))
    sc = make_scene(np.c_[rng.uniform(-1, 1, (n, 2)), rng.uniform(3, 6, n)],
                    rng.uniform(0.1, 0.4, (n, 2)), q, rng.uniform(0.2, 0.9, n))
    xs = rng.uniform(0, 48, 200)
    ys = rng.uniform(0, 40, 200)
    rho, z = orc.eval_points(sc, cam, xs, ys)
    rho_ref, z_ref = _ray_plane_rho(sc, cam, xs, ys)
    ks = orc.keystage(sc, cam, pairs=False)
    vis = ks["cull"] == 0
    assert vis.sum() >= 15
    near = rho_ref[vis] < 50
    np.testing.assert_allclose(rho[vis][near], rho_ref[vis][near], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(z[vis][near], z_ref[vis][near], rtol=1e-11)


def test_two_surfel_composition(orc):
    cam = pinhole(64, 64, f=64.0)
    c1 = np.array([0.9, 0.2, 0.1], np.float32).astype(np.float64)
    c2 = np.array([0.1, 0.3, 0.8], np.float32).astype(np.float64)
    p1 = (0.05, 0.0, 3.0, 0.2, 0.5, 0.4, 0.7)
    p2 = (-0.1, 0.1, 5.0, -0.4, 0.6, 0.9, 0.95)
    sc = make_scene([p1[:3], p2[:3]], [p1[4:6], p2[4:6]], [z_rot_quat(p1[3]), z_rot_quat(p2[3])],
                    [p1[6], p2[6]], rgb=np.stack([c1, c2]))
    r = orc.render(sc, cam, K=2, blend=orc.FULL)
    x, y = pixel_grid(cam)
    a1, _ = closed_form_alpha(x, y, cam, *p1)
    a2, _ = closed_form_alpha(x, y, cam, *p2)
    a1 = np.where(a1 >= 1 / 255, np.minimum(a1, 0.99), 0.0)
    a2 = np.where(a2 >= 1 / 255, np.minimum(a2, 0.99), 0.0)
    ref = c1 * a1[..., None] + c2 * (a2 * (1 - a1))[..., None]
    assert ((a1 > 0) & (a2 > 0)).sum() > 50
    np.testing.assert_allclose(r["rgb"], ref, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["T_final"], (1 - a1) * (1 - a2), rtol=1e-12)


def test_stop_rule_excludes_the_surfel_that_would_end_the_walk(orc):
    # Three stacked opaque surfels: T = 1 -> 0.01 -> 1e-4 (would reach T < 1e-4
    # only at the third); alpha is clamped to 0.99 at the centre pixel.
    cam = pinhole(16, 16, f=16.0)
    sc = make_scene([[0, 0, 2.0], [0, 0, 3.0], [0, 0, 4.0]], [[1, 1]] * 3, [[1, 0, 0, 0]] * 3,
                    [1.0, 1.0, 1.0], rgb=np.eye(3))
    r = orc.render(sc, cam, K=3, blend=orc.FULL)
    c = r["rgb"][8, 8]
    # third surfel: T' = 1e-4 * 0.01 < 1e-4 -> not blended; second: T' = 1e-4 (not < 1e-4)
    a = 0.99
    assert r["ncontrib"][8, 8] == 2
    np.testing.assert_allclose(c, [a, a * (1 - a), 0.0], rtol=1e-12, atol=1e-18)


def test_weights_and_final_transmittance_sum_to_one(orc):
    sc, cam, K, _ = scenes.config("c1_box2k")
    sc.rgb[:] = 1.0
    r = orc.render(sc, cam, K, blend=orc.FULL)
    s = r["rgb"][..., 0] + r["T_final"]
    np.testing.assert_allclose(s, 1.0, atol=1e-12)
    assert r["ncontrib"].max() >= 3


def test_topk_equals_full_when_k_covers_depth_complexity(orc):
    sc, cam, _, _ = scenes.config("c1_box2k")
    rf = orc.render(sc, cam, 8, blend=orc.FULL)
    kmax = int(rf["ncontrib"].max())
    rk = orc.render(sc, cam, kmax, blend=orc.TOPK)
    np.testing.assert_allclose(rk["feat"], rf["feat"], rtol=1e-12, atol=1e-13)


def _tiny_scene(n=40, seed=3, c=None):
    rng = np.random.default_rng(seed)
    c = n if c is None else c
    sc = make_scene(np.c_[rng.uniform(-0.6, 0.6, (n, 2)), rng.uniform(2, 4, n)],
                    np.exp(rng.normal(np.log(0.15), 0.4, (n, 2))), rng.standard_normal((n, 4)),
                    rng.uniform(0.2, 0.95, n), rgb=rng.uniform(0, 1, (n, 3)),
                    feat=np.eye(n, c))
    return sc, pinhole(40, 32, f=36.0)


@pytest.mark.parametrize("K", [1, 2, 4])
def test_topk_selection_brute_force(orc, K):
    """One-hot features make the dense blend return every contributor's weight
    (F[p, j] = w_j); Top-K must keep exactly the K largest of them."""
    sc, cam = _tiny_scene()
    full = orc.render(sc, cam, K, blend=orc.FULL)["feat"]
    topk = orc.render(sc, cam, K, blend=orc.TOPK)["feat"]
    assert (np.count_nonzero(full, axis=-1) > K).sum() > 50
    ref = np.zeros_like(full)
    for idx in np.ndindex(full.shape[:2]):
        w = full[idx]
        order = np.argsort(-w, kind="stable")[:K]
        keep = order[w[order] > 0]
        ref[idx][keep] = w[keep]
    np.testing.assert_array_equal(topk, ref)


def test_topk_truncation_bound(orc):
    sc, cam, K, _ = scenes.config("c1_box2k")
    K = 2
    rf = orc.render(sc, cam, K, blend=orc.FULL)
    rk = orc.render(sc, cam, K, blend=orc.TOPK)
    fmax = np.abs(sc.feat).max()
    wsel = rk["sel_w"].sum(-1)
    bound = fmax * (1.0 - rk["T_final"] - wsel)
    err = np.abs(rk["feat"] - rf["feat"]).max(-1)
    assert (err <= bound + 1e-12).all()
    assert (err > 0).sum() > 20


def test_mirror_symmetry(orc):
    sc, cam, K, _ = scenes.config("c1_box2k")
    m = sc.copy()
    m.means[:, 0] *= -1
    m.quats[:, 2] *= -1
    m.quats[:, 3] *= -1
    a = orc.render(sc, cam, K, blend=orc.TOPK)
    b = orc.render(m, cam, K, blend=orc.TOPK)
    ok = (a["margin"] > 1e-6) & (b["margin"][:, ::-1] > 1e-6)
    assert ok.mean() > 0.99
    for key, sign in (("rgb", 1), ("depth", 1), ("alpha", 1), ("feat", 1)):
        np.testing.assert_allclose(b[key][:, ::-1][ok], a[key][ok], rtol=1e-9, atol=1e-11)
    nb = b["normal"][:, ::-1].copy()
    nb[..., 0] *= -1
    np.testing.assert_allclose(nb[ok], a["normal"][ok], rtol=1e-9, atol=1e-11)
