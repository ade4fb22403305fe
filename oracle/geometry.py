"""SOGMM geometric loss of surfels (Sec. 3.2 eq. (3), Sec. 4.2 eq. (13) and
the anisotropy term), written out plainly.  TEST INFRASTRUCTURE ONLY: the
test-suite, the smoke check and the benchmark's CPU-baseline leg are the only
callers.

Plane prior M_k: mixing weight pi_k, mean mu_k, covariance Sigma_k; its
reference normal n_k is the eigenvector of Sigma_k's smallest eigenvalue
(the normal constraint of Sec. 3.2).

Assignment (a reading: the paper pairs each surfel with the component whose
neighbourhood holds it): surfel i takes the component of largest posterior
pi_k N(mu_i; mu_k, Sigma_k), i.e. the smallest score
    s_k(x) = (x - mu_k)^T P_k (x - mu_k) + ln det Sigma_k - 2 ln pi_k,
with P_k = Sigma_k^-1 and the constant c_k = ln det Sigma_k - 2 ln pi_k
evaluated in FP64 and rounded to FP32; the score itself is evaluated in FP32
in the order written in `scores_f32` (a decision, taken the same way on both
sides; ties go to the lower index).

    d(mu_i, M_k) = |(mu_i - mu_k) . n_k|                           eq. (3)
    L_geo = sum_i d(mu_i, M_k(i)) + lambda_n (1 - |n_i . n_k(i)|)   eq. (13)
    L_iso = sum_i (s_i1 - s_i2)^2
with n_i the surfel normal (third column of the rotation of the normalised
quaternion).  Gradients hold the assignment fixed; at a zero distance or a
zero normal product the sign's subgradient 0 is used.
"""
from __future__ import annotations

import numpy as np

SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def cov_matrix(cov6):
    c = np.asarray(cov6, np.float64)
    S = np.zeros((c.shape[0], 3, 3))
    for k, (i, j) in enumerate(SYM):
        S[:, i, j] = c[:, k]
        S[:, j, i] = c[:, k]
    return S


def prepare(mean, cov6, weight):
    """Per component: FP32 mean, FP32 precision (6 numbers), FP32 constant,
    FP64 reference normal (smallest-eigenvalue eigenvector)."""
    S = cov_matrix(cov6)
    P = np.linalg.inv(S)
    _, logdet = np.linalg.slogdet(S)
    c = logdet - 2.0 * np.log(np.asarray(weight, np.float64))
    w, V = np.linalg.eigh(S)
    normal = V[:, :, 0]                                   # ascending eigenvalues: the smallest first
    P6 = np.stack([P[:, i, j] for i, j in SYM], 1)
    return {"mean": np.asarray(mean, np.float32), "P": P6.astype(np.float32), "c": c.astype(np.float32),
            "normal": normal, "eig": w}


def scores_f32(x, comp):
    """(n, K) FP32 scores:  d = x - mu;  t0 = (P00 d0 + P01 d1) + P02 d2,
    t1 = (P01 d0 + P11 d1) + P12 d2, t2 = (P02 d0 + P12 d1) + P22 d2;
    s = ((d0 t0 + d1 t1) + d2 t2) + c."""
    f = np.float32
    x = np.asarray(x, f)
    mu, P, c = comp["mean"], comp["P"], comp["c"]
    d0 = x[:, None, 0] - mu[None, :, 0]
    d1 = x[:, None, 1] - mu[None, :, 1]
    d2 = x[:, None, 2] - mu[None, :, 2]
    P00, P01, P02, P11, P12, P22 = (P[None, :, k] for k in range(6))
    t0 = (P00 * d0 + P01 * d1) + P02 * d2
    t1 = (P01 * d0 + P11 * d1) + P12 * d2
    t2 = (P02 * d0 + P12 * d1) + P22 * d2
    return ((d0 * t0 + d1 * t1) + d2 * t2) + c[None, :]


def assign(x, comp, chunk=4096):
    out = np.empty(len(x), np.int64)
    for a in range(0, len(x), chunk):
        out[a:a + chunk] = np.argmin(scores_f32(x[a:a + chunk], comp), axis=1)
    return out


def surfel_normal(quats):
    q = np.asarray(quats, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)], 1)


def loss(means, scales, quats, comp, lambda_n, k=None) -> dict:
    """Losses, per-surfel terms and gradients (FP64)."""
    mu = np.asarray(means, np.float64)
    s = np.asarray(scales, np.float64)
    q = np.asarray(quats, np.float64)
    if k is None:
        k = assign(means, comp)
    nk = comp["normal"][k]
    delta = np.einsum("ij,ij->i", mu - comp["mean"][k].astype(np.float64), nk)
    n = surfel_normal(q)
    dot = np.einsum("ij,ij->i", n, nk)
    geo = np.abs(delta) + lambda_n * (1.0 - np.abs(dot))
    iso = (s[:, 0] - s[:, 1]) ** 2
    # gradients
    d_means = np.sign(delta)[:, None] * nk
    dn = -lambda_n * np.sign(dot)[:, None] * nk            # dL/dn
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = qn.T
    # dn/d(w, x, y, z) of n = (2(xz + wy), 2(yz - wx), 1 - 2(x^2 + y^2)) at the unit quaternion
    J = np.stack([np.stack([2 * y, 2 * z, 2 * w, 2 * x], 1),
                  np.stack([-2 * x, -2 * w, 2 * z, 2 * y], 1),
                  np.stack([np.zeros_like(w), -4 * x, -4 * y, np.zeros_like(w)], 1)], 1)   # (n, 3, 4)
    g_unit = np.einsum("ni,nij->nj", dn, J)
    # through q / |q|: (I - qn qn^T) / |q|
    g_q = (g_unit - qn * np.einsum("nj,nj->n", g_unit, qn)[:, None]) / np.linalg.norm(q, axis=1, keepdims=True)
    d_scales = np.stack([2 * (s[:, 0] - s[:, 1]), -2 * (s[:, 0] - s[:, 1])], 1)
    return {"geo": float(geo.sum()), "iso": float(iso.sum()), "assign": k, "geo_i": geo, "iso_i": iso,
            "d_means": d_means, "d_quats": g_q, "d_scales": d_scales, "delta": delta, "dot": dot}
