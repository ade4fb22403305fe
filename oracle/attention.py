"""Frustum-local cross-attention of instance queries over surfels (Sec. 4.1,
eqs. (9)-(11)), written out plainly.  TEST INFRASTRUCTURE ONLY: the
test-suite, the smoke check and the benchmark's CPU-baseline leg are the only
callers.

Active set (the frustum test, a reading of the 3DGS criterion the paper
cites): surfel j takes part when the bounding sphere of its 99% confidence
disk -- rho <= -2 ln(0.01) in its own plane, radius r99 max(s_u, s_v) --
meets the view frustum, i.e. is not wholly behind the near plane or outside
one of the four planes through the camera centre and the image borders.  The
test is evaluated in FP32 in a prescribed operation order (so it is a
decision both sides take identically); every other step is FP64.

    K_j = f_j + psi(mu_j),  V_j = f_j                                eq. (9)
    e_ij = (Q_i W_Q) . (K_j W_K) / sqrt(d)                           eq. (10)
    Q'_i = sum_j softmax_j(e_ij) (V_j W_V)                           eq. (11)

psi (not specified by the paper; a reading): channel c of psi(mu) is
sin(2^b pi mu_a / L) for (c // 3) even and cos(...) for (c // 3) odd, with
axis a = c mod 3 and band b = c // 6, L a scene length.  d is the projection
width (W_Q, W_K, W_V are C x d).  With no active surfel Q' is zero.
"""
from __future__ import annotations

import numpy as np

R99_SQ = -2.0 * np.log(0.01)          # chi-square(2) 99% quantile, 9.2103...
R99_F32 = np.float32(np.sqrt(R99_SQ))  # 99% radius in units of the scale


def frustum_active(means, scales, cam) -> np.ndarray:
    """Boolean mask of the active set, FP32 in the prescribed order."""
    f = np.float32
    mu = np.asarray(means, f)
    sc = np.asarray(scales, f)
    R = np.asarray(cam.R, f).reshape(3, 3)
    t = np.asarray(cam.t, f)
    mc = [((R[i, 0] * mu[:, 0] + R[i, 1] * mu[:, 1]) + R[i, 2] * mu[:, 2]) + t[i] for i in range(3)]
    rr = R99_F32 * np.maximum(sc[:, 0], sc[:, 1])
    fx, fy, cx, cy = f(cam.fx), f(cam.fy), f(cam.cx), f(cam.cy)
    W, H, near = f(cam.width), f(cam.height), f(cam.near)
    nl = np.sqrt(fx * fx + cx * cx)
    nr = np.sqrt(fx * fx + (W - cx) * (W - cx))
    nt = np.sqrt(fy * fy + cy * cy)
    nb = np.sqrt(fy * fy + (H - cy) * (H - cy))
    act = (mc[2] - near) >= -rr
    act &= (fx * mc[0] + cx * mc[2]) >= -(rr * nl)
    act &= ((W - cx) * mc[2] - fx * mc[0]) >= -(rr * nr)
    act &= (fy * mc[1] + cy * mc[2]) >= -(rr * nt)
    act &= ((H - cy) * mc[2] - fy * mc[1]) >= -(rr * nb)
    return act


def posenc(means, C: int, length: float) -> np.ndarray:
    """psi(mu): (n, C), FP64."""
    mu = np.asarray(means, np.float64)
    c = np.arange(C)
    axis, band, phase = c % 3, c // 6, (c // 3) % 2
    arg = (2.0 ** band) * np.pi * mu[:, axis] / float(length)
    return np.where(phase == 0, np.sin(arg), np.cos(arg))


def attention(means, scales, feat, cam, q, wq, wk, wv, length: float) -> dict:
    """Q' (n_q, d) and the intermediate terms, FP64."""
    act = frustum_active(means, scales, cam)
    idx = np.nonzero(act)[0]
    f = np.asarray(feat, np.float64)[idx]
    K = f + posenc(np.asarray(means)[idx], f.shape[1], length)            # eq. (9)
    Qp = np.asarray(q, np.float64) @ np.asarray(wq, np.float64)
    Kp = K @ np.asarray(wk, np.float64)
    Vp = f @ np.asarray(wv, np.float64)
    d = Qp.shape[1]
    out = np.zeros((Qp.shape[0], np.asarray(wv).shape[1]))
    P = np.zeros((Qp.shape[0], idx.size))
    if idx.size:
        e = Qp @ Kp.T / np.sqrt(d)                                          # eq. (10)
        e = e - e.max(axis=1, keepdims=True)
        P = np.exp(e)
        P /= P.sum(axis=1, keepdims=True)
        out = P @ Vp                                                        # eq. (11)
    return {"out": out, "active": act, "idx": idx, "P": P, "Vp": Vp, "Kp": Kp, "Qp": Qp}
