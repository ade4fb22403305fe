"""Instance labels of surfels from localized queries (Sec. 4.1, eqs. (4)-(7)),
written out plainly in FP64 numpy.  TEST INFRASTRUCTURE ONLY: the test-suite,
the smoke check and the benchmark's CPU-baseline leg are the only callers.

For surfel g (centre p_g, instance feature f_g) and query q (feature f_q,
Gaussian with mean mu_q and precision P_q = Sigma_q^-1):

    S(q, g) = sigmoid(f_q . f_g)                              eq. (4)
    D(q, g) = phi_q(p_g) / phi_q(mu_q)
            = exp(-(p_g - mu_q)^T P_q (p_g - mu_q) / 2)       eq. (5)
    A(q, g) = S(q, g) D(q, g)                                 eq. (6)
    l(g)    = softmax over q of A(q, g)                       eq. (7)

The rendered instance map, eq. (8), is the alpha blend of l over the surfels
of a ray; it is the renderer's feature blend applied to l (see oracle.render).

Precisions are given as 6 numbers per query (xx, xy, xz, yy, yz, zz) of the
symmetric matrix; their gradients are with respect to those 6 numbers (an
off-diagonal number appears twice in the matrix).
"""
from __future__ import annotations

import numpy as np

SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def precision_matrix(prec6: np.ndarray) -> np.ndarray:
    """(Q, 6) -> (Q, 3, 3) symmetric."""
    prec6 = np.asarray(prec6, np.float64)
    P = np.zeros((prec6.shape[0], 3, 3))
    for k, (i, j) in enumerate(SYM):
        P[:, i, j] = prec6[:, k]
        P[:, j, i] = prec6[:, k]
    return P


def forward(f_g, p_g, f_q, mu_q, prec6) -> dict:
    """Labels (N, Q) and the intermediate terms, FP64."""
    f_g = np.asarray(f_g, np.float64)
    p_g = np.asarray(p_g, np.float64)
    f_q = np.asarray(f_q, np.float64)
    mu_q = np.asarray(mu_q, np.float64)
    P = precision_matrix(prec6)
    z = f_g @ f_q.T                                   # feature similarity logits
    S = 1.0 / (1.0 + np.exp(-z))                      # eq. (4)
    d = p_g[:, None, :] - mu_q[None, :, :]            # (N, Q, 3)
    Pd = np.einsum("qij,nqj->nqi", P, d)
    m = np.einsum("nqi,nqi->nq", d, Pd)               # squared Mahalanobis distance
    D = np.exp(-0.5 * m)                              # eq. (5)
    A = S * D                                         # eq. (6)
    e = np.exp(A - A.max(axis=1, keepdims=True))      # eq. (7)
    lab = e / e.sum(axis=1, keepdims=True)
    return {"labels": lab, "z": z, "S": S, "D": D, "A": A, "d": d, "Pd": Pd}


def backward(f_g, p_g, f_q, mu_q, prec6, d_labels) -> dict:
    """Gradients of L = sum(d_labels * labels) with respect to every input."""
    fw = forward(f_g, p_g, f_q, mu_q, prec6)
    lab, S, D, d, Pd = fw["labels"], fw["S"], fw["D"], fw["d"], fw["Pd"]
    g = np.asarray(d_labels, np.float64)
    # softmax: dA = l (g - sum_q l g)
    dA = lab * (g - np.sum(lab * g, axis=1, keepdims=True))
    dS = dA * D
    dD = dA * S
    dz = dS * S * (1.0 - S)
    # D = exp(-m/2), m = d^T P d:  dD/dd = -D P d,  dD/dP = -D/2 d d^T
    wD = dD * D                                       # (N, Q)
    out = {
        "f_g": dz @ np.asarray(f_q, np.float64),
        "f_q": dz.T @ np.asarray(f_g, np.float64),
        "p_g": -np.einsum("nq,nqi->ni", wD, Pd),
        "mu_q": np.einsum("nq,nqi->qi", wD, Pd),
    }
    dP = -0.5 * np.einsum("nq,nqi,nqj->qij", wD, d, d)
    out["prec"] = np.stack([dP[:, i, j] if i == j else dP[:, i, j] + dP[:, j, i] for i, j in SYM], axis=1)
    return out
