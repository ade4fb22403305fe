"""Pins of the oracle's instance-label step (Sec. 4.1, eqs. (4)-(7)).

The labels are a softmax over queries of sigmoid(f_q . f_g) times the query
Gaussian's density ratio; pinned by a hand-computed two-query case, the
simplex and invariance properties, and their gradients by central finite
differences and by torch float64 autograd of a separate transcription that
uses the covariance (not the precision) and torch's own softmax."""
import math

import numpy as np
import pytest
import torch

from oracle import labels as LB


def problem(n=7, q=5, c=6, seed=0):
    rng = np.random.default_rng(seed)
    f_g = rng.standard_normal((n, c)) * 0.7
    p_g = rng.uniform(-1, 1, (n, 3))
    f_q = rng.standard_normal((q, c)) * 0.7
    mu_q = rng.uniform(-1, 1, (q, 3))
    # precision = (M M^T + 0.5 I)^-1 scaled, symmetric positive definite
    prec = []
    for _ in range(q):
        M = rng.standard_normal((3, 3)) * 0.5
        P = np.linalg.inv(M @ M.T + 0.5 * np.eye(3))
        prec.append([P[i, j] for i, j in LB.SYM])
    return f_g, p_g, f_q, mu_q, np.array(prec)


def test_two_queries_by_hand():
    # surfel at the origin, f_g = (1, 0); query 1 at the origin with f = (2, 0)
    # (S = sigmoid(2), D = 1); query 2 one unit away along x with identity
    # precision and f = (0, 1) (S = sigmoid(0) = 1/2, D = exp(-1/2)).
    f_g = np.array([[1.0, 0.0]])
    p_g = np.zeros((1, 3))
    f_q = np.array([[2.0, 0.0], [0.0, 1.0]])
    mu_q = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    prec = np.array([[1, 0, 0, 1, 0, 1], [1, 0, 0, 1, 0, 1]], np.float64)
    a1 = 0.8807970779778823            # sigmoid(2)
    a2 = 0.5 * 0.6065306597126334      # sigmoid(0) * exp(-1/2)
    want = np.array([math.exp(a1), math.exp(a2)]) / (math.exp(a1) + math.exp(a2))
    got = LB.forward(f_g, p_g, f_q, mu_q, prec)["labels"][0]
    np.testing.assert_allclose(got, want, rtol=1e-15)


def test_simplex_and_special_cases():
    f_g, p_g, f_q, mu_q, prec = problem()
    lab = LB.forward(f_g, p_g, f_q, mu_q, prec)["labels"]
    np.testing.assert_allclose(lab.sum(1), 1.0, rtol=1e-14)
    assert (lab > 0).all() and (lab < 1).all()
    # one query: every label is 1
    one = LB.forward(f_g, p_g, f_q[:1], mu_q[:1], prec[:1])["labels"]
    np.testing.assert_array_equal(one, 1.0)
    # two identical queries split evenly
    two = LB.forward(f_g, p_g, np.repeat(f_q[:1], 2, 0), np.repeat(mu_q[:1], 2, 0), np.repeat(prec[:1], 2, 0))
    np.testing.assert_allclose(two["labels"], 0.5, rtol=1e-15)
    # a surfel at a query's mean has density ratio exactly 1 for it
    fw = LB.forward(f_g, mu_q[2:3], f_q, mu_q, prec)
    assert fw["D"][0, 2] == 1.0


def test_rigid_motion_and_query_permutation_invariance():
    f_g, p_g, f_q, mu_q, prec = problem(seed=3)
    base = LB.forward(f_g, p_g, f_q, mu_q, prec)["labels"]
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    t = np.array([0.3, -2.0, 5.0])
    P = LB.precision_matrix(prec)
    P2 = np.einsum("ij,qjk,lk->qil", R, P, R)
    prec2 = np.stack([P2[:, i, j] for i, j in LB.SYM], 1)
    moved = LB.forward(f_g, p_g @ R.T + t, f_q, mu_q @ R.T + t, prec2)["labels"]
    np.testing.assert_allclose(moved, base, rtol=1e-12)
    perm = np.array([3, 0, 4, 1, 2])
    np.testing.assert_allclose(LB.forward(f_g, p_g, f_q[perm], mu_q[perm], prec[perm])["labels"], base[:, perm],
                               rtol=1e-14)


def test_gradients_by_central_differences():
    args = list(problem(n=5, q=4, c=3, seed=1))
    rng = np.random.default_rng(2)
    up = rng.standard_normal((5, 4))
    grads = LB.backward(*args, up)
    names = ("f_g", "p_g", "f_q", "mu_q", "prec")
    for ai, name in enumerate(names):
        x = args[ai]
        num = np.zeros_like(x)
        for idx in np.ndindex(x.shape):
            h = 1e-6 * max(1.0, abs(x[idx]))
            xp, xm = x.copy(), x.copy()
            xp[idx] += h
            xm[idx] -= h
            ap, am = list(args), list(args)
            ap[ai], am[ai] = xp, xm
            num[idx] = (np.sum(up * LB.forward(*ap)["labels"]) - np.sum(up * LB.forward(*am)["labels"])) / (2 * h)
        key = {"f_g": "f_g", "p_g": "p_g", "f_q": "f_q", "mu_q": "mu_q", "prec": "prec"}[name]
        np.testing.assert_allclose(grads[key], num, rtol=1e-6, atol=1e-9, err_msg=name)


def _torch_labels(f_g, p_g, f_q, mu_q, cov):
    """Separate transcription: Mahalanobis distance by solving with the
    covariance, torch's sigmoid and softmax."""
    z = f_g @ f_q.T
    d = p_g[:, None, :] - mu_q[None, :, :]                          # (N, Q, 3)
    sol = torch.linalg.solve(cov[None].expand(d.shape[0], -1, -1, -1), d.unsqueeze(-1)).squeeze(-1)
    m = (d * sol).sum(-1)
    return torch.softmax(torch.sigmoid(z) * torch.exp(-0.5 * m), dim=1)


def test_gradients_against_torch_autograd():
    f_g, p_g, f_q, mu_q, prec = problem(n=9, q=6, c=5, seed=4)
    rng = np.random.default_rng(5)
    up = rng.standard_normal((9, 6))
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    tf_g, tp_g, tf_q, tmu = T(f_g), T(p_g), T(f_q), T(mu_q)
    P = LB.precision_matrix(prec)
    tprec = T(prec)
    # covariance as a function of the 6 precision numbers
    idx = torch.tensor([[0, 1, 2], [1, 3, 4], [2, 4, 5]])
    cov = torch.linalg.inv(tprec[:, idx])
    lab = _torch_labels(tf_g, tp_g, tf_q, tmu, cov)
    np.testing.assert_allclose(lab.detach().numpy(), LB.forward(f_g, p_g, f_q, mu_q, prec)["labels"], rtol=1e-12)
    (lab * torch.tensor(up)).sum().backward()
    got = LB.backward(f_g, p_g, f_q, mu_q, prec, up)
    for name, t in (("f_g", tf_g), ("p_g", tp_g), ("f_q", tf_q), ("mu_q", tmu), ("prec", tprec)):
        np.testing.assert_allclose(got[name], t.grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=name)
    assert P.shape == (6, 3, 3)
