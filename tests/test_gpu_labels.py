"""Instance labels (Sec. 4.1, eqs. (4)-(7)) on the matrix cores against the
FP64 oracle, their gradients, and the instance map of eq. (8) rendered in the
same walk and with the same Top-K selection as the semantic features."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, TORCH_DTYPES, decided, render, require_gpu, to_dev
from oracle import labels as LB
from paper_2604_10982_amd import psm, scenes
from paper_2604_10982_amd import render as R

pytestmark = pytest.mark.gpu


def queries(nq, c, seed=0, spread=3.0):
    """Query features N(0,1)/sqrt(c)*3, centres in the scene box, precisions of
    Gaussians with 0.3-2 m axes."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nq, c)) * 3.0 / np.sqrt(c)
    mu = np.c_[rng.uniform(-spread, spread, nq), rng.uniform(-1.5, 1.5, nq), rng.uniform(2.0, 9.0, nq)]
    prec = []
    for _ in range(nq):
        M = np.linalg.qr(rng.standard_normal((3, 3)))[0]
        s = rng.uniform(0.3, 2.0, 3)
        P = M @ np.diag(1.0 / s ** 2) @ M.T
        prec.append([P[i, j] for i, j in LB.SYM])
    return f.astype(np.float32), mu.astype(np.float32), np.array(prec, np.float32)


def surfels(n, c, seed=1):
    rng = np.random.default_rng(seed)
    means = np.c_[rng.uniform(-3, 3, n), rng.uniform(-1.5, 1.5, n), rng.uniform(2, 9, n)].astype(np.float32)
    f = (rng.standard_normal((n, c)) / np.sqrt(c) * 3.0).astype(np.float32)
    return means, f


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


@pytest.mark.parametrize("nq,c", [(1, 4), (7, 32), (16, 32), (64, 32), (100, 128), (256, 16)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_labels_match_oracle(nq, c, dtype):
    require_gpu()
    n = 3001
    means, f_ins = surfels(n, c)
    qf, qm, qp = queries(nq, c)
    tf = T(f_ins).to(TORCH_DTYPES[dtype]).contiguous()
    lab = psm.instance_labels(T(means), tf, T(qf), T(qm), T(qp))
    torch.cuda.synchronize()
    got = lab.cpu().numpy().astype(np.float64)
    ref = LB.forward(tf.float().cpu().numpy(), means, qf, qm, qp)["labels"]
    # FP32 logits (MFMA, c products accumulated), FP32 sigmoid/exp: the label
    # error stays within a few 1e-6 of its value plus 1e-6 absolute
    np.testing.assert_allclose(got[:, :nq], ref, rtol=2e-5, atol=2e-6)
    assert (got[:, nq:] == 0).all()
    np.testing.assert_allclose(got[:, :nq].sum(1), 1.0, rtol=1e-5)


def test_labels_write_into_a_column_slice():
    require_gpu()
    n, nq, c, cs = 500, 10, 8, 24
    means, f_ins = surfels(n, c)
    qf, qm, qp = queries(nq, c)
    big = torch.full((n, cs + psm.label_width(nq) + 8), 7.0, device=DEV)
    psm.instance_labels_into(T(means), T(f_ins), T(qf), T(qm), T(qp), big[:, cs:], big.shape[1])
    torch.cuda.synchronize()
    b = big.cpu().numpy()
    assert (b[:, :cs] == 7.0).all() and (b[:, cs + psm.label_width(nq):] == 7.0).all()
    np.testing.assert_allclose(b[:, cs:cs + nq], LB.forward(f_ins, means, qf, qm, qp)["labels"], rtol=2e-5,
                               atol=2e-6)


@pytest.mark.parametrize("nq,c,dtype", [(16, 32, "f32"), (64, 32, "f16"), (5, 12, "f32"), (130, 64, "f32")])
def test_label_gradients_match_oracle(nq, c, dtype):
    require_gpu()
    n = 2500
    means, f_ins = surfels(n, c, seed=3)
    qf, qm, qp = queries(nq, c, seed=4)
    rng = np.random.default_rng(5)
    up = rng.standard_normal((n, nq)).astype(np.float32)
    tf = T(f_ins).to(TORCH_DTYPES[dtype]).contiguous()
    ld = psm.label_width(nq)
    dl = torch.zeros(n, ld, device=DEV)
    dl[:, :nq] = T(up)
    got = psm.instance_labels_backward(T(means), tf, T(qf), T(qm), T(qp), dl, ld)
    torch.cuda.synchronize()
    ref = LB.backward(tf.float().cpu().numpy(), means, qf, qm, qp, up)
    for key, rk in (("means", "p_g"), ("f_ins", "f_g"), ("q_feat", "f_q"), ("q_mean", "mu_q"), ("q_prec", "prec")):
        g = got[key].cpu().numpy().astype(np.float64)
        r = ref[rk]
        rms = np.sqrt(np.mean(r ** 2))
        err = np.abs(g - r) / np.maximum(np.abs(r), 1e-2 * rms)
        assert float(err.max()) <= 1e-3, (key, float(err.max()))


def test_panoptic_render_one_walk(orc):
    """Semantic and instance maps from one walk: the semantic part equals a
    semantic-only render bit for bit (same selection, channels independent),
    the instance part matches the oracle render of the labels, and the
    autograd chain through labels and render matches the oracle chain."""
    require_gpu()
    sc = scenes.planes7(20_000, 16, seed=5)
    cam = scenes.pinhole(200, 136)
    K = 8
    nq, c = 12, 16
    qf, qm, qp = queries(nq, c, seed=6, spread=8.0)
    rng = np.random.default_rng(7)
    f_ins = (rng.standard_normal((sc.n, c)) / np.sqrt(c) * 3.0).astype(np.float32)
    t = to_dev(sc)
    args = [t["means"].clone().requires_grad_(), t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"],
            T(f_ins).requires_grad_(), T(qf).requires_grad_(), T(qm), T(qp)]
    out = R.render_panoptic(*args, cam, K, "ellipse", "topk")
    sem, ins = out[4], out[5]
    alone, _ = render(t, cam, K)
    assert torch.equal(sem, alone["feat"])
    # oracle: labels, then the render of [semantic | labels]
    lab = LB.forward(f_ins, sc.means, qf, qm, qp)["labels"]
    feat = np.concatenate([sc.feat.astype(np.float64), lab, np.zeros((sc.n, psm.label_width(nq) - nq))], 1)
    sc = scenes.Scene(sc.means, sc.scales, sc.quats, sc.opacity, sc.rgb, feat.astype(np.float32))
    ref = orc.render(sc, cam, K, orc.TOPK, feat=feat)
    ok = decided(ref)
    absf = orc.render(sc, cam, K, orc.TOPK, feat=np.abs(feat))["feat"]
    gi = ins.detach().cpu().numpy().astype(np.float64)
    ri = ref["feat"][..., 16:16 + nq]
    si = absf[..., 16:16 + nq]
    assert float((np.abs(gi - ri) / (1e-5 * si + 1e-7))[ok].max()) <= 1.0
    # gradient chain: loss = sum(w * instance map)
    w = rng.standard_normal(ins.shape).astype(np.float32)
    w[~ok] = 0.0
    (ins * T(w)).sum().backward()
    g_up = {k: np.zeros_like(v) for k, v in scenes.upstream(cam.height, cam.width, feat.shape[1], seed=1).items()}
    g_up["feat"][..., 16:16 + nq] = w
    rb = orc.backward(sc, cam, g_up, K=K, blend=orc.TOPK, feat=feat)
    lb = LB.backward(f_ins, sc.means, qf, qm, qp, rb["feat"][:, 16:16 + nq])
    checks = ((args[6].grad, lb["f_g"]), (args[7].grad, lb["f_q"]), (args[0].grad, rb["means"] + lb["p_g"]))
    for got, r in checks:
        g = got.cpu().numpy().astype(np.float64)
        rms = np.sqrt(np.mean(r ** 2))
        err = np.abs(g - r) / np.maximum(np.abs(r), 1e-2 * rms)
        assert float(err.max()) <= 1e-3, float(err.max())


def test_labels_full_size_1m():
    """The benchmark's shape: labels of the 1M-surfel plane scene from 64
    queries with 32-d instance features.  Labels are per surfel, so a 20k
    sample is checked against the oracle; the query gradients sum over all
    surfels and are checked whole."""
    require_gpu()
    sc, _, _, _ = scenes.config("planes1m_1080p")
    n, nq, c = sc.n, 64, 32
    rng = np.random.default_rng(3)
    f_ins = (rng.standard_normal((n, c)) * 3.0 / np.sqrt(c)).astype(np.float32)
    qf = (rng.standard_normal((nq, c)) * 3.0 / np.sqrt(c)).astype(np.float32)
    qm = np.c_[rng.uniform(-12, 12, nq), rng.uniform(-6, 1.6, nq), rng.uniform(2, 60, nq)].astype(np.float32)
    qp = np.tile(np.array([0.25, 0, 0, 0.25, 0, 0.25], np.float32), (nq, 1))
    args = (T(sc.means), T(f_ins), T(qf), T(qm), T(qp))
    lab = psm.instance_labels(*args)
    ld = psm.label_width(nq)
    up = rng.standard_normal((n, nq)).astype(np.float32)
    dl = torch.zeros(n, ld, device=DEV)
    dl[:, :nq] = T(up)
    got = psm.instance_labels_backward(*args, dl, ld)
    torch.cuda.synchronize()
    idx = np.sort(rng.choice(n, 20_000, replace=False))
    ref = LB.forward(f_ins[idx], sc.means[idx], qf, qm, qp)["labels"]
    np.testing.assert_allclose(lab.cpu().numpy()[idx, :nq].astype(np.float64), ref, rtol=2e-5, atol=2e-6)
    rb = LB.backward(f_ins, sc.means, qf, qm, qp, up)
    for key, rk, rows in (("means", "p_g", idx), ("f_ins", "f_g", idx), ("q_feat", "f_q", None),
                          ("q_mean", "mu_q", None), ("q_prec", "prec", None)):
        g = got[key].cpu().numpy().astype(np.float64)
        r = rb[rk]
        if rows is not None:
            g, r = g[rows], r[rows]
        rms = np.sqrt(np.mean(r ** 2))
        err = np.abs(g - r) / np.maximum(np.abs(r), 1e-2 * rms)
        assert float(err.max()) <= 1e-3, (key, float(err.max()))
