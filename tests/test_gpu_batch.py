"""Several cameras in one call, the persistent tile scheduler, the launch
autotuner and HIP-graph capture.

A batch renders camera b exactly as a single-camera call would (the virtual
surfels of camera b keep the single-camera depth order, so images and the
Top-K selection are bit-identical); its gradients are the sum over cameras
of the single-camera gradients, checked against that sum and against the
FP64 oracle summed over the cameras.  Launch choices (scheduler, pass widths)
never change a result bit."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, decided, np_out, render, require_gpu, stored_feat, to_dev
from paper_2604_10982_amd import psm, scenes
from test_gpu_backward import grad_errors

pytestmark = pytest.mark.gpu

RES4 = ((200, 150), (96, 64), (333, 211), (160, 120))
MAPS = ("rgb", "depth", "normal", "alpha", "feat")
GROUPS = ("means", "scales", "quats", "opacity", "rgb", "feat")


def _street(n=60_000, c=16, seed=3):
    return scenes.street40(n, c, seed), scenes.street_cameras(RES4)


def _args(t):
    return t["means"], t["scales"], t["quats"], t["opacity"], t["rgb"], t["feat"]


def _upstream(cams, c, seed=1):
    """Per-camera upstream maps and their concatenation (camera order)."""
    per = [scenes.upstream(cam.height, cam.width, c, seed=seed + b) for b, cam in enumerate(cams)]
    flat = {k: torch.tensor(np.concatenate([p[k].reshape(cam.height * cam.width, -1) for p, cam in zip(per, cams)]),
                            device=DEV).squeeze(-1).contiguous() for k in per[0]}
    return per, flat


@pytest.mark.parametrize("blend", ["topk", "full"])
def test_batch_images_equal_single_renders(blend):
    require_gpu()
    sc, cams = _street()
    t = to_dev(sc, "f16")
    K = 8
    out, ws, carr = psm.forward_batch(*_args(t), cams, K, "ellipse", blend)
    torch.cuda.synchronize()
    per = psm.split_images(out, carr)
    cfg = psm.config_struct(K, "ellipse", blend)
    sel = psm.read_selection_batch(ws, carr, cfg) if blend == "topk" else None
    p0 = 0
    for b, cam in enumerate(cams):
        single, ws1 = render(t, cam, K, "ellipse", blend)
        for k in MAPS:
            assert torch.equal(per[b][k], single[k]), (b, k)
        if sel is not None:
            s1 = psm.read_selection(ws1, psm.camera_struct(cam), cfg)
            hw = cam.height * cam.width
            assert torch.equal(sel["sel_id"][p0:p0 + hw].reshape(cam.height, cam.width, K), s1["sel_id"])
            assert torch.equal(sel["sel_w"][p0:p0 + hw].reshape(cam.height, cam.width, K), s1["sel_w"])
        p0 += cam.height * cam.width


def test_batch_keys_match_single(orc):
    require_gpu()
    sc, cams = _street()
    t = to_dev(sc, "f16")
    K = 8
    _, ws, carr = psm.forward_batch(*_args(t), cams, K)
    cfg = psm.config_struct(K)
    got = psm.read_pairs_batch(ws, carr, cfg)
    tile = got["tile"].numpy().astype(np.int64)
    ids = got["id"].numpy().astype(np.int64)
    t0 = 0
    for b, cam in enumerate(cams):
        ntiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
        m = (tile >= t0) & (tile < t0 + ntiles)
        ref = orc.keystage(sc, cam, "ellipse")
        np.testing.assert_array_equal(tile[m] - t0, ref["tile"])
        np.testing.assert_array_equal(ids[m] - b * sc.n, ref["id"])
        vb = slice(b * sc.n, (b + 1) * sc.n)
        np.testing.assert_array_equal(got["count"].numpy()[vb], ref["count"])
        t0 += ntiles
    assert int(m.sum()) > 0 and got["P"] == len(tile)


@pytest.mark.parametrize("blend", ["topk", "full"])
def test_batch_gradients(orc, blend):
    require_gpu()
    sc, cams = _street(n=30_000)
    t = to_dev(sc, "f16")
    K = 8
    feat = stored_feat(t)
    b_or = orc.TOPK if blend == "topk" else orc.FULL
    per_g, _ = _upstream(cams, sc.c)
    # zero upstream on pixels whose decisions sit within rounding of a threshold
    for g, cam in zip(per_g, cams):
        ok = decided(orc.render(sc, cam, K, b_or, feat=feat))
        for k in g:
            g[k][~ok] = 0.0
    flat = {k: torch.tensor(np.concatenate([g[k].reshape(cam.height * cam.width, -1) for g, cam in zip(per_g, cams)]),
                            device=DEV).squeeze(-1).contiguous() for k in per_g[0]}
    cfg = psm.config_struct(K, "ellipse", blend)
    _, ws, carr = psm.forward_batch(*_args(t), cams, K, cfg=cfg)
    got = psm.backward_batch(*_args(t), carr, ws, flat, cfg)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    # against the sum of single-camera backward passes
    tot = {k: 0.0 for k in GROUPS}
    mag = {k: 0.0 for k in GROUPS}
    ref = {k: 0.0 for k in GROUPS}
    for g, cam in zip(per_g, cams):
        _, ws1 = render(t, cam, K, "ellipse", blend)
        gt = {k: torch.tensor(v, device=DEV) for k, v in g.items()}
        one = psm.backward(*_args(t), cam, ws1, gt, K, "ellipse", blend)
        torch.cuda.synchronize()
        r = orc.backward(sc, cam, g, K=K, blend=b_or, feat=feat)
        for k in GROUPS:
            v = one[k].cpu().numpy().astype(np.float64)
            tot[k] = tot[k] + v
            mag[k] = mag[k] + np.abs(v)
            ref[k] = ref[k] + r[k]
    # Both sides add the same FP32 per-pair partial sums, associated
    # differently across cameras; with cancellation inside a camera's sum the
    # rounding scales with the running sums, so the bound is the oracle
    # check's form, ten times tighter.
    for k in GROUPS:
        rms = np.sqrt(np.mean(tot[k] ** 2)) + 1e-30
        err = np.abs(got[k] - tot[k]) / np.maximum(np.abs(tot[k]), 1e-2 * rms)
        assert float(err.max()) <= 1e-4, (k, float(err.max()))
    worst = grad_errors(got, ref)
    assert max(worst.values()) <= 1e-3, worst


CHOICES = [(psm.SCHED_GRID, psm.SCHED_GRID, 32, 16), (psm.SCHED_PERSISTENT, psm.SCHED_PERSISTENT, 32, 16),
           (psm.SCHED_GRID, psm.SCHED_PERSISTENT, 16, 32), (psm.SCHED_PERSISTENT, psm.SCHED_GRID, 16, 32)]


@pytest.mark.parametrize("blend", ["topk", "full"])
def test_launch_choices_are_bit_identical(blend):
    """Scheduler and pass widths change the launch, never a result bit; with
    the dense blend the backward's pass width picks the unit of its feature
    contractions (16: vector FMAs, 32: matrix cores), which orders those sums
    differently: bit-identical within a unit, within FP32 rounding across."""
    require_gpu()
    sc = scenes.planes7(20_000, 40, seed=5)
    cams = [scenes.pinhole(328, 200), scenes.pinhole(100, 60)]
    t = to_dev(sc)
    K = 16
    _, flat = _upstream(cams, sc.c)
    res = []
    for sched, sched_b, bp, gp in CHOICES:
        cfg = psm.config_struct(K, "ellipse", blend, schedule=sched, blend_pass=bp, bwd_pass=gp, bwd_schedule=sched_b)
        out, ws, carr = psm.forward_batch(*_args(t), cams, K, cfg=cfg)
        gr = psm.backward_batch(*_args(t), carr, ws, flat, cfg)
        torch.cuda.synchronize()
        res.append(({k: v.clone() for k, v in out.items()}, gr))
    for i, (out, gr) in enumerate(res[1:], 1):
        for k in MAPS:
            assert torch.equal(out[k], res[0][0][k]), k
        same_unit = blend == "topk" or CHOICES[i][3] == CHOICES[0][3]
        for k in GROUPS:
            if same_unit:
                assert torch.equal(gr[k], res[0][1][k]), (i, k)
            else:
                ref = res[0][1][k]
                scale = torch.clamp(ref.abs(), min=1e-2 * float(ref.pow(2).mean().sqrt()))
                # the gradient parity bar (1e-3 of max(|g|, 1e-2 rms)): FP32 sums of
                # hundreds of mixed-sign terms in another order
                assert float(((gr[k] - ref).abs() / scale).max()) < 1e-3, (i, k)


def test_autotune(tmp_path, monkeypatch):
    require_gpu()
    monkeypatch.setenv("PSM_TUNE_CACHE", str(tmp_path / "tune.json"))
    sc = scenes.planes7(20_000, 32, seed=5)
    cams = psm.camera_array([scenes.pinhole(328, 200)])
    t = to_dev(sc)
    K = 16
    cfg = psm.config_struct(K)
    out, ws, _ = psm.forward_batch(*_args(t), cams, K, cfg=cfg)
    ref = {k: v.clone() for k, v in out.items()}
    _, flat = _upstream([scenes.pinhole(328, 200)], sc.c)
    grads = {k: torch.empty_like(v) for k, v in
             psm.backward_batch(*_args(t), cams, ws, flat, cfg).items()}
    s = psm._surfels(*_args(t))
    ctx = psm.context(0)
    ms = psm.autotune(ctx, s, cams, cfg, ws, out, flat, grads, reps=2)
    assert ms is not None and ms > 0
    assert cfg.schedule in (0, 1) and cfg.bwd_schedule in (0, 1) and cfg.blend_pass in (16, 32)
    assert cfg.bwd_pass in (16, 32)
    cfg2 = psm.config_struct(K)
    assert psm.autotune(ctx, s, cams, cfg2, ws, out, flat, grads) is None  # cached
    assert (cfg2.schedule, cfg2.bwd_schedule, cfg2.blend_pass, cfg2.bwd_pass) == \
        (cfg.schedule, cfg.bwd_schedule, cfg.blend_pass, cfg.bwd_pass)
    psm.forward_batch_into(ctx, s, cams, cfg, ws, out)
    torch.cuda.synchronize()
    for k in MAPS:
        assert torch.equal(out[k], ref[k]), k


@pytest.mark.parametrize("sched", [psm.SCHED_GRID, psm.SCHED_PERSISTENT])
def test_graph_captured_step_replays(sched):
    """Forward + backward captured in one HIP graph (capacity mode, no host
    synchronisation); every replay, with eager work in between, reproduces
    the eager step bit for bit."""
    require_gpu()
    sc, cams = _street(n=30_000)
    t = to_dev(sc, "f16")
    K = 16
    cfg = psm.config_struct(K, "ellipse", "topk", psm.FLAG_NO_SYNC, schedule=sched)
    _, ws0, carr = psm.forward_batch(*_args(t), cams, K, cfg=psm.config_struct(K))
    need = psm.read_stats_batch(ws0, carr, psm.config_struct(K)).pairs_required
    ws = psm.alloc_workspace_batch(sc.n, carr, cfg, sc.c, int(need * 1.2) + 1024, DEV)
    del ws0
    out = psm.alloc_images_batch(carr, sc.c, DEV)
    _, flat = _upstream(cams, sc.c)
    n = sc.n
    z = lambda *s: torch.empty(*s, dtype=torch.float32, device=DEV)
    grads = {"means": z(n, 3), "scales": z(n, 2), "quats": z(n, 4), "opacity": z(n), "rgb": z(n, 3),
             "feat": z(n, sc.c)}
    s = psm._surfels(*_args(t))
    ctx = psm.context(0)

    def step():
        psm.forward_batch_into(ctx, s, carr, cfg, ws, out)
        psm.backward_batch_into(ctx, s, carr, cfg, ws, flat, grads)

    step()
    torch.cuda.synchronize()
    eager = ({k: v.clone() for k, v in out.items()}, {k: v.clone() for k, v in grads.items()})
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for r in range(3):
        for v in list(out.values()) + list(grads.values()):
            v.zero_()
        x = torch.randn(512, 512, device=DEV)
        (x @ x).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for k in MAPS:
            assert torch.equal(out[k], eager[0][k]), (r, k)
        for k in GROUPS:
            assert torch.equal(grads[k], eager[1][k]), (r, k)
    st = psm.read_stats_batch(ws, carr, cfg)
    assert st.pairs_required <= st.pair_capacity
