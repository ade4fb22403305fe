"""ctypes binding of libpsm.so (include/psm.h).

Argument marshalling only: torch provides device memory and the stream;
every step of the render runs in the library's HIP kernels.  There is no
fallback: if libpsm.so is missing or the device is not usable, calls raise.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsm.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_CAPACITY, ERR_HIP = 0, -1, -2, -3, -4
TILE_MODES = {"sphere": 0, "aabb": 1, "ellipse": 2}
BLENDS = {"full": 0, "topk": 1}
DTYPES = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}
FLAG_NO_SYNC = 1
FLAG_PROFILE = 2
FLAG_OPACITY_FOOTPRINT = 4
FLAG_FEATURE_ONLY = 8
FLAG_TOPK_RENORM = 16
FLAG_LOWPASS = 32
NUM_STAGES = 12
SCHED_GRID, SCHED_PERSISTENT = 0, 1
MAX_CAMERAS = 8

# Every symbol include/psm.h declares.
EXPORTS = ("psm_create", "psm_destroy", "psm_workspace_size", "psm_forward", "psm_backward",
           "psm_read_stats", "psm_read_pairs", "psm_read_selection", "psm_profile_read", "psm_profile_reset",
           "psm_last_error", "psm_version", "psm_workspace_size_batch", "psm_forward_batch", "psm_backward_batch",
           "psm_read_stats_batch", "psm_read_pairs_batch", "psm_read_selection_batch", "psm_autotune",
           "psm_instance_labels", "psm_instance_labels_workspace_size", "psm_instance_labels_backward",
           "psm_frustum_attention_workspace_size", "psm_frustum_attention",
           "psm_geometry_loss_workspace_size", "psm_geometry_loss", "psm_forward_static")


class PsmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"psm error {status}: {msg}")
        self.status = status


class CapacityError(PsmError):
    pass


class Surfels(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("rgb", C.c_void_p), ("feat", C.c_void_p), ("c", C.c_int32),
                ("feat_dtype", C.c_int32), ("feat_ext", C.c_void_p), ("c_ext", C.c_int32)]

    @property
    def width(self) -> int:
        """Rendered feature channels: feat's and feat_ext's."""
        return self.c + self.c_ext


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("k", C.c_int32), ("tile_mode", C.c_int32), ("blend", C.c_int32), ("flags", C.c_int32),
                ("schedule", C.c_int32), ("blend_pass", C.c_int32), ("bwd_pass", C.c_int32),
                ("bwd_schedule", C.c_int32), ("tile_w", C.c_int32)]


class Queries(C.Structure):
    _fields_ = [("n_q", C.c_int32), ("c", C.c_int32), ("feat", C.c_void_p), ("mean", C.c_void_p),
                ("prec", C.c_void_p)]


class Attention(C.Structure):
    _fields_ = [("n_q", C.c_int32), ("c", C.c_int32), ("d", C.c_int32), ("feat_dtype", C.c_int32),
                ("feat", C.c_void_p), ("q", C.c_void_p), ("wq", C.c_void_p), ("wk", C.c_void_p), ("wv", C.c_void_p),
                ("pos_length", C.c_float)]


class Gmm(C.Structure):
    _fields_ = [("k", C.c_int32), ("mean", C.c_void_p), ("cov", C.c_void_p), ("weight", C.c_void_p)]


class Images(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("rgb", "depth", "normal", "alpha", "feat")]


class ImageGrads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("rgb", "depth", "normal", "alpha", "feat")]


GRAD_KEYS = ("means", "scales", "quats", "opacity", "rgb", "feat", "feat_ext")


class Grads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in GRAD_KEYS]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("visible", C.c_int64), ("culled", C.c_int64 * 5), ("pairs", C.c_int64),
                ("pairs_required", C.c_int64), ("pair_capacity", C.c_int64), ("tiles", C.c_int64),
                ("pairs_walked", C.c_int64), ("contributors", C.c_int64), ("bwd_entries", C.c_int64),
                ("selected_unique", C.c_int64), ("selections", C.c_int64), ("selected_pairs", C.c_int64)]


_lib = None


def lib():
    """Load libpsm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_10982_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.psm_create.argtypes = [C.POINTER(vp), C.c_int]
        L.psm_destroy.argtypes = [vp]
        L.psm_destroy.restype = None
        L.psm_workspace_size.argtypes = [i64, C.POINTER(Camera), C.POINTER(Config), i32, i64, C.POINTER(C.c_size_t)]
        L.psm_forward.argtypes = [vp, C.POINTER(Surfels), C.POINTER(Camera), C.POINTER(Config), vp, C.c_size_t,
                                  i64, C.POINTER(Images), vp]
        L.psm_backward.argtypes = [vp, C.POINTER(Surfels), C.POINTER(Camera), C.POINTER(Config), vp, C.c_size_t,
                                   i64, C.POINTER(ImageGrads), C.POINTER(Grads), vp]
        L.psm_read_stats.argtypes = [vp, vp, i64, C.POINTER(Camera), C.POINTER(Config), i32, i64,
                                     C.POINTER(Stats), vp]
        L.psm_read_pairs.argtypes = [vp, vp, i64, C.POINTER(Camera), C.POINTER(Config), i32, i64, vp, vp, i64,
                                     vp, vp, vp, C.POINTER(i64), vp]
        L.psm_read_selection.argtypes = [vp, vp, i64, C.POINTER(Camera), C.POINTER(Config), i32, i64, vp, vp,
                                         vp, vp, vp]
        L.psm_forward_static.argtypes = [vp, C.POINTER(Surfels), C.POINTER(Camera), C.POINTER(Config), i64,
                                         C.POINTER(Images), vp]
        CamP, CfgP = C.POINTER(Camera), C.POINTER(Config)
        L.psm_workspace_size_batch.argtypes = [i64, CamP, i32, CfgP, i32, i64, C.POINTER(C.c_size_t)]
        L.psm_forward_batch.argtypes = [vp, C.POINTER(Surfels), CamP, i32, CfgP, vp, C.c_size_t, i64,
                                        C.POINTER(Images), vp]
        L.psm_backward_batch.argtypes = [vp, C.POINTER(Surfels), CamP, i32, CfgP, vp, C.c_size_t, i64,
                                         C.POINTER(ImageGrads), C.POINTER(Grads), vp]
        L.psm_read_stats_batch.argtypes = [vp, vp, i64, CamP, i32, CfgP, i32, i64, C.POINTER(Stats), vp]
        L.psm_read_pairs_batch.argtypes = [vp, vp, i64, CamP, i32, CfgP, i32, i64, vp, vp, i64, vp, vp, vp,
                                           C.POINTER(i64), vp]
        L.psm_read_selection_batch.argtypes = [vp, vp, i64, CamP, i32, CfgP, i32, i64, vp, vp, vp, vp, vp]
        L.psm_autotune.argtypes = [vp, C.POINTER(Surfels), CamP, i32, CfgP, vp, C.c_size_t, i64, C.POINTER(Images),
                                   C.POINTER(ImageGrads), C.POINTER(Grads), i32, C.POINTER(C.c_double), vp]
        QP = C.POINTER(Queries)
        L.psm_instance_labels.argtypes = [vp, i64, vp, vp, i32, QP, vp, i32, vp]
        L.psm_instance_labels_workspace_size.argtypes = [i64, QP, C.POINTER(C.c_size_t)]
        L.psm_instance_labels_backward.argtypes = [vp, i64, vp, vp, i32, QP, vp, i32, vp, C.c_size_t, vp, vp, vp,
                                                   vp, vp, vp]
        GP = C.POINTER(Gmm)
        L.psm_geometry_loss_workspace_size.argtypes = [i64, GP, C.POINTER(C.c_size_t)]
        L.psm_geometry_loss.argtypes = [vp, i64, vp, vp, vp, GP, C.c_float, vp, C.c_size_t, vp, vp, vp, vp, vp, vp]
        AP = C.POINTER(Attention)
        L.psm_frustum_attention_workspace_size.argtypes = [vp, i64, AP, C.POINTER(C.c_size_t)]
        L.psm_frustum_attention.argtypes = [vp, i64, vp, vp, C.POINTER(Camera), AP, vp, C.c_size_t, vp, vp, vp]
        L.psm_profile_read.argtypes = [vp, i32, C.POINTER(C.c_char_p), C.POINTER(C.c_double), C.POINTER(i64)]
        L.psm_profile_reset.argtypes = [vp]
        L.psm_last_error.restype = C.c_char_p
        L.psm_version.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("psm_destroy", "psm_last_error", "psm_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != OK:
        msg = lib().psm_last_error().decode()
        if status == ERR_CAPACITY:
            raise CapacityError(status, f"{what}: {msg}")
        raise PsmError(status, f"{what}: {msg}")


class Context:
    """Library context bound to one HIP device."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(lib().psm_create(C.byref(h), device), "psm_create")
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.psm_destroy(self.handle)
            self.handle = None


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def camera_struct(cam) -> Camera:
    """From a scenes.Camera (or anything with R, t, fx, fy, cx, cy, width, height, near)."""
    c = Camera()
    R = [float(v) for v in torch.as_tensor(cam.R, dtype=torch.float32).reshape(9).tolist()]
    t = [float(v) for v in torch.as_tensor(cam.t, dtype=torch.float32).reshape(3).tolist()]
    c.R[:] = R
    c.t[:] = t
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.near_plane = float(getattr(cam, "near", 0.2))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def config_struct(k: int, tile_mode="ellipse", blend="topk", flags: int = 0, schedule: int = SCHED_GRID,
                  blend_pass: int = 0, bwd_pass: int = 0, bwd_schedule: int | None = None,
                  tile_w: int = 0) -> Config:
    """bwd_schedule defaults to the forward's schedule; tile_w 0 = 16 x 16
    tiles (else tile_w x 256 / tile_w, tile_w in 8, 16, 32, 64)."""
    tm = TILE_MODES[tile_mode] if isinstance(tile_mode, str) else int(tile_mode)
    bl = BLENDS[blend] if isinstance(blend, str) else int(blend)
    bs = int(schedule) if bwd_schedule is None else int(bwd_schedule)
    return Config(int(k), tm, bl, int(flags), int(schedule), int(blend_pass), int(bwd_pass), bs, int(tile_w))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Workspace:
    """Caller-owned device workspace; also the state saved for the backward."""
    buf: torch.Tensor
    capacity: int
    n: int
    c: int
    k: int
    tile_w: int = 0

    @property
    def nbytes(self) -> int:
        return self.buf.numel()


def workspace_size(n: int, cam: Camera, cfg: Config, c: int, capacity: int) -> int:
    out = C.c_size_t()
    _check(lib().psm_workspace_size(n, C.byref(cam), C.byref(cfg), c, capacity, C.byref(out)), "psm_workspace_size")
    return int(out.value)


def alloc_workspace(n, cam: Camera, cfg: Config, c: int, capacity: int, device) -> Workspace:
    nbytes = workspace_size(n, cam, cfg, c, capacity)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return Workspace(buf[off:off + nbytes], capacity, n, c, cfg.k, int(cfg.tile_w))


def alloc_workspace_shapes(n, cams, cfg: Config, c: int, capacity: int, device, tile_ws=(8, 16, 32, 64)) -> Workspace:
    """A workspace that holds the layout of every listed tile width (for the
    autotuner, which times each shape in the same workspace)."""
    carr = camera_array(list(cams))
    nbytes = 0
    for tw in tile_ws:
        c2 = Config.from_buffer_copy(cfg)
        c2.tile_w = int(tw)
        nbytes = max(nbytes, workspace_size_batch(n, carr, c2, c, capacity))
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return Workspace(buf[off:off + nbytes], capacity, n, c, cfg.k, int(cfg.tile_w))


def _surfels(means, scales, quats, opacity, rgb, feat, feat_ext=None) -> Surfels:
    n = means.shape[0]
    for name, t, w in (("means", means, 3), ("scales", scales, 2), ("quats", quats, 4), ("rgb", rgb, 3)):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (n, w):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape ({n}, {w})")
    if opacity.dtype != torch.float32 or not opacity.is_cuda or not opacity.is_contiguous() or opacity.numel() != n:
        raise ValueError("opacity must be a contiguous float32 CUDA tensor of shape (n,)")
    c, dt, fp = 0, 0, None
    if feat is not None:
        if (feat.dtype not in DTYPES or not feat.is_cuda or not feat.is_contiguous() or feat.dim() != 2
                or feat.shape[0] != n):
            raise ValueError("feat must be a contiguous (n, C) float32/float16/bfloat16 CUDA tensor")
        c, dt, fp = int(feat.shape[1]), DTYPES[feat.dtype], feat.data_ptr()
    ce, ep = 0, None
    if feat_ext is not None:
        if (feat_ext.dtype != torch.float32 or not feat_ext.is_cuda or not feat_ext.is_contiguous()
                or feat_ext.dim() != 2 or feat_ext.shape[0] != n):
            raise ValueError("feat_ext must be a contiguous (n, C_ext) float32 CUDA tensor")
        ce, ep = int(feat_ext.shape[1]), feat_ext.data_ptr()
    return Surfels(n, means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opacity.data_ptr(), rgb.data_ptr(),
                   fp, c, dt, ep, ce)


def alloc_images(cam: Camera, c: int, device, feature_only: bool = False) -> dict:
    """Output maps; with ``feature_only`` (FLAG_FEATURE_ONLY) only the feature map."""
    H, W = cam.height, cam.width
    e = lambda *s: torch.empty(*s, dtype=torch.float32, device=device)
    if feature_only:
        return {"rgb": None, "depth": None, "normal": None, "alpha": None, "feat": e(H, W, c)}
    return {"rgb": e(H, W, 3), "depth": e(H, W), "normal": e(H, W, 3), "alpha": e(H, W),
            "feat": e(H, W, c) if c > 0 else None}


def capacity_guess(n: int, cam: Camera) -> int:
    tiles = math.ceil(cam.width / 16) * math.ceil(cam.height / 16)
    return int(min(2**31 - 1, 8 * n + 4 * tiles + 1024))


def forward_into(ctx: Context, s: Surfels, cam: Camera, cfg: Config, ws: Workspace, out: dict, stream=None):
    """Raw forward into preallocated outputs (no allocation, no retry)."""
    imgs = Images(*(_ptr(out.get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    st = stream if stream is not None else _stream(ctx.device)
    _check(lib().psm_forward(ctx.handle, C.byref(s), C.byref(cam), C.byref(cfg), _ptr(ws.buf), ws.nbytes,
                             ws.capacity, C.byref(imgs), st), "psm_forward")


STATIC_WORKSPACE_BYTES = 64 << 20


def forward_static_into(ctx: Context, s: Surfels, cam: Camera, cfg: Config, out: dict, pair_capacity: int = -1,
                        stream=None):
    """psm_forward_static: the forward with the library's static device
    workspace (no caller workspace, no device allocation)."""
    imgs = Images(*(_ptr(out.get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    st = stream if stream is not None else _stream(ctx.device)
    _check(lib().psm_forward_static(ctx.handle, C.byref(s), C.byref(cam), C.byref(cfg), int(pair_capacity),
                                    C.byref(imgs), st), "psm_forward_static")


def backward_into(ctx: Context, s: Surfels, cam: Camera, cfg: Config, ws: Workspace, gout: dict, grads: dict,
                  stream=None):
    g = ImageGrads(*(_ptr(gout.get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    gr = Grads(*(_ptr(grads.get(k)) for k in GRAD_KEYS))
    st = stream if stream is not None else _stream(ctx.device)
    _check(lib().psm_backward(ctx.handle, C.byref(s), C.byref(cam), C.byref(cfg), _ptr(ws.buf), ws.nbytes,
                              ws.capacity, C.byref(g), C.byref(gr), st), "psm_backward")


def launch_config(k: int, tile_mode="ellipse", blend="topk", flags: int = 0, launch=None) -> Config:
    """Config with the launch choices ``launch`` = (schedule, bwd_schedule,
    blend_pass, bwd_pass[, tile_w]), or the defaults (grid schedules, default
    passes, 16 x 16 tiles)."""
    if launch is None:
        return config_struct(k, tile_mode, blend, flags)
    v = [int(x) for x in launch]
    sched, bsched, bp, fp = v[:4]
    tw = v[4] if len(v) > 4 else 0
    return config_struct(k, tile_mode, blend, flags, sched, bp, fp, bsched, tw)


def forward(means, scales, quats, opacity, rgb, feat, camera, k=16, tile_mode="ellipse", blend="topk",
            capacity: int | None = None, ws: Workspace | None = None, flags: int = 0, launch=None, feat_ext=None):
    """Render; returns (images dict, workspace).  The workspace holds the
    state the backward needs.  Re-allocates once if the pairs do not fit.
    ``flags``: FLAG_* options of the key stage and the walks (e.g.
    FLAG_OPACITY_FOOTPRINT); the backward takes the same flags.  ``launch``:
    (schedule, bwd_schedule, blend_pass, bwd_pass), see launch_config.
    ``feat_ext``: optional FP32 (n, C_ext) features blended after ``feat``'s
    channels by the same walk (the feature map has C + C_ext channels)."""
    device = means.device
    ctx = context(device.index or 0)
    s = _surfels(means, scales, quats, opacity, rgb, feat, feat_ext)
    cam = camera if isinstance(camera, Camera) else camera_struct(camera)
    cfg = launch_config(k, tile_mode, blend, flags, launch)
    out = alloc_images(cam, s.width, device, feature_only=bool(flags & FLAG_FEATURE_ONLY))
    cap = capacity if capacity is not None else (ws.capacity if ws is not None else capacity_guess(s.n, cam))
    for attempt in range(3):
        if (ws is None or ws.capacity < cap or ws.n != s.n or ws.c != s.width or ws.k != cfg.k
                or ws.tile_w != cfg.tile_w):
            ws = alloc_workspace(s.n, cam, cfg, s.width, cap, device)
        try:
            forward_into(ctx, s, cam, cfg, ws, out)
            return out, ws
        except CapacityError:
            st = read_stats(ws, s.n, cam, cfg, s.width, ws.capacity, device)
            cap = int(min(2**31 - 1, st.pairs_required * 1.15 + 1024))
            ws = None
    raise RuntimeError("pair capacity could not be satisfied")


def backward(means, scales, quats, opacity, rgb, feat, camera, ws: Workspace, gout: dict, k=16,
             tile_mode="ellipse", blend="topk", flags: int = 0, launch=None, feat_ext=None) -> dict:
    device = means.device
    ctx = context(device.index or 0)
    s = _surfels(means, scales, quats, opacity, rgb, feat, feat_ext)
    cam = camera if isinstance(camera, Camera) else camera_struct(camera)
    cfg = launch_config(k, tile_mode, blend, flags, launch)
    n = s.n
    z = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=device)
    grads = {"means": z(n, 3), "scales": z(n, 2), "quats": z(n, 4), "opacity": z(n), "rgb": z(n, 3),
             "feat": z(n, s.c) if s.c > 0 else None}
    if s.c_ext > 0:  # the second source's gradient, only when there is one
        grads["feat_ext"] = z(n, s.c_ext)
    gout = {kk: (None if v is None else v.contiguous().float()) for kk, v in gout.items()}
    if flags & FLAG_FEATURE_ONLY:  # only the feature map was rendered
        gout = {kk: (v if kk == "feat" else None) for kk, v in gout.items()}
    backward_into(ctx, s, cam, cfg, ws, gout, grads)
    return grads


def read_stats(ws: Workspace, n, cam: Camera, cfg: Config, c, capacity, device=None) -> Stats:
    ctx = context(ws.buf.device.index or 0)
    st = Stats()
    _check(lib().psm_read_stats(ctx.handle, _ptr(ws.buf), n, C.byref(cam), C.byref(cfg), c, capacity, C.byref(st),
                                _stream(ctx.device)), "psm_read_stats")
    return st


def read_pairs(ws: Workspace, cam: Camera, cfg: Config) -> dict:
    """Sorted pair list and per-surfel key-stage results, as CPU tensors."""
    ctx = context(ws.buf.device.index or 0)
    dev = ws.buf.device
    st = read_stats(ws, ws.n, cam, cfg, ws.c, ws.capacity)
    P = int(st.pairs)
    tile = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    ids = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    n = max(ws.n, 1)
    cull = torch.empty(n, dtype=torch.int32, device=dev)
    depth = torch.empty(n, dtype=torch.int32, device=dev)
    count = torch.empty(n, dtype=torch.int32, device=dev)
    got = C.c_int64()
    _check(lib().psm_read_pairs(ctx.handle, _ptr(ws.buf), ws.n, C.byref(cam), C.byref(cfg), ws.c, ws.capacity,
                                _ptr(tile), _ptr(ids), P, _ptr(cull), _ptr(depth), _ptr(count), C.byref(got),
                                _stream(ctx.device)), "psm_read_pairs")
    return {"P": int(got.value), "tile": tile[:P].cpu(), "id": ids[:P].cpu(), "cull": cull[:ws.n].cpu(),
            "depth_bits": depth[:ws.n].cpu().view(torch.int32), "count": count[:ws.n].cpu(), "stats": st}


def read_selection(ws: Workspace, cam: Camera, cfg: Config) -> dict:
    ctx = context(ws.buf.device.index or 0)
    dev = ws.buf.device
    H, W, K = cam.height, cam.width, cfg.k
    sid = torch.empty(H, W, K, dtype=torch.int32, device=dev)
    sw = torch.empty(H, W, K, dtype=torch.float32, device=dev)
    nl = torch.empty(H, W, dtype=torch.int32, device=dev)
    tf = torch.empty(H, W, dtype=torch.float32, device=dev)
    _check(lib().psm_read_selection(ctx.handle, _ptr(ws.buf), ws.n, C.byref(cam), C.byref(cfg), ws.c, ws.capacity,
                                    _ptr(sid), _ptr(sw), _ptr(nl), _ptr(tf), _stream(ctx.device)),
           "psm_read_selection")
    return {"sel_id": sid, "sel_w": sw, "n_last": nl, "T_final": tf}


def profile_read(ctx: Context) -> dict:
    """{stage name: (total ms, calls)} accumulated since the last reset."""
    out = {}
    for i in range(NUM_STAGES):
        name, ms, calls = C.c_char_p(), C.c_double(), C.c_int64()
        _check(lib().psm_profile_read(ctx.handle, i, C.byref(name), C.byref(ms), C.byref(calls)), "psm_profile_read")
        out[name.value.decode()] = (float(ms.value), int(calls.value))
    return out


def profile_reset(ctx: Context):
    _check(lib().psm_profile_reset(ctx.handle), "psm_profile_reset")


def version() -> str:
    return lib().psm_version().decode()


# ------------------------------------------------------------ camera batches
def camera_array(cams) -> C.Array:
    """ctypes array of Camera from scenes.Camera objects (or Camera structs)."""
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, Camera) else camera_struct(c)
    return arr


def _cam_ptr(cams: C.Array):
    return C.cast(cams, C.POINTER(Camera))


def workspace_size_batch(n: int, cams: C.Array, cfg: Config, c: int, capacity: int) -> int:
    out = C.c_size_t()
    _check(lib().psm_workspace_size_batch(n, _cam_ptr(cams), len(cams), C.byref(cfg), c, capacity, C.byref(out)),
           "psm_workspace_size_batch")
    return int(out.value)


def alloc_workspace_batch(n, cams: C.Array, cfg: Config, c: int, capacity: int, device) -> Workspace:
    nbytes = workspace_size_batch(n, cams, cfg, c, capacity)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return Workspace(buf[off:off + nbytes], capacity, n, c, cfg.k, int(cfg.tile_w))


def total_pixels(cams: C.Array) -> int:
    return sum(int(c.width) * int(c.height) for c in cams)


def alloc_images_batch(cams: C.Array, c: int, device) -> dict:
    """Concatenated maps of all cameras: (sum W*H, channels)."""
    P = total_pixels(cams)
    e = lambda *s: torch.empty(*s, dtype=torch.float32, device=device)
    return {"rgb": e(P, 3), "depth": e(P), "normal": e(P, 3), "alpha": e(P), "feat": e(P, c) if c > 0 else None}


def split_images(maps: dict, cams: C.Array) -> list:
    """Per-camera (H, W, ...) views of concatenated maps."""
    out, p = [], 0
    for cam in cams:
        H, W = int(cam.height), int(cam.width)
        out.append({k: None if v is None else v[p:p + H * W].reshape(H, W, *v.shape[1:]) for k, v in maps.items()})
        p += H * W
    return out


def capacity_guess_batch(n: int, cams: C.Array) -> int:
    return int(min(2**31 - 1, sum(capacity_guess(n, c) for c in cams)))


def forward_batch_into(ctx: Context, s: Surfels, cams: C.Array, cfg: Config, ws: Workspace, out: dict,
                       stream=None):
    imgs = Images(*(_ptr(out.get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    st = stream if stream is not None else _stream(ctx.device)
    _check(lib().psm_forward_batch(ctx.handle, C.byref(s), _cam_ptr(cams), len(cams), C.byref(cfg), _ptr(ws.buf),
                                   ws.nbytes, ws.capacity, C.byref(imgs), st), "psm_forward_batch")


def backward_batch_into(ctx: Context, s: Surfels, cams: C.Array, cfg: Config, ws: Workspace, gout: dict,
                        grads: dict, stream=None):
    g = ImageGrads(*(_ptr(gout.get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    gr = Grads(*(_ptr(grads.get(k)) for k in GRAD_KEYS))
    st = stream if stream is not None else _stream(ctx.device)
    _check(lib().psm_backward_batch(ctx.handle, C.byref(s), _cam_ptr(cams), len(cams), C.byref(cfg),
                                    _ptr(ws.buf), ws.nbytes, ws.capacity, C.byref(g), C.byref(gr), st),
           "psm_backward_batch")


def read_stats_batch(ws: Workspace, cams: C.Array, cfg: Config) -> Stats:
    ctx = context(ws.buf.device.index or 0)
    st = Stats()
    _check(lib().psm_read_stats_batch(ctx.handle, _ptr(ws.buf), ws.n, _cam_ptr(cams), len(cams), C.byref(cfg),
                                      ws.c, ws.capacity, C.byref(st), _stream(ctx.device)), "psm_read_stats_batch")
    return st


def forward_batch(means, scales, quats, opacity, rgb, feat, cams, k=16, tile_mode="ellipse", blend="topk",
                  cfg: Config | None = None, capacity: int | None = None, ws: Workspace | None = None,
                  feat_ext=None):
    """Render several cameras in one call; returns (concatenated maps, workspace, camera array)."""
    device = means.device
    ctx = context(device.index or 0)
    s = _surfels(means, scales, quats, opacity, rgb, feat, feat_ext)
    cams = cams if isinstance(cams, C.Array) else camera_array(cams)
    cfg = cfg if cfg is not None else config_struct(k, tile_mode, blend)
    out = alloc_images_batch(cams, s.width, device)
    cap = capacity if capacity is not None else (ws.capacity if ws is not None else capacity_guess_batch(s.n, cams))
    for attempt in range(3):
        if (ws is None or ws.capacity < cap or ws.n != s.n or ws.c != s.width or ws.k != cfg.k
                or ws.tile_w != cfg.tile_w):
            ws = alloc_workspace_batch(s.n, cams, cfg, s.width, cap, device)
        try:
            forward_batch_into(ctx, s, cams, cfg, ws, out)
            return out, ws, cams
        except CapacityError:
            st = read_stats_batch(ws, cams, cfg)
            cap = int(min(2**31 - 1, st.pairs_required * 1.15 + 1024))
            ws = None
    raise RuntimeError("pair capacity could not be satisfied")


def backward_batch(means, scales, quats, opacity, rgb, feat, cams: C.Array, ws: Workspace, gout: dict,
                   cfg: Config, feat_ext=None) -> dict:
    device = means.device
    ctx = context(device.index or 0)
    s = _surfels(means, scales, quats, opacity, rgb, feat, feat_ext)
    n = s.n
    z = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=device)
    grads = {"means": z(n, 3), "scales": z(n, 2), "quats": z(n, 4), "opacity": z(n), "rgb": z(n, 3),
             "feat": z(n, s.c) if s.c > 0 else None}
    if s.c_ext > 0:  # the second source's gradient, only when there is one
        grads["feat_ext"] = z(n, s.c_ext)
    gout = {kk: (None if v is None else v.contiguous().float()) for kk, v in gout.items()}
    backward_batch_into(ctx, s, cams, cfg, ws, gout, grads)
    return grads


def read_pairs_batch(ws: Workspace, cams: C.Array, cfg: Config) -> dict:
    """Sorted pair list (global tile ids, virtual surfel ids b * n + i) and
    per-virtual-surfel key-stage results, as CPU tensors."""
    ctx = context(ws.buf.device.index or 0)
    dev = ws.buf.device
    st = read_stats_batch(ws, cams, cfg)
    P = int(st.pairs)
    nv = ws.n * len(cams)
    tile = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    ids = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    cull = torch.empty(max(nv, 1), dtype=torch.int32, device=dev)
    depth = torch.empty(max(nv, 1), dtype=torch.int32, device=dev)
    count = torch.empty(max(nv, 1), dtype=torch.int32, device=dev)
    got = C.c_int64()
    _check(lib().psm_read_pairs_batch(ctx.handle, _ptr(ws.buf), ws.n, _cam_ptr(cams), len(cams), C.byref(cfg),
                                      ws.c, ws.capacity, _ptr(tile), _ptr(ids), P, _ptr(cull), _ptr(depth),
                                      _ptr(count), C.byref(got), _stream(ctx.device)), "psm_read_pairs_batch")
    return {"P": int(got.value), "tile": tile[:P].cpu(), "id": ids[:P].cpu(), "cull": cull[:nv].cpu(),
            "depth_bits": depth[:nv].cpu(), "count": count[:nv].cpu(), "stats": st}


def read_selection_batch(ws: Workspace, cams: C.Array, cfg: Config) -> dict:
    ctx = context(ws.buf.device.index or 0)
    dev = ws.buf.device
    P, K = total_pixels(cams), cfg.k
    sid = torch.empty(P, K, dtype=torch.int32, device=dev)
    sw = torch.empty(P, K, dtype=torch.float32, device=dev)
    nl = torch.empty(P, dtype=torch.int32, device=dev)
    tf = torch.empty(P, dtype=torch.float32, device=dev)
    _check(lib().psm_read_selection_batch(ctx.handle, _ptr(ws.buf), ws.n, _cam_ptr(cams), len(cams),
                                          C.byref(cfg), ws.c, ws.capacity, _ptr(sid), _ptr(sw), _ptr(nl), _ptr(tf),
                                          _stream(ctx.device)), "psm_read_selection_batch")
    return {"sel_id": sid, "sel_w": sw, "n_last": nl, "T_final": tf}


# ---------------------------------------------------------------- autotuner
def tune_cache_path() -> str:
    return os.environ.get("PSM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "psm", "tune.json"))


def _tune_key(s: Surfels, cams, cfg: Config, bwd: bool) -> str:
    dims = ",".join(f"{int(c.width)}x{int(c.height)}" for c in cams)
    return f"n={s.n};c={s.c}+{s.c_ext};dt={s.feat_dtype};k={cfg.k};tm={cfg.tile_mode};bl={cfg.blend};bwd={int(bwd)};cams={dims}"


def autotune(ctx: Context, s: Surfels, cams: C.Array, cfg: Config, ws: Workspace, out: dict,
             gout: dict | None = None, grads: dict | None = None, reps: int = 3, cache: bool = True) -> float | None:
    """Pick the launch choices for these shapes (the library times the
    candidates) and write them into cfg.  Choices persist in a JSON file
    (PSM_TUNE_CACHE); returns the best time in ms, or None on a cache hit."""
    bwd = grads is not None
    key = _tune_key(s, cams, cfg, bwd)
    path = tune_cache_path()
    table = {}
    if cache and os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if cache and key in table and len(table[key]) == 5:
        cfg.schedule, cfg.bwd_schedule, cfg.blend_pass, cfg.bwd_pass, cfg.tile_w = (int(v) for v in table[key])
        return None
    imgs = Images(*(_ptr(out.get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    g = ImageGrads(*(_ptr((gout or {}).get(k)) for k in ("rgb", "depth", "normal", "alpha", "feat")))
    gr = Grads(*(_ptr((grads or {}).get(k)) for k in GRAD_KEYS))
    best = C.c_double()
    _check(lib().psm_autotune(ctx.handle, C.byref(s), _cam_ptr(cams), len(cams), C.byref(cfg), _ptr(ws.buf),
                              ws.nbytes, ws.capacity, C.byref(imgs), C.byref(g) if bwd else None,
                              C.byref(gr) if bwd else None, int(reps), C.byref(best), _stream(ctx.device)),
           "psm_autotune")
    if cache:
        table[key] = [int(cfg.schedule), int(cfg.bwd_schedule), int(cfg.blend_pass), int(cfg.bwd_pass),
                      int(cfg.tile_w)]
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".tmp{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass
    return float(best.value)


# ------------------------------------------------------------ instance labels
def label_width(n_q: int) -> int:
    """Feature columns the labels of n_q queries occupy (n_q rounded up to 8)."""
    return (int(n_q) + 7) // 8 * 8


def _queries(q_feat, q_mean, q_prec) -> Queries:
    nq = q_feat.shape[0]
    for name, t, w in (("q_feat", q_feat, q_feat.shape[1]), ("q_mean", q_mean, 3), ("q_prec", q_prec, 6)):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (nq, w):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape ({nq}, {w})")
    return Queries(int(nq), int(q_feat.shape[1]), q_feat.data_ptr(), q_mean.data_ptr(), q_prec.data_ptr())


def _check_surfel_side(means, f_ins):
    n = means.shape[0]
    if means.dtype != torch.float32 or not means.is_cuda or not means.is_contiguous() or tuple(means.shape) != (n, 3):
        raise ValueError("means must be a contiguous float32 CUDA tensor of shape (n, 3)")
    if f_ins.dtype not in DTYPES or not f_ins.is_cuda or not f_ins.is_contiguous() or f_ins.shape[0] != n:
        raise ValueError("f_ins must be a contiguous (n, c) float32/float16/bfloat16 CUDA tensor")


def instance_labels_into(means, f_ins, q_feat, q_mean, q_prec, out: torch.Tensor, ld: int, stream=None):
    """Labels into out (FP32, row stride ld; out may be a column slice of a
    larger feature array whose row stride is ld)."""
    _check_surfel_side(means, f_ins)
    q = _queries(q_feat, q_mean, q_prec)
    ctx = context(means.device.index or 0)
    st = stream if stream is not None else _stream(ctx.device)
    _check(lib().psm_instance_labels(ctx.handle, means.shape[0], _ptr(means), _ptr(f_ins), DTYPES[f_ins.dtype],
                                     C.byref(q), C.c_void_p(out.data_ptr()), int(ld), st), "psm_instance_labels")


def instance_labels(means, f_ins, q_feat, q_mean, q_prec) -> torch.Tensor:
    """(n, label_width(n_q)) FP32 labels; columns >= n_q are zero."""
    out = torch.empty(means.shape[0], label_width(q_feat.shape[0]), dtype=torch.float32, device=means.device)
    instance_labels_into(means, f_ins, q_feat, q_mean, q_prec, out, out.shape[1])
    return out


def instance_labels_backward(means, f_ins, q_feat, q_mean, q_prec, d_labels: torch.Tensor, ld: int) -> dict:
    _check_surfel_side(means, f_ins)
    q = _queries(q_feat, q_mean, q_prec)
    ctx = context(means.device.index or 0)
    dev = means.device
    ws_bytes = C.c_size_t()
    _check(lib().psm_instance_labels_workspace_size(means.shape[0], C.byref(q), C.byref(ws_bytes)),
           "psm_instance_labels_workspace_size")
    buf = torch.empty(int(ws_bytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    ws = buf[off:off + int(ws_bytes.value)]
    n, nq, c = means.shape[0], q_feat.shape[0], q_feat.shape[1]
    z = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=dev)
    g = {"means": z(n, 3), "f_ins": z(n, c), "q_feat": z(nq, c), "q_mean": z(nq, 3), "q_prec": z(nq, 6)}
    _check(lib().psm_instance_labels_backward(ctx.handle, n, _ptr(means), _ptr(f_ins), DTYPES[f_ins.dtype],
                                              C.byref(q), C.c_void_p(d_labels.data_ptr()), int(ld), _ptr(ws),
                                              ws.numel(), _ptr(g["means"]), _ptr(g["f_ins"]), _ptr(g["q_feat"]),
                                              _ptr(g["q_mean"]), _ptr(g["q_prec"]), _stream(ctx.device)),
           "psm_instance_labels_backward")
    return g


# ------------------------------------------------------------ frustum attention
def _attention(feat, q, wq, wk, wv, pos_length) -> Attention:
    for name, t in (("feat", feat), ("q", q), ("wq", wq), ("wk", wk), ("wv", wv)):
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    for name, t in (("q", q), ("wq", wq), ("wk", wk), ("wv", wv)):
        if t.dtype != torch.float32:
            raise ValueError(f"{name} must be float32")
    return Attention(int(q.shape[0]), int(q.shape[1]), int(wq.shape[1]), DTYPES[feat.dtype], _ptr(feat), _ptr(q),
                     _ptr(wq), _ptr(wk), _ptr(wv), float(pos_length))


def frustum_attention(means, scales, feat, q, wq, wk, wv, camera, pos_length: float, return_active: bool = False):
    """Cross-attention of the queries q [n_q, C] over the surfels whose 99%
    disk meets the camera's frustum (Sec. 4.1, eqs. (9)-(11)): [n_q, d] FP32,
    and with ``return_active`` the uint8 active mask [n]."""
    dev = means.device
    ctx = context(dev.index or 0)
    cam = camera if isinstance(camera, Camera) else camera_struct(camera)
    a = _attention(feat, q, wq, wk, wv, pos_length)
    n = int(means.shape[0])
    ws_bytes = C.c_size_t()
    _check(lib().psm_frustum_attention_workspace_size(ctx.handle, n, C.byref(a), C.byref(ws_bytes)),
           "psm_frustum_attention_workspace_size")
    buf = torch.empty(int(ws_bytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    ws = buf[off:off + int(ws_bytes.value)]
    out = torch.empty(a.n_q, a.d, dtype=torch.float32, device=dev)
    act = torch.empty(max(n, 1), dtype=torch.uint8, device=dev) if return_active else None
    _check(lib().psm_frustum_attention(ctx.handle, n, _ptr(means), _ptr(scales), C.byref(cam), C.byref(a), _ptr(ws),
                                       ws.numel(), _ptr(out), _ptr(act), _stream(ctx.device)),
           "psm_frustum_attention")
    return (out, act[:n]) if return_active else out


# ------------------------------------------------------------ geometric loss
def geometry_loss(means, scales, quats, g_mean, g_cov, g_weight, lambda_n: float, return_assign: bool = False):
    """SOGMM geometric loss (eq. (3), eq. (13)) and anisotropy term: returns
    {"geo", "iso" (FP64 device scalars), "d_means", "d_scales", "d_quats"} and
    with ``return_assign`` the int32 component of every surfel."""
    for name, t in (("means", means), ("scales", scales), ("quats", quats), ("g_mean", g_mean), ("g_cov", g_cov),
                    ("g_weight", g_weight)):
        if not t.is_contiguous() or t.dtype != torch.float32:
            raise ValueError(f"{name} must be contiguous float32")
    dev = means.device
    ctx = context(dev.index or 0)
    n = int(means.shape[0])
    g = Gmm(int(g_mean.shape[0]), _ptr(g_mean), _ptr(g_cov), _ptr(g_weight))
    ws_bytes = C.c_size_t()
    _check(lib().psm_geometry_loss_workspace_size(n, C.byref(g), C.byref(ws_bytes)), "psm_geometry_loss_workspace_size")
    buf = torch.empty(int(ws_bytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    ws = buf[off:off + int(ws_bytes.value)]
    losses = torch.empty(2, dtype=torch.float64, device=dev)
    z = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=dev)
    out = {"d_means": z(n, 3), "d_scales": z(n, 2), "d_quats": z(n, 4)}
    asg = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if return_assign else None
    _check(lib().psm_geometry_loss(ctx.handle, n, _ptr(means), _ptr(scales), _ptr(quats), C.byref(g),
                                   float(lambda_n), _ptr(ws), ws.numel(), _ptr(losses), _ptr(asg),
                                   _ptr(out["d_means"]), _ptr(out["d_scales"]), _ptr(out["d_quats"]),
                                   _stream(ctx.device)), "psm_geometry_loss")
    out["geo"], out["iso"] = losses[0], losses[1]
    if return_assign:
        out["assign"] = asg[:n]
    return out
