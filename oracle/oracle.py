"""ctypes bindings of the CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here imports the HIP package;
features arrive already rounded to their storage dtype, as float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.cpp")

SPHERE, AABB, ELLIPSE = 0, 1, 2
FULL, TOPK = 0, 1
# Top-K with the feature-only stop: a pixel's walk ends once no later surfel can
# enter its K largest weights (selection and feature map unchanged).
TOPK_FEATURE_ONLY = 2
# Top-K with the selected weights renormalised to sum 1 (F = sum w f / sum w).
TOPK_RENORM = 3
MODES = {"sphere": SPHERE, "aabb": AABB, "ellipse": ELLIPSE}

_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile liboracle.so (g++, FP64 model + FP32 key stage, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["g++", "-std=c++17", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", SRC, "-o", f"{LIB_PATH}.tmp{os.getpid()}"]
        subprocess.run(cmd, check=True)
        os.replace(f"{LIB_PATH}.tmp{os.getpid()}", LIB_PATH)  # several test workers may build at once
    return LIB_PATH


def _vp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.orc_keystage.restype = i64
        L.orc_keystage.argtypes = [i64, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, i64, vp, vp]
        L.orc_eval_points.restype = None
        L.orc_eval_points.argtypes = [i64, vp, vp, vp, vp, i64, vp, vp, vp, vp]
        L.orc_render.restype = None
        L.orc_render.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, vp, i32, i32, i32, i32, i32, i64, vp,
                                 vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_backward.restype = None
        L.orc_backward.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, vp, i32, i32, i32, i32, i32, i64, vp,
                                   vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_decisions.restype = None
        L.orc_decisions.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, vp, i32, i32, i32, i32, i32, i64, vp, vp]
        L.orc_num_threads.restype = i32
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [i32]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only)."""
    lib().orc_set_threads(int(n))


def _c32(a):
    return np.ascontiguousarray(a, np.float32)


def _scene_args(scene):
    return (_c32(scene.means), _c32(scene.scales), _c32(scene.quats))


def keystage(scene, cam, mode="ellipse", tile=16, pairs=True, opacity_footprint=False, lowpass=False) -> dict:
    """FP32 key stage: cull codes, depth bits, flips, counts, footprint floats
    and (optionally) the sorted pair list (tile ids, surfel ids).
    ``tile``: the tile size (square) or its (width, height).
    ``opacity_footprint``: list the footprint of rho <= min(9, 2 ln(255 o))
    (widened and rounded up, see oracle.cpp) instead of rho <= 9.
    ``lowpass``: the footprint also covers the screen-space low-pass filter's
    disk 2 |x - c|^2 <= 9 (widened, see oracle.cpp)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    tw, th = (tile, tile) if np.isscalar(tile) else (int(tile[0]), int(tile[1]))
    n = scene.n
    mu, sc, q = _scene_args(scene)
    op = _c32(scene.opacity) if opacity_footprint else None
    camv = cam.as_array()
    cull = np.zeros(n, np.int32)
    depth = np.zeros(n, np.uint32)
    flip = np.zeros(n, np.int32)
    count = np.zeros(n, np.int32)
    fp = np.zeros((n, 8), np.float32)
    L = lib()
    P = L.orc_keystage(n, _vp(mu), _vp(sc), _vp(q), _vp(op), _vp(camv), tw, th, m, int(lowpass),
                       _vp(cull), _vp(depth), _vp(flip), _vp(count), _vp(fp), 0, None, None)
    out = {"cull": cull, "depth_bits": depth, "flip": flip, "count": count, "fp": fp, "P": int(P)}
    if pairs:
        tiles = np.zeros(max(P, 1), np.int32)
        ids = np.zeros(max(P, 1), np.int32)
        L.orc_keystage(n, _vp(mu), _vp(sc), _vp(q), _vp(op), _vp(camv), tw, th, m, int(lowpass),
                       None, None, None, None, None, P, _vp(tiles), _vp(ids))
        out["tile"] = tiles[:P]
        out["id"] = ids[:P]
    return out


def eval_points(scene, cam, xs, ys):
    """FP64 rho and intersection depth of every surfel at the given image points."""
    mu, sc, q = _scene_args(scene)
    xs = np.ascontiguousarray(xs, np.float64)
    ys = np.ascontiguousarray(ys, np.float64)
    rho = np.zeros((scene.n, xs.size), np.float64)
    z = np.zeros((scene.n, xs.size), np.float64)
    lib().orc_eval_points(scene.n, _vp(mu), _vp(sc), _vp(q), _vp(cam.as_array()), xs.size,
                          _vp(xs), _vp(ys), _vp(rho), _vp(z))
    return rho, z


def _pix(pix):
    return None if pix is None else np.ascontiguousarray(pix, np.int64)


def render(scene, cam, K=16, blend=TOPK, feat=None, pix=None, tile=16, lowpass=False) -> dict:
    """FP64 forward render.  ``feat`` overrides scene.feat (e.g. the values of
    a bf16-rounded copy); ``pix`` restricts the render to listed pixels;
    ``lowpass`` applies the screen-space low-pass filter,
    rho = min(u^2 + v^2, 2 |x - c|^2)."""
    n, Cn = scene.n, scene.c
    mu, sc, q = _scene_args(scene)
    f64 = np.ascontiguousarray(scene.feat if feat is None else feat, np.float64)
    pix = _pix(pix)
    cnt = cam.width * cam.height if pix is None else pix.size
    o = {
        "rgb": np.zeros((cnt, 3)), "depth": np.zeros(cnt), "normal": np.zeros((cnt, 3)),
        "alpha": np.zeros(cnt), "feat": np.zeros((cnt, Cn)), "ncontrib": np.zeros(cnt, np.int32),
        "T_final": np.zeros(cnt), "last": np.zeros(cnt, np.int64),
        "sel_id": np.zeros((cnt, K), np.int64), "sel_w": np.zeros((cnt, K)), "margins": np.zeros((cnt, 4)),
    }
    lib().orc_render(n, _vp(mu), _vp(sc), _vp(q), _vp(_c32(scene.opacity)), _vp(_c32(scene.rgb)),
                     _vp(f64), Cn, _vp(cam.as_array()), tile, tile, K, int(blend), int(lowpass),
                     0 if pix is None else pix.size, _vp(pix),
                     _vp(o["rgb"]), _vp(o["depth"]), _vp(o["normal"]), _vp(o["alpha"]), _vp(o["feat"]),
                     _vp(o["ncontrib"]), _vp(o["T_final"]), _vp(o["last"]), _vp(o["sel_id"]),
                     _vp(o["sel_w"]), _vp(o["margins"]))
    o["margin"] = o["margins"].min(-1)
    if pix is None:
        H, W = cam.height, cam.width
        for key in ("rgb", "normal", "feat", "sel_id", "sel_w", "margins"):
            o[key] = o[key].reshape(H, W, -1)
        for key in ("depth", "alpha", "ncontrib", "T_final", "last", "margin"):
            o[key] = o[key].reshape(H, W)
    return o


def backward(scene, cam, grads: dict, K=16, blend=TOPK, feat=None, pix=None, mask=None, tile=16,
             lowpass=False) -> dict:
    """FP64 gradients of L = sum(upstream * outputs).  ``grads`` holds the
    upstream maps (full images, or per listed pixel when ``pix`` is given)."""
    n, Cn = scene.n, scene.c
    mu, sc, q = _scene_args(scene)
    f64 = np.ascontiguousarray(scene.feat if feat is None else feat, np.float64)
    pix = _pix(pix)
    cnt = cam.width * cam.height if pix is None else pix.size
    g = {k: np.ascontiguousarray(np.asarray(grads[k], np.float64).reshape(cnt, -1))
         for k in ("rgb", "depth", "normal", "alpha", "feat")}
    mask_a = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    d = {"means": np.zeros((n, 3)), "scales": np.zeros((n, 2)), "quats": np.zeros((n, 4)),
         "opacity": np.zeros(n), "rgb": np.zeros((n, 3)), "feat": np.zeros((n, Cn))}
    lib().orc_backward(n, _vp(mu), _vp(sc), _vp(q), _vp(_c32(scene.opacity)), _vp(_c32(scene.rgb)),
                       _vp(f64), Cn, _vp(cam.as_array()), tile, tile, K, int(blend), int(lowpass),
                       0 if pix is None else pix.size, _vp(pix),
                       _vp(g["rgb"]), _vp(g["depth"]), _vp(g["normal"]), _vp(g["alpha"]), _vp(g["feat"]),
                       _vp(mask_a), _vp(d["means"]), _vp(d["scales"]), _vp(d["quats"]),
                       _vp(d["opacity"]), _vp(d["rgb"]), _vp(d["feat"]))
    return d


def decisions(scene, cam, pix, K=16, blend=TOPK, feat=None, tile=16, lowpass=False) -> np.ndarray:
    """Per-pixel hash of the ordered contributor set, clamp flags, low-pass
    branches and Top-K set."""
    mu, sc, q = _scene_args(scene)
    f64 = np.ascontiguousarray(scene.feat if feat is None else feat, np.float64)
    pix = _pix(pix)
    sig = np.zeros(pix.size, np.uint64)
    lib().orc_decisions(scene.n, _vp(mu), _vp(sc), _vp(q), _vp(_c32(scene.opacity)),
                        _vp(_c32(scene.rgb)), _vp(f64), scene.c, _vp(cam.as_array()), tile, tile,
                        K, int(blend), int(lowpass), pix.size, _vp(pix), _vp(sig))
    return sig
