"""Host code under AddressSanitizer, on the CPU (no GPU needed).

* The oracle (oracle.cpp), built with g++ -fsanitize=address, renders and
  differentiates a small scene in a child process that preloads the
  sanitizer runtime; its results equal the regular build's.
* The C-ABI library with api.cpp's host code instrumented (clang's host-side
  sanitizer, device code unchanged) runs the host-side validation of every
  entry point -- bad sizes, bad enums, null pointers, no device -- without a
  sanitizer report and with the documented status codes.
"""
import glob
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2604_10982_amd")
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _child(code, preload, tmp):
    env = dict(os.environ, LD_PRELOAD=preload, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=23")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900, cwd=tmp)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, (r.returncode, r.stderr[-6000:])
    return r.stdout


def test_oracle_under_asan(tmp_path):
    runtime = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(runtime) or not os.path.exists(runtime):
        pytest.skip("g++ has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", os.path.join(ROOT, "oracle", "oracle.cpp"),
                    "-o", lib], check=True)
    out = str(tmp_path / "asan.npz")
    code = f"""
import numpy as np
from oracle import oracle as O
from paper_2604_10982_amd import scenes
O.LIB_PATH = {lib!r}
sc = scenes.uniform_box(300, 16, seed=4, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12))
cam = scenes.pinhole(64, 48, f=56.0)
r = {{}}
for m in ("sphere", "aabb", "ellipse"):
    ks = O.keystage(sc, cam, m)
    r["tile_" + m], r["id_" + m] = ks["tile"], ks["id"]
ks = O.keystage(sc, cam, "ellipse", tile=(32, 8), lowpass=True)
r["tile_w32lp"] = ks["tile"]
for b in (O.TOPK, O.FULL):
    f = O.render(sc, cam, 4, b)
    r["feat_%d" % b], r["rgb_%d" % b] = f["feat"], f["rgb"]
g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
d = O.backward(sc, cam, g, K=4, blend=O.TOPK)
for k, v in d.items():
    r["d_" + k] = v
r["sig"] = O.decisions(sc, cam, np.arange(64 * 48), K=4, blend=O.TOPK)
np.savez({out!r}, **r)
print("ok")
"""
    assert "ok" in _child(code, runtime, str(tmp_path))
    from oracle import oracle as O
    from paper_2604_10982_amd import scenes
    got = np.load(out)
    sc = scenes.uniform_box(300, 16, seed=4, xy=1.0, z=(2.0, 5.0), scale_mu=np.log(0.12))
    cam = scenes.pinhole(64, 48, f=56.0)
    for m in ("sphere", "aabb", "ellipse"):
        ks = O.keystage(sc, cam, m)
        np.testing.assert_array_equal(got["tile_" + m], ks["tile"])
        np.testing.assert_array_equal(got["id_" + m], ks["id"])
    np.testing.assert_array_equal(got["tile_w32lp"], O.keystage(sc, cam, "ellipse", tile=(32, 8), lowpass=True)["tile"])
    for b in (O.TOPK, O.FULL):
        f = O.render(sc, cam, 4, b)
        np.testing.assert_array_equal(got["feat_%d" % b], f["feat"])
        np.testing.assert_array_equal(got["rgb_%d" % b], f["rgb"])
    g = scenes.upstream(cam.height, cam.width, sc.c, seed=1)
    d = O.backward(sc, cam, g, K=4, blend=O.TOPK)
    for k, v in d.items():  # per-thread buffers: equal up to the order of their final sums
        np.testing.assert_allclose(got["d_" + k], v, rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(got["sig"], O.decisions(sc, cam, np.arange(64 * 48), K=4, blend=O.TOPK))


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_library_host_validation_under_asan(tmp_path):
    runtime = _clang_asan_runtime()
    objs = [os.path.join(PKG, "_build", os.path.splitext(s)[0] + ".o") for s in
            ("keystage.hip", "sort.hip", "raster_fwd.hip", "raster_bwd.hip", "labels.hip", "attention.hip",
             "geometry.hip")]
    if runtime is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs the clang sanitizer runtime and the package build (python -m paper_2604_10982_amd.build)")
    from paper_2604_10982_amd import build as B
    api = str(tmp_path / "api_asan.o")
    flags = [f for f in B.COMMON if f != "-O3"] + ["-O1", "-g"] + HOST_ASAN
    subprocess.run([B.HIPCC, *flags, "-x", "hip", "-c", os.path.join(PKG, "csrc", "api.cpp"), "-o", api],
                   check=True, capture_output=True)
    lib = str(tmp_path / "libpsm_asan.so")
    subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", api, *objs, "-o", lib], check=True,
                   capture_output=True)
    code = f"""
import ctypes as C
L = C.CDLL({lib!r})
class Cam(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32)]
class Cfg(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("k", "tile_mode", "blend", "flags", "schedule", "blend_pass", "bwd_pass",
                                         "bwd_schedule", "tile_w")]
class Surf(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(n, C.c_void_p) for n in ("means", "scales", "quats", "opacity", "rgb",
                                                             "feat")] + [("c", C.c_int32), ("dt", C.c_int32),
                                                                         ("feat_ext", C.c_void_p),
                                                                         ("c_ext", C.c_int32)]
def cam(w=64, h=48, near=0.2):
    c = Cam(); c.R[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]; c.fx = c.fy = 50.0; c.cx, c.cy = w / 2, h / 2
    c.near_plane = near; c.width, c.height = w, h
    return c
L.psm_last_error.restype = C.c_char_p
L.psm_version.restype = C.c_char_p
out = C.c_size_t()
ws = lambda n, cm, cf, c, cap: L.psm_workspace_size(C.c_int64(n), C.byref(cm), C.byref(cf), c, C.c_int64(cap),
                                                   C.byref(out))
assert ws(100, cam(), Cfg(16), 16, 1000) == 0 and out.value > 0
assert ws(100, cam(), Cfg(16, 2, 1, 0, 0, 0, 0, 0, 32), 16, 1000) == 0
assert ws(100, cam(), Cfg(0), 16, 1000) == -1            # k
assert ws(100, cam(), Cfg(33), 16, 1000) == -1
assert ws(100, cam(), Cfg(16, 3), 16, 1000) == -1        # tile mode
assert ws(100, cam(), Cfg(16, 2, 2), 16, 1000) == -1     # blend
assert ws(100, cam(), Cfg(16, 2, 1, 1 << 20), 16, 1000) == -1   # flags
assert ws(100, cam(), Cfg(16, 2, 1, 0, 0, 0, 0, 0, 12), 16, 1000) == -1   # tile width
assert ws(100, cam(), Cfg(16), 12, 1000) == -2           # c % 8
assert ws(100, cam(), Cfg(16), 2048, 1000) == -1         # c too large
assert ws(-1, cam(), Cfg(16), 16, 1000) == -1
assert ws(100, cam(), Cfg(16), 16, -5) == -1
assert ws(100, cam(near=0.0), Cfg(16), 16, 1000) == -1
assert ws(100, cam(w=0), Cfg(16), 16, 1000) == -1
assert len(L.psm_last_error()) > 0
assert L.psm_workspace_size(C.c_int64(10), None, C.byref(Cfg(16)), 16, C.c_int64(10), C.byref(out)) == -1
assert L.psm_workspace_size(C.c_int64(10), C.byref(cam()), C.byref(Cfg(16)), 16, C.c_int64(10), None) == -1
s, imgs = Surf(), (C.c_void_p * 5)()
assert L.psm_forward(None, C.byref(s), C.byref(cam()), C.byref(Cfg(16)), None, C.c_size_t(0), C.c_int64(0),
                     imgs, None) == -1
assert L.psm_backward(None, C.byref(s), C.byref(cam()), C.byref(Cfg(16)), None, C.c_size_t(0), C.c_int64(0), None,
                      None, None) == -1
assert L.psm_forward_static(None, C.byref(s), C.byref(cam()), C.byref(Cfg(16)), C.c_int64(-1), imgs, None) == -1
assert L.psm_create(None, 0) == -1
ctx = C.c_void_p()
assert L.psm_create(C.byref(ctx), 0) == -4 and not ctx.value  # no HIP device on this host
assert L.psm_version().startswith(b"psm")
print("ok")
"""
    assert "ok" in _child(code, runtime, str(tmp_path))
