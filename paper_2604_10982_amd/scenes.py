"""Seeded synthetic surfel scenes, cameras and upstream gradients.

This module only draws inputs; it contains none of the renderer's arithmetic,
so both the CPU oracle (tests) and the HIP path consume the same arrays.

The paper's workloads (ScanNet-V2/++ indoor rooms, KITTI-360 streets; Sec. 6.1)
are not available here.  The generators reproduce their *structure*: the
SOGMM initialisation of Sec. 3.2 places surfels on planar surfaces with
normals close to the plane normal, plus free-floating clutter.

Conventions (Sec. 3.1, D1 of the design notes):
  * camera: OpenCV axes (x right, y down, z forward), world->camera (R, t),
    pinhole intrinsics fx, fy, cx, cy;
  * surfel: centre mu (3), tangent scales (s_u, s_v), quaternion (w, x, y, z)
    whose rotation's columns are (t_u, t_v, n), activated opacity in (0, 1),
    RGB and a C-dim feature.

Draw order for every generator: placement (means and orientation), scales,
opacity, rgb, feat -- all from one ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Camera", "Scene", "pinhole", "uniform_box", "planes7", "street40",
    "room6", "upstream", "config", "CONFIGS", "street_cameras", "batch_config", "BATCH_RES",
]


@dataclass
class Camera:
    R: np.ndarray          # (3,3) float32, world -> camera rotation
    t: np.ndarray          # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    def as_array(self) -> np.ndarray:
        """Flat float32 record: R(9) t(3) fx fy cx cy near W H (19 floats)."""
        return np.concatenate([
            self.R.astype(np.float32).reshape(9), self.t.astype(np.float32),
            np.array([self.fx, self.fy, self.cx, self.cy, self.near,
                      self.width, self.height], np.float32)])


@dataclass
class Scene:
    means: np.ndarray      # (N,3) float32
    scales: np.ndarray     # (N,2) float32
    quats: np.ndarray      # (N,4) float32, (w,x,y,z), not necessarily unit
    opacity: np.ndarray    # (N,)  float32
    rgb: np.ndarray        # (N,3) float32
    feat: np.ndarray       # (N,C) float32 (round to bf16/fp16 by the caller)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def c(self) -> int:
        return int(self.feat.shape[1])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.scales[idx], self.quats[idx],
                     self.opacity[idx], self.rgb[idx], self.feat[idx], dict(self.meta))

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.scales.copy(), self.quats.copy(),
                     self.opacity.copy(), self.rgb.copy(), self.feat.copy(), dict(self.meta))


def pinhole(width: int, height: int, f: float | None = None, near: float = 0.2,
            R=None, t=None) -> Camera:
    """Pinhole camera with the principal point at the image centre.

    Focal length defaults to 0.75*W (a 67-degree horizontal field of view).
    """
    f = 0.75 * width if f is None else f
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    t = np.zeros(3, np.float32) if t is None else np.asarray(t, np.float32)
    return Camera(R, t, float(f), float(f), width / 2.0, height / 2.0,
                  int(width), int(height), float(near))


# ---------------------------------------------------------------- quaternions
def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of (...,4) arrays in (w,x,y,z) order."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def _qaxis(axis, angle) -> np.ndarray:
    axis = np.asarray(axis, np.float64)
    angle = np.asarray(angle, np.float64)
    h = 0.5 * angle
    s = np.sin(h)[..., None]
    return np.concatenate([np.cos(h)[..., None], s * axis], -1)


def _random_quats(rng, n) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _plane_quats(rng, n, q_plane, max_tilt_deg=5.0) -> np.ndarray:
    """Orientation whose local z (normal) is within ``max_tilt_deg`` of the
    plane normal q_plane*e_z: tilt with cos(theta) ~ U(cos max, 1) about a
    uniformly drawn in-plane axis, then a uniform spin about the normal."""
    cos_t = rng.uniform(math.cos(math.radians(max_tilt_deg)), 1.0, n)
    theta = np.arccos(np.clip(cos_t, -1.0, 1.0))
    beta = rng.uniform(0.0, 2 * math.pi, n)
    spin = rng.uniform(0.0, 2 * math.pi, n)
    q_tilt = _qaxis(np.stack([np.cos(beta), np.sin(beta), np.zeros(n)], -1), theta)
    q_spin = _qaxis(np.array([0.0, 0.0, 1.0]), spin)
    qp = np.broadcast_to(np.asarray(q_plane, np.float64), (n, 4))
    return _qmul(_qmul(qp, q_tilt), q_spin)


def _q_yaw(deg) -> np.ndarray:
    """Rotation about the camera y axis (OpenCV: y down)."""
    return _qaxis(np.array([0.0, 1.0, 0.0]), math.radians(deg))


_Q_GROUND = _qaxis(np.array([1.0, 0.0, 0.0]), math.pi / 2)   # e_z -> -y (up)


def _facade_quat(yaw_deg) -> np.ndarray:
    """Vertical facade whose normal is R_y(yaw) * (0,0,-1)."""
    return _q_yaw(yaw_deg + 180.0)


def _allocate(n: int, areas) -> np.ndarray:
    """Deterministic area-proportional split of n items."""
    areas = np.asarray(areas, np.float64)
    raw = n * areas / areas.sum()
    cnt = np.floor(raw).astype(np.int64)
    rest = n - int(cnt.sum())
    order = np.argsort(-(raw - cnt), kind="stable")
    cnt[order[:rest]] += 1
    return cnt


def _rect_points(rng, n, origin, du, dv):
    """n points uniform on the rectangle origin + a*du + b*dv, a,b in [0,1]."""
    a = rng.uniform(0.0, 1.0, (n, 1))
    b = rng.uniform(0.0, 1.0, (n, 1))
    return np.asarray(origin) + a * np.asarray(du) + b * np.asarray(dv)


def _finish(rng, means, quats, n, c, scale_mu, scale_sigma, meta) -> Scene:
    scales = np.exp(rng.normal(scale_mu, scale_sigma, (n, 2)))
    opacity = rng.uniform(0.1, 0.99, n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    feat = rng.standard_normal((n, c))
    return Scene(np.ascontiguousarray(means, np.float32),
                 np.ascontiguousarray(scales, np.float32),
                 np.ascontiguousarray(quats, np.float32),
                 np.ascontiguousarray(opacity, np.float32),
                 np.ascontiguousarray(rgb, np.float32),
                 np.ascontiguousarray(feat, np.float32), meta)


# ---------------------------------------------------------------- generators
def uniform_box(n: int, c: int, seed: int = 0, xy: float = 2.5, z=(2.0, 10.0),
                scale_mu: float = math.log(0.05), scale_sigma: float = 0.5) -> Scene:
    """Means uniform in [-xy,xy]^2 x [z0,z1], uniform random orientations."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-xy, xy, n), rng.uniform(-xy, xy, n),
                      rng.uniform(z[0], z[1], n)], -1)
    quats = _random_quats(rng, n)
    return _finish(rng, means, quats, n, c, scale_mu, scale_sigma,
                   {"generator": "uniform_box", "seed": seed})


def planes7(n: int, c: int, seed: int = 0, clutter: float = 0.3,
            scale_mu: float = math.log(0.05), scale_sigma: float = 0.5) -> Scene:
    """Ground plane, two side facades, a back facade and three yawed facades
    (70% of surfels, area-proportional) plus 30% uniformly placed clutter."""
    rng = np.random.default_rng(seed)
    ground_y, top = 1.6, -8.0
    rects = [  # (origin, du, dv, q_plane)
        ((-12.0, ground_y, 1.0), (24.0, 0, 0), (0, 0, 59.0), _Q_GROUND),
        ((-6.0, top, 2.0), (0, 0, 48.0), (0, ground_y - top, 0), _facade_quat(-90.0)),
        ((6.0, top, 2.0), (0, 0, 48.0), (0, ground_y - top, 0), _facade_quat(90.0)),
        ((-12.0, top, 60.0), (24.0, 0, 0), (0, ground_y - top, 0), _facade_quat(0.0)),
    ]
    for cx_, cz_, yaw, width in ((-3.0, 25.0, 45.0, 6.0), (3.0, 35.0, -30.0, 8.0),
                                 (0.0, 45.0, 0.0, 10.0)):
        # facade normal R_y(yaw)(0,0,-1) = (-sin, 0, -cos); in-plane axis along (cos, 0, -sin)
        ux, uz = math.cos(math.radians(yaw)), -math.sin(math.radians(yaw))
        origin = (cx_ - 0.5 * width * ux, -6.0, cz_ - 0.5 * width * uz)
        rects.append((origin, (width * ux, 0, width * uz), (0, ground_y + 6.0, 0),
                      _facade_quat(yaw)))
    n_clutter = int(round(clutter * n))
    n_plane = n - n_clutter
    areas = [np.linalg.norm(np.cross(r[1], r[2])) for r in rects]
    counts = _allocate(n_plane, areas)
    means, quats = [], []
    for (o, du, dv, qp), k in zip(rects, counts):
        means.append(_rect_points(rng, k, o, du, dv))
        quats.append(_plane_quats(rng, k, qp))
    means.append(np.stack([rng.uniform(-6, 6, n_clutter), rng.uniform(-4, ground_y, n_clutter),
                           rng.uniform(2, 50, n_clutter)], -1))
    quats.append(_random_quats(rng, n_clutter))
    return _finish(rng, np.concatenate(means), np.concatenate(quats), n, c,
                   scale_mu, scale_sigma, {"generator": "planes7", "seed": seed})


def street40(n: int, c: int, seed: int = 0, clutter: float = 0.2,
             scale_mu: float = math.log(0.1), scale_sigma: float = 0.7) -> Scene:
    """200 m x 40 m street: ground, 40 facades (20 per side in 10 m slots along
    z, width U(6,10), height U(8,25), yaw jitter +-5 deg) and 20% clutter."""
    rng = np.random.default_rng(seed)
    ground_y = 1.6
    rects = [((-20.0, ground_y, -20.0), (40.0, 0, 0), (0, 0, 200.0), _Q_GROUND)]
    for side in (-1.0, 1.0):
        for k in range(20):
            x = side * (12.0 + rng.uniform(0.0, 6.0))
            width = rng.uniform(6.0, 10.0)
            height = rng.uniform(8.0, 25.0)
            jitter = rng.uniform(-5.0, 5.0)
            # facing the street: normal -side*x  => yaw = side*90 (+ jitter)
            yaw = side * 90.0 + jitter
            ux, uz = math.cos(math.radians(yaw)), -math.sin(math.radians(yaw))
            zc = -20.0 + 10.0 * k + 5.0
            origin = (x - 0.5 * width * ux, ground_y - height, zc - 0.5 * width * uz)
            rects.append((origin, (width * ux, 0, width * uz), (0, height, 0),
                          _facade_quat(yaw)))
    n_clutter = int(round(clutter * n))
    n_plane = n - n_clutter
    areas = [np.linalg.norm(np.cross(r[1], r[2])) for r in rects]
    counts = _allocate(n_plane, areas)
    means, quats = [], []
    for (o, du, dv, qp), k in zip(rects, counts):
        means.append(_rect_points(rng, k, o, du, dv))
        quats.append(_plane_quats(rng, k, qp))
    means.append(np.stack([rng.uniform(-12, 12, n_clutter), rng.uniform(-4, ground_y, n_clutter),
                           rng.uniform(0, 180, n_clutter)], -1))
    quats.append(_random_quats(rng, n_clutter))
    return _finish(rng, np.concatenate(means), np.concatenate(quats), n, c,
                   scale_mu, scale_sigma, {"generator": "street40", "seed": seed})


def room6(n: int, c: int, seed: int = 0, clutter: float = 0.2,
          scale_mu: float = math.log(0.05), scale_sigma: float = 0.5) -> Scene:
    """Indoor room 6 m x 5 m x 3 m (floor, ceiling, four walls) seen from
    inside, plus 20% clutter: a stand-in for the indoor scans of Sec. 6."""
    rng = np.random.default_rng(seed)
    x0, x1, y0, y1, z0, z1 = -3.0, 3.0, -1.5, 1.5, -1.0, 4.0
    rects = [
        ((x0, y1, z0), (6.0, 0, 0), (0, 0, 5.0), _Q_GROUND),                       # floor
        ((x0, y0, z0), (6.0, 0, 0), (0, 0, 5.0), _qaxis(np.array([1.0, 0, 0]), -math.pi / 2)),
        ((x0, y0, z0), (0, 0, 5.0), (0, 3.0, 0), _facade_quat(-90.0)),            # left
        ((x1, y0, z0), (0, 0, 5.0), (0, 3.0, 0), _facade_quat(90.0)),             # right
        ((x0, y0, z1), (6.0, 0, 0), (0, 3.0, 0), _facade_quat(0.0)),              # front
        ((x0, y0, z0), (6.0, 0, 0), (0, 3.0, 0), _facade_quat(180.0)),            # back
    ]
    n_clutter = int(round(clutter * n))
    n_plane = n - n_clutter
    areas = [np.linalg.norm(np.cross(r[1], r[2])) for r in rects]
    counts = _allocate(n_plane, areas)
    means, quats = [], []
    for (o, du, dv, qp), k in zip(rects, counts):
        means.append(_rect_points(rng, k, o, du, dv))
        quats.append(_plane_quats(rng, k, qp))
    means.append(np.stack([rng.uniform(x0, x1, n_clutter), rng.uniform(y0, y1, n_clutter),
                           rng.uniform(0.5, z1, n_clutter)], -1))
    quats.append(_random_quats(rng, n_clutter))
    return _finish(rng, np.concatenate(means), np.concatenate(quats), n, c,
                   scale_mu, scale_sigma, {"generator": "room6", "seed": seed})


def upstream(height: int, width: int, c: int, seed: int = 1) -> dict:
    """Random upstream gradients dL/d(output) ~ N(0,1) for every rendered map."""
    rng = np.random.default_rng(seed)
    return {
        "rgb": rng.standard_normal((height, width, 3)).astype(np.float32),
        "depth": rng.standard_normal((height, width)).astype(np.float32),
        "normal": rng.standard_normal((height, width, 3)).astype(np.float32),
        "alpha": rng.standard_normal((height, width)).astype(np.float32),
        "feat": rng.standard_normal((height, width, c)).astype(np.float32),
    }


# ------------------------------------------------------------------- presets
CONFIGS = {
    # name: (generator, n, C, W, H, f, K, feature storage dtype)
    "c1_box2k": ("uniform_box", 2_000, 16, 128, 128, 128.0, 8, "f32"),
    "c2_planes200k": ("planes7", 200_000, 64, 1280, 720, None, 16, "f32"),
    "c3_planes500k": ("planes7", 500_000, 128, 1920, 1080, None, 16, "f32"),
    "c4_street1m": ("street40", 1_000_000, 256, 1920, 1080, None, 16, "bf16"),
    "planes1m_1080p": ("planes7", 1_000_000, 128, 1920, 1080, None, 16, "f32"),
    "room_1296x968": ("room6", 400_000, 128, 1296, 968, None, 16, "f32"),
}


# Camera rig of the batched workload: 8 cameras of uneven resolution.
BATCH_RES = ((640, 480), (800, 600), (1024, 768), (1280, 720), (1280, 960), (1600, 900),
             (1920, 1080), (1920, 1080))


def street_cameras(res=BATCH_RES, near: float = 0.2) -> list:
    """Camera k at (+-2 m alternating, 0, 20 k m) looking down the street with
    yaw +-10 deg alternating; focal length 0.75 W."""
    cams = []
    for k, (w, h) in enumerate(res):
        x = 2.0 if k % 2 == 0 else -2.0
        a = math.radians(10.0 if k % 2 == 0 else -10.0)
        centre = np.array([x, 0.0, 20.0 * k])
        to_world = np.array([[math.cos(a), 0.0, math.sin(a)], [0.0, 1.0, 0.0], [-math.sin(a), 0.0, math.cos(a)]])
        R = to_world.T
        cams.append(pinhole(w, h, None, near, R, -R @ centre))
    return cams


def batch_config(seed: int = 0, n: int | None = None, k: int = 16):
    """(scene, cameras, K, feature dtype) of the batched workload: a shared
    2M-surfel street scene, 128-d FP16 features, 8 cameras."""
    scene = street40(2_000_000 if n is None else n, 128, seed)
    scene.meta["config"] = "c5_street2m_8cam"
    return scene, street_cameras(), k, "f16"


def config(name: str, seed: int = 0, n: int | None = None):
    """(scene, camera, K, feature dtype) for a named workload."""
    gen, n0, c, w, h, f, k, dtype = CONFIGS[name]
    fn = {"uniform_box": uniform_box, "planes7": planes7, "street40": street40,
          "room6": room6}[gen]
    scene = fn(n0 if n is None else n, c, seed)
    scene.meta["config"] = name
    return scene, pinhole(w, h, f), k, dtype


def plane_gmm(scene, k: int, seed: int = 0, extent=(1.5, 1.5, 0.03)):
    """Synthetic plane prior standing in for a LiDAR SOGMM: k components
    centred on random surfels of the scene, each flat along that surfel's own
    plane (standard deviations `extent` times U(0.7, 1.3) along the surfel's
    tangent axes and its normal), Dirichlet(1) mixing weights.
    Returns FP32 (mean [k,3], cov [k,6] as xx xy xz yy yz zz, weight [k])."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(scene.n, k, replace=False)
    q = scene.quats[pick].astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
                  np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
                  np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)
    sd = np.asarray(extent) * rng.uniform(0.7, 1.3, (k, 3))
    S = np.einsum("kij,kj,klj->kil", R, sd ** 2, R)
    cov6 = np.stack([S[:, i, j] for i, j in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))], 1)
    return (scene.means[pick].astype(np.float32), cov6.astype(np.float32),
            rng.dirichlet(np.ones(k)).astype(np.float32))
