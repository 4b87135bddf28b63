"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and builds camera poses.  It holds none of
the rendering or propagation arithmetic: the HIP path and the CPU oracle each
implement that on their own.

Distributions follow the learned-field statistics of Supplementary F (scales
mostly below 0.05, bimodal opacity, phase spread over [0, 2pi), amplitude in
[0, 1]); the five workloads follow the benchmark configurations listed in
``WORKLOADS``.  There is no dataset here: the NeRF-Synthetic / LLFF /
Mip-NeRF-360 scenes the paper trains on (Sec. 6) are replaced by these draws.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Camera", "Scene", "Optics", "Workload", "WORKLOADS",
    "make_gaussians", "identity_camera", "ring_cameras", "yaw_cameras",
    "make_targets", "make_workload",
]


@dataclass
class Camera:
    """Pinhole camera: x_cam = R @ x_world + t; axes x right, y down, z forward.

    Pixel (row r, column c) has its centre at (c + 0.5, r + 0.5).
    """
    R: np.ndarray            # (3, 3) float32, world -> camera rotation, row-major
    t: np.ndarray            # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.01

    def as_array(self) -> np.ndarray:
        """Packed float32 record (R[9], t[3], fx, fy, cx, cy, z_near, pad[3])."""
        out = np.zeros(20, np.float32)
        out[0:9] = np.asarray(self.R, np.float32).reshape(9)
        out[9:12] = np.asarray(self.t, np.float32)
        out[12:17] = [self.fx, self.fy, self.cx, self.cy, self.z_near]
        return out


@dataclass
class Scene:
    """Complex Gaussians, structure-of-arrays, float32 (Eq. 9 minus the plane logits)."""
    means: np.ndarray        # (N, 3)
    log_scales: np.ndarray   # (N, 3)
    quats: np.ndarray        # (N, 4) (w, x, y, z), any norm
    opacity: np.ndarray      # (N,) activated, in (0, 1)
    amp: np.ndarray          # (N, L) amplitude per wavelength
    phase: np.ndarray        # (N, L) radians

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_lambda(self) -> int:
        return int(self.amp.shape[1])

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity, self.amp, self.phase)

    def subset(self, idx) -> "Scene":
        return Scene(*(np.ascontiguousarray(a[idx]) for a in self.arrays()))


@dataclass
class Optics:
    wavelengths: tuple       # metres
    distances: tuple         # metres, signed
    pitch: float             # metres
    pad: int = 2
    band_limit: int = 2      # 0 none, 1 evanescent cut (Eq. 7), 2 Eq. 7 + sampling limit


@dataclass
class Workload:
    name: str
    scene: Scene
    cameras: list
    optics: Optics
    backward: bool
    targets: np.ndarray | None = None
    notes: dict = field(default_factory=dict)


def make_gaussians(n, n_lambda, seed, *, x_range=(-0.5, 0.5), y_range=(-0.5, 0.5),
                   z_range=(1.0, 3.0), log_scale_mean=-4.0, log_scale_std=0.5, opacity_logit_mean=0.0,
                   opacity_logit_std=1.0) -> Scene:
    """opacity = sigmoid(N(opacity_logit_mean, opacity_logit_std)); a large mean
    draws the near-opaque Gaussians of the learned fields (Supplementary F),
    whose alpha clamps at alpha_max and whose stacks end pixel walks early."""
    rng = np.random.default_rng(seed)
    means = np.stack([
        rng.uniform(*x_range, n), rng.uniform(*y_range, n), rng.uniform(*z_range, n)
    ], axis=1)
    log_scales = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    quats = rng.normal(0.0, 1.0, (n, 4))          # uniform rotation once normalised
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(opacity_logit_mean, opacity_logit_std, n)))
    amp = rng.uniform(0.0, 1.0, (n, n_lambda))
    phase = rng.uniform(0.0, 2.0 * math.pi, (n, n_lambda))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(means), f32(log_scales), f32(quats), f32(opacity), f32(amp), f32(phase))


def identity_camera(width, height, f=None, z_near=0.01) -> Camera:
    f = float(width) if f is None else float(f)
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f,
                  width / 2.0, height / 2.0, int(width), int(height), z_near)


def _look_at(center, target, down=(0.0, 1.0, 0.0)):
    center = np.asarray(center, np.float64)
    zc = np.asarray(target, np.float64) - center
    zc /= np.linalg.norm(zc)
    yc = np.asarray(down, np.float64) - np.dot(down, zc) * zc
    yc /= np.linalg.norm(yc)
    xc = np.cross(yc, zc)
    R = np.stack([xc, yc, zc])           # rows: camera axes in world coordinates
    t = -R @ center
    return R.astype(np.float32), t.astype(np.float32)


def ring_cameras(n_views, radius, width, height, f=None, z_near=0.01):
    """Cameras on a ring in the xz-plane at azimuth 2*pi*v/n, looking at the origin."""
    cams = []
    f = float(width) if f is None else float(f)
    for v in range(n_views):
        a = 2.0 * math.pi * v / n_views
        center = (radius * math.sin(a), 0.0, -radius * math.cos(a))
        R, t = _look_at(center, (0.0, 0.0, 0.0))
        cams.append(Camera(R, t, f, f, width / 2.0, height / 2.0, width, height, z_near))
    return cams


def yaw_cameras(yaws_deg, pivot, width, height, f=None, z_near=0.01):
    """Identity camera yawed about the world y axis through ``pivot``."""
    cams = []
    f = float(width) if f is None else float(f)
    p = np.asarray(pivot, np.float64)
    for yd in yaws_deg:
        a = math.radians(yd)
        Ry = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
        center = p + Ry @ (-p)
        R = Ry.T                       # camera axes rotated by Ry: world->camera is Ry^T
        t = -R @ center
        cams.append(Camera(R.astype(np.float32), t.astype(np.float32), f, f,
                           width / 2.0, height / 2.0, width, height, z_near))
    return cams


def make_targets(shape, seed) -> np.ndarray:
    """Target intensities U[0, 1), drawn directly in single precision."""
    rng = np.random.default_rng(seed)
    return rng.random(shape, dtype=np.float32)


def make_plane_masks(n_views, n_planes, height, width, seed) -> np.ndarray:
    """Binary plane masks uint8 [views, planes, H, W]: a smooth synthetic depth
    map per view (a tilted plane plus random bumps) cut into n_planes equal
    depth bins, so every pixel belongs to exactly one plane."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    out = np.zeros((n_views, n_planes, height, width), np.uint8)
    for v in range(n_views):
        d = rng.uniform(-1, 1) * xx / width + rng.uniform(-1, 1) * yy / height
        for _ in range(6):
            cx, cy = rng.uniform(0, width), rng.uniform(0, height)
            s = rng.uniform(0.05, 0.3) * max(height, width)
            d += rng.uniform(-1.5, 1.5) * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s))
        lo, hi = d.min(), d.max()
        q = np.minimum(((d - lo) / max(hi - lo, 1e-12) * n_planes).astype(np.int64), n_planes - 1)
        for k in range(n_planes):
            out[v, k] = q == k
    return out


def _c1():
    scene = make_gaussians(1000, 1, 1001)
    cam = identity_camera(128, 128, f=128)
    opt = Optics((515e-9,), (1e-3,), 8e-6, 2, 2)
    return Workload("c1_plain_fwd_128", scene, [cam], opt, backward=False)


def _c2(backward=False, seed=1002):
    scene = make_gaussians(100_000, 3, seed)
    cam = identity_camera(1920, 1080, f=1920)
    opt = Optics((639e-9, 515e-9, 473e-9), (0.5e-3, 1.0e-3, 1.5e-3, 2.0e-3), 8e-6, 2, 2)
    name = "c3_fwd_bwd_1080p_3l_4z_100k" if backward else "c2_fwd_1080p_3l_4z_100k"
    w = Workload(name, scene, [cam], opt, backward=backward)
    if backward:
        w.targets = make_targets((1, 3, 4, 1080, 1920), seed + 10_000)
        w.notes["masks_seed"] = seed + 30_000
    return w


def _c4():
    scene = make_gaussians(500_000, 3, 1004, x_range=(-2.0, 2.0), y_range=(-0.25, 0.25),
                           z_range=(-0.25, 0.25))
    cams = ring_cameras(16, 2.0, 1920, 1080, f=1920)
    z = tuple(float(v) for v in np.linspace(0.25e-3, 2e-3, 8))
    opt = Optics((639e-9, 515e-9, 473e-9), z, 8e-6, 2, 2)
    w = Workload("c4_batched_16view_ring_500k", scene, cams, opt, backward=True)
    w.targets = make_targets((16, 3, 8, 1080, 1920), 1004 + 10_000)
    return w


def _c5():
    scene = make_gaussians(2_000_000, 3, 1005, log_scale_mean=-5.0, log_scale_std=0.7)
    cams = yaw_cameras((0.0, -10.0, 10.0, 20.0), (0.0, 0.0, 2.0), 3840, 2160, f=3840)
    z = tuple(float(v) for v in np.linspace(0.1e-3, 3e-3, 16))
    opt = Optics((639e-9, 515e-9, 473e-9), z, 4e-6, 2, 2)
    w = Workload("c5_train_2160p_4view_2m", scene, cams, opt, backward=True)
    # 1.6e9 target values (6.4 GB): callers draw them on the device from this seed
    w.notes["target_shape"] = (4, 3, 16, 2160, 3840)
    w.notes["target_seed"] = 1005 + 10_000
    return w


def _c3_layers():
    """The 100,000-Gaussian 1080p scene as a four-layer hologram: layers
    symmetric about d = 2 mm over a 4 mm volume (Sec. 4.1 layer placement with
    the distance and depth of the paper's holographic configuration), layer
    logits N(0, 1)."""
    w = _c2(True)
    lg = np.random.default_rng(1002 + 20_000).normal(0.0, 1.0, (w.scene.n, 4)).astype(np.float32)
    z = tuple(float(v) for v in np.linspace(0.0, 4e-3, 4))
    w.optics = Optics(w.optics.wavelengths, z, w.optics.pitch, w.optics.pad, w.optics.band_limit)
    w.name = "c3_layers_fwd_bwd_1080p_3l_4layers_100k"
    w.notes["logits"] = lg
    return w


def _c3_fd(second=False):
    """The finite-difference subset of the 1080p training workload: its first
    50 Gaussians rendered at 64 x 64 with fx = fy = 64, same wavelengths,
    planes and pitch; the second case redraws the log-scales N(-2.5, 0.3)
    for footprints of several pixels.  Targets U[0, 1)."""
    full = make_gaussians(100_000, 3, 1002)
    scene = full.subset(np.arange(50))
    if second:
        rng = np.random.default_rng(1002 + 40_000)
        scene.log_scales = rng.normal(-2.5, 0.3, (50, 3)).astype(np.float32)
    cam = identity_camera(64, 64, f=64)
    opt = Optics((639e-9, 515e-9, 473e-9), (0.5e-3, 1.0e-3, 1.5e-3, 2.0e-3), 8e-6, 2, 2)
    name = "c3_fd_subset_64_wide" if second else "c3_fd_subset_64"
    w = Workload(name, scene, [cam], opt, backward=True)
    w.targets = make_targets((1, 3, 4, 64, 64), 1002 + 50_000 + int(second))
    return w


WORKLOADS = {"c1": _c1, "c2": lambda: _c2(False), "c3": lambda: _c2(True), "c4": _c4, "c5": _c5,
             "c3_layers": _c3_layers, "c3_fd": _c3_fd, "c3_fd_wide": lambda: _c3_fd(True)}


def make_workload(key: str) -> Workload:
    return WORKLOADS[key]()
