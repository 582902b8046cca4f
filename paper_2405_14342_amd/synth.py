"""Seeded synthetic inputs for the meshgrid-surfel splatting path.

This module holds the *recipe* for the inputs only: surfel grids laid on a
road-like surface, camera rigs moving along a trajectory, and random training
targets.  It holds none of the method's arithmetic (no projection, compositing,
loss or optimiser maths), so both the GPU path and the FP64 oracle can consume
exactly the same FP32 bits from it.

The workloads stand in for the paper's nuScenes / KITTI captures (Sec. 4.1),
which are not available: a 0.1 m square surfel lattice (Sec. 3.1, "Meshgrid
Layout"), a gently curving trajectory, six surround cameras with 60 degree yaw
offsets (the nuScenes rig of Sec. 4.1) and targets with the per-pixel RGB,
hard semantic label and road mask of Sec. 3.3.2.

Everything is generated in FP64 with ``numpy.random.default_rng`` and cast to
FP32 exactly once.  Seeds follow ``1000 * config_index + sub_stream``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# sub-stream ids (seed = 1000 * config_index + sub_stream)
_SS_TRAJ, _SS_NOISE, _SS_RGB, _SS_SEM, _SS_TARGET0 = 0, 1, 2, 3, 10

SPACING = 0.1          # grid pitch in metres
SCALE0 = 0.06          # initial (s_x, s_y) in metres
ALPHA0 = 0.9           # initial opacity
CAM_HEIGHT = 1.5       # camera height above the road (m)
CAM_PITCH_DEG = -10.0  # cameras look 10 degrees down
HFOV_DEG = 70.0        # horizontal field of view of the surround cameras
CULL_LAT = 20.0        # ground rectangle half-width along camera x (m), supp. Sec. 2.1
CULL_FWD = 40.0        # ground rectangle length along camera z (m), supp. Sec. 2.1
Z_NEAR = 0.1


def surface_height(x, y):
    """Analytic road height used to place the synthetic surfels (metres)."""
    return 0.2 * np.sin(0.3 * x) * np.cos(0.2 * y)


def surface_slope(x, y):
    """Partial derivatives (dz/dx, dz/dy) of :func:`surface_height`."""
    zx = 0.06 * np.cos(0.3 * x) * np.cos(0.2 * y)
    zy = -0.04 * np.sin(0.3 * x) * np.sin(0.2 * y)
    return zx, zy


def focal_from_hfov(width: int, hfov_deg: float = HFOV_DEG) -> float:
    return (0.5 * width) / math.tan(math.radians(0.5 * hfov_deg))


@dataclass
class Camera:
    """One view: intrinsics, world-to-camera pose and its ground cull rectangle.

    OpenCV convention (x right, y down, z forward); ``t = R_cw @ mu + t_cw``.
    ``model`` 0 = pinhole (fx, fy, cx, cy in pixels); 1 = orthographic, where
    fx, fy are pixels per metre.  The cull rectangle is given by its origin
    (camera centre, xy), the unit ground directions of the camera x and z axes,
    a half-width and a forward length; ``cull_lat <= 0`` disables it.
    ``tile`` is the renderer's per-view tile code (``tile_w | tile_h << 16``,
    0 = the render options' shape); it changes no rendered value.
    """
    w: int
    h: int
    model: int
    fx: float
    fy: float
    cx: float
    cy: float
    R_cw: np.ndarray            # float32 [3, 3]
    t_cw: np.ndarray            # float32 [3]
    z_near: float = Z_NEAR
    cull_o: np.ndarray = field(default_factory=lambda: np.zeros(2, np.float32))
    cull_ex: np.ndarray = field(default_factory=lambda: np.array([1, 0], np.float32))
    cull_ez: np.ndarray = field(default_factory=lambda: np.array([0, 1], np.float32))
    cull_lat: float = 0.0
    cull_fwd: float = 0.0
    tile: int = 0

    @property
    def npix(self) -> int:
        return self.w * self.h


@dataclass
class Targets:
    rgb: np.ndarray     # float32 [3, H, W]
    label: np.ndarray   # uint8 [H, W]
    mask: np.ndarray    # uint8 [H, W]


@dataclass
class Scene:
    n_sem: int
    x: np.ndarray       # float32 [N]   fixed grid vertex x
    y: np.ndarray       # float32 [N]   fixed grid vertex y
    z: np.ndarray       # float32 [N]   height (learnable)
    q: np.ndarray       # float32 [4,N] rotation quaternion, w first (learnable, raw)
    log_s: np.ndarray   # float32 [2,N] raw log-scales (learnable)
    s: np.ndarray       # float32 [2,N] activated scales exp(log_s)
    logit_a: np.ndarray  # float32 [N]  raw opacity logit (learnable)
    alpha: np.ndarray   # float32 [N]   activated opacity sigmoid(logit_a)
    rgb: np.ndarray     # float32 [3,N]
    sem: np.ndarray     # float32 [C,N] semantic logits
    cams: List[Camera]
    targets: List[Targets]
    extent: float       # grid bounding-box diagonal (m), scales the z learning rate
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_views(self) -> int:
        return len(self.cams)

    @property
    def npix(self) -> int:
        return sum(c.npix for c in self.cams)


# ---------------------------------------------------------------- cameras

def pinhole_camera(pos, yaw: float, pitch: float, w: int, h: int, f: float,
                   cull: bool = True, cx: Optional[float] = None,
                   cy: Optional[float] = None) -> Camera:
    """Pinhole camera at ``pos`` looking along heading ``yaw`` (rad, from +x
    towards +y), tilted by ``pitch`` (rad, negative = down)."""
    pos = np.asarray(pos, np.float64)
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
                    math.sin(pitch)])
    down = np.cross(fwd, right)
    R_cw = np.stack([right, down, fwd])            # rows = camera axes in world
    t_cw = -R_cw @ pos
    cam = Camera(w=w, h=h, model=0, fx=float(np.float32(f)), fy=float(np.float32(f)),
                 cx=0.5 * w if cx is None else cx, cy=0.5 * h if cy is None else cy,
                 R_cw=R_cw.astype(np.float32), t_cw=t_cw.astype(np.float32))
    if cull:
        ex = right[:2] / np.linalg.norm(right[:2])
        ez = fwd[:2] / np.linalg.norm(fwd[:2])
        cam.cull_o = pos[:2].astype(np.float32)
        cam.cull_ex = ex.astype(np.float32)
        cam.cull_ez = ez.astype(np.float32)
        cam.cull_lat = CULL_LAT
        cam.cull_fwd = CULL_FWD
    return cam


def ortho_bev_camera(center_xy, height: float, w: int, h: int,
                     m_per_px: float = 0.05) -> Camera:
    """Orthographic camera looking straight down from ``height`` metres above
    the xy point ``center_xy``; image x = world +x, image y = world -y."""
    R_cw = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0]])
    pos = np.array([center_xy[0], center_xy[1], height], np.float64)
    t_cw = -R_cw @ pos
    k = 1.0 / m_per_px
    return Camera(w=w, h=h, model=1, fx=k, fy=k, cx=0.5 * w, cy=0.5 * h,
                  R_cw=R_cw.astype(np.float32), t_cw=t_cw.astype(np.float32))


# ---------------------------------------------------------------- surfels

def _quat_from_rot(R: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z), w >= 0, for rotation matrices R [..., 3, 3]."""
    m = R
    tr = m[..., 0, 0] + m[..., 1, 1] + m[..., 2, 2]
    w = 0.5 * np.sqrt(np.maximum(1.0 + tr, 0.0))
    x = 0.5 * np.sqrt(np.maximum(1.0 + m[..., 0, 0] - m[..., 1, 1] - m[..., 2, 2], 0.0))
    y = 0.5 * np.sqrt(np.maximum(1.0 - m[..., 0, 0] + m[..., 1, 1] - m[..., 2, 2], 0.0))
    z = 0.5 * np.sqrt(np.maximum(1.0 - m[..., 0, 0] - m[..., 1, 1] + m[..., 2, 2], 0.0))
    x = np.copysign(x, m[..., 2, 1] - m[..., 1, 2])
    y = np.copysign(y, m[..., 0, 2] - m[..., 2, 0])
    z = np.copysign(z, m[..., 1, 0] - m[..., 0, 1])
    q = np.stack([w, x, y, z], axis=0)
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def _surfel_params(x: np.ndarray, y: np.ndarray, n_sem: int, seed0: int,
                   noise_std: float = 0.01):
    """Height, slope-aligned rotation and appearance for grid vertices (x, y)."""
    n = x.shape[0]
    rng_n = np.random.default_rng(seed0 + _SS_NOISE)
    z = surface_height(x, y) + rng_n.normal(0.0, noise_std, n)
    zx, zy = surface_slope(x, y)
    nrm = np.stack([-zx, -zy, np.ones_like(zx)], axis=-1)
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    ex = np.array([1.0, 0.0, 0.0])
    e1 = ex[None, :] - (nrm @ ex)[:, None] * nrm
    e1 /= np.linalg.norm(e1, axis=-1, keepdims=True)
    e2 = np.cross(nrm, e1)
    R = np.stack([e1, e2, nrm], axis=-1)              # columns e1, e2, n
    q = _quat_from_rot(R)
    log_s = np.full((2, n), math.log(SCALE0))
    logit_a = np.full(n, math.log(ALPHA0 / (1.0 - ALPHA0)))
    rgb = np.random.default_rng(seed0 + _SS_RGB).uniform(0.0, 1.0, (3, n))
    sem = np.random.default_rng(seed0 + _SS_SEM).normal(0.0, 1.0, (n_sem, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(z=f32(z), q=f32(q), log_s=f32(log_s),
                s=f32(np.full((2, n), SCALE0)), logit_a=f32(logit_a),
                alpha=f32(np.full(n, ALPHA0)), rgb=f32(rgb), sem=f32(sem))


def _targets(cams: Sequence[Camera], n_sem: int, seed0: int,
             mask_keep: float = 1.0) -> List[Targets]:
    out = []
    for v, c in enumerate(cams):
        rng = np.random.default_rng(seed0 + _SS_TARGET0 + v)
        rgb = rng.uniform(0.0, 1.0, (3, c.h, c.w)).astype(np.float32)
        label = rng.integers(0, n_sem, (c.h, c.w), dtype=np.uint8)
        if mask_keep >= 1.0:
            mask = np.ones((c.h, c.w), np.uint8)
        else:
            mask = (rng.uniform(0.0, 1.0, (c.h, c.w)) < mask_keep).astype(np.uint8)
        out.append(Targets(rgb=rgb, label=label, mask=mask))
    return out


class Trajectory:
    """Planar trajectory with heading theta(s) = theta0 + A sin(2 pi s / L + phi),
    integrated with the midpoint rule at 0.1 m."""

    def __init__(self, length_m: float, seed: int):
        rng = np.random.default_rng(seed)
        self.theta0 = rng.uniform(0.0, 2.0 * math.pi)
        self.A = rng.uniform(0.1, 0.3)
        self.L = rng.uniform(80.0, 150.0)
        self.phi = rng.uniform(0.0, 2.0 * math.pi)
        n = int(round(length_m / SPACING)) + 1
        self.s = np.arange(n) * SPACING
        mid = self.heading(self.s[:-1] + 0.5 * SPACING)
        steps = SPACING * np.stack([np.cos(mid), np.sin(mid)], axis=-1)
        self.p = np.concatenate([np.zeros((1, 2)), np.cumsum(steps, axis=0)], axis=0)

    def heading(self, s):
        return self.theta0 + self.A * np.sin(2.0 * math.pi * np.asarray(s) / self.L + self.phi)

    def at(self, s: float):
        k = int(round(s / SPACING))
        k = min(max(k, 0), len(self.s) - 1)
        return self.p[k], float(self.heading(self.s[k]))


def curvilinear_grid(traj: Trajectory, n_along: int, n_across: int):
    """Lattice of arclength (0.1 m) x lateral offset (0.1 m) vertices."""
    k = np.arange(n_along)
    th = traj.heading(traj.s[k])
    nrm = np.stack([-np.sin(th), np.cos(th)], axis=-1)
    lat = SPACING * (np.arange(n_across) - 0.5 * (n_across - 1))
    pts = traj.p[k][:, None, :] + lat[None, :, None] * nrm[:, None, :]
    return pts[..., 0].reshape(-1), pts[..., 1].reshape(-1)


def surround_rig(traj: Trajectory, s: float, sizes: Sequence[tuple]) -> List[Camera]:
    """Six cameras at arclength ``s``: yaw offsets 0, 60, ..., 300 degrees
    (front first, back = index 3), HFOV 70 degrees, 1.5 m above the road."""
    p, th = traj.at(s)
    zc = float(surface_height(p[0], p[1])) + CAM_HEIGHT
    cams = []
    for k in range(6):
        w, h = sizes[k]
        cams.append(pinhole_camera((p[0], p[1], zc), th + math.radians(60.0 * k),
                                   math.radians(CAM_PITCH_DEG), w, h, focal_from_hfov(w)))
    return cams


def vehicle_poses(traj: Trajectory, step_m: float = 0.5, s0: float = 0.0,
                  s1: Optional[float] = None) -> np.ndarray:
    """Vehicle poses along the trajectory every ``step_m`` metres: the rear
    axle's ground point on the road surface, rotation with columns forward,
    left, up, where up is the surface normal and forward the heading projected
    onto the surface.  float32 [P, 12] = x, y, z, R (row-major)."""
    s1 = traj.s[-1] if s1 is None else s1
    out = []
    for s in np.arange(s0, s1 + 1e-9, step_m):
        p, th = traj.at(float(s))
        z = float(surface_height(p[0], p[1]))
        zx, zy = surface_slope(p[0], p[1])
        up = np.array([-zx, -zy, 1.0])
        up /= np.linalg.norm(up)
        f = np.array([math.cos(th), math.sin(th), 0.0])
        f = f - (f @ up) * up
        f /= np.linalg.norm(f)
        left = np.cross(up, f)
        R = np.stack([f, left, up], axis=-1)
        out.append(np.concatenate([[p[0], p[1], z], R.reshape(-1)]))
    return np.ascontiguousarray(np.array(out), np.float32)


def lidar_points(traj: Trajectory, n: int, seed: int, half_width: float = 8.0,
                 noise_std: float = 0.02, s0: float = 0.0, s1: Optional[float] = None) -> np.ndarray:
    """Synthetic LiDAR returns on the road surface near the trajectory (the
    paper's nuScenes sweeps are not available): xy uniform in a band of
    +-half_width metres around the path, z = surface height + N(0, noise_std).
    float32 [3, n]."""
    rng = np.random.default_rng(seed)
    s1 = traj.s[-1] if s1 is None else s1
    s = rng.uniform(s0, s1, n)
    lat = rng.uniform(-half_width, half_width, n)
    k = np.clip(np.round(s / SPACING).astype(np.int64), 0, len(traj.s) - 1)
    th = traj.heading(traj.s[k])
    x = traj.p[k, 0] - lat * np.sin(th)
    y = traj.p[k, 1] + lat * np.cos(th)
    z = surface_height(x, y) + rng.normal(0.0, noise_std, n)
    return np.ascontiguousarray(np.stack([x, y, z]), np.float32)


def grid_neighbours(n_along: int, n_across: int) -> np.ndarray:
    """Four-neighbour table [4, n] (up, down, left, right; own index at the
    border) of the curvilinear lattice, whose vertex (k, j) has index
    k * n_across + j: up/down step along the path, left/right across."""
    k, j = np.meshgrid(np.arange(n_along), np.arange(n_across), indexing="ij")
    idx = k * n_across + j
    up = np.where(k > 0, idx - n_across, idx)
    down = np.where(k < n_along - 1, idx + n_across, idx)
    left = np.where(j > 0, idx - 1, idx)
    right = np.where(j < n_across - 1, idx + 1, idx)
    return np.ascontiguousarray(np.stack([up, down, left, right]).reshape(4, -1), np.int32)


# ---------------------------------------------------------------- configs

def _assemble(x, y, n_sem, cams, seed0, name, mask_keep=1.0, with_targets=True):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    prm = _surfel_params(x, y, n_sem, seed0)
    ext = float(math.hypot(x.max() - x.min(), y.max() - y.min()))
    tg = _targets(cams, n_sem, seed0, mask_keep) if with_targets else []
    return Scene(n_sem=n_sem, x=x.astype(np.float32), y=y.astype(np.float32),
                 cams=list(cams), targets=tg, extent=ext, name=name, **prm)


def config1(n_sem: int = 8, mask_keep: float = 1.0) -> Scene:
    """64 x 64 axis-aligned grid, one 160 x 90 pinhole (f = 120) at
    (-1, 0, 1.5), yaw 0, pitched 10 degrees down."""
    seed0 = 1000 * 0
    i = np.arange(64)
    gx, gy = np.meshgrid(SPACING * i, SPACING * (i - 31.5), indexing="xy")
    cam = pinhole_camera((-1.0, 0.0, 1.5), 0.0, math.radians(CAM_PITCH_DEG), 160, 90, 120.0)
    sc = _assemble(gx.reshape(-1), gy.reshape(-1), n_sem, [cam], seed0, "C1-4096", mask_keep)
    sc.grid_shape = (64, 64)       # vertex (row j, column i) has index 64 j + i
    return sc


def strip_scene(cfg_index: int, n_along: int, n_across: int, n_sem: int,
                frames: Sequence[float], sizes: Sequence[tuple], name: str,
                mask_keep: float = 1.0, with_targets: bool = True) -> Scene:
    seed0 = 1000 * cfg_index
    traj = Trajectory(n_along * SPACING, seed0 + _SS_TRAJ)
    x, y = curvilinear_grid(traj, n_along, n_across)
    cams = []
    for s in frames:
        cams += surround_rig(traj, s, sizes)
    sc = _assemble(x, y, n_sem, cams, seed0, name, mask_keep, with_targets)
    sc.trajectory = traj
    sc.grid_shape = (n_along, n_across)
    return sc


def config2(**kw) -> Scene:
    """200k surfels (1000 x 200), six 1600 x 900 cameras at s = 50 m, C = 8."""
    return strip_scene(1, 1000, 200, 8, [50.0], [(1600, 900)] * 6, "C2-200k-6x1600x900", **kw)


def config3(**kw) -> Scene:
    """800k surfels (2000 x 400), 4 frames x 6 cameras (front/back 1600 x 900,
    sides 1280 x 720) = 24 views, C = 8."""
    sizes = [(1600, 900), (1280, 720), (1280, 720), (1600, 900), (1280, 720), (1280, 720)]
    return strip_scene(2, 2000, 400, 8, [70.0, 90.0, 110.0, 130.0], sizes,
                       "C3-800k-24views", **kw)


def config4(**kw) -> Scene:
    """3M surfels (10000 x 300), six 1920 x 1080 cameras at s = 500 m, C = 16."""
    return strip_scene(3, 10000, 300, 16, [500.0], [(1920, 1080)] * 6, "C4-3M-6x1920x1080", **kw)


def mini_strip(n_along=240, n_across=60, n_sem=8, w=320, h=180, n_frames=1,
               cfg_index=7, mask_keep=0.8, sides=None) -> Scene:
    """Small strip scene for parity tests: same recipe, fewer surfels and pixels."""
    sizes = sides or [(w, h)] * 6
    frames = [0.5 * n_along * SPACING + 4.0 * k for k in range(n_frames)]
    return strip_scene(cfg_index, n_along, n_across, n_sem, frames, sizes,
                       f"mini-{n_along}x{n_across}", mask_keep=mask_keep)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4}

# serving request classes over the 3M-surfel map (pinhole sizes with HFOV 70
# degrees, and a 512 x 512 top-down orthographic view at 0.05 m/px)
SERVE_CLASSES = [(640, 360), (1280, 720), (1600, 900), (1920, 1080), "bev"]
SERVE_KINDS_PINHOLE = ["rgb", "rgb_sem", "rgb_sem_d_a"]
BEV_HEIGHT = 50.0


@dataclass
class ServeRequest:
    t: float             # arrival time (s) from the start of the schedule
    cam: Camera
    kind: str            # "rgb", "rgb_sem", "rgb_sem_d_a" (pinhole) or "elev_sem" (BEV)
    elev_ref: float      # camera height for the elevation channel


def serve_schedule(traj: Trajectory, rate: float, duration: float, seed: int = 5000,
                   length_m: float = 1000.0) -> List[ServeRequest]:
    """Poisson arrivals at ``rate`` per second over ``duration`` seconds; pose
    s ~ U[0, length_m], rig camera ~ U{0..5}; class uniform over
    SERVE_CLASSES; pinhole channel set uniform over SERVE_KINDS_PINHOLE."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        s = rng.uniform(0.0, length_m)
        k = int(rng.integers(0, 6))
        cls = SERVE_CLASSES[int(rng.integers(0, len(SERVE_CLASSES)))]
        p, th = traj.at(s)
        if cls == "bev":
            zc = float(surface_height(p[0], p[1])) + BEV_HEIGHT
            out.append(ServeRequest(t, ortho_bev_camera((p[0], p[1]), zc, 512, 512, 0.05),
                                    "elev_sem", zc))
            continue
        w, h = cls
        zc = float(surface_height(p[0], p[1])) + CAM_HEIGHT
        cam = pinhole_camera((p[0], p[1], zc), th + math.radians(60.0 * k),
                             math.radians(CAM_PITCH_DEG), w, h, focal_from_hfov(w))
        kind = SERVE_KINDS_PINHOLE[int(rng.integers(0, 3))]
        out.append(ServeRequest(t, cam, kind, zc))


def custom_scene(x, y, z, q, s, alpha, rgb, sem, cams, targets=None, name="custom",
                 seed: int = 99) -> Scene:
    """Scene from explicit per-surfel arrays (cast to FP32).  Raw parameters
    (log-scales, opacity logits) are derived from the activated ones; random
    targets are drawn when none are given."""
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    x, y, z, alpha = f32(x), f32(y), f32(z), f32(alpha)
    q, s, rgb, sem = f32(q), f32(s), f32(rgb), f32(sem)
    n_sem = sem.shape[0]
    if targets is None:
        targets = _targets(cams, n_sem, seed * 1000, mask_keep=0.8)
    ext = float(math.hypot(float(x.max() - x.min()), float(y.max() - y.min())))
    a64 = alpha.astype(np.float64)
    return Scene(n_sem=n_sem, x=x, y=y, z=z, q=q, log_s=f32(np.log(s.astype(np.float64))), s=s,
                 logit_a=f32(np.log(a64 / (1.0 - a64))), alpha=alpha, rgb=rgb, sem=sem,
                 cams=list(cams), targets=list(targets), extent=ext, name=name)


def quat_wxyz_from_matrix(R) -> np.ndarray:
    """Unit quaternion (w, x, y, z), w >= 0, of one 3x3 rotation matrix."""
    return _quat_from_rot(np.asarray(R, np.float64)[None])[:, 0]


def tiny_scene(nx=8, ny=8, n_sem=4, w=32, h=32, f=40.0, seed=5, alpha_range=(0.3, 0.8),
               n_views=1) -> Scene:
    """A few dozen surfels seen by one or two small cameras: the size used for
    finite-difference checks."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = 1.0 + SPACING * i.reshape(-1)
    y = SPACING * (j.reshape(-1) - 0.5 * (ny - 1))
    n = x.size
    z = surface_height(x, y) + rng.normal(0.0, 0.01, n)
    ang = rng.normal(0.0, 0.15, (n, 3))
    qs = []
    for a in ang:
        cx, cy, cz = np.cos(a), np.sin(a), None
        Rx = np.array([[1, 0, 0], [0, cx[0], -cy[0]], [0, cy[0], cx[0]]])
        Ry = np.array([[cx[1], 0, cy[1]], [0, 1, 0], [-cy[1], 0, cx[1]]])
        Rz = np.array([[cx[2], -cy[2], 0], [cy[2], cx[2], 0], [0, 0, 1]])
        qs.append(quat_wxyz_from_matrix(Rz @ Ry @ Rx))
    q = np.stack(qs, axis=1) * rng.uniform(0.8, 1.25, (1, n))   # unnormalised on purpose
    s = rng.uniform(0.04, 0.08, (2, n))
    alpha = rng.uniform(alpha_range[0], alpha_range[1], n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    sem = rng.normal(0.0, 1.0, (n_sem, n))
    cams = [pinhole_camera((0.0, 0.0, 0.6), 0.0, math.radians(-20.0), w, h, f, cull=True)]
    if n_views > 1:
        cams.append(pinhole_camera((0.3, -0.4, 0.7), math.radians(25.0), math.radians(-25.0),
                                   w + 8, h - 8, f * 1.1, cull=True))
    return custom_scene(x, y, z, q, s, alpha, rgb, sem, cams, name="tiny", seed=seed)


def clamp_scene() -> Scene:
    """The tiny scene's recipe with opacities in [0.995, 0.999] and footprints
    three times larger, seen by a 48 x 40 camera (f = 60): near the centre of
    every surfel alpha g exceeds the opacity clamp 0.99, on about 70
    (pixel, surfel) pairs."""
    sc = tiny_scene(w=48, h=40, f=60.0, alpha_range=(0.995, 0.999))
    sc.s[:] = sc.s * np.float32(3.0)
    sc.log_s[:] = np.log(sc.s.astype(np.float64)).astype(np.float32)
    return sc
