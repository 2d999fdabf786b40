"""Seeded synthetic depth workloads (inputs only).

This module renders the depth images and camera poses that stand in for the
paper's recorded sequences (Replica, Redwood; §V).  It holds none of the
integration method's arithmetic: it only casts rays through pixel centres
against analytic geometry (an axis-aligned room, spheres, axis-aligned boxes)
in float64 and rounds the z-depth to float32.  Both the HIP path and the CPU
oracle consume exactly the arrays produced here.

Conventions
-----------
* World frame: rooms are ``[0, Lx] x [0, Ly] x [0, Lz]`` with z up, metres.
* Camera frame: x right, y down, z forward.  A depth image stores z-depth
  (the camera-frame z of the hit point), as a pinhole depth camera does
  (§III, the depth map D: Omega -> d).
* Pixel (i, j) covers ``[i, i+1) x [j, j+1)``; its ray passes through the
  centre ``(i + 0.5, j + 0.5)``.
* ``T_world_cam`` is the 4x4 float32 row-major pose of the camera in the world
  (the paper's T_LC).  The renderer uses exactly this float32 pose (widened to
  float64), so the images agree with the pose handed to the integrators.

Every random draw comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch


# --------------------------------------------------------------------------
# Cameras and poses
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class PinholeCamera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @property
    def K(self) -> np.ndarray:
        """Intrinsics as float32 ``[fx, fy, cx, cy]``."""
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)


def pose_from_forward(position: Sequence[float], yaw: float, pitch: float,
                      roll: float = 0.0) -> np.ndarray:
    """Camera pose (float32 4x4, row-major) from a position and yaw/pitch/roll.

    yaw rotates about world +z from the +x axis, pitch tilts the optical axis
    up (positive) or down, roll turns the image about the optical axis.
    Columns of the rotation are the camera x (right), y (down), z (forward)
    axes expressed in the world.
    """
    cp, sp = math.cos(pitch), math.sin(pitch)
    cyw, syw = math.cos(yaw), math.sin(yaw)
    fwd = np.array([cp * cyw, cp * syw, sp])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    if roll != 0.0:
        cr, sr = math.cos(roll), math.sin(roll)
        right, down = cr * right + sr * down, -sr * right + cr * down
    T = np.eye(4)
    T[:3, 0] = right
    T[:3, 1] = down
    T[:3, 2] = fwd
    T[:3, 3] = np.asarray(position, dtype=np.float64)
    return T.astype(np.float32)


def pose_look_along(position: Sequence[float], forward: Sequence[float],
                    down_hint: Sequence[float]) -> np.ndarray:
    """Camera pose looking along ``forward`` with image-down close to ``down_hint``."""
    f = np.asarray(forward, dtype=np.float64)
    f = f / np.linalg.norm(f)
    d = np.asarray(down_hint, dtype=np.float64)
    d = d - f * np.dot(d, f)
    d = d / np.linalg.norm(d)
    r = np.cross(d, f)
    T = np.eye(4)
    T[:3, 0] = r
    T[:3, 1] = d
    T[:3, 2] = f
    T[:3, 3] = np.asarray(position, dtype=np.float64)
    return T.astype(np.float32)


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------
@dataclass
class Scene:
    """Analytic scene: an optional room (ray exits its walls), spheres and
    boxes (rays enter them), and optional infinite planes."""
    room: Optional[Tuple[float, float, float]] = None
    spheres: List[Tuple[Tuple[float, float, float], float]] = field(default_factory=list)
    boxes: List[Tuple[Tuple[float, float, float], Tuple[float, float, float]]] = field(default_factory=list)
    # plane n . x = c, hit only from the side where n . x < c
    planes: List[Tuple[Tuple[float, float, float], float]] = field(default_factory=list)


def _ray_dirs_cam(cam: PinholeCamera, dev, dtype=torch.float64):
    j, i = torch.meshgrid(torch.arange(cam.height, device=dev, dtype=dtype),
                          torch.arange(cam.width, device=dev, dtype=dtype), indexing="ij")
    dx = (i + 0.5 - cam.cx) / cam.fx
    dy = (j + 0.5 - cam.cy) / cam.fy
    dz = torch.ones_like(dx)
    return torch.stack([dx, dy, dz], dim=-1)  # (H, W, 3); z component is 1


def _cast(scene: Scene, o, dirs, chunk: int = 1 << 16):
    """Distance t along each direction (o + t d) to the first surface, inf if none."""
    dev, f64 = dirs.device, torch.float64
    dirs = torch.where(dirs == 0, torch.full_like(dirs, 1e-300), dirs)
    inf = float("inf")
    room = torch.tensor(scene.room, device=dev, dtype=f64) if scene.room is not None else None
    if scene.spheres:
        sc = torch.tensor([c for c, _ in scene.spheres], device=dev, dtype=f64)      # (S, 3)
        sr = torch.tensor([r for _, r in scene.spheres], device=dev, dtype=f64)      # (S,)
        oc = o[None, :] - sc
        cc = (oc * oc).sum(-1) - sr * sr
    if scene.boxes:
        blo = torch.tensor([b[0] for b in scene.boxes], device=dev, dtype=f64)       # (B, 3)
        bhi = torch.tensor([b[1] for b in scene.boxes], device=dev, dtype=f64)
    if scene.planes:
        pn = torch.tensor([n for n, _ in scene.planes], device=dev, dtype=f64)       # (P, 3)
        pc = torch.tensor([c for _, c in scene.planes], device=dev, dtype=f64)
    out = []
    for a in range(0, dirs.shape[0], chunk):
        d = dirs[a:a + chunk]
        t_best = torch.full(d.shape[:1], inf, device=dev, dtype=f64)
        if room is not None:
            bound = torch.where(d > 0, room, torch.zeros_like(room))
            t_axes = (bound - o) / d
            t_axes = torch.where(t_axes > 0, t_axes, torch.full_like(t_axes, inf))
            t_best = torch.minimum(t_best, t_axes.min(dim=-1).values)
        if scene.spheres:
            aa = (d * d).sum(-1)[:, None]                            # (N, 1)
            b = d @ oc.T                                             # (N, S)
            disc = b * b - aa * cc[None, :]
            sq = torch.sqrt(torch.clamp(disc, min=0.0))
            t0 = (-b - sq) / aa
            t1 = (-b + sq) / aa
            t = torch.where(t0 > 0, t0, t1)
            t = torch.where((disc >= 0) & (t > 0), t, torch.full_like(t, inf))
            t_best = torch.minimum(t_best, t.min(dim=-1).values)
        if scene.boxes:
            inv = 1.0 / d
            t1 = (blo[None] - o) * inv[:, None, :]                   # (N, B, 3)
            t2 = (bhi[None] - o) * inv[:, None, :]
            tn = torch.minimum(t1, t2).max(dim=-1).values
            tf = torch.maximum(t1, t2).min(dim=-1).values
            t = torch.where((tn <= tf) & (tn > 0), tn, torch.full_like(tn, inf))
            t_best = torch.minimum(t_best, t.min(dim=-1).values)
        if scene.planes:
            denom = d @ pn.T                                         # (N, P)
            t = (pc[None, :] - (pn @ o)[None, :]) / denom
            t = torch.where((denom > 0) & (t > 0), t, torch.full_like(t, inf))
            t_best = torch.minimum(t_best, t.min(dim=-1).values)
        out.append(t_best)
    return torch.cat(out)


def render_depth(scene: Scene, cam: PinholeCamera, T_world_cam: np.ndarray,
                 device: str = "cpu") -> np.ndarray:
    """Ray-cast z-depth (float32, H x W) of ``scene`` seen from ``T_world_cam``.

    Every object is intersected with every ray in float64 (spheres and boxes
    vectorised over objects, rays processed in chunks); pixels whose ray hits
    nothing get depth 0 (invalid).  Ray directions have camera-frame z = 1, so
    the distance along them is the z-depth.
    """
    dev = torch.device(device)
    T = torch.as_tensor(np.asarray(T_world_cam, dtype=np.float64), device=dev)
    R, o = T[:3, :3], T[:3, 3]
    dirs = (_ray_dirs_cam(cam, dev) @ R.T).reshape(-1, 3)
    t = _cast(scene, o, dirs).reshape(cam.height, cam.width)
    depth = torch.where(torch.isfinite(t), t, torch.zeros_like(t))
    return depth.to(torch.float32).cpu().numpy()


@dataclass(frozen=True)
class LidarModel:
    """Spherical range image (rotating LiDAR).  Sensor frame: x forward, y left,
    z up.  Column i spans azimuths (atan2(y, x)) azimuth_start + [i, i+1) *
    azimuth_fov / width, row j polar angles (from +z) polar_start + [j, j+1) *
    polar_fov / height; each beam points at the centre of its pixel."""
    width: int = 1024
    height: int = 64
    azimuth_start: float = -math.pi
    azimuth_fov: float = 2.0 * math.pi
    polar_start: float = math.radians(74.0)
    polar_fov: float = math.radians(32.0)
    interp_max_diff: float = 0.2
    max_range: float = 25.0

    def params(self) -> np.ndarray:
        """float32 [azimuth start, azimuth fov, polar start, polar fov, interp max diff, max range]."""
        return np.array([self.azimuth_start, self.azimuth_fov, self.polar_start, self.polar_fov,
                         self.interp_max_diff, self.max_range], dtype=np.float32)


def render_range(scene: Scene, lidar: LidarModel, T_world_sensor: np.ndarray,
                 device: str = "cpu") -> np.ndarray:
    """Ray-cast Euclidean range (float32, height x width) along the beam of
    every pixel centre; 0 where a beam hits nothing."""
    dev = torch.device(device)
    p = lidar.params().astype(np.float64)
    j, i = torch.meshgrid(torch.arange(lidar.height, device=dev, dtype=torch.float64),
                          torch.arange(lidar.width, device=dev, dtype=torch.float64), indexing="ij")
    theta = p[0] + (i + 0.5) * (p[1] / lidar.width)
    phi = p[2] + (j + 0.5) * (p[3] / lidar.height)
    ds = torch.stack([torch.sin(phi) * torch.cos(theta), torch.sin(phi) * torch.sin(theta), torch.cos(phi)], -1)
    T = torch.as_tensor(np.asarray(T_world_sensor, dtype=np.float64), device=dev)
    dirs = (ds @ T[:3, :3].T).reshape(-1, 3)
    t = _cast(scene, T[:3, 3], dirs).reshape(lidar.height, lidar.width)
    rng = torch.where(torch.isfinite(t), t, torch.zeros_like(t))
    return rng.to(torch.float32).cpu().numpy()


def pose_lidar(position: Sequence[float], yaw: float) -> np.ndarray:
    """Level LiDAR pose (float32 4x4): x forward at ``yaw``, y left, z up."""
    c, s_ = math.cos(yaw), math.sin(yaw)
    T = np.eye(4)
    T[:3, 0] = (c, s_, 0.0)
    T[:3, 1] = (-s_, c, 0.0)
    T[:3, 2] = (0.0, 0.0, 1.0)
    T[:3, 3] = np.asarray(position, dtype=np.float64)
    return T.astype(np.float32)


def add_range_noise(rng_img: np.ndarray, rng: np.random.Generator, sigma: float = 0.02) -> np.ndarray:
    """Range noise N(0, sigma^2) on valid returns."""
    r = rng_img.astype(np.float64)
    out = np.where(r > 0, r + sigma * rng.standard_normal(r.shape), 0.0)
    return out.astype(np.float32)


def add_depth_noise(depth: np.ndarray, rng: np.random.Generator, sigma_a: float = 0.0012,
                    dropout: float = 0.05) -> np.ndarray:
    """Axial noise d += N(0, (sigma_a d^2)^2), then a fraction of pixels set to 0."""
    d = depth.astype(np.float64)
    n = rng.standard_normal(d.shape)
    out = d + sigma_a * d * d * n
    out = np.where(d > 0, out, 0.0)
    drop = rng.random(d.shape) < dropout
    out = np.where(drop, 0.0, out)
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# Trajectories
# --------------------------------------------------------------------------
def _catmull_rom_centripetal(pts: np.ndarray, samples_per_seg: int = 2000) -> np.ndarray:
    """Dense samples of a centripetal Catmull-Rom spline through ``pts``.

    End segments use mirrored phantom points so the curve passes through every
    waypoint.
    """
    P = np.vstack([2 * pts[0] - pts[1], pts, 2 * pts[-1] - pts[-2]])
    out = []
    for k in range(1, len(P) - 2):
        p0, p1, p2, p3 = P[k - 1], P[k], P[k + 1], P[k + 2]
        t0 = 0.0
        t1 = t0 + np.linalg.norm(p1 - p0) ** 0.5
        t2 = t1 + np.linalg.norm(p2 - p1) ** 0.5
        t3 = t2 + np.linalg.norm(p3 - p2) ** 0.5
        t = np.linspace(t1, t2, samples_per_seg, endpoint=(k == len(P) - 3))[:, None]
        A1 = (t1 - t) / (t1 - t0) * p0 + (t - t0) / (t1 - t0) * p1
        A2 = (t2 - t) / (t2 - t1) * p1 + (t - t1) / (t2 - t1) * p2
        A3 = (t3 - t) / (t3 - t2) * p2 + (t - t2) / (t3 - t2) * p3
        B1 = (t2 - t) / (t2 - t0) * A1 + (t - t0) / (t2 - t0) * A2
        B2 = (t3 - t) / (t3 - t1) * A2 + (t - t1) / (t3 - t1) * A3
        out.append((t2 - t) / (t2 - t1) * B1 + (t - t1) / (t2 - t1) * B2)
    return np.vstack(out)


def spline_trajectory(room: Tuple[float, float, float], n_frames: int, rng: np.random.Generator,
                      margin: float, speed: float = 0.5, fps: float = 30.0,
                      height: Tuple[float, float] = (1.0, 2.0), n_waypoints: int = 6,
                      pitch_deg: float = -10.0) -> List[np.ndarray]:
    """Smooth camera path: centripetal Catmull-Rom through random waypoints,
    sampled by arc length at ``speed`` m/s and ``fps`` frames/s.  The camera
    looks along the path tangent, pitched by ``pitch_deg``.  Waypoints are
    redrawn (from the same generator) until the path is long enough."""
    need = (n_frames - 1) * speed / fps
    while True:
        wp = np.empty((n_waypoints, 3))
        wp[:, 0] = rng.uniform(margin, room[0] - margin, n_waypoints)
        wp[:, 1] = rng.uniform(margin, room[1] - margin, n_waypoints)
        wp[:, 2] = rng.uniform(height[0], height[1], n_waypoints)
        curve = _catmull_rom_centripetal(wp)
        seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
        s = np.concatenate([[0.0], np.cumsum(seg)])
        inside = np.all((curve[:, :2] > 0.2) & (curve[:, :2] < np.asarray(room[:2]) - 0.2)) and \
            np.all((curve[:, 2] > 0.2) & (curve[:, 2] < room[2] - 0.2))
        if s[-1] >= need + 0.05 and inside:
            break
    poses = []
    for k in range(n_frames):
        sk = k * speed / fps
        idx = int(np.searchsorted(s, sk, side="right") - 1)
        idx = min(max(idx, 0), len(curve) - 2)
        a = (sk - s[idx]) / max(s[idx + 1] - s[idx], 1e-12)
        pos = (1 - a) * curve[idx] + a * curve[idx + 1]
        tang = curve[min(idx + 8, len(curve) - 1)] - curve[max(idx - 8, 0)]
        yaw = math.atan2(tang[1], tang[0])
        poses.append(pose_from_forward(pos, yaw, math.radians(pitch_deg)))
    return poses


def _path_positions(poses: Sequence[np.ndarray]) -> np.ndarray:
    return np.stack([p[:3, 3].astype(np.float64) for p in poses])


def random_objects(room: Tuple[float, float, float], rng: np.random.Generator,
                   n_spheres: int, n_boxes: int, path: np.ndarray, clearance: float,
                   r_range=(0.1, 0.6), half_range=(0.1, 0.5)):
    """Spheres and axis-aligned boxes inside the room, each kept at least
    ``clearance`` metres (surface distance) away from every path position."""
    L = np.asarray(room)
    spheres, boxes = [], []
    while len(spheres) < n_spheres:
        r = rng.uniform(*r_range)
        c = rng.uniform(r, L - r)
        if np.min(np.linalg.norm(path - c, axis=1)) - r >= clearance:
            spheres.append((tuple(float(v) for v in c), float(r)))
    while len(boxes) < n_boxes:
        h = rng.uniform(half_range[0], half_range[1], 3)
        c = rng.uniform(h, L - h)
        q = np.maximum(np.abs(path - c) - h, 0.0)
        if np.min(np.linalg.norm(q, axis=1)) >= clearance:
            boxes.append((tuple(float(v) for v in c - h), tuple(float(v) for v in c + h)))
    return spheres, boxes


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
@dataclass
class MapParams:
    voxel_size: float
    truncation_vox: float
    weighting: str          # "constant" or "linear_dropoff"
    max_weight: float = 100.0
    max_range: float = 5.0


@dataclass
class Workload:
    name: str
    camera: PinholeCamera
    scene: Scene
    poses: List[np.ndarray]
    params: MapParams
    noise_seed: Optional[int] = None
    dropout: float = 0.0

    def frames(self, device: str = "cpu", count: Optional[int] = None) -> List[np.ndarray]:
        """Render (and, if configured, corrupt) the first ``count`` depth frames."""
        n = len(self.poses) if count is None else min(count, len(self.poses))
        rng = np.random.default_rng(self.noise_seed) if self.noise_seed is not None else None
        out = []
        for k in range(n):
            d = render_depth(self.scene, self.camera, self.poses[k], device=device)
            if rng is not None:
                d = add_depth_noise(d, rng, dropout=self.dropout)
            out.append(d)
        return out


CAM_160 = PinholeCamera(160, 120, 140.0, 140.0, 80.0, 60.0)
CAM_640 = PinholeCamera(640, 480, 560.0, 560.0, 320.0, 240.0)


def box_room_single(seed: int = 0) -> Workload:
    """Plain FP32 single frame: 160x120 view of an empty 4 x 3 x 2.5 m box room,
    5 cm voxels, truncation 4 voxels, constant weight, no noise."""
    rng = np.random.default_rng(seed)
    room = (4.0, 3.0, 2.5)
    pos = rng.uniform([0.5, 0.5, 0.5], [3.5, 2.5, 2.0])
    yaw = rng.uniform(-math.pi, math.pi)
    pitch = math.radians(rng.uniform(-15.0, 15.0))
    pose = pose_from_forward(pos, yaw, pitch)
    return Workload("box_room_160x120_5cm", CAM_160, Scene(room=room), [pose],
                    MapParams(0.05, 4.0, "constant"))


def cluttered_room_sequence(n_frames: int = 300) -> Workload:
    """Plain FP32 sequence: 640x480 frames along a spline path (0.5 m/s, 30 fps)
    through an 8 x 6 x 3 m room with 40 spheres and 20 boxes; axial noise
    sigma = 0.0012 z^2 and 5 % dropped pixels; 4 cm voxels, truncation 4 voxels,
    linear-dropoff weight, max range 5 m."""
    room = (8.0, 6.0, 3.0)
    poses = spline_trajectory(room, n_frames, np.random.default_rng(1), margin=1.0)
    spheres, boxes = random_objects(room, np.random.default_rng(0), 40, 20,
                                    _path_positions(poses), clearance=0.6)
    return Workload("cluttered_room_640x480_4cm", CAM_640, Scene(room=room, spheres=spheres, boxes=boxes),
                    poses, MapParams(0.04, 4.0, "linear_dropoff"), noise_seed=2, dropout=0.05)


def box_room_sequence(voxel_size: float, n_frames: int = 300) -> Workload:
    """Precision workload: the 4 x 3 x 2.5 m box room at 640x480 along a spline
    path kept 0.6 m from the walls; no noise; constant weight."""
    room = (4.0, 3.0, 2.5)
    poses = spline_trajectory(room, n_frames, np.random.default_rng(1), margin=0.6)
    name = f"box_room_640x480_{int(round(voxel_size * 100))}cm"
    return Workload(name, CAM_640, Scene(room=room), poses,
                    MapParams(voxel_size, 4.0, "constant"))


def depth_edge_range(depth: np.ndarray) -> np.ndarray:
    """max - min of the valid depths in each pixel's 3x3 neighbourhood (0 where
    fewer than two are valid)."""
    d = np.asarray(depth, dtype=np.float64)
    valid = d > 0
    big = np.where(valid, d, -np.inf)
    small = np.where(valid, d, np.inf)
    H, W = d.shape
    pad_hi = np.pad(big, 1, constant_values=-np.inf)
    pad_lo = np.pad(small, 1, constant_values=np.inf)
    mx = np.full((H, W), -np.inf)
    mn = np.full((H, W), np.inf)
    for dj in range(3):
        for di in range(3):
            mx = np.maximum(mx, pad_hi[dj:dj + H, di:di + W])
            mn = np.minimum(mn, pad_lo[dj:dj + H, di:di + W])
    r = mx - mn
    return np.where(np.isfinite(r), r, 0.0), np.where(np.isfinite(mn), mn, 0.0), np.where(np.isfinite(mx), mx, 0.0)


def add_flying_pixels(noisy: np.ndarray, clean: np.ndarray, rng: np.random.Generator, frac: float = 0.03,
                      edge_range: float = 0.1) -> np.ndarray:
    """Flying pixels at depth edges: pixels whose 3x3 neighbourhood (in the clean
    render) spans more than `edge_range` metres are candidates; `frac` of all
    pixels (at most every candidate) take a value between the neighbourhood's
    nearest and farthest depth, d_fg + u (d_bg - d_fg) with u ~ U(0, 1)."""
    r, mn, mx = depth_edge_range(clean)
    cand = np.flatnonzero((r > edge_range) & (np.asarray(clean) > 0))
    k = min(len(cand), int(round(frac * clean.size)))
    out = np.array(noisy, dtype=np.float32, copy=True)
    if k == 0:
        return out
    pick = rng.choice(cand, size=k, replace=False)
    u = rng.uniform(0.0, 1.0, k)
    flat = out.reshape(-1)
    flat[pick] = (mn.reshape(-1)[pick] + u * (mx.reshape(-1)[pick] - mn.reshape(-1)[pick])).astype(np.float32)
    return out


@dataclass
class LearningRoom:
    """One room of the learned-sensor-model data: clean renders and their
    corrupted versions (axial noise sigma = 0.0012 z^2, then flying pixels)
    from the same poses."""
    seed: int
    camera: PinholeCamera
    scene: Scene
    poses: List[np.ndarray]

    def frames(self, device: str = "cpu", count: Optional[int] = None):
        n = len(self.poses) if count is None else min(count, len(self.poses))
        rng = np.random.default_rng(self.seed + 20000)
        clean, noisy = [], []
        for k in range(n):
            c = render_depth(self.scene, self.camera, self.poses[k], device=device)
            nz = add_depth_noise(c, rng, dropout=0.0)
            noisy.append(add_flying_pixels(nz, c, rng))
            clean.append(c)
        return clean, noisy


def learning_room(seed: int, n_frames: int = 100, camera: Optional[PinholeCamera] = None) -> LearningRoom:
    """The cluttered-room generator (8 x 6 x 3 m, 40 spheres, 20 boxes, spline
    path at 0.5 m/s and 30 fps) with scene seed `seed` and path seed
    seed + 10000.  Rooms 1000-1019 are the training set."""
    camera = camera or CAM_640
    room = (8.0, 6.0, 3.0)
    poses = spline_trajectory(room, n_frames, np.random.default_rng(seed + 10000), margin=1.0)
    spheres, boxes = random_objects(room, np.random.default_rng(seed), 40, 20, _path_positions(poses),
                                    clearance=0.6)
    return LearningRoom(seed, camera, Scene(room=room, spheres=spheres, boxes=boxes), poses)


def random_frame(cam: PinholeCamera, rng: np.random.Generator, lo: float = 0.3, hi: float = 6.0,
                 invalid_frac: float = 0.1) -> np.ndarray:
    """Unstructured depth (uniform in [lo, hi]) with a fraction of invalid
    pixels drawn from {0, -1, NaN, +Inf}; used for edge-case tests."""
    d = rng.uniform(lo, hi, (cam.height, cam.width))
    bad = rng.random(d.shape) < invalid_frac
    choice = rng.integers(0, 4, d.shape)
    vals = np.array([0.0, -1.0, np.nan, np.inf])[choice]
    return np.where(bad, vals, d).astype(np.float32)


# --------------------------------------------------------------------------
# Multi-sensor rig
# --------------------------------------------------------------------------
RIG_SIZES = ((640, 480), (848, 480), (424, 240), (1280, 720))


@dataclass
class RigStep:
    cameras: List[PinholeCamera]
    poses: List[np.ndarray]
    lidar_pose: Optional[np.ndarray] = None


def rig_cameras() -> List[PinholeCamera]:
    """Four pinhole depth cameras of uneven sizes, f = 0.875 W, centred principal point."""
    return [PinholeCamera(w, h, 0.875 * w, 0.875 * w, w / 2.0, h / 2.0) for (w, h) in RIG_SIZES]


def rig_extrinsics(seed: int = 3) -> List[Tuple[float, float]]:
    """Yaw (0, 90, 180, 270 deg, each +- U(10 deg)) and pitch U(+-5 deg) of the rig cameras."""
    rng = np.random.default_rng(seed)
    return [(math.radians(90.0 * k + rng.uniform(-10, 10)), math.radians(rng.uniform(-5, 5)))
            for k in range(4)]


def rig_sequence(n_steps: int, room=(20.0, 15.0, 3.0), speed: float = 0.5, rate: float = 10.0,
                 seed_path: int = 1, seed_scene: int = 0, seed_rig: int = 3):
    """Cameras of the rig carried along a spline path through a cluttered room
    (40 spheres, 20 boxes): returns (scene, steps)."""
    base = spline_trajectory(room, n_steps, np.random.default_rng(seed_path), margin=1.0,
                             speed=speed, fps=rate, pitch_deg=0.0)
    spheres, boxes = random_objects(room, np.random.default_rng(seed_scene), 40, 20,
                                    _path_positions(base), clearance=0.6)
    cams = rig_cameras()
    ext = rig_extrinsics(seed_rig)
    steps = []
    for T in base:
        Tb = T.astype(np.float64)
        yaw0 = math.atan2(Tb[1, 2], Tb[0, 2])
        poses = [pose_from_forward(Tb[:3, 3], yaw0 + dy, dp) for (dy, dp) in ext]
        lidar_pose = pose_lidar(Tb[:3, 3] + np.array([0.0, 0.0, 0.15]), yaw0)
        steps.append(RigStep(cams, poses, lidar_pose))
    return Scene(room=room, spheres=spheres, boxes=boxes), steps
