"""Closed-form geometry used by the pins (float64, independent of the oracle).

Nothing here performs the integration method; these are signed distances of
analytic shapes and a camera-frustum membership test, used to state what the
fused field must equal.
"""
import numpy as np


def voxel_centres(blocks: np.ndarray, voxel_size: float) -> np.ndarray:
    """(n, 512, 3) float64 centres of the voxels of integer blocks, voxel
    (lx, ly, lz) at index lx + 8 ly + 64 lz."""
    l = np.arange(512)
    local = np.stack([l % 8, (l // 8) % 8, l // 64], axis=1)          # (512, 3)
    g = blocks[:, None, :].astype(np.int64) * 8 + local[None]
    return (g.astype(np.float64) + 0.5) * float(np.float32(voxel_size))


def world_to_camera(T_world_cam: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Camera-frame coordinates using a float64 matrix inverse of the pose."""
    T = np.asarray(T_world_cam, np.float64)
    Ti = np.linalg.inv(T)
    return p @ Ti[:3, :3].T + Ti[:3, 3]


def frustum_margin(cam, pc: np.ndarray) -> np.ndarray:
    """Signed pixel distance of each camera-frame point's projection to the
    image border (positive inside); -inf behind the camera."""
    z = pc[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam.fx * pc[..., 0] / z + cam.cx
        v = cam.fy * pc[..., 1] / z + cam.cy
    m = np.minimum.reduce([u, cam.width - u, v, cam.height - v])
    return np.where(z > 0, m, -np.inf)


def plane_sdf(p: np.ndarray, n, c: float) -> np.ndarray:
    """Signed distance to the plane n.x = c, positive on the side n.x < c."""
    n = np.asarray(n, np.float64)
    return c - p @ n


def sphere_sdf(p: np.ndarray, centre, r: float) -> np.ndarray:
    return np.linalg.norm(p - np.asarray(centre, np.float64), axis=-1) - r


def room_sdf(p: np.ndarray, L):
    """Distance to the nearest wall of the box room [0, L] (positive inside),
    the index of that wall, and the gap to the second-nearest wall."""
    L = np.asarray(L, np.float64)
    walls = np.concatenate([p, L - p], axis=-1)                        # (..., 6)
    order = np.sort(walls, axis=-1)
    return order[..., 0], np.argmin(walls, axis=-1), order[..., 1] - order[..., 0]


ROOM_NORMALS = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1],
                         [-1, 0, 0], [0, -1, 0], [0, 0, -1]], np.float64)   # into the room
