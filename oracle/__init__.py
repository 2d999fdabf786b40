"""Python view of the CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``libtsdf_oracle.so`` (plain C, see
``tsdf_oracle.h``) with numpy arrays; it shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TSDF_ORACLE_LIB points the wrapper at another build of the same sources
# (the mutation test builds deliberately broken copies to check the pins).
_LIB_PATH = os.environ.get("TSDF_ORACLE_LIB") or os.path.join(_HERE, "libtsdf_oracle.so")
_lib = None

WEIGHTINGS = {"constant": 0, "linear_dropoff": 1}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = C.CDLL(_LIB_PATH)
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    lib.ora_create.restype = C.c_void_p
    lib.ora_create.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int]
    lib.ora_destroy.argtypes = [C.c_void_p]
    lib.ora_set_storage16.restype = C.c_int
    lib.ora_set_storage16.argtypes = [C.c_void_p]
    lib.ora_round_binary16.restype = C.c_float
    lib.ora_round_binary16.argtypes = [C.c_float]
    lib.ora_integrate_depth.restype = C.c_longlong
    lib.ora_integrate_depth.argtypes = [C.c_void_p, f32p, C.c_int, C.c_int, f32p, f32p]
    lib.ora_integrate_depth_threads.restype = C.c_longlong
    lib.ora_integrate_depth_threads.argtypes = [C.c_void_p, f32p, C.c_int, C.c_int, f32p, f32p, C.c_int]
    lib.ora_integrate_depth_range.restype = C.c_longlong
    lib.ora_integrate_depth_range.argtypes = [C.c_void_p, f32p, C.c_int, C.c_int, f32p, f32p, C.c_float]
    lib.ora_integrate_range.restype = C.c_longlong
    lib.ora_integrate_range.argtypes = [C.c_void_p, f32p, C.c_int, C.c_int, f32p, f32p]
    lib.ora_dense_integrate_range.restype = C.c_longlong
    lib.ora_dense_integrate_range.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int,
                                              f32p, C.c_int, C.c_int, f32p, f32p, i32p, i32p, f64p, f64p]
    lib.ora_atan2_f32.restype = C.c_float
    lib.ora_atan2_f32.argtypes = [C.c_float, C.c_float]
    lib.ora_num_blocks.restype = C.c_longlong
    lib.ora_num_blocks.argtypes = [C.c_void_p]
    lib.ora_blocks.argtypes = [C.c_void_p, i32p]
    lib.ora_voxels.argtypes = [C.c_void_p, f64p, f64p]
    lib.ora_find_block.restype = C.c_longlong
    lib.ora_find_block.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    lib.ora_touched.restype = C.c_longlong
    lib.ora_touched.argtypes = [C.c_void_p, C.c_void_p]
    lib.ora_last_scan.argtypes = [C.c_void_p, i32p, i32p]
    lib.ora_camera_from_world.argtypes = [C.c_int, f32p, f64p, f64p]
    lib.ora_dense_integrate.restype = C.c_longlong
    lib.ora_dense_integrate.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int,
                                        f32p, C.c_int, C.c_int, f32p, f32p, i32p, i32p, f64p, f64p]
    lib.ora_integrate_depth_dda.restype = C.c_longlong
    lib.ora_integrate_depth_dda.argtypes = [C.c_void_p, f32p, C.c_int, C.c_int, f32p, f32p]
    lib.ora_round_bf16.restype = C.c_float
    lib.ora_round_bf16.argtypes = [C.c_float]
    lib.ora_sm_features.restype = None
    lib.ora_sm_features.argtypes = [f32p, C.c_int, C.c_int, f32p, C.c_float, f32p]
    lib.ora_sm_maps.restype = C.c_int
    lib.ora_sm_maps.argtypes = [f32p, C.c_int, C.c_int, f32p, C.c_float, C.c_float, f32p, f32p, f32p]
    lib.ora_integrate_learned.restype = C.c_longlong
    lib.ora_integrate_learned.argtypes = [C.c_void_p, f32p, C.c_int, C.c_int, f32p, f32p, f32p, f32p]
    lib.ora_sm_loss_grad.restype = C.c_double
    lib.ora_sm_loss_grad.argtypes = [f32p, C.c_int, f32p, C.c_int, C.c_int, f32p, f32p, C.c_float, C.c_float,
                                     C.c_longlong, i32p, f64p, C.c_int, f64p, C.POINTER(C.c_longlong)]
    _lib = lib
    return lib


def _f32(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if n is not None:
        a = a.reshape(n)
    return a


class OracleMap:
    """Sparse TSDF map integrated on the CPU in binary32 (``precision=32``,
    the parity oracle) or binary64 (``precision=64``, the error oracle)."""

    def __init__(self, voxel_size: float, truncation_vox: float, *, precision: int = 32,
                 max_weight: float = 100.0, max_range: float = 5.0, weighting: str = "constant",
                 storage: str = "fp32"):
        lib = _load()
        self.precision = precision
        self.voxel_size = voxel_size
        self._h = lib.ora_create(precision, voxel_size, truncation_vox, max_weight, max_range,
                                 WEIGHTINGS[weighting])
        if not self._h:
            raise ValueError("invalid oracle map parameters")
        if storage == "fp16" and lib.ora_set_storage16(self._h) != 0:
            raise ValueError("binary16 storage needs precision 32")

    @classmethod
    def from_params(cls, params, precision: int = 32, storage: str = "fp32") -> "OracleMap":
        return cls(params.voxel_size, params.truncation_vox, precision=precision,
                   max_weight=params.max_weight, max_range=params.max_range,
                   weighting=params.weighting, storage=storage)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ora_destroy(h)
            self._h = None

    def integrate(self, depth: np.ndarray, K, T_world_cam, max_range: float = 0.0) -> int:
        """One frame; max_range > 0 replaces the map's max range for it."""
        depth = _f32(depth)
        H, W = depth.shape
        if max_range > 0:
            n = _lib.ora_integrate_depth_range(self._h, depth, W, H, _f32(K, 4), _f32(T_world_cam, 16),
                                               max_range)
        else:
            n = _lib.ora_integrate_depth(self._h, depth, W, H, _f32(K, 4), _f32(T_world_cam, 16))
        if n < 0:
            raise ValueError("oracle rejected the frame")
        return int(n)

    def integrate_threads(self, depth: np.ndarray, K, T_world_cam, threads: int) -> int:
        """integrate() on `threads` OpenMP threads (bitwise the same map)."""
        depth = _f32(depth)
        H, W = depth.shape
        n = _lib.ora_integrate_depth_threads(self._h, depth, W, H, _f32(K, 4), _f32(T_world_cam, 16), int(threads))
        if n < 0:
            raise ValueError("oracle rejected the frame")
        return int(n)

    def integrate_range(self, rng: np.ndarray, lidar, T_world_sensor) -> int:
        """One spherical range image; lidar has .params() = float32 [azimuth
        start, azimuth fov, polar start, polar fov, interp max diff, max range]."""
        rng = _f32(rng)
        H, W = rng.shape
        n = _lib.ora_integrate_range(self._h, rng, W, H, _f32(lidar.params(), 6), _f32(T_world_sensor, 16))
        if n < 0:
            raise ValueError("oracle rejected the range image")
        return int(n)

    def integrate_dda(self, depth: np.ndarray, K, T_world_cam) -> int:
        """One pinhole frame with ray-DDA allocation (blocks along pixel rays)."""
        depth = _f32(depth)
        H, W = depth.shape
        n = _lib.ora_integrate_depth_dda(self._h, depth, W, H, _f32(K, 4), _f32(T_world_cam, 16))
        if n < 0:
            raise ValueError("oracle rejected the frame")
        return int(n)

    def integrate_learned(self, depth: np.ndarray, K, T_world_cam, w_map, eps_map) -> int:
        """One pinhole frame with per-pixel weight and truncation maps."""
        depth = _f32(depth)
        H, W = depth.shape
        n = _lib.ora_integrate_learned(self._h, depth, W, H, _f32(K, 4), _f32(T_world_cam, 16),
                                       _f32(w_map).reshape(H, W), _f32(eps_map).reshape(H, W))
        if n < 0:
            raise ValueError("oracle rejected the frame")
        return int(n)

    def num_blocks(self) -> int:
        return int(_lib.ora_num_blocks(self._h))

    def blocks(self) -> np.ndarray:
        out = np.empty((self.num_blocks(), 3), np.int32)
        if out.size:
            _lib.ora_blocks(self._h, out)
        return out

    def voxels(self) -> Tuple[np.ndarray, np.ndarray]:
        n = self.num_blocks()
        d = np.zeros((n, 512), np.float64)
        w = np.zeros((n, 512), np.float64)
        if n:
            _lib.ora_voxels(self._h, d, w)
        return d, w

    def find(self, x: int, y: int, z: int) -> int:
        return int(_lib.ora_find_block(self._h, x, y, z))

    def touched(self) -> np.ndarray:
        n = int(_lib.ora_touched(self._h, None))
        out = np.empty((n, 3), np.int32)
        if n:
            _lib.ora_touched(self._h, out.ctypes.data_as(C.c_void_p))
        return out

    def last_scan(self) -> Tuple[np.ndarray, np.ndarray]:
        lo = np.empty(3, np.int32)
        hi = np.empty(3, np.int32)
        _lib.ora_last_scan(self._h, lo, hi)
        return lo, hi

    def sorted_state(self):
        """(blocks, dist, weight) sorted by block index (x, y, z)."""
        b = self.blocks()
        d, w = self.voxels()
        order = np.lexsort((b[:, 2], b[:, 1], b[:, 0]))
        return b[order], d[order], w[order]


def _dense_state(state, n):
    """Flat (dist, weight) binary64 arrays: zeros, or a copy of an earlier
    call's result on the same box to continue from."""
    if state is None:
        return np.zeros(n, np.float64), np.zeros(n, np.float64)
    return (np.array(state[0], dtype=np.float64).reshape(n), np.array(state[1], dtype=np.float64).reshape(n))


def dense_integrate_range(params, images, lidar, poses, gmin, gdim, precision: int = 32, state=None):
    """Dense brute force of range images over a voxel box; (dist, weight)
    shaped (gdim[2], gdim[1], gdim[0]).  `state`: the (dist, weight) of an
    earlier dense call on the same box, to continue from (frames of several
    sensors in their order)."""
    lib = _load()
    gmin = np.ascontiguousarray(np.asarray(gmin, np.int32))
    gdim = np.ascontiguousarray(np.asarray(gdim, np.int32))
    n = int(np.prod(gdim.astype(np.int64)))
    dist, weight = _dense_state(state, n)
    for img, T in zip(images, poses):
        img = _f32(img)
        H, W = img.shape
        r = lib.ora_dense_integrate_range(precision, params.voxel_size, params.truncation_vox, params.max_weight,
                                          params.max_range, WEIGHTINGS[params.weighting], img, W, H,
                                          _f32(lidar.params(), 6), _f32(T, 16), gmin, gdim, dist, weight)
        if r < 0:
            raise ValueError("oracle rejected the range image")
    shape = (int(gdim[2]), int(gdim[1]), int(gdim[0]))
    return dist.reshape(shape), weight.reshape(shape)


def atan2_f32(y: float, x: float) -> float:
    return float(_load().ora_atan2_f32(y, x))


def round_binary16(x: float) -> float:
    return float(_load().ora_round_binary16(x))


def camera_from_world(T_world_cam, precision: int = 32):
    lib = _load()
    R = np.empty(9, np.float64)
    t = np.empty(3, np.float64)
    lib.ora_camera_from_world(precision, _f32(T_world_cam, 16), R, t)
    return R.reshape(3, 3), t


def dense_integrate(params, frames, K, poses, gmin, gdim, precision: int = 32, state=None):
    """Brute force over a dense voxel box (no blocks, hash or candidates).
    Returns (dist, weight) arrays shaped (gdim[2], gdim[1], gdim[0]); `state`
    as in dense_integrate_range."""
    lib = _load()
    gmin = np.ascontiguousarray(np.asarray(gmin, np.int32))
    gdim = np.ascontiguousarray(np.asarray(gdim, np.int32))
    n = int(np.prod(gdim.astype(np.int64)))
    dist, weight = _dense_state(state, n)
    for depth, T in zip(frames, poses):
        depth = _f32(depth)
        H, W = depth.shape
        r = lib.ora_dense_integrate(precision, params.voxel_size, params.truncation_vox,
                                    params.max_weight, params.max_range,
                                    WEIGHTINGS[params.weighting], depth, W, H, _f32(K, 4),
                                    _f32(T, 16), gmin, gdim, dist, weight)
        if r < 0:
            raise ValueError("oracle rejected the frame")
    shape = (int(gdim[2]), int(gdim[1]), int(gdim[0]))
    return dist.reshape(shape), weight.reshape(shape)


SM_NPARAM = 2018


def round_bf16(x: float) -> float:
    return float(_load().ora_round_bf16(x))


def sm_features(depth, K, max_range: float) -> np.ndarray:
    """(H, W, 27) binary32 input features of the learned sensor model."""
    lib = _load()
    depth = _f32(depth)
    H, W = depth.shape
    out = np.empty((H, W, 27), np.float32)
    lib.ora_sm_features(depth, W, H, _f32(K, 4), max_range, out)
    return out


def sm_maps(depth, K, max_range: float, voxel_size: float, params) -> Tuple[np.ndarray, np.ndarray]:
    """Per-pixel (weight, truncation) maps of the bfloat16-emulating forward."""
    lib = _load()
    depth = _f32(depth)
    H, W = depth.shape
    w = np.empty((H, W), np.float32)
    e = np.empty((H, W), np.float32)
    if lib.ora_sm_maps(depth, W, H, _f32(K, 4), max_range, voxel_size, _f32(params, SM_NPARAM), w, e) != 0:
        raise ValueError("oracle rejected the sensor-model inputs")
    return w, e


def sm_loss_grad(params, frames, K, poses, voxel_size: float, max_range: float, vox, target,
                 emulate_bf16: bool = True):
    """(loss, gradient (2018,), voxels used) of the learned sensor model's
    training loss in binary64 (see sensor_model_impl.h)."""
    lib = _load()
    frames = np.ascontiguousarray(np.stack([_f32(f) for f in frames]))
    n, H, W = frames.shape
    T = np.ascontiguousarray(np.stack([_f32(t, 16) for t in poses]))
    vox = np.ascontiguousarray(np.asarray(vox, np.int32).reshape(-1, 3))
    target = np.ascontiguousarray(np.asarray(target, np.float64).reshape(-1))
    grad = np.zeros(SM_NPARAM, np.float64)
    used = C.c_longlong()
    loss = lib.ora_sm_loss_grad(_f32(params, SM_NPARAM), n, frames.reshape(-1), W, H, _f32(K, 4), T.reshape(-1),
                                voxel_size, max_range, len(vox), vox.reshape(-1), target, int(emulate_bf16),
                                grad, C.byref(used))
    if loss < 0:
        raise MemoryError("oracle out of memory")
    return float(loss), grad, int(used.value)
