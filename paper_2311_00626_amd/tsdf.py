"""Thin ctypes binding of ``lib/libtsdf.so`` (the C ABI in include/tsdf.h).

Argument marshalling only: every step of integration and every query runs in
the library's HIP kernels.  PyTorch supplies device memory and the current
stream.  Importing this module raises if the library has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libtsdf.so")

OK, EINVAL, ENOMEM, EFULL, EDEVICE, ESTATE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6
WEIGHTINGS = {"constant": 0, "linear_dropoff": 1, "learned": 2}
SM_NPARAM = 2018
SM_MAX_FRAMES = 16
STORAGES = {"fp32": 0, "fp16": 1}
ALLOCATIONS = {"exact": 0, "ray_walk": 1}


class TsdfError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {strerror(status)} (status {status})")
        self.status = status


class tsdf_stats(C.Structure):
    _fields_ = [("blocks", C.c_longlong), ("voxel_updates", C.c_longlong),
                ("voxel_writes", C.c_longlong), ("touched_blocks", C.c_longlong),
                ("launches", C.c_longlong), ("candidate_blocks", C.c_longlong),
                ("block_capacity", C.c_longlong), ("hash_capacity", C.c_longlong),
                ("error_bits", C.c_longlong)]

# tsdf_stats.error_bits
ERR_POOL_FULL, ERR_HASH_FULL, ERR_TOUCHED_OVERFLOW, ERR_INSERT_RACE, ERR_WALK_OUTSIDE = 1, 2, 4, 8, 16


class tsdf_depth_view(C.Structure):
    _fields_ = [("depth_dev", C.c_void_p), ("width", C.c_int), ("height", C.c_int),
                ("model", C.c_int), ("max_range_m", C.c_float), ("K", C.c_float * 4),
                ("interp_max_diff_m", C.c_float), ("reserved", C.c_float), ("T_world_cam", C.c_float * 16)]


class tsdf_lidar_model(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("azimuth_start_rad", C.c_float),
                ("azimuth_fov_rad", C.c_float), ("polar_start_rad", C.c_float), ("polar_fov_rad", C.c_float),
                ("interp_max_diff_m", C.c_float), ("max_range_m", C.c_float)]


MODEL_PINHOLE, MODEL_SPHERICAL = 0, 1


def lidar_struct(lidar) -> tsdf_lidar_model:
    """tsdf_lidar_model of an object with width, height and params() (see synth.LidarModel)."""
    if isinstance(lidar, tsdf_lidar_model):
        return lidar
    p = [float(x) for x in np.asarray(lidar.params(), dtype=np.float32)]
    return tsdf_lidar_model(int(lidar.width), int(lidar.height), *p)


MAX_VIEWS = 16
FOOTPRINT = {"auto": 0, "never": 1, "always": 2}
COMPACTION = {"auto": 0, "never": 1, "always": 2}
STAGING = {"auto": 0, "never": 1, "always": 2}


class tsdf_launch_config(C.Structure):
    _fields_ = [("max_groups", C.c_int), ("partitions", C.c_int), ("chunk", C.c_int), ("footprint", C.c_int),
                ("compaction", C.c_int), ("staging", C.c_int)]


class tsdf_params(C.Structure):
    _fields_ = [("voxel_size_m", C.c_float), ("truncation_vox", C.c_float),
                ("max_weight", C.c_float), ("max_range_m", C.c_float),
                ("weighting", C.c_int), ("storage", C.c_int),
                ("block_capacity", C.c_longlong), ("hash_capacity", C.c_longlong),
                ("allocation", C.c_int), ("reserved", C.c_int)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, ll, i = C.c_void_p, C.c_longlong, C.c_int
    fp = C.POINTER(C.c_float)
    lib.tsdf_default_params.argtypes = [C.POINTER(tsdf_params), C.c_float, C.c_float]
    lib.tsdf_default_params.restype = None
    lib.create_map.argtypes = [C.c_float, C.c_float, C.POINTER(vp)]
    lib.create_map_ex.argtypes = [C.POINTER(tsdf_params), C.POINTER(vp)]
    lib.destroy_map.argtypes = [vp]
    lib.reserve.argtypes = [vp, ll]
    lib.integrate_depth.argtypes = [vp, vp, i, i, vp, vp, vp]
    lib.integrate_depth_noalloc.argtypes = [vp, vp, i, i, vp, vp, vp]
    lib.query_blocks.argtypes = [vp, vp, ll, C.POINTER(ll), vp]
    lib.query_tsdf.argtypes = [vp, vp, ll, vp, vp, vp]
    lib.insert_blocks.argtypes = [vp, vp, ll, vp, vp, vp]
    lib.query_touched.argtypes = [vp, vp, ll, C.POINTER(ll), vp]
    lib.map_stats.argtypes = [vp, C.POINTER(tsdf_stats), vp]
    lib.integrate_depth_views.argtypes = [vp, C.POINTER(tsdf_depth_view), i, vp]
    lib.integrate_range.argtypes = [vp, vp, C.POINTER(tsdf_lidar_model), vp, vp]
    lib.map_status.argtypes = [vp]
    lib.tsdf_strerror.argtypes = [i]
    lib.tsdf_strerror.restype = C.c_char_p
    lib.tsdf_profile.argtypes = [vp, i]
    lib.tsdf_set_launch_config.argtypes = [vp, C.POINTER(tsdf_launch_config)]
    lib.tsdf_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(ll)]
    lib.tsdf_step_create.argtypes = [vp, i, C.POINTER(vp)]
    lib.tsdf_step_run.argtypes = [vp, C.POINTER(tsdf_depth_view), i, vp]
    lib.tsdf_step_destroy.argtypes = [vp]
    lib.tsdf_set_sensor_model.argtypes = [vp, vp]
    lib.tsdf_sensor_maps.argtypes = [vp, i, i, vp, C.c_float, C.c_float, vp, vp, vp]
    lib.tsdf_sm_trainer_create.argtypes = [i, i, i, C.POINTER(vp)]
    lib.tsdf_sm_trainer_destroy.argtypes = [vp]
    lib.tsdf_sm_loss_grad.argtypes = [vp, vp, i, vp, vp, vp, C.c_float, C.c_float, ll, vp, vp, vp, vp, vp]
    lib.tsdf_sm_adam.argtypes = [vp, vp, vp, vp, vp, i, C.c_float, C.c_float, C.c_float, C.c_float, i, vp]
    for name in ("create_map", "create_map_ex", "destroy_map", "reserve", "integrate_depth",
                 "integrate_depth_noalloc", "integrate_depth_views",
                 "integrate_range",
                 "query_blocks", "insert_blocks",
                 "query_tsdf", "query_touched", "map_stats", "map_status", "tsdf_profile",
                 "tsdf_profile_read", "tsdf_set_launch_config", "tsdf_step_create", "tsdf_step_run",
                 "tsdf_step_destroy", "tsdf_set_sensor_model", "tsdf_sensor_maps", "tsdf_sm_trainer_create",
                 "tsdf_sm_trainer_destroy", "tsdf_sm_loss_grad", "tsdf_sm_adam"):
        getattr(lib, name).restype = C.c_int
    return lib


lib = _load()

EXPORTED = ("tsdf_default_params", "create_map", "create_map_ex", "destroy_map", "reserve", "integrate_depth",
            "integrate_depth_noalloc",
            "integrate_depth_views", "integrate_range",
            "query_blocks", "insert_blocks", "query_tsdf", "query_touched", "map_stats", "map_status",
            "tsdf_strerror", "tsdf_profile", "tsdf_profile_read", "tsdf_set_launch_config",
            "tsdf_step_create", "tsdf_step_run", "tsdf_step_destroy", "tsdf_set_sensor_model", "tsdf_sensor_maps",
            "tsdf_sm_trainer_create", "tsdf_sm_trainer_destroy", "tsdf_sm_loss_grad", "tsdf_sm_adam")


def strerror(status: int) -> str:
    return lib.tsdf_strerror(status).decode()


def _check(status: int, where: str) -> None:
    if status != OK:
        raise TsdfError(status, where)


_RAW_STREAM = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_ptr(stream: Optional[torch.cuda.Stream], device: Optional[int] = None) -> int:
    """HIP stream handle: `stream`, else torch's current stream on `device`
    (the current device if None)."""
    if stream is not None:
        return stream.cuda_stream
    if _RAW_STREAM is not None:      # a plain integer, without building a Stream object
        return _RAW_STREAM(torch.cuda.current_device() if device is None else device)
    return torch.cuda.current_stream(device).cuda_stream


def _host_f32(a, n: int) -> np.ndarray:
    if type(a) is np.ndarray and a.dtype == np.float32 and a.size == n and a.flags.c_contiguous:
        return a.reshape(n)
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(n))


def default_params(voxel_size: float, truncation_vox: float) -> tsdf_params:
    p = tsdf_params()
    lib.tsdf_default_params(C.byref(p), voxel_size, truncation_vox)
    return p


# tsdf_depth_view as a NumPy record (same 112-byte layout), so that a batch's
# arguments are filled column by column instead of field by field.
_VIEW_DTYPE = np.dtype({"names": ["depth_dev", "width", "height", "model", "max_range_m", "K",
                                  "interp_max_diff_m", "reserved", "T_world_cam"],
                        "formats": ["<u8", "<i4", "<i4", "<i4", "<f4", ("<f4", 4), "<f4", "<f4", ("<f4", 16)],
                        "offsets": [0, 8, 12, 16, 20, 24, 40, 44, 48], "itemsize": C.sizeof(tsdf_depth_view)})


class ViewBatch:
    """The tsdf_depth_view array of a batch of views (see views_array)."""

    def __init__(self, rec: np.ndarray):
        self.rec = rec
        self.ptr = C.cast(rec.ctypes.data, C.POINTER(tsdf_depth_view))

    def __getitem__(self, k):
        return self.ptr[k]


def views_array(depths: Sequence[torch.Tensor], Ks, Ts, max_ranges=None):
    """(ViewBatch, n) of a batch of depth / range images: the tsdf_depth_view
    array the C entry points take (ViewBatch.ptr), kept alive by the batch."""
    n = len(depths)
    if not 1 <= n <= MAX_VIEWS or len(Ks) != n or len(Ts) != n:
        raise ValueError(f"need 1..{MAX_VIEWS} views with matching K and T")
    rec = np.zeros(n, _VIEW_DTYPE)
    ptrs, shapes = [], []
    for d in depths:
        if not (d.is_cuda and d.dtype == torch.float32 and d.dim() == 2 and d.is_contiguous()):
            raise ValueError("each depth must be a contiguous 2-D float32 CUDA tensor")
        ptrs.append(d.data_ptr())
        shapes.append(d.shape)
    rec["depth_dev"] = ptrs
    rec["height"] = [h for h, _ in shapes]
    rec["width"] = [w for _, w in shapes]
    T = np.asarray(Ts, dtype=np.float32)
    if T.size != 16 * n:
        raise ValueError("each pose must hold 16 values (row-major 4x4)")
    rec["T_world_cam"] = T.reshape(n, 16)
    if max_ranges is not None:
        rec["max_range_m"] = np.asarray(max_ranges, dtype=np.float32).reshape(n)
    if not any(hasattr(K, "params") for K in Ks):
        rec["K"] = np.asarray(Ks, dtype=np.float32).reshape(n, 4)
    else:
        for k, K in enumerate(Ks):
            if hasattr(K, "params"):
                lm = lidar_struct(K)
                rec["model"][k] = MODEL_SPHERICAL
                rec["K"][k] = [lm.azimuth_start_rad, lm.azimuth_fov_rad, lm.polar_start_rad, lm.polar_fov_rad]
                rec["interp_max_diff_m"][k] = lm.interp_max_diff_m
                if rec["max_range_m"][k] == 0.0:
                    rec["max_range_m"][k] = lm.max_range_m
            else:
                rec["K"][k] = _host_f32(K, 4)
    return ViewBatch(rec), n


class TsdfMap:
    """A block-sparse TSDF layer on the current GPU (see include/tsdf.h)."""

    def __init__(self, voxel_size: float, truncation_vox: float, *, max_weight: float = 100.0,
                 max_range: float = 5.0, weighting: str = "constant", storage: str = "fp32",
                 block_capacity: int = 1 << 18, hash_capacity: int = 0, allocation: str = "exact"):
        p = default_params(voxel_size, truncation_vox)
        p.max_weight = max_weight
        p.max_range_m = max_range
        p.weighting = WEIGHTINGS[weighting]
        p.storage = STORAGES[storage]
        p.block_capacity = block_capacity
        p.hash_capacity = hash_capacity
        p.allocation = ALLOCATIONS[allocation]
        h = C.c_void_p()
        _check(lib.create_map_ex(C.byref(p), C.byref(h)), "create_map_ex")
        self._h = h
        self.params = p
        self.block_capacity = block_capacity
        # per-map host staging of K and the pose: the library copies both by
        # value during a call, so one buffer each is reused call after call
        # (filled in place, their addresses taken once)
        self._K = (C.c_float * 4)()
        self._K_addr = C.addressof(self._K)
        self._T = np.empty(16, np.float32)
        self._T44 = self._T.reshape(4, 4)     # the same memory: a 4x4 pose is copied in one step
        self._T_addr = self._T.ctypes.data

    @classmethod
    def from_params(cls, params, **kw) -> "TsdfMap":
        """A map with the fields of `params` (synth.MapParams); keyword
        arguments override them."""
        args = dict(max_weight=params.max_weight, max_range=params.max_range, weighting=params.weighting)
        args.update(kw)
        return cls(params.voxel_size, params.truncation_vox, **args)

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib.destroy_map(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, block_capacity: int) -> None:
        """Grows the block pool (and the hash) to block_capacity blocks; every
        block keeps its voxels.  Also clears a sticky overflow (see tsdf.h)."""
        _check(lib.reserve(self._h, int(block_capacity)), "reserve")
        self.block_capacity = max(self.block_capacity, int(block_capacity))

    # -- integration --------------------------------------------------------
    def _set_pose(self, T) -> None:
        """Copies a 4x4 (or 16-element) row-major pose into the call's binary32 buffer."""
        if getattr(T, "shape", None) == (4, 4):
            self._T44[...] = T
        else:
            self._T[:] = np.reshape(T, 16)

    def integrate_depth(self, depth: torch.Tensor, K: Sequence[float], T_world_cam,
                        stream: Optional[torch.cuda.Stream] = None) -> None:
        if not (depth.is_cuda and depth.dtype == torch.float32 and depth.dim() == 2
                and depth.is_contiguous()):
            raise ValueError("depth must be a contiguous 2-D float32 CUDA tensor")
        self._K[:] = K
        self._set_pose(T_world_cam)
        H, W = depth.shape
        st = lib.integrate_depth(self._h, depth.data_ptr(), W, H, self._K_addr, self._T_addr,
                                 _stream_ptr(stream, depth.get_device()))
        _check(st, "integrate_depth")

    def integrate_depth_noalloc(self, depth: torch.Tensor, K: Sequence[float], T_world_cam,
                                stream: Optional[torch.cuda.Stream] = None) -> None:
        """integrate_depth with the library's fixed device scratch: the call
        allocates no device memory (see tsdf.h for its limits)."""
        if not (depth.is_cuda and depth.dtype == torch.float32 and depth.dim() == 2
                and depth.is_contiguous()):
            raise ValueError("depth must be a contiguous 2-D float32 CUDA tensor")
        self._K[:] = K
        self._set_pose(T_world_cam)
        H, W = depth.shape
        st = lib.integrate_depth_noalloc(self._h, depth.data_ptr(), W, H, self._K_addr, self._T_addr,
                                         _stream_ptr(stream, depth.get_device()))
        _check(st, "integrate_depth_noalloc")

    def integrate_range(self, rng: torch.Tensor, lidar, T_world_sensor,
                        stream: Optional[torch.cuda.Stream] = None) -> None:
        """One LiDAR range image; lidar is a LidarModel (or tsdf_lidar_model)."""
        if not (rng.is_cuda and rng.dtype == torch.float32 and rng.dim() == 2 and rng.is_contiguous()):
            raise ValueError("range must be a contiguous 2-D float32 CUDA tensor")
        lm = lidar_struct(lidar)
        if (lm.height, lm.width) != tuple(rng.shape):
            raise ValueError("range image shape does not match the LiDAR model")
        self._set_pose(T_world_sensor)
        _check(lib.integrate_range(self._h, rng.data_ptr(), C.byref(lm), self._T_addr, _stream_ptr(stream)),
               "integrate_range")

    def integrate_depth_views(self, depths: Sequence[torch.Tensor], Ks, Ts, max_ranges=None,
                              stream: Optional[torch.cuda.Stream] = None) -> None:
        """Fuses up to MAX_VIEWS views in one launch; bit-identical to calling
        integrate_depth / integrate_range on each in order (per-view max range,
        0 = map default).  A view whose K is a LidarModel is a range image."""
        arr, n = views_array(depths, Ks, Ts, max_ranges)
        _check(lib.integrate_depth_views(self._h, arr.ptr, n, C.c_void_p(_stream_ptr(stream))),
               "integrate_depth_views")

    def set_sensor_model(self, params) -> None:
        """Parameters of the learned sensor model (TSDF_SM_NPARAM bfloat16 values)."""
        h = _host_f32(params.detach().cpu().numpy() if isinstance(params, torch.Tensor) else params, SM_NPARAM)
        _check(lib.tsdf_set_sensor_model(self._h, h.ctypes.data), "tsdf_set_sensor_model")

    def step(self, with_spherical: bool = False) -> "TsdfStep":
        """A graph-replayed batched step on this map (see TsdfStep)."""
        return TsdfStep(self, with_spherical)

    # -- queries --------------------------------------------------------------
    def query_blocks(self, stream=None) -> torch.Tensor:
        """Allocated block indices, int32 (n, 3), sorted by (x, y, z)."""
        n = C.c_longlong()
        _check(lib.query_blocks(self._h, None, 0, C.byref(n), C.c_void_p(_stream_ptr(stream))), "query_blocks")
        out = torch.empty((max(n.value, 1), 3), dtype=torch.int32, device="cuda")
        n2 = C.c_longlong()
        _check(lib.query_blocks(self._h, C.c_void_p(out.data_ptr()), n.value, C.byref(n2),
                                C.c_void_p(_stream_ptr(stream))), "query_blocks")
        return out[: n2.value]

    def query_tsdf(self, blocks: torch.Tensor, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
        """(dist, weight) float32 (n, 512) of int32 (n, 3) device block indices."""
        blocks = blocks.to(device="cuda", dtype=torch.int32).contiguous()
        n = blocks.shape[0]
        d = torch.empty((n, 512), dtype=torch.float32, device="cuda")
        w = torch.empty((n, 512), dtype=torch.float32, device="cuda")
        if n:
            _check(lib.query_tsdf(self._h, C.c_void_p(blocks.data_ptr()), n, C.c_void_p(d.data_ptr()),
                                  C.c_void_p(w.data_ptr()), C.c_void_p(_stream_ptr(stream))), "query_tsdf")
        return d, w

    def insert_blocks(self, blocks: torch.Tensor, dist: torch.Tensor, weight: torch.Tensor, stream=None) -> None:
        """Writes blocks (int32 (n, 3)) with their (n, 512) distances and
        weights into the map (see insert_blocks in tsdf.h)."""
        blocks = blocks.to(device="cuda", dtype=torch.int32).contiguous()
        dist = dist.to(device="cuda", dtype=torch.float32).contiguous()
        weight = weight.to(device="cuda", dtype=torch.float32).contiguous()
        n = blocks.shape[0]
        if blocks.shape != (n, 3) or dist.shape != (n, 512) or weight.shape != (n, 512):
            raise ValueError("blocks (n, 3), dist and weight (n, 512)")
        if n:
            _check(lib.insert_blocks(self._h, C.c_void_p(blocks.data_ptr()), n, C.c_void_p(dist.data_ptr()),
                                     C.c_void_p(weight.data_ptr()), C.c_void_p(_stream_ptr(stream))),
                   "insert_blocks")
            (stream or torch.cuda.current_stream()).synchronize()   # the buffers may go once this returns

    def save(self, path: str) -> None:
        """Writes the map's parameters, blocks and voxels to an .npz file
        (plain arrays: numpy.load with its default allow_pickle=False reads it)."""
        b, d, w = self.sorted_state()
        p = self.params
        np.savez(path, format_version=np.int32(1), voxel_size_m=np.float32(p.voxel_size_m),
                 truncation_vox=np.float32(p.truncation_vox), max_weight=np.float32(p.max_weight),
                 max_range_m=np.float32(p.max_range_m), weighting=np.int32(p.weighting), storage=np.int32(p.storage),
                 allocation=np.int32(p.allocation), blocks=b, dist=d, weight=w)

    @classmethod
    def load(cls, path: str, block_capacity: Optional[int] = None) -> "TsdfMap":
        """A map restored from save(): same parameters, blocks and voxel
        values; block_capacity defaults to twice the saved blocks (at least
        2^16)."""
        z = np.load(path)
        if int(z["format_version"]) != 1:
            raise ValueError("unknown map file version")
        names = {v: k for k, v in WEIGHTINGS.items()}
        stor = {v: k for k, v in STORAGES.items()}
        alloc = {v: k for k, v in ALLOCATIONS.items()}
        n = int(z["blocks"].shape[0])
        m = cls(float(z["voxel_size_m"]), float(z["truncation_vox"]), max_weight=float(z["max_weight"]),
                max_range=float(z["max_range_m"]), weighting=names[int(z["weighting"])],
                storage=stor[int(z["storage"])], allocation=alloc[int(z["allocation"])],
                block_capacity=block_capacity or max(1 << 16, 2 * n))
        m.insert_blocks(torch.as_tensor(z["blocks"]), torch.as_tensor(z["dist"]), torch.as_tensor(z["weight"]))
        return m

    def query_touched(self, stream=None) -> torch.Tensor:
        """Blocks updated by the last integrate_depth call, int32 (n, 3), unordered."""
        n = C.c_longlong()
        _check(lib.query_touched(self._h, None, 0, C.byref(n), C.c_void_p(_stream_ptr(stream))), "query_touched")
        out = torch.empty((max(n.value, 1), 3), dtype=torch.int32, device="cuda")
        n2 = C.c_longlong()
        _check(lib.query_touched(self._h, C.c_void_p(out.data_ptr()), n.value, C.byref(n2),
                                 C.c_void_p(_stream_ptr(stream))), "query_touched")
        return out[: n2.value]

    def stats(self, stream=None) -> Tuple[int, int]:
        """(allocated blocks, running total of voxel updates)."""
        b, u, _ = self.counters(stream)
        return b, u

    def counters(self, stream=None) -> Tuple[int, int, int]:
        """(allocated blocks, total voxel updates, total touched blocks)."""
        st = self.full_stats(stream)
        return st["blocks"], st["voxel_updates"], st["touched_blocks"]

    def full_stats(self, stream=None) -> dict:
        out = tsdf_stats()
        _check(lib.map_stats(self._h, C.byref(out), C.c_void_p(_stream_ptr(stream))), "map_stats")
        return {name: getattr(out, name) for name, _ in tsdf_stats._fields_}

    def status(self) -> int:
        return lib.map_status(self._h)

    def sorted_state(self):
        """(blocks, dist, weight) on the host, sorted by block index."""
        b = self.query_blocks()
        d, w = self.query_tsdf(b)
        torch.cuda.synchronize()
        return b.cpu().numpy(), d.cpu().numpy(), w.cpu().numpy()

    def set_launch_config(self, max_groups: int = 0, partitions: int = 0, chunk: int = 0,
                          footprint: str = "auto", compaction: str = "auto", staging: str = "auto") -> None:
        """Launch shape of the integration kernels (0 = automatic); footprint
        culling, compacted launches and LDS footprint staging "auto", "never"
        or "always"."""
        c = tsdf_launch_config(max_groups, partitions, chunk, FOOTPRINT[footprint], COMPACTION[compaction],
                               STAGING[staging])
        _check(lib.tsdf_set_launch_config(self._h, C.byref(c)), "tsdf_set_launch_config")

    # -- kernel timing -------------------------------------------------------
    def profile(self, enable: bool) -> None:
        _check(lib.tsdf_profile(self._h, 1 if enable else 0), "tsdf_profile")

    def profile_read(self) -> Tuple[float, int]:
        ms, n = C.c_double(), C.c_longlong()
        _check(lib.tsdf_profile_read(self._h, C.byref(ms), C.byref(n)), "tsdf_profile_read")
        return ms.value, n.value


class TsdfStep:
    """A batched step replayed from a captured hipGraph (tsdf_step_* in the C
    ABI): run() has the effect of TsdfMap.integrate_depth_views, with one
    graph launch per step.  Close it (or let it go) before its map."""

    def __init__(self, m: TsdfMap, with_spherical: bool = False):
        h = C.c_void_p()
        _check(lib.tsdf_step_create(m.handle, 1 if with_spherical else 0, C.byref(h)), "tsdf_step_create")
        self._h = h
        self.map = m

    def run(self, depths: Sequence[torch.Tensor], Ks, Ts, max_ranges=None,
            stream: Optional[torch.cuda.Stream] = None) -> None:
        arr, n = views_array(depths, Ks, Ts, max_ranges)
        _check(lib.tsdf_step_run(self._h, arr.ptr, n, C.c_void_p(_stream_ptr(stream))), "tsdf_step_run")

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib.tsdf_step_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_f32(t: torch.Tensor, name: str, n: Optional[int] = None) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must hold {n} values")
    return t


def sensor_maps(depth: torch.Tensor, K, max_range: float, voxel_size: float, params: torch.Tensor,
                stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """(H, W, 2) per-pixel (weight, truncation) of the learned sensor model."""
    _dev_f32(depth, "depth")
    _dev_f32(params, "params", SM_NPARAM)
    H, W = depth.shape
    out = torch.empty((H, W, 2), dtype=torch.float32, device=depth.device)
    Kh = _host_f32(K, 4)
    _check(lib.tsdf_sensor_maps(depth.data_ptr(), W, H, Kh.ctypes.data, max_range, voxel_size, params.data_ptr(),
                                out.data_ptr(), C.c_void_p(_stream_ptr(stream))), "tsdf_sensor_maps")
    return out


class SmTrainer:
    """Work buffers for loss/gradient evaluations of the learned sensor model
    on windows of up to max_frames depth images of one size."""

    def __init__(self, width: int, height: int, max_frames: int = SM_MAX_FRAMES):
        h = C.c_void_p()
        _check(lib.tsdf_sm_trainer_create(width, height, max_frames, C.byref(h)), "tsdf_sm_trainer_create")
        self._h = h
        self.width, self.height, self.max_frames = width, height, max_frames

    def loss_grad(self, params: torch.Tensor, depths: Sequence[torch.Tensor], K, poses, voxel_size: float,
                  max_range: float, vox: torch.Tensor, target: torch.Tensor, grad: torch.Tensor,
                  want_loss: bool = True, stream=None):
        """Writes dL/dparams into grad; returns (L, voxels reached) if want_loss."""
        _dev_f32(params, "params", SM_NPARAM)
        _dev_f32(grad, "grad", SM_NPARAM)
        _dev_f32(target, "target")
        if not (vox.is_cuda and vox.dtype == torch.int32 and vox.is_contiguous() and vox.numel() == 3 * target.numel()):
            raise ValueError("vox must be a contiguous int32 CUDA tensor of shape (n, 3)")
        n = len(depths)
        if not 1 <= n <= self.max_frames:
            raise ValueError(f"need 1..{self.max_frames} frames")
        for d in depths:
            if tuple(_dev_f32(d, "depth").shape) != (self.height, self.width):
                raise ValueError(f"depth must be ({self.height}, {self.width})")
        if len(poses) != n:
            raise ValueError("one pose per frame")
        ptrs = (C.c_void_p * n)(*[d.data_ptr() for d in depths])
        T = np.ascontiguousarray(np.stack([_host_f32(t, 16) for t in poses]).reshape(-1))
        Kh = _host_f32(K, 4)
        out = (C.c_double * 2)()
        _check(lib.tsdf_sm_loss_grad(self._h, params.data_ptr(), n, ptrs, Kh.ctypes.data, T.ctypes.data, voxel_size,
                                     max_range, target.numel(), vox.data_ptr(), target.data_ptr(), grad.data_ptr(),
                                     out if want_loss else None, C.c_void_p(_stream_ptr(stream))),
               "tsdf_sm_loss_grad")
        return (out[0], int(out[1])) if want_loss else None

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib.tsdf_sm_trainer_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sm_adam(master, m1, m2, grad, params, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
            eps: float = 1e-8, stream=None) -> None:
    for t, name in ((master, "master"), (m1, "m1"), (m2, "m2"), (grad, "grad"), (params, "params")):
        _dev_f32(t, name, SM_NPARAM)
    _check(lib.tsdf_sm_adam(master.data_ptr(), m1.data_ptr(), m2.data_ptr(), grad.data_ptr(), params.data_ptr(),
                            SM_NPARAM, lr, beta1, beta2, eps, step, C.c_void_p(_stream_ptr(stream))), "tsdf_sm_adam")
