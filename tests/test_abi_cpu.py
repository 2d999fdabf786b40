"""The C-ABI library loads, exports every symbol include/tsdf.h declares, and
rejects bad arguments before touching a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsdf.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"TSDF_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)


@pytest.fixture(scope="module")
def t():
    from paper_2311_00626_amd import tsdf
    return tsdf


def test_header_declares_expected_entry_points():
    names = set(declared_functions())
    for n in ("create_map", "create_map_ex", "destroy_map", "reserve", "integrate_depth", "integrate_depth_noalloc",
              "integrate_range", "integrate_depth_views", "query_blocks", "query_tsdf", "query_touched", "map_stats",
              "map_status", "tsdf_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(t):
    for name in declared_functions():
        assert hasattr(t.lib, name), name
    assert set(t.EXPORTED) == set(declared_functions())


def test_struct_layouts(t):
    assert C.sizeof(t.tsdf_depth_view) == 112
    assert C.sizeof(t.tsdf_lidar_model) == 32
    assert C.sizeof(t.tsdf_stats) == 72
    assert C.sizeof(t.tsdf_launch_config) == 24


def test_struct_layouts_match_the_c_compiler(t, tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal the C layout of
    include/tsdf.h (a small C program prints sizeof / offsetof)."""
    import subprocess
    exe = tmp_path / "abi_sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    os.path.join(ROOT, "tests", "abi_sizes.c")], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    c_layout = dict(line.rsplit(" ", 1) for line in out.splitlines())
    checked = 0
    for key, value in c_layout.items():
        struct, _, field = key.partition(".")
        cls = getattr(t, struct)
        got = C.sizeof(cls) if not field else getattr(cls, field).offset
        assert got == int(value), (key, got, value)
        checked += 1
    assert checked >= 15


def test_params_struct_layout(t):
    assert C.sizeof(t.tsdf_params) == 48
    p = t.default_params(0.04, 4.0)
    assert p.voxel_size_m == pytest.approx(0.04) and p.truncation_vox == 4.0
    assert p.max_weight == 100.0 and p.max_range_m == 5.0 and p.weighting == 0
    assert p.block_capacity == 1 << 18 and p.hash_capacity == 0


def test_strerror(t):
    for s in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(t.strerror(s), str) and t.strerror(s)
    assert t.strerror(-3).startswith("map capacity")


def test_invalid_create_arguments_rejected_before_device(t):
    h = C.c_void_p()
    for vs, tau in ((0.0, 4.0), (-1.0, 4.0), (float("nan"), 4.0), (0.05, 0.0), (0.05, float("inf"))):
        assert t.lib.create_map(vs, tau, C.byref(h)) == t.EINVAL
        assert not h.value
    p = t.default_params(0.05, 4.0)
    for field, bad in (("max_weight", 0.0), ("max_range_m", -1.0), ("weighting", 7), ("storage", 2),
                       ("block_capacity", 0), ("hash_capacity", 3), ("hash_capacity", -8), ("allocation", 2),
                       ("reserved", 1)):
        q = t.default_params(0.05, 4.0)
        setattr(q, field, bad)
        assert t.lib.create_map_ex(C.byref(q), C.byref(h)) == t.EINVAL, field
    q = t.default_params(0.05, 4.0)
    q.block_capacity, q.hash_capacity = 1024, 512          # hash smaller than the pool
    assert t.lib.create_map_ex(C.byref(q), C.byref(h)) == t.EINVAL
    assert t.lib.create_map_ex(None, C.byref(h)) == t.EINVAL
    assert t.lib.create_map_ex(C.byref(p), None) == t.EINVAL


def test_null_map_rejected(t):
    K = (C.c_float * 4)(1, 1, 0, 0)
    T = (C.c_float * 16)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1)
    n = C.c_longlong()
    assert t.lib.integrate_depth(None, C.c_void_p(16), 4, 4, K, T, None) == t.EINVAL
    assert t.lib.query_blocks(None, None, 0, C.byref(n), None) == t.EINVAL
    assert t.lib.query_touched(None, None, 0, C.byref(n), None) == t.EINVAL
    assert t.lib.query_tsdf(None, None, 0, None, None, None) == t.EINVAL
    st = t.tsdf_stats()
    assert t.lib.map_stats(None, C.byref(st), None) == t.EINVAL
    views = (t.tsdf_depth_view * 2)()
    assert t.lib.integrate_depth_views(None, views, 1, None) == t.EINVAL
    assert t.lib.map_status(None) == t.EINVAL
    assert t.lib.destroy_map(None) == t.OK
    assert t.lib.reserve(None, 1024) == t.EINVAL
    step = C.c_void_p()
    assert t.lib.tsdf_step_create(None, 0, C.byref(step)) == t.EINVAL and not step.value
    assert t.lib.tsdf_step_run(None, views, 1, None) == t.EINVAL
    assert t.lib.tsdf_step_destroy(None) == t.OK
    P = (C.c_float * 2018)()
    assert t.lib.tsdf_set_sensor_model(None, P) == t.EINVAL


def test_sensor_model_arguments_rejected_before_device(t):
    K = (C.c_float * 4)(1, 1, 0, 0)
    tr = C.c_void_p()
    for w, h, n in ((0, 10, 1), (10, 0, 1), (10, 10, 0), (10, 10, 17)):
        assert t.lib.tsdf_sm_trainer_create(w, h, n, C.byref(tr)) == t.EINVAL and not tr.value
    assert t.lib.tsdf_sm_trainer_create(10, 10, 1, None) == t.EINVAL
    assert t.lib.tsdf_sm_trainer_destroy(None) == t.OK
    assert t.lib.tsdf_sm_loss_grad(None, None, 1, None, K, None, 0.05, 5.0, 0, None, None, None, None, None) == t.EINVAL
    assert t.lib.tsdf_sensor_maps(None, 4, 4, K, 5.0, 0.05, None, None, None) == t.EINVAL
    assert t.lib.tsdf_sensor_maps(C.c_void_p(16), 0, 4, K, 5.0, 0.05, C.c_void_p(16), C.c_void_p(16), None) == t.EINVAL
    assert t.lib.tsdf_sm_adam(None, None, None, None, None, 2018, 1e-3, 0.9, 0.999, 1e-8, 1, None) == t.EINVAL
    # learned weighting is a valid map parameter, other codes are not
    q = t.default_params(0.05, 4.0)
    q.weighting = 3
    h = C.c_void_p()
    assert t.lib.create_map_ex(C.byref(q), C.byref(h)) == t.EINVAL


def test_view_record_layout_matches_struct():
    """The NumPy record a batch's arguments are filled in has the C struct's
    layout: every field written through the record reads back through the
    ctypes view of the same memory."""
    import numpy as np
    from paper_2311_00626_amd import tsdf as t
    rec = np.zeros(3, t._VIEW_DTYPE)
    assert rec.itemsize == C.sizeof(t.tsdf_depth_view) == 112
    rec["depth_dev"] = [0x1000, 0x2000, 0x3000]
    rec["width"], rec["height"], rec["model"] = [640, 1024, 5], [480, 64, 7], [0, 1, 0]
    rec["max_range_m"] = [0.0, 25.0, 3.5]
    rec["K"] = np.arange(12, dtype=np.float32).reshape(3, 4)
    rec["interp_max_diff_m"] = [0.0, 0.2, 0.0]
    rec["T_world_cam"] = np.arange(48, dtype=np.float32).reshape(3, 16) + 0.5
    b = t.ViewBatch(rec)
    for k in range(3):
        v = b[k]
        assert v.depth_dev == 0x1000 * (k + 1)
        assert (v.width, v.height, v.model) == (int(rec["width"][k]), int(rec["height"][k]), int(rec["model"][k]))
        assert v.max_range_m == rec["max_range_m"][k] and v.interp_max_diff_m == rec["interp_max_diff_m"][k]
        assert list(v.K) == list(rec["K"][k]) and list(v.T_world_cam) == list(rec["T_world_cam"][k])


def test_hash_capacity_rules(t):
    """hash_capacity: 0 (automatic) or a power of two no smaller than the
    pool, down to tiny tables whose 32 slots the 64-lane probe window covers
    twice; rejected values fail before any device call, accepted ones get
    past validation (on a machine without a GPU the device call then fails)."""
    h = C.c_void_p()
    for bc, hc, ok in ((32, 32, True), (32, 64, True), (1, 1, True), (1000, 1024, True), (1024, 1024, True),
                       (33, 32, False), (32, 48, False), (32, 16, False), ((1 << 30) + 1, 0, False),
                       (1 << 20, 1 << 32, False)):
        q = t.default_params(0.05, 4.0)
        q.block_capacity, q.hash_capacity = bc, hc
        st = t.lib.create_map_ex(C.byref(q), C.byref(h))
        if ok:
            assert st != t.EINVAL, (bc, hc)
            if st == t.OK:
                t.lib.destroy_map(h)
        else:
            assert st == t.EINVAL and not h.value, (bc, hc)
