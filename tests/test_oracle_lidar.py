"""Pins of the oracle's spherical (LiDAR) path, Eq. (3) of the paper, against
facts that do not come from the oracle: the accuracy of the atan2 it evaluates,
the closed-form field of a constant range image (a sphere around the sensor),
the wall distance in a box room, dense brute force, the interpolation guard
and the azimuth wrap."""
import math

import numpy as np
import pytest

from paper_2311_00626_amd import synth
from tests import geometry as geo
from tests.test_oracle_pins import lookup


def sensor_frame(T, p):
    Ti = np.linalg.inv(np.asarray(T, np.float64))
    return p @ Ti[:3, :3].T + Ti[:3, 3]


def test_atan2_accuracy(oracle_mod):
    """binary32 atan2 from the Abramowitz & Stegun 4.4.49 polynomial: within
    a few binary32 ulps of the exact angle, every octant, exact special values."""
    rng = np.random.default_rng(0)
    y = rng.standard_normal(20000) * 10.0 ** rng.uniform(-3, 3, 20000)
    x = rng.standard_normal(20000) * 10.0 ** rng.uniform(-3, 3, 20000)
    y32, x32 = y.astype(np.float32), x.astype(np.float32)
    got = np.array([oracle_mod.atan2_f32(float(a), float(b)) for a, b in zip(y32, x32)])
    ref = np.arctan2(y32.astype(np.float64), x32.astype(np.float64))
    assert np.abs(got - ref).max() < 6e-7
    assert oracle_mod.atan2_f32(0.0, 0.0) == 0.0
    assert oracle_mod.atan2_f32(0.0, 1.0) == 0.0
    assert oracle_mod.atan2_f32(1.0, 0.0) == np.float32(math.pi / 2)
    assert oracle_mod.atan2_f32(0.0, -1.0) == np.float32(math.pi)
    assert oracle_mod.atan2_f32(-1.0, 0.0) == -np.float32(math.pi / 2)


@pytest.mark.parametrize("pol_start_deg,pol_fov_deg", [(60.0, 40.0), (74.0, 32.0)])
def test_constant_range_is_a_sphere(oracle_mod, pol_start_deg, pol_fov_deg):
    """A range image holding R0 everywhere describes the sphere |p| = R0: every
    voxel whose direction lies inside the polar band (with all four neighbouring
    beams in the image) gets D = min(R0 - |p|, eps), W = 1; all azimuths wrap."""
    L = synth.LidarModel(width=128, height=12, polar_start=math.radians(pol_start_deg),
                         polar_fov=math.radians(pol_fov_deg), max_range=10.0)
    R0 = 2.0
    rimg = np.full((L.height, L.width), R0, np.float32)
    T = synth.pose_lidar([0.3, -0.2, 0.5], 0.7)
    vs, eps = 0.05, 0.2
    params = synth.MapParams(vs, 4.0, "constant", max_range=10.0)
    m = oracle_mod.OracleMap.from_params(params)
    m.integrate_range(rimg, L, T)
    state = m.sorted_state()
    # every voxel within R0 + eps + margin of the sensor
    o = T[:3, 3].astype(np.float64)
    lo = np.floor((o - 2.4) / vs).astype(int)
    hi = np.ceil((o + 2.4) / vs).astype(int)
    axes = [np.arange(a, b + 1) for a, b in zip(lo, hi)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    p = (g + 0.5) * float(np.float32(vs))
    ps = sensor_frame(T, p)
    r = np.linalg.norm(ps, axis=1)
    phi = np.arctan2(np.hypot(ps[:, 0], ps[:, 1]), ps[:, 2])
    beta = L.height / L.polar_fov
    v = (phi - L.polar_start) * beta - 0.5          # row coordinate between beam centres
    inside = (v > 1e-3) & (v < L.height - 1 - 1e-3) & (r > 0.05) & (R0 - r > -eps + 1e-4)
    outside = (v < -1e-3) | (v > L.height - 1 + 1e-3) | (R0 - r < -eps - 1e-4)
    d, w, _ = lookup(state, g)
    assert inside.sum() > 5000
    assert np.all(w[inside] == 1.0) and np.all(w[outside] == 0.0)
    exp = np.minimum(R0 - r[inside], eps)
    assert np.abs(d[inside] - exp).max() < 2e-6
    # the wrap: voxels straight behind the sensor (azimuth near +-pi) are covered
    theta = np.arctan2(ps[:, 1], ps[:, 0])
    behind = inside & (np.abs(np.abs(theta) - math.pi) < 0.02)
    assert behind.sum() > 20


def test_box_room_wall_distance(oracle_mod):
    """Near a wall, hit at incidence angle a, the fused distance is the
    along-beam distance s / cos(a) up to the interpolation error of range
    between neighbouring beams."""
    L = synth.LidarModel(width=1024, height=64, polar_start=math.radians(60), polar_fov=math.radians(60),
                         max_range=10.0)
    room = (4.0, 3.0, 2.5)
    T = synth.pose_lidar([1.7, 1.4, 1.3], 0.4)
    rimg = synth.render_range(synth.Scene(room=room), L, T)
    vs = 0.04
    params = synth.MapParams(vs, 4.0, "constant", max_range=10.0)
    m = oracle_mod.OracleMap.from_params(params)
    m.integrate_range(rimg, L, T)
    blocks, dist, weight = m.sorted_state()
    cen = geo.voxel_centres(blocks, vs).reshape(-1, 3)
    D, W = dist.reshape(-1), weight.reshape(-1)
    s, wall, gap = geo.room_sdf(cen, room)
    o = T[:3, 3].astype(np.float64)
    ray = cen - o
    rn = np.linalg.norm(ray, axis=1)
    cos_a = np.abs(np.sum(ray / rn[:, None] * geo.ROOM_NORMALS[wall], axis=1))
    sel = (W > 0) & (np.abs(s) <= vs) & (cos_a > 0.7) & (gap > 0.4)
    assert sel.sum() > 500
    dth = L.azimuth_fov / L.width
    dph = L.polar_fov / L.height
    tan2 = (1 - cos_a ** 2) / cos_a ** 2
    bound = rn * (dth ** 2 + dph ** 2) * (1 + 3 * tan2) + np.abs(s) * 1e-3 + 2e-5
    err = np.abs(D - s / cos_a)
    assert np.all(err[sel] <= bound[sel]), (err[sel] / bound[sel]).max()
    # deep free space carries eps exactly
    free = (W > 0) & (s > 0.5)
    assert free.sum() > 1000 and np.all(D[free] == np.float32(4 * vs))


def test_interpolation_guard(oracle_mod):
    """A range image stepping from 2 m to 3 m between two column blocks: voxels
    interpolating across the step are updated only if the guard allows the 1 m
    spread."""
    L = synth.LidarModel(width=64, height=8, polar_start=math.radians(80), polar_fov=math.radians(20),
                         interp_max_diff=0.5, max_range=10.0)
    rimg = np.full((L.height, L.width), 2.0, np.float32)
    rimg[:, 32:] = 3.0
    T = np.eye(4, dtype=np.float32)
    params = synth.MapParams(0.05, 4.0, "constant", max_range=10.0)
    strict = oracle_mod.OracleMap.from_params(params)
    strict.integrate_range(rimg, L, T)
    loose_model = synth.LidarModel(width=64, height=8, polar_start=math.radians(80), polar_fov=math.radians(20),
                                   interp_max_diff=1.5, max_range=10.0)
    loose = oracle_mod.OracleMap.from_params(params)
    loose.integrate_range(rimg, loose_model, T)
    bs, ds, ws = strict.sorted_state()
    bl, dl, wl = loose.sorted_state()
    assert (wl > 0).sum() > (ws > 0).sum()
    # on the strict map, voxels whose azimuth lies between the centres of
    # columns 31 and 32 (or 63 and 0) are never updated
    cen = geo.voxel_centres(bs, 0.05).reshape(-1, 3)
    theta = np.arctan2(cen[:, 1], cen[:, 0])
    u = (theta - L.azimuth_start) * (L.width / L.azimuth_fov) - 0.5
    straddle = ((u > 31 + 1e-3) & (u < 32 - 1e-3)) | (u > 63 + 1e-3) | (u < -1e-3)
    assert np.all(ws.reshape(-1)[straddle] == 0)


def test_lidar_sparse_equals_dense(oracle_mod):
    """Sparse LiDAR integration (scan box, blocks, hash) is bitwise equal to a
    dense evaluation of every voxel of a box that holds every update."""
    L = synth.LidarModel(width=96, height=10, polar_start=math.radians(70), polar_fov=math.radians(40),
                         max_range=3.0)
    room = (4.0, 3.0, 2.5)
    rng = np.random.default_rng(4)
    poses = [synth.pose_lidar([2.1, 1.3, 1.2], -0.6), synth.pose_lidar([1.6, 1.1, 1.0], 0.9)]
    imgs = [synth.add_range_noise(synth.render_range(synth.Scene(room=room), L, T), rng) for T in poses]
    params = synth.MapParams(0.1, 3.0, "linear_dropoff", max_range=3.0)
    m = oracle_mod.OracleMap.from_params(params)
    for img, T in zip(imgs, poses):
        m.integrate_range(img, L, T)
    gmin = np.array([-24, -24, -24])
    gdim = np.array([90, 80, 70])
    Dd, Wd = oracle_mod.dense_integrate_range(params, imgs, L, poses, gmin, gdim)
    zz, yy, xx = np.nonzero(Wd > 0)
    assert len(xx) > 500
    assert xx.min() > 0 and yy.min() > 0 and zz.min() > 0
    assert xx.max() < gdim[0] - 1 and yy.max() < gdim[1] - 1 and zz.max() < gdim[2] - 1
    g = np.stack([xx, yy, zz], 1) + gmin
    state = m.sorted_state()
    d, w, present = lookup(state, g)
    assert present.all()
    assert np.array_equal(d, Dd[zz, yy, xx]) and np.array_equal(w, Wd[zz, yy, xx])
    blocks, dist, weight = state
    assert np.all((weight > 0).any(axis=1)) and int((weight > 0).sum()) == len(xx)


def test_partial_azimuth_fov(oracle_mod):
    """A sensor covering azimuths [-45, 45] deg updates nothing behind it."""
    L = synth.LidarModel(width=90, height=10, azimuth_start=math.radians(-45), azimuth_fov=math.radians(90),
                         polar_start=math.radians(70), polar_fov=math.radians(40), max_range=10.0)
    rimg = np.full((L.height, L.width), 2.0, np.float32)
    T = np.eye(4, dtype=np.float32)
    params = synth.MapParams(0.05, 4.0, "constant", max_range=10.0)
    m = oracle_mod.OracleMap.from_params(params)
    m.integrate_range(rimg, L, T)
    blocks, dist, weight = m.sorted_state()
    cen = geo.voxel_centres(blocks, 0.05).reshape(-1, 3)
    theta = np.arctan2(cen[:, 1], cen[:, 0])
    W = weight.reshape(-1)
    assert (W > 0).sum() > 1000
    assert np.all(np.abs(theta[W > 0]) < math.radians(45) + 0.02)
