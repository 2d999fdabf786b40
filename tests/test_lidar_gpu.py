"""GPU parity of the spherical (LiDAR) path, Eq. (3): integrate_range and
spherical views in a batch, against the binary32 oracle -- blocks bit-exact,
weights exact, distances bit-identical."""
import math

import numpy as np
import pytest
import torch

from paper_2311_00626_amd import synth
from tests.gpu_util import assert_parity, gpu_map, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_00626_amd.tsdf  # noqa: F401


def both(params, **kw):
    import oracle
    return gpu_map(params, **kw), oracle.OracleMap.from_params(params, storage=kw.get("storage", "fp32"))


def test_range_box_room():
    L = synth.LidarModel(width=256, height=16, max_range=10.0)
    room = synth.Scene(room=(4.0, 3.0, 2.5), spheres=[((2.5, 2.0, 1.0), 0.3)])
    rng = np.random.default_rng(0)
    poses = [synth.pose_lidar([1.5 + 0.2 * k, 1.2, 1.1], 0.3 * k) for k in range(4)]
    imgs = [synth.add_range_noise(synth.render_range(room, L, T), rng) for T in poses]
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=10.0)
    say("case: LiDAR 256x16 in a box room, 4 scans")
    gm, om = both(params)
    for img, T in zip(imgs, poses):
        gm.integrate_range(torch.as_tensor(img, device="cuda"), L, T)
        om.integrate_range(img, L, T)
        gt = {tuple(x) for x in gm.query_touched().cpu().numpy()}
        assert gt == {tuple(x) for x in om.touched()}
    say(assert_parity(gm, om, exact_dist=True))


@pytest.mark.parametrize("az_start", [-math.pi, 2.5, -9.0, 15.0, -40.0])
def test_range_full_circle_azimuth_starts(az_start):
    """Full-circle column wrap for azimuth starts within and beyond two turns
    of the azimuth range (the kernel wraps the former by conditional adds, the
    latter by the integer remainder)."""
    L = synth.LidarModel(width=200, height=12, azimuth_start=az_start, max_range=10.0, interp_max_diff=0.3)
    room = synth.Scene(room=(4.0, 3.0, 2.5), spheres=[((2.6, 1.9, 1.2), 0.35)])
    rng = np.random.default_rng(5)
    poses = [synth.pose_lidar([1.4 + 0.3 * k, 1.3, 1.2], 0.4 * k) for k in range(3)]
    imgs = [synth.add_range_noise(synth.render_range(room, L, T), rng) for T in poses]
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=10.0)
    say(f"case: full-circle LiDAR 200x12, azimuth start {az_start} rad, 3 scans")
    gm, om = both(params)
    for img, T in zip(imgs, poses):
        gm.integrate_range(torch.as_tensor(img, device="cuda"), L, T)
        om.integrate_range(img, L, T)
    say(assert_parity(gm, om, exact_dist=True))


@pytest.mark.parametrize("pol", [(60.0, 40.0), (74.0, 32.0), (30.0, 120.0)])
def test_range_constant_sphere(pol):
    L = synth.LidarModel(width=128, height=12, polar_start=math.radians(pol[0]), polar_fov=math.radians(pol[1]),
                         max_range=10.0)
    img = np.full((L.height, L.width), 2.0, np.float32)
    T = synth.pose_lidar([0.3, -0.2, 0.5], 0.7)
    params = synth.MapParams(0.05, 4.0, "constant", max_range=10.0)
    say(f"case: constant range image, polar band {pol}")
    gm, om = both(params)
    gm.integrate_range(torch.as_tensor(img, device="cuda"), L, T)
    om.integrate_range(img, L, T)
    say(assert_parity(gm, om, exact_dist=True))


def test_range_partial_fov_invalid_pixels_fp16():
    L = synth.LidarModel(width=90, height=10, azimuth_start=math.radians(-45), azimuth_fov=math.radians(90),
                         polar_start=math.radians(70), polar_fov=math.radians(40), interp_max_diff=0.3,
                         max_range=6.0)
    rng = np.random.default_rng(1)
    img = rng.uniform(1.0, 7.0, (L.height, L.width)).astype(np.float32)
    img[rng.random(img.shape) < 0.1] = np.nan
    img[rng.random(img.shape) < 0.1] = 0.0
    T = synth.pose_lidar([0.0, 0.0, 0.0], 0.2)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=10.0)
    for storage in ("fp32", "fp16"):
        say(f"case: partial azimuth, invalid pixels, {storage}")
        gm, om = both(params, storage=storage)
        for _ in range(3):
            gm.integrate_range(torch.as_tensor(img, device="cuda"), L, T)
            om.integrate_range(img, L, T)
        assert_parity(gm, om, exact_dist=True)


def test_rig_step_cameras_plus_lidar():
    """Batched multi-sensor step: 4 cameras of uneven sizes and a 1024x64 LiDAR
    (+-16 deg, 25 m) fused in one launch per step, in a 20 x 15 x 3 m room."""
    scene, steps = synth.rig_sequence(4)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(2)
    say("case: rig step, 4 cameras + LiDAR, 2 steps, one launch each")
    gm, om = both(params)
    for st in steps[:2]:
        depths, Ks, poses = [], [], []
        for cam, T in zip(st.cameras, st.poses):
            d = synth.add_depth_noise(synth.render_depth(scene, cam, T, device="cuda"), rng)
            depths.append(d)
            Ks.append(cam.K)
            poses.append(T)
        r = synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose, device="cuda"), rng)
        gm.integrate_depth_views([torch.as_tensor(x, device="cuda") for x in depths + [r]],
                                 Ks + [L], poses + [st.lidar_pose])
        union = set()
        for d, K, T in zip(depths, Ks, poses):
            om.integrate(d, K, T)
            union |= {tuple(x) for x in om.touched()}
        om.integrate_range(r, L, st.lidar_pose)
        union |= {tuple(x) for x in om.touched()}
        assert {tuple(x) for x in gm.query_touched().cpu().numpy()} == union
    say(assert_parity(gm, om, exact_dist=True))
