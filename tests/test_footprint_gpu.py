"""Footprint culling (per-view pyramid of tile depth maxima) only skips blocks
that hold no updated voxel: maps integrated with it forced on, forced off and
automatic are bitwise identical, and equal to the binary32 oracle, for
pinhole views at fine voxels, a cluttered scene, batched views and a
full-circle LiDAR."""
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


def states_equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a.sorted_state(), b.sorted_state()))


@pytest.mark.parametrize("vs,n", [(0.02, 12), (0.01, 4)])
def test_footprint_box_room_fine_voxels(vs, n):
    import oracle
    w = synth.box_room_sequence(vs, n_frames=n)
    say(f"case: footprint culling, box room {int(vs * 100)} cm, {n} frames, never/always/auto")
    frames = w.frames(device="cuda")
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    maps = {}
    for mode in ("never", "always", "auto"):
        m = gpu_map(w.params, block_capacity=1 << 17)
        m.set_launch_config(footprint=mode)
        for d, T in zip(dev, w.poses):
            m.integrate_depth(d, w.camera.K, T)
        maps[mode] = m
    torch.cuda.synchronize()
    assert states_equal(maps["never"], maps["always"]) and states_equal(maps["never"], maps["auto"])
    om = oracle.OracleMap.from_params(w.params)
    for f, T in zip(frames, w.poses):
        om.integrate(f, w.camera.K, T)
    t_always = {tuple(x) for x in maps["always"].query_touched().cpu().numpy()}
    assert t_always == {tuple(x) for x in om.touched()}
    say(assert_parity(maps["always"], om, exact_dist=True))


def test_footprint_cluttered_room_plain_and_batched():
    import oracle
    w = synth.cluttered_room_sequence()
    n = 20
    say("case: footprint culling forced on, cluttered room, plain and batched (5 per launch)")
    frames = w.frames(device="cuda", count=n)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    K = w.camera.K
    plain = gpu_map(w.params)
    plain.set_launch_config(footprint="always")
    for d, T in zip(dev, w.poses):
        plain.integrate_depth(d, K, T)
    batched = gpu_map(w.params)
    batched.set_launch_config(footprint="always")
    step = batched.step()
    for a in range(0, n, 5):
        if a % 10 == 0:
            batched.integrate_depth_views(dev[a:a + 5], [K] * 5, w.poses[a:a + 5])
        else:
            step.run(dev[a:a + 5], [K] * 5, w.poses[a:a + 5])
    torch.cuda.synchronize()
    step.close()
    om = oracle.OracleMap.from_params(w.params)
    for f, T in zip(frames, w.poses):
        om.integrate(f, K, T)
    say(assert_parity(plain, om, exact_dist=True))
    say(assert_parity(batched, om, exact_dist=True))


@pytest.mark.parametrize("az_start_deg", [-180.0, 37.0])
def test_footprint_lidar_full_circle(az_start_deg):
    import math
    import oracle
    scene, steps = synth.rig_sequence(3)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2,
                         azimuth_start=math.radians(az_start_deg))
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(9)
    say(f"case: footprint culling, LiDAR 1024x64 full circle from {az_start_deg} deg, 3 scans, never/always")
    imgs = [synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose, device="cuda"), rng)
            for st in steps]
    maps = {}
    for mode in ("never", "always"):
        m = gpu_map(params, block_capacity=1 << 17)
        m.set_launch_config(footprint=mode)
        for img, st in zip(imgs, steps):
            m.integrate_range(torch.as_tensor(img, device="cuda"), L, st.lidar_pose)
        maps[mode] = m
    torch.cuda.synchronize()
    assert states_equal(maps["never"], maps["always"])
    om = oracle.OracleMap.from_params(params)
    for img, st in zip(imgs, steps):
        om.integrate_range(img, L, st.lidar_pose)
    say(assert_parity(maps["always"], om, exact_dist=True))


def test_footprint_lidar_partial_fov_seam():
    """A partial-azimuth sensor whose field of view spans the +-pi seam's
    neighbourhood, with invalid returns."""
    import math
    import oracle
    L = synth.LidarModel(width=180, height=16, azimuth_start=math.radians(100), azimuth_fov=math.radians(150),
                         polar_start=math.radians(70), polar_fov=math.radians(40), interp_max_diff=0.3,
                         max_range=8.0)
    room = synth.Scene(room=(6.0, 5.0, 3.0), spheres=[((1.0, 2.5, 1.5), 0.4)])
    T = synth.pose_lidar([3.0, 2.5, 1.5], 0.3)
    rng = np.random.default_rng(3)
    img = synth.add_range_noise(synth.render_range(room, L, T), rng)
    img[rng.random(img.shape) < 0.1] = 0.0
    params = synth.MapParams(0.05, 4.0, "constant", max_range=10.0)
    say("case: footprint culling, partial-azimuth LiDAR across the seam")
    gm = gpu_map(params)
    gm.set_launch_config(footprint="always")
    gm.integrate_range(torch.as_tensor(img, device="cuda"), L, T)
    om = oracle.OracleMap.from_params(params)
    om.integrate_range(img, L, T)
    say(assert_parity(gm, om, exact_dist=True))
