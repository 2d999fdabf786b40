"""Compacted launches (a cull pass writes the surviving blocks of the lattice to
a list that the integration kernel deals out to its waves) change only the
order in which blocks are visited: maps integrated with compaction forced on,
forced off and automatic are bitwise identical, equal to the binary32 oracle,
and count the same voxel updates, for single frames, batched views (eager and
graph replays), a LiDAR, FP16 storage and learned weighting."""
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


@pytest.mark.parametrize("vs,n,storage", [(0.02, 10, "fp32"), (0.01, 3, "fp32"), (0.02, 6, "fp16")])
def test_compaction_box_room(vs, n, storage):
    import oracle
    w = synth.box_room_sequence(vs, n_frames=n)
    say(f"case: compacted launches, box room {int(vs * 100)} cm, {n} frames, {storage}, never/always/auto"
        " and always on an explicit 512-workgroup grid")
    frames = w.frames(device="cuda")
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    maps = {}
    # "always" runs the list kernel on every resident workgroup; "always_512"
    # on the explicit grid of the lattice walk
    for mode, groups in (("never", 0), ("always", 0), ("auto", 0), ("always_512", 512)):
        m = gpu_map(w.params, block_capacity=1 << 17, storage=storage)
        m.set_launch_config(max_groups=groups, compaction=mode.split("_")[0])
        for d, T in zip(dev, w.poses):
            m.integrate_depth(d, w.camera.K, T)
        maps[mode] = m
    torch.cuda.synchronize()
    assert states_equal(maps["never"], maps["always"]) and states_equal(maps["never"], maps["auto"])
    assert states_equal(maps["never"], maps["always_512"])
    s_never, s_always = maps["never"].full_stats(), maps["always"].full_stats()
    assert s_never["voxel_updates"] == s_always["voxel_updates"]
    assert s_never["touched_blocks"] == s_always["touched_blocks"]
    if storage == "fp32":
        om = oracle.OracleMap.from_params(w.params)
        for f, T in zip(frames, w.poses):
            om.integrate(f, w.camera.K, T)
        t_always = {tuple(x) for x in maps["always"].query_touched().cpu().numpy()}
        assert t_always == {tuple(x) for x in om.touched()}
        say(assert_parity(maps["always"], om, exact_dist=True))


def test_compaction_batched_eager_and_graph():
    import oracle
    w = synth.cluttered_room_sequence()
    n = 20
    say("case: compacted launches forced on, cluttered room, batched eager and graph replays (5 per launch)")
    frames = w.frames(device="cuda", count=n)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    K = w.camera.K
    batched = gpu_map(w.params)
    batched.set_launch_config(compaction="always", footprint="always")
    step = batched.step()
    for a in range(0, n, 5):
        if a % 10 == 0:
            batched.integrate_depth_views(dev[a:a + 5], [K] * 5, w.poses[a:a + 5])
        else:
            step.run(dev[a:a + 5], [K] * 5, w.poses[a:a + 5])
        torch.cuda.synchronize()
    step.close()
    # the same graph alternating between compacted and walking replays
    mixed = gpu_map(w.params)
    mstep = mixed.step()
    for k, a in enumerate(range(0, n, 5)):
        mixed.set_launch_config(compaction="always" if k % 2 else "never")
        mstep.run(dev[a:a + 5], [K] * 5, w.poses[a:a + 5])
    torch.cuda.synchronize()
    mstep.close()
    om = oracle.OracleMap.from_params(w.params)
    for f, T in zip(frames, w.poses):
        om.integrate(f, K, T)
    say(assert_parity(batched, om, exact_dist=True))
    say(assert_parity(mixed, om, exact_dist=True))
    assert states_equal(batched, mixed)


def test_compaction_lidar():
    import math
    import oracle
    scene, steps = synth.rig_sequence(3)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2,
                         azimuth_start=math.radians(-180.0))
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(11)
    say("case: compacted launches, LiDAR 1024x64, 3 scans, never/always")
    imgs = [synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose, device="cuda"), rng)
            for st in steps]
    maps = {}
    for mode in ("never", "always"):
        m = gpu_map(params, block_capacity=1 << 17)
        m.set_launch_config(compaction=mode)
        for img, st in zip(imgs, steps):
            m.integrate_range(torch.as_tensor(img, device="cuda"), L, st.lidar_pose)
        maps[mode] = m
    torch.cuda.synchronize()
    assert states_equal(maps["never"], maps["always"])
    om = oracle.OracleMap.from_params(params)
    for img, st in zip(imgs, steps):
        om.integrate_range(img, L, st.lidar_pose)
    say(assert_parity(maps["always"], om, exact_dist=True))


def test_compaction_learned_weighting():
    import oracle
    from paper_2311_00626_amd import sensor_model as sm
    from paper_2311_00626_amd.tsdf import TsdfMap
    cam = synth.PinholeCamera(160, 120, 140.0, 140.0, 80.0, 60.0)
    r = synth.learning_room(1003, n_frames=6, camera=cam)
    _, noisy = r.frames()
    P = sm.init_params(5, scale=4.0)
    vs = 0.05
    say("case: compacted launches, learned weighting, 6 corrupted frames at 5 cm, plain and batched")
    plain = TsdfMap(vs, 4.0, weighting="learned")
    plain.set_sensor_model(P)
    plain.set_launch_config(compaction="always")
    batched = TsdfMap(vs, 4.0, weighting="learned")
    batched.set_sensor_model(P)
    batched.set_launch_config(compaction="always")
    dev = [torch.as_tensor(d, device="cuda") for d in noisy]
    om = oracle.OracleMap(vs, 4.0, weighting="constant")
    for d, dt, T in zip(noisy, dev, r.poses):
        plain.integrate_depth(dt, cam.K, T)
        w, e = oracle.sm_maps(d, cam.K, 5.0, vs, P)
        om.integrate_learned(d, cam.K, T, w, e)
    batched.integrate_depth_views(dev[:3], [cam.K] * 3, r.poses[:3])
    batched.integrate_depth_views(dev[3:], [cam.K] * 3, r.poses[3:])
    torch.cuda.synchronize()
    say(assert_parity(plain, om, exact_dist=True))
    say(assert_parity(batched, om, exact_dist=True))


def test_compaction_rejected_with_ray_walk_is_ignored():
    """Ray-walk allocation marks its own candidates: a compaction request is
    ignored there and the map still matches the oracle's walk."""
    import oracle
    w = synth.box_room_sequence(0.05, n_frames=3)
    say("case: compaction requested with ray-walk allocation (ignored), box room 5 cm")
    frames = w.frames(device="cuda")
    m = gpu_map(w.params, allocation="ray_walk")
    m.set_launch_config(compaction="always")
    om = oracle.OracleMap.from_params(w.params)
    for f, T in zip(frames, w.poses):
        m.integrate_depth(torch.as_tensor(f, device="cuda"), w.camera.K, T)
        om.integrate_dda(f, w.camera.K, T)
    torch.cuda.synchronize()
    say(assert_parity(m, om, exact_dist=True))


def test_step_switches_cull_layout_between_batches():
    """One graph step alternating between camera-only batches (the cull kernel
    gives each view a lane) and camera + LiDAR batches (each lane tests all of
    its block's views), with compaction forced on: bitwise equal to eager
    launches and to the oracle."""
    import oracle
    scene, steps = synth.rig_sequence(4)
    L = synth.LidarModel(width=512, height=32, max_range=12.0, interp_max_diff=0.2)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(17)
    say("case: graph step alternating camera-only and camera+LiDAR batches, compaction forced on")
    batches = []
    for k, st in enumerate(steps):
        cams = [synth.add_depth_noise(synth.render_depth(scene, c, T, device="cuda"), rng)
                for c, T in zip(st.cameras, st.poses)]
        imgs, Ks, Ts = cams, [c.K for c in st.cameras], list(st.poses)
        if k % 2:
            imgs = imgs + [synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose, device="cuda"), rng)]
            Ks, Ts = Ks + [L], Ts + [st.lidar_pose]
        batches.append((imgs, Ks, Ts))
    graph = gpu_map(params, block_capacity=1 << 16)
    graph.set_launch_config(compaction="always")
    eager = gpu_map(params, block_capacity=1 << 16)
    eager.set_launch_config(compaction="always")
    step = graph.step(with_spherical=True)
    om = oracle.OracleMap.from_params(params)
    for imgs, Ks, Ts in batches:
        dev = [torch.as_tensor(x, device="cuda") for x in imgs]
        step.run(dev, Ks, Ts)
        eager.integrate_depth_views(dev, Ks, Ts)
        torch.cuda.synchronize()
        for x, K, T in zip(imgs, Ks, Ts):
            if hasattr(K, "params"):
                om.integrate_range(x, K, T)
            else:
                om.integrate(x, K, T)
    step.close()
    assert states_equal(graph, eager)
    say(assert_parity(graph, om, exact_dist=True))
