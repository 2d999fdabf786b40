"""The graph-replayed batched step (tsdf_step_*): a captured hipGraph of
[argument upload + batched integration kernel], replayed once per step with
eager work on the same map and stream in between, must leave exactly the map
that integrate_depth_views leaves (bitwise), and so the binary32 oracle's."""
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


def same_state(a, b):
    sa, sb = a.sorted_state(), b.sorted_state()
    return all(np.array_equal(x, y) for x, y in zip(sa, sb))


def test_step_replays_match_eager_and_oracle():
    import oracle
    w = synth.cluttered_room_sequence()
    n = 40
    say(f"case: graph step, cluttered room, {n} frames in uneven batches, eager calls between replays")
    frames = w.frames(device="cuda", count=n)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    K = w.camera.K
    ge, gs = gpu_map(w.params), gpu_map(w.params)
    om = oracle.OracleMap.from_params(w.params)
    step = gs.step()
    batches, a = [], 0
    for size in (1, 3, 16, 5, 2, 8, 1, 4):
        batches.append(list(range(a, min(a + size, n))))
        a += size
    for b_i, idx in enumerate(batches):
        if not idx:
            continue
        args = ([dev[k] for k in idx], [K] * len(idx), [w.poses[k] for k in idx])
        if b_i % 3 == 2:
            # eager work on both maps between replays
            for k in idx:
                ge.integrate_depth(dev[k], K, w.poses[k])
                gs.integrate_depth(dev[k], K, w.poses[k])
        else:
            ge.integrate_depth_views(*args)
            step.run(*args)
        union = set()
        for k in idx:
            om.integrate(frames[k], K, w.poses[k])
            last = {tuple(x) for x in om.touched()}
            union |= last
        if b_i % 3 == 2:
            union = last          # one launch per frame: the touched list is the last frame's
        ts = {tuple(x) for x in gs.query_touched().cpu().numpy()}
        assert ts == union, f"touched set differs after batch {b_i}"
        assert same_state(ge, gs), f"graph step differs from eager after batch {b_i}"
    torch.cuda.synchronize()
    step.close()
    se, ss = ge.full_stats(), gs.full_stats()
    assert se["voxel_updates"] == ss["voxel_updates"] and se["blocks"] == ss["blocks"]
    say(assert_parity(gs, om, exact_dist=True))


def test_step_back_to_back_replays_fp16():
    """Many replays queued without host synchronisation (the staging slots
    alternate), binary16 storage."""
    import oracle
    w = synth.box_room_sequence(0.05, n_frames=48)
    say("case: graph step, box room 5 cm fp16, 12 back-to-back replays of 4 views")
    frames = w.frames(device="cuda")
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    gs = gpu_map(w.params, storage="fp16")
    om = oracle.OracleMap.from_params(w.params, storage="fp16")
    step = gs.step()
    for a in range(0, 48, 4):
        step.run(dev[a:a + 4], [w.camera.K] * 4, w.poses[a:a + 4])
    for f, T in zip(frames, w.poses):
        om.integrate(f, w.camera.K, T)
    torch.cuda.synchronize()
    step.close()
    say(assert_parity(gs, om, exact_dist=True))


def test_step_rig_with_lidar():
    import oracle
    from paper_2311_00626_amd.tsdf import TsdfError
    scene, steps = synth.rig_sequence(3)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(5)
    say("case: graph step, rig of 4 cameras + LiDAR, 3 steps")
    gs, ge = gpu_map(params), gpu_map(params)
    om = oracle.OracleMap.from_params(params)
    pinhole_only = gs.step(with_spherical=False)
    step = gs.step(with_spherical=True)
    for st in steps:
        depths = [torch.as_tensor(synth.add_depth_noise(synth.render_depth(scene, c, T, device="cuda"), rng),
                                  device="cuda") for c, T in zip(st.cameras, st.poses)]
        r = torch.as_tensor(synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose, device="cuda"), rng),
                            device="cuda")
        views = depths + [r]
        Ks = [c.K for c in st.cameras] + [L]
        Ts = list(st.poses) + [st.lidar_pose]
        with pytest.raises(TsdfError):
            pinhole_only.run(views, Ks, Ts)
        step.run(views, Ks, Ts)
        ge.integrate_depth_views(views, Ks, Ts)
        for d, c, T in zip(depths, st.cameras, st.poses):
            om.integrate(d.cpu().numpy(), c.K, T)
        om.integrate_range(r.cpu().numpy(), L, st.lidar_pose)
    torch.cuda.synchronize()
    pinhole_only.close()
    step.close()
    assert same_state(ge, gs)
    say(assert_parity(gs, om, exact_dist=True))
