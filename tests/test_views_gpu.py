"""GPU parity of the batched path (integrate_depth_views): one launch for up
to 16 views must equal integrating the views one by one, in order, in the
binary32 oracle (blocks bit-exact, weights exact, distances within 1e-5 m)."""
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


def run_batches(params, frames, Ks, poses, batch, max_ranges=None, check_touched=True):
    import oracle
    gm = gpu_map(params)
    om = oracle.OracleMap.from_params(params)
    dev = [torch.as_tensor(np.ascontiguousarray(d), device="cuda") for d in frames]
    max_ranges = max_ranges or [0.0] * len(frames)
    total = 0
    for a in range(0, len(frames), batch):
        idx = list(range(a, min(a + batch, len(frames))))
        gm.integrate_depth_views([dev[k] for k in idx], [Ks[k] for k in idx], [poses[k] for k in idx],
                                 max_ranges=[max_ranges[k] for k in idx])
        union = set()
        for k in idx:
            total += om.integrate(frames[k], Ks[k], poses[k], max_range=max_ranges[k])
            union |= {tuple(x) for x in om.touched()}
        if check_touched:
            gt = gm.query_touched().cpu().numpy()
            assert {tuple(x) for x in gt} == union and len(gt) == len(union), f"touched differs, batch at {a}"
    torch.cuda.synchronize()
    st = gm.full_stats()
    assert st["voxel_updates"] == total
    assert st["voxel_writes"] <= total
    return gm, om


@pytest.mark.parametrize("batch", [16, 5, 1])
def test_views_cluttered_room(batch):
    w = synth.cluttered_room_sequence()
    n = 37
    say(f"case: cluttered room, {n} frames in batches of {batch}")
    frames = w.frames(device="cuda", count=n)
    gm, om = run_batches(w.params, frames, [w.camera.K] * n, w.poses[:n], batch)
    say(assert_parity(gm, om, exact_dist=True))


def test_views_box_room_2cm():
    w = synth.box_room_sequence(0.02, n_frames=20)
    say("case: box room 2 cm, 20 frames in batches of 8")
    frames = w.frames(device="cuda")
    gm, om = run_batches(w.params, frames, [w.camera.K] * 20, w.poses, 8)
    say(assert_parity(gm, om, exact_dist=True))


def test_views_equal_plain_path_bitwise():
    w = synth.box_room_sequence(0.04, n_frames=24)
    say("case: views vs plain integrate_depth, bitwise")
    frames = [torch.as_tensor(f, device="cuda") for f in w.frames(device="cuda")]
    a = gpu_map(w.params)
    for d, T in zip(frames, w.poses):
        a.integrate_depth(d, w.camera.K, T)
    b = gpu_map(w.params)
    for k in range(0, 24, 12):
        b.integrate_depth_views(frames[k:k + 12], [w.camera.K] * 12, w.poses[k:k + 12])
    for x, y in zip(a.sorted_state(), b.sorted_state()):
        assert np.array_equal(x, y)
    sa, sb = a.full_stats(), b.full_stats()
    assert sa["voxel_updates"] == sb["voxel_updates"] and sa["blocks"] == sb["blocks"]
    assert sb["voxel_writes"] < sa["voxel_writes"]


def test_views_heterogeneous_rig():
    scene, steps = synth.rig_sequence(12)
    say("case: rig of 4 cameras (640x480, 848x480, 424x240, 1280x720), 6 steps")
    frames, Ks, poses = [], [], []
    for st in steps[::2]:
        for cam, T in zip(st.cameras, st.poses):
            frames.append(synth.render_depth(scene, cam, T, device="cuda"))
            Ks.append(cam.K)
            poses.append(T)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff")
    gm, om = run_batches(params, frames, Ks, poses, 4)
    say(assert_parity(gm, om, exact_dist=True))


def test_views_per_view_max_range():
    w = synth.cluttered_room_sequence()
    frames = w.frames(device="cuda", count=8)
    ranges = [5.0, 3.0, 0.0, 7.5, 2.0, 5.0, 6.0, 1.0]
    say("case: per-view max range")
    import oracle
    gm = gpu_map(w.params)
    om = oracle.OracleMap.from_params(w.params)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    gm.integrate_depth_views(dev, [w.camera.K] * 8, w.poses[:8], max_ranges=ranges)
    for d, T, r in zip(frames, w.poses, ranges):
        om.integrate(d, w.camera.K, T, max_range=r)
    assert_parity(gm, om, exact_dist=True)


def test_views_max_batch_and_invalid():
    from paper_2311_00626_amd import tsdf
    w = synth.box_room_single(0)
    d = torch.as_tensor(w.frames()[0], device="cuda")
    gm = gpu_map(w.params)
    with pytest.raises(ValueError):
        gm.integrate_depth_views([d] * 17, [w.camera.K] * 17, w.poses * 17)
    bad = w.poses[0].copy()
    bad[3, 3] = 2.0
    with pytest.raises(tsdf.TsdfError):
        gm.integrate_depth_views([d, d], [w.camera.K] * 2, [w.poses[0], bad])
    assert gm.stats() == (0, 0)
    say("case: 16 identical views in one launch")
    import oracle
    gm.integrate_depth_views([d] * 16, [w.camera.K] * 16, w.poses * 16)
    om = oracle.OracleMap.from_params(w.params)
    for _ in range(16):
        om.integrate(w.frames()[0], w.camera.K, w.poses[0])
    assert_parity(gm, om, exact_dist=True)
