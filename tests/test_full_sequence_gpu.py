"""Parity at the measured workloads' full sizes, in the launch configurations
the benchmark times.

The headline 300-frame cluttered room (640x480, 4 cm) and the 300-frame box
room at 1 cm are fused whole by the sparse oracle (the 1 cm room on all host
cores through its multi-threaded entry point, bitwise the single-threaded
map): every allocated block, every voxel and the touched set after every
launch are compared, one frame per launch and (4 cm) 16 per launch.  500 rig
steps (4 cameras + a LiDAR reaching 25 m, whose scan box holds ~10^8 voxels
per range image) replayed from graphs would take the oracle many minutes, so
there sampled blocks are checked against its dense evaluator (every voxel of
a box fused frame by frame, no hash or candidates), which computes any voxel
on its own: allocated sampled blocks hold bit-identical (D, W), sampled
blocks the GPU did not allocate receive no update, and every allocated block
holds an updated voxel (the allocation rule, checked over the whole map)."""
import numpy as np
import pytest
import torch

from paper_2311_00626_amd import synth
from tests.gpu_util import gpu_map, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_00626_amd.tsdf  # noqa: F401


def sample_blocks(blocks: np.ndarray, rng, n_alloc: int, n_absent: int):
    """Random allocated blocks, and random blocks of their bounding box that
    are not allocated."""
    pick = blocks[rng.choice(len(blocks), size=min(n_alloc, len(blocks)), replace=False)]
    have = {tuple(b) for b in blocks}
    lo, hi = blocks.min(0), blocks.max(0)
    absent = []
    while len(absent) < n_absent:
        b = tuple(int(v) for v in rng.integers(lo, hi + 1))
        if b not in have:
            absent.append(b)
    return pick, np.array(absent, np.int32).reshape(-1, 3)


def check_map(gm, rng, dense_of_block, n_alloc=10, n_absent=6):
    blocks = gm.query_blocks().cpu().numpy()
    assert len(blocks) > 0 and gm.status() == 0
    # every allocated block holds an updated voxel
    _, w_all = gm.query_tsdf(torch.as_tensor(blocks, device="cuda"))
    assert bool((w_all.max(dim=1).values > 0).all()), "an allocated block has no updated voxel"
    alloc, absent = sample_blocks(blocks, rng, n_alloc, n_absent)
    d, w = gm.query_tsdf(torch.as_tensor(alloc, device="cuda"))
    d, w = d.cpu().numpy(), w.cpu().numpy()
    updated = 0
    for k, b in enumerate(alloc):
        dd, dw = dense_of_block(b)
        assert np.array_equal(w[k].astype(np.float64), dw.reshape(-1)), f"weights differ in block {tuple(b)}"
        assert np.array_equal(d[k].astype(np.float64), dd.reshape(-1)), f"distances differ in block {tuple(b)}"
        updated += int((dw > 0).sum())
    for b in absent:
        _, dw = dense_of_block(b)
        assert not (dw > 0).any(), f"block {tuple(b)} has updated voxels but was not allocated"
    return {"blocks": len(blocks), "sampled_allocated": len(alloc), "sampled_absent": len(absent),
            "updated_voxels_in_sample": updated}


@pytest.fixture(scope="module")
def cluttered():
    w = synth.cluttered_room_sequence(300)
    frames = w.frames(device="cuda", count=300)
    return w, frames, [torch.as_tensor(f, device="cuda") for f in frames]


@pytest.fixture(scope="module")
def cluttered_oracle(cluttered):
    """The binary32 oracle over all 300 frames: its sorted final state and
    the touched set of every frame."""
    import oracle
    w, frames, _ = cluttered
    om = oracle.OracleMap.from_params(w.params)
    touched = []
    for d, T in zip(frames, w.poses):
        om.integrate(d, w.camera.K, T)
        touched.append({tuple(x) for x in om.touched()})
    return om.sorted_state(), touched


def dense_frames(params, frames, K, poses):
    import oracle

    def of_block(b):
        return oracle.dense_integrate(params, frames, K, poses, 8 * np.asarray(b), (8, 8, 8))
    return of_block


def test_cluttered_room_300_frames_one_per_launch(cluttered, cluttered_oracle):
    w, frames, dev = cluttered
    (ob, od, ow), touched = cluttered_oracle
    say("case: cluttered room 640x480 / 4 cm, all 300 frames one per launch (default launch shape), "
        "whole map and every touched set against the sparse oracle")
    gm = gpu_map(w.params, block_capacity=1 << 16)
    for k, (d, T) in enumerate(zip(dev, w.poses)):
        gm.integrate_depth(d, w.camera.K, T)
        gt = gm.query_touched().cpu().numpy()
        assert len(gt) == len(touched[k]) and {tuple(x) for x in gt} == touched[k], f"touched set differs at frame {k}"
    torch.cuda.synchronize()
    say(compare_whole(gm, ob, od, ow))


def test_cluttered_room_300_frames_16_per_launch(cluttered, cluttered_oracle):
    w, frames, dev = cluttered
    (ob, od, ow), touched = cluttered_oracle
    B = 16
    first = len(dev) % B or B
    say("case: cluttered room 640x480 / 4 cm, 300 frames 16 per launch (compacted launches), "
        "whole map and every launch's touched set against the sparse oracle")
    gm = gpu_map(w.params, block_capacity=1 << 16)
    K = w.camera.K
    for a, b in [(0, first)] + [(a, a + B) for a in range(first, len(dev), B)]:
        gm.integrate_depth_views(dev[a:b], [K] * (b - a), w.poses[a:b])
        want = set().union(*touched[a:b])
        gt = gm.query_touched().cpu().numpy()
        assert len(gt) == len(want) and {tuple(x) for x in gt} == want, f"touched set differs at launch {a}"
    torch.cuda.synchronize()
    say(compare_whole(gm, ob, od, ow))


def compare_whole(gm, ob, od, ow):
    """Every allocated block and every voxel of the GPU map against the
    oracle's sorted state: block sets and weights identical, distances
    bit-identical."""
    gb, gd, gw = gm.sorted_state()
    assert gm.status() == 0
    assert gb.shape == ob.shape and np.array_equal(gb, ob), f"{len(gb)} GPU blocks vs {len(ob)} oracle blocks"
    assert np.array_equal(gw.astype(np.float64), ow), "weights differ"
    assert np.array_equal(gd.astype(np.float64), od), "distances differ"
    return {"blocks": len(gb), "updated_voxels": int((gw > 0).sum()), "bit_identical": True}


def test_box_room_1cm_300_frames():
    import os
    import oracle
    w = synth.box_room_sequence(0.01, n_frames=300)
    frames = w.frames(device="cuda")
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    say(f"case: box room 640x480 / 1 cm, 300 frames (footprint culling and compacted launches), whole map "
        f"and every touched set against the sparse oracle ({threads} threads)")
    gm = gpu_map(w.params, block_capacity=1 << 17)
    om = oracle.OracleMap.from_params(w.params)
    for k, (f, T) in enumerate(zip(frames, w.poses)):
        gm.integrate_depth(torch.as_tensor(f, device="cuda"), w.camera.K, T)
        om.integrate_threads(f, w.camera.K, T, threads)
        gt = gm.query_touched().cpu().numpy()
        ot = om.touched()
        assert len(gt) == len(ot), f"touched count differs at frame {k}"
        assert np.array_equal(np.unique(gt, axis=0), np.unique(ot, axis=0)), f"touched set differs at frame {k}"
    torch.cuda.synchronize()
    ob, od, ow = om.sorted_state()
    del om
    say(compare_whole(gm, ob, od, ow))


def test_rig_500_steps_graph():
    import oracle
    scene, steps = synth.rig_sequence(500)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(11)
    say("case: rig 4 cameras + LiDAR, 500 graph-replayed steps (compacted launch, footprint culling), sampled blocks")
    host = []
    gm = gpu_map(params, block_capacity=1 << 16)
    gm.set_launch_config(max_groups=512, footprint="always", compaction="always")
    step = gm.step(with_spherical=True)
    for st in steps:
        cams = [synth.add_depth_noise(synth.render_depth(scene, c, T, device="cuda"), rng)
                for c, T in zip(st.cameras, st.poses)]
        lid = synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose, device="cuda"), rng)
        host.append((cams, lid))
        views = [torch.as_tensor(v, device="cuda") for v in cams + [lid]]
        step.run(views, [c.K for c in st.cameras] + [L], list(st.poses) + [st.lidar_pose])
    torch.cuda.synchronize()
    step.close()

    def of_block(b):
        state = None
        for st, (cams, lid) in zip(steps, host):
            for img, c, T in zip(cams, st.cameras, st.poses):
                state = oracle.dense_integrate(params, [img], c.K, [T], 8 * np.asarray(b), (8, 8, 8), state=state)
            state = oracle.dense_integrate_range(params, [lid], L, [st.lidar_pose], 8 * np.asarray(b), (8, 8, 8),
                                                 state=state)
        return state
    say(check_map(gm, np.random.default_rng(23), of_block, n_alloc=6, n_absent=4))
