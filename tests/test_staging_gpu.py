"""LDS staging of block depth footprints (§IV-B's per-voxel nearest-pixel
sample read from a staged copy of the block's pixel rectangle): maps
integrated with staging forced on, forced off and automatic are bitwise
identical to each other and to the binary32 oracle, with the touched set
checked after every frame; for the compacted launch at 1 cm (footprints that
mostly fit the 1024-pixel region), the lattice walk at 4 cm (mostly larger
footprints, which fall back to direct reads), binary16 storage, frames seen
from close up and from far away, and ragged images whose rectangles clip at
the image edges."""
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


def run_modes(w, frames, K, poses, storage="fp32", launch=None, crop=None):
    import oracle
    maps = {}
    for mode in ("never", "always", "auto"):
        m = gpu_map(w.params, block_capacity=1 << 17, storage=storage)
        m.set_launch_config(staging=mode, **(launch or {}))
        maps[mode] = m
    om = oracle.OracleMap.from_params(w.params, storage=storage)
    for k, (f, T) in enumerate(zip(frames, poses)):
        if crop is not None:
            f = np.ascontiguousarray(f[crop[0]:, crop[1]:])
        d = torch.as_tensor(f, device="cuda")
        for m in maps.values():
            m.integrate_depth(d, K, T)
        om.integrate(f, K, T)
        want = {tuple(x) for x in om.touched()}
        for mode, m in maps.items():
            got = m.query_touched().cpu().numpy()
            assert {tuple(x) for x in got} == want and len(got) == len(want), f"touched set ({mode}), frame {k}"
    torch.cuda.synchronize()
    ref = maps["never"].sorted_state()
    for mode in ("always", "auto"):
        st = maps[mode].sorted_state()
        assert all(np.array_equal(a, b) for a, b in zip(ref, st)), f"staging {mode} differs from direct reads"
    return maps, om


@pytest.mark.parametrize("vs,n", [(0.01, 6), (0.02, 10)])
def test_staging_box_room(vs, n):
    w = synth.box_room_sequence(vs, n_frames=300)
    say(f"case: LDS staging never/always/auto, box room 640x480 / {int(vs * 100)} cm, {n} frames (every 30th)")
    idx = list(range(0, 30 * n, 30))
    frames = w.frames(device="cuda", count=30 * n)
    maps, om = run_modes(w, [frames[i] for i in idx], w.camera.K, [w.poses[i] for i in idx])
    say(assert_parity(maps["always"], om, exact_dist=True))


def test_staging_cluttered_room_walk_and_fp16():
    w = synth.cluttered_room_sequence(300)
    n = 12
    say("case: LDS staging never/always/auto, cluttered room 640x480 / 4 cm, 12 frames, fp32 and fp16")
    frames = w.frames(device="cuda", count=n)
    maps, om = run_modes(w, frames, w.camera.K, w.poses[:n])
    say(assert_parity(maps["always"], om, exact_dist=True))
    maps16, om16 = run_modes(w, frames, w.camera.K, w.poses[:n], storage="fp16")
    say(assert_parity(maps16["always"], om16, exact_dist=True))


def test_staging_ragged_image_compacted():
    """A 517x389 crop of the 1 cm frames (the principal point stays, so rays
    are unchanged and rectangles clip at the crop's edges), compacted launch
    forced on."""
    w = synth.box_room_sequence(0.01, n_frames=300)
    say("case: LDS staging, box room 1 cm, frames cropped to 517x389 from (91, 123), compacted")
    frames = w.frames(device="cuda", count=90)
    K = list(w.camera.K)
    K[2] -= 123
    K[3] -= 91
    sel = [0, 45, 89]
    maps, om = run_modes(w, [frames[i] for i in sel], K, [w.poses[i] for i in sel],
                         launch={"compaction": "always"}, crop=(91, 123))
    say(assert_parity(maps["always"], om, exact_dist=True))
