"""Saving and restoring a map (query_blocks + query_tsdf to .npz, insert_blocks
back): the restored map holds the same blocks and every distance and weight
bit for bit, and integration continues from it exactly -- after more frames
it equals the map that was never saved and the oracle fed every frame, for
binary32 and binary16 storage.  Restoring into a pool too small records the
sticky overflow."""
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
    return (np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1].view(np.uint32), sb[1].view(np.uint32))
            and np.array_equal(sa[2].view(np.uint32), sb[2].view(np.uint32)))


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_save_restore_continue(tmp_path, storage):
    import oracle
    from paper_2311_00626_amd.tsdf import TsdfMap
    w = synth.cluttered_room_sequence(300)
    n1, n2 = 20, 40
    say(f"case: save after {n1} frames, restore, {n2 - n1} more frames, cluttered room 4 cm, {storage}")
    frames = w.frames(device="cuda", count=n2)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    m = gpu_map(w.params, block_capacity=1 << 15, storage=storage)
    om = oracle.OracleMap.from_params(w.params, storage=storage)
    for k in range(n1):
        m.integrate_depth(dev[k], w.camera.K, w.poses[k])
        om.integrate(frames[k], w.camera.K, w.poses[k])
    path = str(tmp_path / "map.npz")
    m.save(path)
    r = TsdfMap.load(path)
    assert same_state(m, r), "restored map differs"
    st = r.full_stats()
    assert st["blocks"] == m.full_stats()["blocks"] and r.status() == 0
    for k in range(n1, n2):
        m.integrate_depth(dev[k], w.camera.K, w.poses[k])
        r.integrate_depth(dev[k], w.camera.K, w.poses[k])
        om.integrate(frames[k], w.camera.K, w.poses[k])
        assert {tuple(x) for x in r.query_touched().cpu().numpy()} == {tuple(x) for x in om.touched()}
    torch.cuda.synchronize()
    assert same_state(m, r), "integration after the restore differs"
    say(assert_parity(r, om, exact_dist=True))
    z = np.load(path)   # plain arrays only
    assert z["blocks"].dtype == np.int32 and z["dist"].shape == (z["blocks"].shape[0], 512)


def test_restore_overflow_is_sticky(tmp_path):
    from paper_2311_00626_amd.tsdf import EFULL, TsdfMap
    w = synth.cluttered_room_sequence(300)
    say("case: restore ~1 000 blocks into a 256-block pool")
    m = gpu_map(w.params, block_capacity=1 << 14)
    d = torch.as_tensor(w.frames(device="cuda", count=1)[0], device="cuda")
    m.integrate_depth(d, w.camera.K, w.poses[0])
    path = str(tmp_path / "map.npz")
    m.save(path)
    n = m.full_stats()["blocks"]
    assert n > 256
    r = TsdfMap.load(path, block_capacity=256)
    assert r.status() == EFULL
    assert r.full_stats()["blocks"] == 256
