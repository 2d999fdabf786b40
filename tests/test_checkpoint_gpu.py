"""Saving and restoring a map (query_blocks + query_tsdf to .npz, insert_blocks
back): the restored map holds the same blocks and every distance and weight
bit for bit, and integration continues from it exactly -- after more frames
it equals the map that was never saved and the oracle fed every frame, for
binary32 and binary16 storage.  Restoring into a pool too small records the
sticky overflow.  Many waves inserting the same keys in one call allocate
each block once."""
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


def test_insert_same_keys_from_many_waves():
    """Race stress of the hash insert: 1 000 distinct blocks, each listed 64
    times in one insert_blocks call (64 waves racing on one key's atomicCAS,
    thousands of keys competing for free slots of a hash at load ~0.5), with
    the same voxel values in every copy: exactly the distinct blocks are
    allocated, each once, with its values, and no error bit is set.  Run twice
    on fresh maps, the two maps are bitwise identical (run-to-run
    determinism of the stored state)."""
    from paper_2311_00626_amd.tsdf import TsdfMap
    say("case: insert 1 000 distinct blocks x 64 copies each (one call), hash load ~0.5")
    rng = np.random.default_rng(7)
    uniq = np.unique(rng.integers(-40, 40, size=(1400, 3)).astype(np.int32), axis=0)[:1000]
    assert len(uniq) == 1000
    dist = rng.standard_normal((1000, 512)).astype(np.float32) * 0.1
    weight = rng.integers(1, 100, size=(1000, 512)).astype(np.float32)
    order = rng.permutation(np.repeat(np.arange(1000), 64))
    states = []
    for _ in range(2):
        m = TsdfMap(0.05, 4.0, block_capacity=1024, hash_capacity=2048)
        m.insert_blocks(torch.as_tensor(uniq[order]), torch.as_tensor(dist[order]), torch.as_tensor(weight[order]))
        st = m.full_stats()
        assert m.status() == 0 and st["error_bits"] == 0
        assert st["blocks"] == 1000
        b, d, w = m.sorted_state()
        idx = np.lexsort((uniq[:, 2], uniq[:, 1], uniq[:, 0]))
        assert np.array_equal(b, uniq[idx])
        assert np.array_equal(d, dist[idx]) and np.array_equal(w, weight[idx])
        states.append((b, d, w))
        m.close()
    assert all(np.array_equal(x, y) for x, y in zip(*states))
