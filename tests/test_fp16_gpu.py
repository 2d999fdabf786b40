"""GPU parity of binary16 voxel storage: the kernel (binary32 update, binary16
round-to-nearest-even store) against the binary32 oracle with binary16
storage -- bit-exact blocks, weights and distances."""
import numpy as np
import pytest
import torch

from paper_2311_00626_amd import synth
from tests.gpu_util import assert_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_00626_amd.tsdf  # noqa: F401


def maps(params):
    import oracle
    from paper_2311_00626_amd.tsdf import TsdfMap
    return (TsdfMap.from_params(params, storage="fp16"),
            oracle.OracleMap.from_params(params, storage="fp16"))


def test_fp16_box_room_single():
    w = synth.box_room_single(0)
    say("case: fp16 storage, box room 160x120")
    gm, om = maps(w.params)
    d = w.frames()[0]
    gm.integrate_depth(torch.as_tensor(d, device="cuda"), w.camera.K, w.poses[0])
    om.integrate(d, w.camera.K, w.poses[0])
    say(assert_parity(gm, om, exact_dist=True))


def test_fp16_cluttered_room_plain_and_batched():
    w = synth.cluttered_room_sequence()
    n = 30
    say(f"case: fp16 storage, cluttered room, {n} frames, plain and batched")
    frames = w.frames(device="cuda", count=n)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    gm, om = maps(w.params)
    gb, _ = maps(w.params)
    for d, dd, T in zip(frames, dev, w.poses):
        gm.integrate_depth(dd, w.camera.K, T)
        om.integrate(d, w.camera.K, T)
    for a in range(0, n, 8):
        k = list(range(a, min(a + 8, n)))
        gb.integrate_depth_views([dev[i] for i in k], [w.camera.K] * len(k), [w.poses[i] for i in k])
    say(assert_parity(gm, om, exact_dist=True))
    say(assert_parity(gb, om, exact_dist=True))


def test_fp16_box_room_2cm_weights_saturate():
    w = synth.box_room_sequence(0.02, n_frames=10)
    frames = w.frames(device="cuda")
    say("case: fp16 storage, box room 2 cm, 10 frames x 12 repeats (weights reach the cap)")
    gm, om = maps(w.params)
    dev = [torch.as_tensor(f, device="cuda") for f in frames]
    for rep in range(12):
        gm.integrate_depth_views(dev, [w.camera.K] * 10, w.poses)
        for d, T in zip(frames, w.poses):
            om.integrate(d, w.camera.K, T)
    r = assert_parity(gm, om, exact_dist=True)
    say(r)
    _, _, gw = gm.sorted_state()
    assert gw.max() == 100.0
