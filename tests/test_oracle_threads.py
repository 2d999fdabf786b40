"""The multi-threaded oracle entry point (used to time the CPU baseline on all
host cores) gives the single-threaded oracle's map bit for bit: same blocks in
the same insertion order, same voxels, same touched list, same update count,
in binary32, binary64 and with binary16 storage."""
import os

import numpy as np
import pytest

from paper_2311_00626_amd import synth


def run(params, frames, K, poses, threads, precision=32, storage="fp32"):
    import oracle
    om = oracle.OracleMap.from_params(params, precision=precision, storage=storage)
    counts, touched = [], []
    for d, T in zip(frames, poses):
        counts.append(om.integrate(d, K, T) if threads == 0 else om.integrate_threads(d, K, T, threads))
        touched.append(om.touched().copy())
    d, w = om.voxels()
    return om.blocks(), d, w, counts, touched


def assert_same(a, b):
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert a[3] == b[3]
    for x, y in zip(a[4], b[4]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,storage", [(32, "fp32"), (64, "fp32"), (32, "fp16")])
def test_threads_bitwise_box_room(precision, storage):
    threads = max(2, min(8, os.cpu_count() or 2))
    ws = [synth.box_room_single(s) for s in range(4)]
    frames = [w.frames()[0] for w in ws]
    poses = [w.poses[0] for w in ws]
    p = ws[0].params
    one = run(p, frames, ws[0].camera.K, poses, 0, precision, storage)
    many = run(p, frames, ws[0].camera.K, poses, threads, precision, storage)
    assert len(one[0]) > 100 and sum(one[3]) > 0
    assert_same(one, many)


def test_threads_bitwise_cluttered_room_dropoff():
    w = synth.cluttered_room_sequence(300)
    frames = w.frames(count=3)
    one = run(w.params, frames, w.camera.K, w.poses[:3], 0)
    many = run(w.params, frames, w.camera.K, w.poses[:3], max(2, min(8, os.cpu_count() or 2)))
    assert len(one[0]) > 500
    assert_same(one, many)
