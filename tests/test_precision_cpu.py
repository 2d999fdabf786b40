"""The zero-crossing measure used by the precision report: on exact signed
distance fields of the room (and of the room with its walls moved by a known
amount) it recovers the walls' offsets exactly."""
import numpy as np
import pytest

from tests.test_precision_gpu import crossing_stats, wall_crossings


def exact_room_state(vs, room, shift):
    nb = [int(np.ceil((L / vs + 2) / 8)) + 1 for L in room]
    blocks = np.array([[x, y, z] for x in range(-1, nb[0]) for y in range(-1, nb[1]) for z in range(-1, nb[2])],
                      np.int32)
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    loc = np.stack([lx, ly, lz], -1).reshape(-1, 3)
    p = (blocks[:, None, :].astype(np.float64) * 8 + loc[None] + 0.5) * vs
    # walls moved inward by `shift`: the surface sits `shift` inside each wall
    dist = np.min(np.stack([p[..., 0] - shift, room[0] - shift - p[..., 0], p[..., 1] - shift,
                            room[1] - shift - p[..., 1], p[..., 2] - shift, room[2] - shift - p[..., 2]], -1), -1)
    return blocks, dist.astype(np.float32), np.ones_like(dist, dtype=np.float32)


@pytest.mark.parametrize("shift", [0.0, 0.03, -0.04])
def test_wall_crossings_recover_wall_offsets(shift):
    vs, room = 0.1, (2.0, 1.5, 1.0)
    c = wall_crossings(exact_room_state(vs, room, shift), vs, room, margin_vox=2)
    v = np.concatenate([x[np.isfinite(x)] for x in c.values()])
    assert v.size > 300 and len(c) == 6
    assert np.allclose(v, shift, atol=1e-6)
    st = crossing_stats(c)
    assert abs(st["mean_abs_m"] - abs(shift)) < 1e-6
    assert crossing_stats(c, c)["max_abs_m"] == 0.0
