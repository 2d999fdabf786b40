"""Launch shapes never change results: the rig workload (4 cameras + LiDAR,
graph-replayed steps) leaves a bit-identical map under every tuned launch
configuration, and the tuner picks one of its candidates."""
import numpy as np
import pytest
import torch

from paper_2311_00626_amd import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_00626_amd.tsdf  # noqa: F401


def rig_views(n):
    scene, steps = synth.rig_sequence(n)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2)
    rng = np.random.default_rng(7)
    out = []
    for st in steps:
        views = [torch.as_tensor(synth.add_depth_noise(synth.render_depth(scene, c, T, device="cuda"), rng),
                                 device="cuda") for c, T in zip(st.cameras, st.poses)]
        views.append(torch.as_tensor(synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose,
                                                                              device="cuda"), rng), device="cuda"))
        out.append((views, [c.K for c in st.cameras] + [L], list(st.poses) + [st.lidar_pose]))
    return out


def test_launch_shapes_bit_identical_and_tuner_choice():
    from paper_2311_00626_amd import autotune as at
    from paper_2311_00626_amd.tsdf import TsdfMap
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    data = rig_views(6)
    say("case: rig, 6 graph steps under 6 launch shapes")

    def make_map():
        return TsdfMap.from_params(params, block_capacity=1 << 17)

    def make_runner(m):
        s = m.step(with_spherical=True)
        return (lambda k: s.run(*data[k])), s.close

    cands = [at.LaunchConfig(256, 1, 1), at.LaunchConfig(512, 1, 0), at.LaunchConfig(512, 8, 8),
             at.LaunchConfig(1024, 1, 4), at.LaunchConfig(2048, 1, 8), at.LaunchConfig(2048, 8, 1)]
    ref = None
    for c in cands:
        m = make_map()
        c.apply(m)
        st = m.step(with_spherical=True)
        for k in range(len(data)):
            st.run(*data[k])
        torch.cuda.synchronize()
        st.close()
        state = m.sorted_state()
        if ref is None:
            ref = state
        else:
            assert all(np.array_equal(a, b) for a, b in zip(ref, state)), f"{c} changed the map"
    choice, trials = at.tune("rig-test", make_map, None, range(len(data)), candidates=cands, rounds=1,
                             make_runner=make_runner, refresh=True)
    say("trials:", [(t.config, round(t.kernel_ms_per_launch, 4)) for t in trials])
    assert choice in cands and len(trials) == len(cands)
    assert all(t.launches == len(data) - 2 for t in trials)
