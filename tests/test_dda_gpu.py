"""GPU parity of the paper-literal ray-walk allocation (TSDF_ALLOC_RAY_WALK):
the visited block set, the touched list and every voxel are bit-identical to
the binary32 oracle; the walk allocates weight-0 blocks that exact-touch
allocation does not, and the two modes agree on every voxel they share."""
import json

import numpy as np
import pytest
import torch

from paper_2311_00626_amd import synth
from tests.gpu_util import assert_parity, gpu_map, say, write_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_00626_amd.tsdf  # noqa: F401


@pytest.mark.parametrize("name", ["cluttered_640", "box_160"])
def test_ray_walk_bit_exact(name):
    import oracle
    if name == "cluttered_640":
        w = synth.cluttered_room_sequence()
        n = 6
    else:
        w = synth.box_room_sequence(0.05, n_frames=6)
        w.camera = synth.CAM_160
        n = 6
    frames = w.frames(device="cuda", count=n)
    say(f"case: ray-walk allocation, {name}, {n} frames")
    gm = gpu_map(w.params, allocation="ray_walk")
    ge = gpu_map(w.params)
    om = oracle.OracleMap.from_params(w.params)
    for k, (d, T) in enumerate(zip(frames, w.poses)):
        dt = torch.as_tensor(d, device="cuda")
        gm.integrate_depth(dt, w.camera.K, T)
        ge.integrate_depth(dt, w.camera.K, T)
        om.integrate_dda(d, w.camera.K, T)
        gt = gm.query_touched().cpu().numpy()
        ot = om.touched()
        assert {tuple(x) for x in gt} == {tuple(x) for x in ot} and len(gt) == len(ot), f"frame {k}"
    torch.cuda.synchronize()
    assert gm.status() == 0
    say(assert_parity(gm, om, exact_dist=True))
    bw, dw, ww = gm.sorted_state()
    be, de, we = ge.sorted_state()
    kw = {tuple(b): i for i, b in enumerate(bw)}
    ke = {tuple(b): i for i, b in enumerate(be)}
    zero = [b for b in kw if not np.any(ww[kw[b]] > 0)]
    report = {"workload": name, "frames": n, "blocks_ray_walk": len(bw), "blocks_exact": len(be),
              "weight0_blocks_ray_walk": len(zero), "exact_blocks_not_visited": len(set(ke) - set(kw))}
    say(json.dumps(report))
    write_report(f"ray_walk_{name}.json", report)
    assert len(zero) > 0
    assert len(set(ke) - set(kw)) <= 0.02 * len(be)


def test_ray_walk_rejections():
    from paper_2311_00626_amd.tsdf import TsdfError
    params = synth.MapParams(0.05, 4.0, "constant")
    m = gpu_map(params, allocation="ray_walk")
    d = torch.full((120, 160), 2.0, device="cuda")
    K = synth.CAM_160.K
    T = np.eye(4, dtype=np.float32)
    with pytest.raises(TsdfError):
        m.integrate_depth_views([d], [K], [T])
    with pytest.raises(TsdfError):
        m.step()
    L = synth.LidarModel(width=64, height=8, max_range=10.0)
    with pytest.raises(TsdfError):
        m.integrate_range(torch.full((8, 64), 2.0, device="cuda"), L, T)
