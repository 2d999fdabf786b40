"""GPU parity and gain of the learned sensor model: the per-pixel (weight,
truncation) maps and the fusion that uses them are bit-identical to the CPU
oracle; the loss and gradient kernels agree with the oracle's binary64 loss
and gradient; training on corrupted renders lowers the surface error below the
linear-dropoff fallback on rooms it has not seen."""
import json

import numpy as np
import pytest
import torch

from paper_2311_00626_amd import synth
from tests.gpu_util import assert_parity, say, write_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_00626_amd.tsdf  # noqa: F401


CAM = synth.PinholeCamera(160, 120, 140.0, 140.0, 80.0, 60.0)


def room_frames(seed, n, cam=CAM):
    r = synth.learning_room(seed, n_frames=n, camera=cam)
    clean, noisy = r.frames()
    return r, clean, noisy


@pytest.mark.parametrize("scale", [1.0, 6.0])
def test_maps_bit_exact(scale):
    import oracle
    from paper_2311_00626_amd import sensor_model as sm
    from paper_2311_00626_amd.tsdf import sensor_maps
    r, clean, noisy = room_frames(1000, 12)
    P = sm.init_params(3, scale=scale)
    P[sm.B3:] = sm.round_bf16(np.array([0.3, -0.4], np.float32))
    say(f"case: sensor-model maps, 160x120 corrupted frames, parameter scale {scale}")
    pt = torch.as_tensor(P, device="cuda")
    for k in (0, 5, 11):
        d = noisy[k]
        got = sensor_maps(torch.as_tensor(d, device="cuda"), CAM.K, 5.0, 0.02, pt).cpu().numpy()
        w, e = oracle.sm_maps(d, CAM.K, 5.0, 0.02, P)
        assert np.array_equal(got[..., 0], w) and np.array_equal(got[..., 1], e)
        valid = (d > 0) & (d <= 5)
        assert np.all(w[valid] > 0) and np.all((e[valid] > 0.02) & (e[valid] < 0.16))
        assert np.std(w[valid]) > 0.01 or scale == 1.0


def test_learned_fusion_bit_exact_plain_and_batched():
    import oracle
    from paper_2311_00626_amd import sensor_model as sm
    from paper_2311_00626_amd.tsdf import TsdfMap
    r, clean, noisy = room_frames(1001, 10)
    P = sm.init_params(5, scale=4.0)
    vs = 0.05
    say("case: learned fusion, 10 corrupted frames at 5 cm, plain and batched, vs oracle")
    plain = TsdfMap(vs, 4.0, weighting="learned")
    plain.set_sensor_model(P)
    batched = TsdfMap(vs, 4.0, weighting="learned")
    batched.set_sensor_model(P)
    om = oracle.OracleMap(vs, 4.0, weighting="constant")
    dev = [torch.as_tensor(d, device="cuda") for d in noisy]
    for d, dt, T in zip(noisy, dev, r.poses):
        plain.integrate_depth(dt, CAM.K, T)
        w, e = oracle.sm_maps(d, CAM.K, 5.0, vs, P)
        om.integrate_learned(d, CAM.K, T, w, e)
        gt = {tuple(x) for x in plain.query_touched().cpu().numpy()}
        assert gt == {tuple(x) for x in om.touched()}
    for a in range(0, 10, 5):
        batched.integrate_depth_views(dev[a:a + 5], [CAM.K] * 5, r.poses[a:a + 5])
    torch.cuda.synchronize()
    say(assert_parity(plain, om, exact_dist=True))
    say(assert_parity(batched, om, exact_dist=True))


def test_learned_map_rejections():
    from paper_2311_00626_amd.tsdf import TsdfError, TsdfMap
    m = TsdfMap(0.05, 4.0, weighting="learned")
    d = torch.full((120, 160), 2.0, device="cuda")
    with pytest.raises(TsdfError):
        m.integrate_depth(d, CAM.K, np.eye(4, dtype=np.float32))       # no parameters yet
    bad = np.full(2018, 0.1, np.float32)                                # not bfloat16 values
    with pytest.raises(TsdfError):
        m.set_sensor_model(bad)
    with pytest.raises(TsdfError):
        m.step()


def loss_case(width=48, height=36, idx=(0, 8, 16, 23)):
    import oracle
    cam = synth.PinholeCamera(width, height, 40.0, 40.0, width / 2, height / 2)
    r, clean, noisy = room_frames(1002, 24, cam)
    vs = 0.1
    om = oracle.OracleMap(vs, 4.0, precision=64, weighting="constant")
    for k in idx:
        om.integrate(clean[k], cam.K, r.poses[k])
    blocks, dist, weight = om.sorted_state()
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    loc = np.stack([lx, ly, lz], -1).reshape(-1, 3)
    g = (blocks[:, None, :] * 8 + loc[None]).reshape(-1, 3)
    D, W = dist.reshape(-1), weight.reshape(-1)
    keep = (W > 0) & (np.abs(D) < 4 * vs)
    return cam, [noisy[k] for k in idx], [r.poses[k] for k in idx], g[keep].astype(np.int32), D[keep], vs


@pytest.mark.parametrize("width,height,idx", [(48, 36, (0, 8, 16, 23)), (50, 37, tuple(range(0, 24, 2)))],
                         ids=["48x36-4frames", "50x37-12frames-partial-tile"])
def test_loss_and_gradient_match_oracle(width, height, idx):
    """50x37 = 1850 pixels leaves a partial 64-pixel tile at the end of every
    frame of the backward pass; 12 frames is a window longer than the 8 of
    training."""
    import oracle
    from paper_2311_00626_amd import sensor_model as sm
    from paper_2311_00626_amd.tsdf import SmTrainer
    cam, frames, poses, vox, target, vs = loss_case(width, height, idx)
    P = sm.init_params(7, scale=3.0)
    say(f"case: loss/gradient, {len(idx)} frames {width}x{height}, {len(vox)} target voxels, vs oracle "
        "(bfloat16-emulating binary64)")
    loss_o, grad_o, used_o = oracle.sm_loss_grad(P, frames, cam.K, poses, vs, 5.0, vox, target, emulate_bf16=True)
    tr = SmTrainer(cam.width, cam.height, len(idx))
    grad = torch.zeros(2018, device="cuda")
    loss_g, used_g = tr.loss_grad(torch.as_tensor(P, device="cuda"), [torch.as_tensor(f, device="cuda") for f in frames],
                                  cam.K, poses, vs, 5.0, torch.as_tensor(vox, device="cuda"),
                                  torch.as_tensor(target.astype(np.float32), device="cuda"), grad)
    g = grad.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - grad_o) / np.linalg.norm(grad_o)
    blocks = check_gradient_blocks(g, grad_o)
    say({"loss_gpu": loss_g, "loss_oracle": loss_o, "used": [used_g, used_o], "grad_rel_err": rel,
         "blocks": blocks})
    # the voxels reached and the loss: the GPU projects and fuses in binary32,
    # the oracle in binary64, so a voxel on a pixel or band boundary may go
    # the other way (none did in the recorded runs)
    assert abs(used_g - used_o) <= 2
    assert abs(loss_g - loss_o) <= 1e-5 * loss_o


# Parameter blocks of the perceptron (offsets into the 2018 parameters).
GRAD_BLOCKS = {"W1": (0, 864), "b1": (864, 896), "W2": (896, 1920), "b2": (1920, 1952), "W3": (1952, 2016),
               "b3": (2016, 2018)}
# Tolerances of the binary32 gradient kernels against the binary64 oracle.
# Every parameter gradient is a sum over 10^3 - 10^4 pixels of products of
# bfloat16 values accumulated in binary32 (order set by atomics and matrix
# cores): rounding contributes a relative error of order sqrt(n) 2^-24,
# ~1e-5 in the worst block, and the recorded runs stay near 2e-6.  The bounds
# below sit above that and far below what a wrong term moves: a sign error, a
# transposed operand or a dropped term (a ReLU mask, a bias, the clamp's
# truncation path) changes its block by a sizeable fraction of its norm.
GRAD_BLOCK_RTOL = 1e-4         # |g_b - o_b| / |o_b| per block
GRAD_ELEM_RTOL = 1e-3          # per element, relative to the element
GRAD_ELEM_ATOL = 1e-4          # per element, relative to the block's largest magnitude


def check_gradient_blocks(g, o):
    """Per parameter block: relative L2 error and an element-wise bound."""
    out = {}
    for name, (a, b) in GRAD_BLOCKS.items():
        gb, ob = g[a:b], o[a:b]
        scale = np.abs(ob).max()
        assert scale > 0, f"{name} receives no gradient"
        rel = float(np.linalg.norm(gb - ob) / np.linalg.norm(ob))
        worst = float((np.abs(gb - ob) / (GRAD_ELEM_RTOL * np.abs(ob) + GRAD_ELEM_ATOL * scale)).max())
        out[name] = {"rel": rel, "elem_bound_used": worst}
        assert rel < GRAD_BLOCK_RTOL, f"{name}: relative error {rel:.3g}"
        assert worst <= 1.0, f"{name}: an element is off by {worst:.3g}x its bound"
    return out


def test_training_beats_linear_dropoff_on_held_out_rooms():
    """Reduced configuration (160x120, 2 cm, 6 training rooms of 40 frames):
    the trained model fuses the held-out rooms' corrupted frames closer to the
    clean fusion than the linear-dropoff fallback does."""
    from paper_2311_00626_amd import sensor_model as sm
    vs = 0.02
    say("case: training, 6 rooms x 40 frames (windows of 8) at 160x120 / 2 cm, 300 steps; 2 held-out rooms")
    rooms = [sm.prepare_room(1000 + k, 40, CAM, vs, window=8) for k in range(6)]
    held = [sm.prepare_room(2000 + k, 40, CAM, vs, window=8) for k in range(2)]
    p0 = sm.init_params(0)
    before = sm.window_loss(p0, held, vs)
    res = sm.train(rooms, vs, steps=300, lr=3e-3)
    after = sm.window_loss(res.params, held, vs)
    errs = [sm.surface_error(r, vs, res.params) for r in held]
    say(json.dumps({"held_out_loss_before": before, "held_out_loss_after": after, "loss_log": res.losses[:4] +
                    res.losses[-4:], "surface_error": errs}))
    write_report("sensor_model_gain.json", {"before": before, "after": after, "errors": errs, "losses": res.losses})
    assert after < before
    for e in errs:
        assert e["learned"]["rms_m"] < e["fallback"]["rms_m"]


def test_training_full_configuration_gain():
    """The full learned-model configuration: 20 training rooms (seeds
    1000-1019) x 100 corrupted 640x480 frames = 2000 frames, 2 cm voxels,
    windows of 8 frames, 2400 Adam steps; held-out rooms 2000-2002.  On
    every held-out room the learned model's fusion is closer to the clean
    fusion than the linear-dropoff fallback's, by at least a tenth in RMS
    (runs of this configuration have measured 24-31 %)."""
    from paper_2311_00626_amd import sensor_model as sm
    say("case: full configuration, 20 rooms x 100 frames at 640x480 / 2 cm, 2400 steps; held-out rooms 2000-2002")
    out = sm.gain_run()
    gains = {}
    for seed, e in out["surface_error"].items():
        gains[seed] = 1.0 - e["learned"]["rms_m"] / e["fallback"]["rms_m"]
    say(json.dumps({"held_out_loss_before": out["held_out_loss_before"],
                    "held_out_loss_after": out["held_out_loss_after"], "rms_gain": gains,
                    "data_s": out["data_s"], "train_s": out["train_s"]}))
    write_report("sensor_model_gain_full.json", {**out, "rms_gain": gains})
    assert out["held_out_loss_after"] < out["held_out_loss_before"]
    assert len(gains) == 3
    for seed, g in gains.items():
        assert g >= 0.10, (seed, g)
        e = out["surface_error"][seed]
        assert e["learned"]["mean_abs_m"] < e["fallback"]["mean_abs_m"]
        assert e["voxels"] > 10000
