"""Learned sensor model: training data, training loop and evaluation.

The model (a per-pixel perceptron giving each depth pixel its measurement
weight and truncation distance, see include/tsdf.h) is trained on the GPU by
the library's own kernels (tsdf_sm_loss_grad, tsdf_sm_adam); this module only
prepares the data and drives them.

Data: rooms from the cluttered-room generator (8 x 6 x 3 m, 40 spheres, 20
boxes) seen along a spline path; each frame is rendered twice from the same
pose, clean and corrupted (axial noise sigma = 0.0012 z^2 m, then 3 % flying
pixels at depth edges).  A training window is a run of consecutive frames; its
targets are the voxels within epsilon of the surface in the constant-weight
fusion of the clean renders of the same window, with their fused distance.
The loss compares the fusion of the corrupted window under the model with
those targets.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import synth
from .tsdf import SM_NPARAM, SmTrainer, TsdfMap, sm_adam

N_IN, N_HID, N_OUT = 27, 32, 2
W1, B1 = 0, N_HID * N_IN
W2, B2 = B1 + N_HID, B1 + N_HID + N_HID * N_HID
W3, B3 = B2 + N_HID, B2 + N_HID + N_OUT * N_HID


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 values (ties to even) of a float32 array, as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    u = np.where(finite, r, u).astype(np.uint32)
    return u.view(np.float32)


def init_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """He-style initialisation with small outputs: the untrained model gives
    weights near 1 and truncations near 4.5 voxels."""
    rng = np.random.default_rng(seed)
    p = np.zeros(SM_NPARAM, np.float32)
    p[W1:B1] = rng.standard_normal(N_HID * N_IN) * math.sqrt(2.0 / N_IN) * 0.5 * scale
    p[B1:W2] = 0.05
    p[W2:B2] = rng.standard_normal(N_HID * N_HID) * math.sqrt(2.0 / N_HID) * 0.5 * scale
    p[B2:W3] = 0.05
    p[W3:B3] = rng.standard_normal(N_OUT * N_HID) * 0.02 * scale
    p[B3:] = 0.0
    return round_bf16(p)


@dataclass
class Window:
    frames: List[torch.Tensor]      # corrupted depth, device
    poses: List[np.ndarray]
    vox: torch.Tensor               # (n, 3) int32 global voxel indices, device
    target: torch.Tensor            # (n,) float32 target distances, device


@dataclass
class Room:
    seed: int
    camera: synth.PinholeCamera
    windows: List[Window] = field(default_factory=list)
    clean: List[torch.Tensor] = field(default_factory=list)
    noisy: List[torch.Tensor] = field(default_factory=list)
    poses: List[np.ndarray] = field(default_factory=list)


def fused_targets(frames: Sequence[torch.Tensor], K, poses, vs: float, max_range: float,
                  band_vox: float = 4.0):
    """Voxels within band_vox voxels of the surface in the constant-weight
    fusion of `frames` (truncation band_vox voxels), and their distances."""
    m = TsdfMap(vs, band_vox, weighting="constant", max_range=max_range, block_capacity=1 << 18)
    for d, T in zip(frames, poses):
        m.integrate_depth(d, K, T)
    blocks = m.query_blocks()
    dist, weight = m.query_tsdf(blocks)
    lz, ly, lx = torch.meshgrid(torch.arange(8), torch.arange(8), torch.arange(8), indexing="ij")
    loc = torch.stack([lx, ly, lz], -1).reshape(-1, 3).to(blocks.device, torch.int32)
    g = (blocks[:, None, :] * 8 + loc[None]).reshape(-1, 3)
    D, W = dist.reshape(-1), weight.reshape(-1)
    keep = (W > 0) & (D.abs() < band_vox * vs)
    m.close()
    return g[keep].contiguous(), D[keep].contiguous()


def prepare_room(seed: int, n_frames: int, camera: synth.PinholeCamera, vs: float, window: int,
                 max_range: float = 5.0, stride: Optional[int] = None) -> Room:
    lr = synth.learning_room(seed, n_frames=n_frames, camera=camera)
    clean, noisy = lr.frames(device="cuda")
    room = Room(seed, camera)
    room.clean = [torch.as_tensor(c, device="cuda") for c in clean]
    room.noisy = [torch.as_tensor(n, device="cuda") for n in noisy]
    room.poses = [np.ascontiguousarray(p, dtype=np.float32) for p in lr.poses]
    stride = stride or window
    for a in range(0, n_frames - window + 1, stride):
        idx = range(a, a + window)
        vox, target = fused_targets([room.clean[k] for k in idx], camera.K, [room.poses[k] for k in idx], vs,
                                    max_range)
        room.windows.append(Window([room.noisy[k] for k in idx], [room.poses[k] for k in idx], vox, target))
    return room


@dataclass
class TrainResult:
    params: np.ndarray
    losses: List[float]
    steps: int


def train(rooms: Sequence[Room], vs: float, steps: int, lr: float = 2e-3, seed: int = 0,
          init: Optional[np.ndarray] = None, max_range: float = 5.0, log_every: int = 25) -> TrainResult:
    """Adam on the windows of `rooms`, one window per step (drawn at random)."""
    cam = rooms[0].camera
    win = max(len(w.frames) for r in rooms for w in r.windows)
    p0 = init if init is not None else init_params(seed)
    master = torch.as_tensor(p0.astype(np.float32), device="cuda").contiguous()
    params = master.clone()
    m1 = torch.zeros_like(master)
    m2 = torch.zeros_like(master)
    grad = torch.zeros_like(master)
    trainer = SmTrainer(cam.width, cam.height, win)
    rng = np.random.default_rng(seed + 1)
    pairs = [(r, w) for r in rooms for w in r.windows]
    losses = []
    for step in range(1, steps + 1):
        room, w = pairs[int(rng.integers(len(pairs)))]
        want = step % log_every == 0 or step == 1
        out = trainer.loss_grad(params, w.frames, cam.K, w.poses, vs, max_range, w.vox, w.target, grad,
                                want_loss=want)
        if want:
            losses.append(out[0])
        sm_adam(master, m1, m2, grad, params, lr, step)
    torch.cuda.synchronize()
    trainer.close()
    return TrainResult(params.cpu().numpy(), losses, steps)


def window_loss(params: np.ndarray, rooms: Sequence[Room], vs: float, max_range: float = 5.0) -> float:
    """Mean training loss over every window of `rooms` (voxel-weighted)."""
    cam = rooms[0].camera
    win = max(len(w.frames) for r in rooms for w in r.windows)
    trainer = SmTrainer(cam.width, cam.height, win)
    p = torch.as_tensor(params, device="cuda").contiguous()
    g = torch.zeros_like(p)
    tot, n = 0.0, 0
    for r in rooms:
        for w in r.windows:
            loss, used = trainer.loss_grad(p, w.frames, cam.K, w.poses, vs, max_range, w.vox, w.target, g)
            tot += loss * used
            n += used
    trainer.close()
    return tot / max(n, 1)


def surface_error(room: Room, vs: float, params: Optional[np.ndarray], max_range: float = 5.0,
                  fallback_trunc_vox: float = 4.0) -> dict:
    """Fuses the room's corrupted frames with the learned model and with the
    linear-dropoff fallback, and compares each with the constant-weight fusion
    of the clean renders, over voxels within one voxel of the clean surface
    that all three maps observe: RMS and mean absolute distance error."""
    cam = room.camera
    ref = TsdfMap(vs, fallback_trunc_vox, weighting="constant", max_range=max_range, block_capacity=1 << 18)
    fb = TsdfMap(vs, fallback_trunc_vox, weighting="linear_dropoff", max_range=max_range, block_capacity=1 << 18)
    maps = {"reference": ref, "fallback": fb}
    if params is not None:
        lm = TsdfMap(vs, fallback_trunc_vox, weighting="learned", max_range=max_range, block_capacity=1 << 18)
        lm.set_sensor_model(params)
        maps["learned"] = lm
    for c, nz, T in zip(room.clean, room.noisy, room.poses):
        ref.integrate_depth(c, cam.K, T)
        fb.integrate_depth(nz, cam.K, T)
        if "learned" in maps:
            maps["learned"].integrate_depth(nz, cam.K, T)
    blocks = ref.query_blocks()
    states = {k: m.query_tsdf(blocks) for k, m in maps.items()}
    Dr, Wr = states["reference"]
    sel = (Wr > 0) & (Dr.abs() <= vs)
    for k in ("fallback", "learned"):
        if k in states:
            sel &= states[k][1] > 0
    out = {"voxels": int(sel.sum().item())}
    for k in ("fallback", "learned"):
        if k in states:
            e = (states[k][0] - Dr)[sel].double()
            out[k] = {"rms_m": float(e.pow(2).mean().sqrt().item()), "mean_abs_m": float(e.abs().mean().item())}
    for m in maps.values():
        m.close()
    return out


def gain_run(n_rooms: int = 20, n_held_out: int = 3, frames: int = 100, vs: float = 0.02, window: int = 8,
             steps: int = 2400, lr: float = 3e-3, log_every: int = 0) -> dict:
    """Trains on rooms 1000.. and compares the learned model with the
    linear-dropoff fallback on held-out rooms 2000.. (640x480 frames); the
    defaults are the full configuration.  Returns the losses, timings and
    per-room surface errors."""
    import time
    cam = synth.CAM_640
    t0 = time.perf_counter()
    rooms = [prepare_room(1000 + k, frames, cam, vs, window=window) for k in range(n_rooms)]
    held = [prepare_room(2000 + k, frames, cam, vs, window=window) for k in range(n_held_out)]
    t_data = time.perf_counter() - t0
    before = window_loss(init_params(0), held, vs)
    t1 = time.perf_counter()
    res = train(rooms, vs, steps=steps, lr=lr, seed=0, log_every=log_every or max(1, steps // 12))
    t_train = time.perf_counter() - t1
    return {"train_rooms": n_rooms, "frames_per_room": frames, "resolution": f"{cam.width}x{cam.height}",
            "voxel_m": vs, "window": window, "steps": steps, "data_s": t_data, "train_s": t_train,
            "held_out_loss_before": before, "held_out_loss_after": window_loss(res.params, held, vs),
            "loss_log": res.losses,
            "surface_error": {str(r.seed): surface_error(r, vs, res.params) for r in held}}


def main(argv=None) -> dict:
    """Trains at a chosen scale and compares with the linear-dropoff fallback
    on held-out rooms.  Defaults: the full configuration -- 20 training rooms
    (seeds 1000-1019) x 100 corrupted 640x480 frames, 2 cm voxels, windows of
    8 frames, 2400 Adam steps; held-out rooms 2000-2002.  Prints one JSON
    object (and writes it to --out if given)."""
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--rooms", type=int, default=20)
    ap.add_argument("--held-out", type=int, default=3)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--voxel", type=float, default=0.02)
    ap.add_argument("--window", type=int, default=8)
    ap.add_argument("--steps", type=int, default=2400)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    out = gain_run(args.rooms, args.held_out, args.frames, args.voxel, args.window, args.steps, args.lr)
    text = json.dumps(out)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    return out


if __name__ == "__main__":
    main()
