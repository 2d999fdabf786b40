"""Throughput of projective TSDF integration on one MI355X.

Workload: the 300-frame cluttered-room sequence (640x480 float32 depth, 8 x 6
x 3 m room with 40 spheres and 20 boxes, spline path at 0.5 m/s and 30 fps,
axial noise 0.0012 z^2 and 5 % dropped pixels; 4 cm voxels, truncation 4
voxels, linear-dropoff weight, max range 5 m).  All frames are rendered and
uploaded to HBM before timing.  One step = one integrate_depth call (all
stages of the path: culling, allocation, projection, update, touched-block
compaction) on the next frame of the sequence, into one running map.

Prints one JSON line (rank 0) with voxel updates/s as the value, frames/s,
the integration kernel's roofline (algorithmic bytes per launch over its mean
HIP-event duration, against 8 TB/s) and the CPU oracle timed on a bounded
sample of the same frames.
"""
import argparse
import hashlib
import json
from dataclasses import asdict
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGING = "auto"   # LDS footprint staging of the one-frame-per-launch legs (--staging)
PARTITIONS = 0     # image bands of the one-frame-per-launch legs (--partitions; 0 = automatic)
CHUNK = 0          # lattice blocks a wave culls per pass (--chunk; 0 = automatic)
COMPACTION = "auto"  # compacted launches of the one-frame-per-launch legs (--compaction)
PMC_SUMMARY = os.path.join(ROOT, "profiles", "integrate_depth_cluttered_room_pmc.json")
KERNEL_SOURCES = ["paper_2311_00626_amd/csrc/integrate.hip", "paper_2311_00626_amd/csrc/device_common.hpp",
                  "paper_2311_00626_amd/csrc/tsdf_internal.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_of(text: str) -> str:
    """C++ source without its comments, trailing blanks and empty lines: what
    the compiler sees, up to layout.  String and character literals are kept
    whole, so a '//' inside one is not taken for a comment."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash() -> str:
    """Hash of the measured kernels' code (comments and blank lines left out,
    so a comment edit keeps the committed counter profile valid)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(_code_of(f.read()).encode("utf-8"))
    return h.hexdigest()[:16]


def algorithmic_bytes(voxel_rw: int, touched: int, new_blocks: int, pixels: int, frames: int,
                      voxel_bytes: int = 8) -> int:
    """Bytes the method must move: one (distance, weight) read and one write per
    voxel read-modify-written (2 x 8 B binary32, 2 x 4 B binary16), one read of
    every depth pixel per frame (4 B), a hash key and value read per touched
    block (12 B) plus its touched-list entry (4 B), and a key, value and slot
    key per new block (20 B).  A single-frame launch read-modify-writes a voxel
    once per update; a batched launch once per launch (voxel writes)."""
    return 2 * voxel_bytes * voxel_rw + 4 * pixels * frames + 16 * touched + 20 * new_blocks


def _pmc_summary():
    """The committed rocprofv3 PMC summary, if it was taken on the current
    kernel source; else None."""
    try:
        with open(PMC_SUMMARY) as f:
            s = json.load(f)
    except (OSError, ValueError):
        return None
    if s.get("kernel_source_hash") != kernel_source_hash():
        return None
    return s


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the PMC summary."""
    s = _pmc_summary()
    return None if s is None else s.get("hbm_bytes_per_launch")


def measured_traffic_record():
    """The frames the PMC figure averages over, and the algorithmic bytes of
    those same frames, so that their ratio is read off one frame set."""
    s = _pmc_summary()
    if s is None:
        return None
    keys = ("frames", "algorithmic_bytes_per_launch", "traffic_over_algorithmic", "fetch_scale", "write_scale",
            "calibration")
    return {k: s[k] for k in keys if k in s}


def host_cpu() -> dict:
    """CPU model and core counts of the host the benchmark runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def oracle_threads() -> int:
    """Threads for the all-cores oracle: the CPUs this process may use,
    capped by OMP_NUM_THREADS when that is set."""
    n = host_cpu()["usable_cpus"]
    try:
        cap = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        cap = 0
    return max(1, min(n, cap) if cap > 0 else n)


def time_oracle(params, frames_host, K, poses, threads: int, min_s: float, budget_s: float, precision: int = 32):
    """Passes of the oracle over the frames, each into a fresh map, until
    `min_s` seconds have passed (at most `budget_s`); threads 0 = the
    single-threaded entry point."""
    import oracle
    updates, n, passes, t0 = 0, 0, 0, time.perf_counter()
    while True:
        om = oracle.OracleMap.from_params(params, precision=precision)
        passes += 1
        for d, T in zip(frames_host, poses):
            updates += om.integrate(d, K, T) if threads == 0 else om.integrate_threads(d, K, T, threads)
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        del om
        if time.perf_counter() - t0 > min(min_s, budget_s):
            break
    dt = time.perf_counter() - t0
    return {"updates_per_s": updates / dt, "frames": n, "passes": passes, "seconds": dt, "frames_per_s": n / dt}


def cpu_baseline(w, frames_host, budget_s: float) -> dict:
    """The oracle on the host: binary32 on all usable cores (the value) and
    on one thread, over the 300-frame sequence, each pass into a fresh map;
    and binary64 on all cores over the first frames of the 1 cm box room."""
    from paper_2311_00626_amd import synth
    threads = oracle_threads()
    share = budget_s / 3.0
    many = time_oracle(w.params, frames_host, w.camera.K, w.poses, threads, 0.6 * share, share)
    one = time_oracle(w.params, frames_host, w.camera.K, w.poses, 0, 0.6 * share, share)
    fine = synth.box_room_sequence(0.01, n_frames=300)
    fine_frames = fine.frames(count=30)
    f64 = time_oracle(fine.params, fine_frames, fine.camera.K, fine.poses[:30], threads, 0.5 * share, share,
                      precision=64)
    return {"value": many["updates_per_s"], "unit": "voxel updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{many['frames']} frames ({many['passes']} pass(es) over the 300-frame sequence, each into a "
                      f"fresh map), binary32 oracle on {threads} threads (bitwise the one-thread map), "
                      f"{many['seconds']:.1f} s, {many['frames_per_s']:.1f} frames/s",
            "host": host_cpu(),
            "one_thread": {"value": one["updates_per_s"], "unit": "voxel updates/s", "cores": 1,
                           "frames_per_s": one["frames_per_s"],
                           "sample": f"{one['frames']} frames, {one['seconds']:.1f} s"},
            "binary64_box_room_1cm": {"value": f64["updates_per_s"], "unit": "voxel updates/s", "cores": threads,
                                      "frames_per_s": f64["frames_per_s"], "workload": fine.name,
                                      "sample": f"{f64['frames']} frames (first 30 of 300, passes into fresh maps), "
                                                f"binary64 oracle, {f64['seconds']:.1f} s"}}


def calibration_kernels(mib: int, dev) -> list:
    """Kernels of known traffic for scaling the FETCH_SIZE / WRITE_SIZE
    counters, launched in this order after the buffers are filled: a plain
    copy of `mib` MiB (contiguous 16-byte accesses), and two gathers of one
    4-byte word per 128-byte and per 64-byte line (the access pattern of the
    integration kernel's depth and hash reads) over buffers far larger than
    the L2 caches, each line touched once.  Returns (kind, bytes read,
    bytes written) per kernel, in launch order."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device=dev)
    dst = torch.zeros_like(src)
    g128 = torch.ones(n // 4, dtype=torch.float32, device=dev)        # n bytes, n / 128 lines
    g64 = torch.ones(n // 8, dtype=torch.float32, device=dev)         # n / 2 bytes, n / 128 lines
    o128 = torch.zeros(n // 128, dtype=torch.float32, device=dev)
    o64 = torch.zeros(n // 128, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    dst.copy_(src)
    o128.copy_(g128.view(-1, 32)[:, 0])
    o64.copy_(g64.view(-1, 16)[:, 0])
    torch.cuda.synchronize()
    plan = [("copy", n, n), ("gather_4B_per_128B_line", n // 128 * 128, n // 32),
            ("gather_4B_per_64B_line", n // 128 * 64, n // 32)]
    log("calibration kernels (kind, algorithmic bytes read, written), in launch order: " + json.dumps(plan))
    return plan


def counters(m):
    st = m.full_stats()
    return st["blocks"], st["voxel_updates"], st["voxel_writes"], st["touched_blocks"]


def candidates(m) -> int:
    return m.full_stats()["candidate_blocks"]


def region_events():
    """Start/stop events for a timed region on the current stream, the stream
    every launch of the region goes to."""
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed_plain(w, frames, poses, storage: str, steps: int, warmup: int, block_capacity: int,
                setup=None, per_frame: bool = False, **map_kw) -> dict:
    """One integrate_depth launch per frame over `steps` frames (cycling the
    sequence) after `warmup` untimed ones.  One HIP event pair on the launch
    stream brackets the timed region; the mean launch duration is its time over
    the launches (it includes the gap between consecutive launches, so it bounds
    the kernel's own duration from above; per-launch events would add several
    microseconds of their own to every launch)."""
    import torch
    from paper_2311_00626_amd.tsdf import TsdfMap
    n_frames = frames.shape[0]
    fl = list(frames.unbind(0))   # one view per frame, made before timing
    H, W = frames.shape[1], frames.shape[2]
    K = w.camera.K
    log(f"leg: {w.name} {storage} {map_kw or ''} one frame per launch, {steps} timed after {warmup}")
    m = TsdfMap.from_params(w.params, storage=storage, block_capacity=block_capacity, **map_kw)
    m.set_launch_config(partitions=PARTITIONS, chunk=CHUNK, compaction=COMPACTION, staging=STAGING)
    if setup is not None:
        setup(m)
    for k in range(warmup):
        m.integrate_depth(fl[k % n_frames], K, poses[k % n_frames])
    torch.cuda.synchronize()
    b0, u0, _, t0_ = counters(m)
    c0 = candidates(m)
    ev = region_events()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record()
    for k in range(warmup, warmup + steps):
        m.integrate_depth(fl[k % n_frames], K, poses[k % n_frames])
    ev[1].record()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    kernel_ms, launches = ev[0].elapsed_time(ev[1]), steps
    b1, u1, _, t1_ = counters(m)
    assert m.status() == 0, "map overflowed"
    vb = 4 if storage == "fp16" else 8
    alg = algorithmic_bytes(u1 - u0, t1_ - t0_, b1 - b0, H * W, steps, vb) / steps
    kern = kernel_ms / 1e3 / max(launches, 1)
    out = {"elapsed": t_end - t_start, "updates": u1 - u0, "touched": t1_ - t0_, "new_blocks": b1 - b0,
           "alg_per_launch": alg, "kernel_s": kern, "launches": launches, "achieved": alg / kern / 1e9,
           "blocks": b1, "candidates": candidates(m) - c0,
           "block_granular_per_launch": block_granular_bytes(t1_ - t0_, vb) / steps,
           "frames_timed": f"{warmup}-{warmup + steps - 1}" if steps <= n_frames - warmup
                           else f"{warmup}.. ({steps} frames, the sequence cycled)"}
    del m
    if per_frame:
        out["per_frame"] = per_frame_times(w, frames, poses, storage, steps, warmup, block_capacity, setup, **map_kw)
    return out


def block_granular_bytes(touched: int, voxel_bytes: int) -> int:
    """Whole touched blocks read and written once (512 voxels each way)."""
    return 2 * 512 * voxel_bytes * touched


def per_frame_times(w, frames, poses, storage: str, steps: int, warmup: int, block_capacity: int,
                    setup=None, **map_kw) -> dict:
    """Median and 90th percentile of one integrate_depth call's GPU time over
    the timed frames, from a second pass over the same frames into a fresh
    map with the library's per-call events (they cost a few microseconds a
    call, so the timed region above uses one event pair instead)."""
    import torch
    from paper_2311_00626_amd.tsdf import TsdfMap
    n_frames = frames.shape[0]
    fl = list(frames.unbind(0))   # one view per frame, made before timing
    K = w.camera.K
    m = TsdfMap.from_params(w.params, storage=storage, block_capacity=block_capacity, **map_kw)
    m.set_launch_config(partitions=PARTITIONS, chunk=CHUNK, compaction=COMPACTION, staging=STAGING)
    if setup is not None:
        setup(m)
    for k in range(warmup):
        m.integrate_depth(fl[k % n_frames], K, poses[k % n_frames])
    torch.cuda.synchronize()
    m.profile(True)
    ms = []
    for k in range(warmup, warmup + steps):
        m.integrate_depth(fl[k % n_frames], K, poses[k % n_frames])
        t, n = m.profile_read()
        assert n == 1
        ms.append(t)
    m.profile(False)
    a = np.asarray(ms)
    return {"median_ms": float(np.median(a)), "p90_ms": float(np.percentile(a, 90)),
            "min_ms": float(a.min()), "max_ms": float(a.max()), "frames": len(ms),
            "note": "GPU time of one call (all of its kernels), library events per call"}


def precision_leg(voxel_size: float, steps: int, warmup: int) -> dict:
    """The 640x480 box-room sequence at a fine voxel size, binary32 and
    binary16 storage one frame per launch (the configuration whose per-frame
    voxel traffic is large enough for the HBM roofline to bind), and binary32
    16 frames per launch."""
    import torch
    from paper_2311_00626_amd import synth
    w = synth.box_room_sequence(voxel_size, n_frames=300)
    frames = torch.stack([torch.as_tensor(f) for f in w.frames(device="cuda")]).cuda().contiguous()
    poses = [np.ascontiguousarray(p, dtype=np.float32) for p in w.poses]
    out = {"workload": w.name, "voxel_size_m": voxel_size}
    for storage in ("fp32", "fp16"):
        r = timed_plain(w, frames, poses, storage, min(steps, 290), warmup, 1 << 17, per_frame=True)
        out[storage] = {"value": r["updates"] / r["elapsed"], "unit": "voxel updates/s",
                        "frames_per_s": min(steps, 290) / r["elapsed"],
                        "updates_per_frame": r["updates"] / min(steps, 290),
                        "touched_blocks_per_frame": r["touched"] / min(steps, 290),
                        "candidate_blocks_per_frame": r["candidates"] / min(steps, 290),
                        "roofline": {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": r["achieved"] / HBM_PEAK_GBS,
                                     "kernel": f"integrate_depth<{storage}> per frame (footprint and cull "
                                               "pre-passes included on lattices large enough to use them)",
                                     "kernel_ms_mean": r["kernel_s"] * 1e3,
                                     "algorithmic_bytes_per_launch": r["alg_per_launch"],
                                     "block_granular_bytes_per_launch": r["block_granular_per_launch"],
                                     "frames_timed": r["frames_timed"]},
                        "per_frame": r["per_frame"]}
    out["fp32_16_per_launch"] = timed_views(w, frames, poses, 16, 1 << 18)
    del frames
    torch.cuda.empty_cache()
    return out


def timed_views(w, frames, poses, B: int, block_capacity: int) -> dict:
    """The same sequence with B frames per integrate_depth_views launch
    (binary32): every voxel is read and written once per launch, and the
    footprint and cull pre-passes run once per launch.  One event pair around
    the timed launches, as in timed_plain."""
    import torch
    from paper_2311_00626_amd.tsdf import TsdfMap
    K = w.camera.K
    n = frames.shape[0]
    fl = list(frames.unbind(0))   # one view per frame, made before timing
    H, W = frames.shape[1], frames.shape[2]
    log(f"leg: {w.name} {B} frames per launch")
    m = TsdfMap.from_params(w.params, block_capacity=block_capacity)
    first = n % B or B
    m.integrate_depth_views(fl[:first], [K] * first, poses[:first])
    torch.cuda.synchronize()
    b0, u0, wr0, t0_ = counters(m)
    ev = region_events()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record()
    for a in range(first, n, B):
        m.integrate_depth_views(fl[a:a + B], [K] * B, poses[a:a + B])
    ev[1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t_start
    launches = (n - first) // B
    kms = ev[0].elapsed_time(ev[1])
    b1, u1, wr1, t1_ = counters(m)
    assert m.status() == 0, "map overflowed"
    alg = algorithmic_bytes(wr1 - wr0, t1_ - t0_, b1 - b0, H * W, n - first) / max(launches, 1)
    ks = kms / 1e3 / max(launches, 1)
    return {"views_per_launch": B, "frames": n - first, "value": (u1 - u0) / el, "unit": "voxel updates/s",
            "frames_per_s": (n - first) / el, "ms_per_launch": el / launches * 1e3,
            "roofline": {"bound": "hbm", "achieved": alg / ks / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / ks / 1e9 / HBM_PEAK_GBS, "kernel": "integrate_depth_views per launch",
                         "kernel_ms_mean": ks * 1e3, "algorithmic_bytes_per_launch": alg}}


def walk_leg(w, frames, poses, steps: int, warmup: int) -> dict:
    """The paper-literal ray-walk allocation on the same frames."""
    r = timed_plain(w, frames, poses, "fp32", steps, warmup, 1 << 16, allocation="ray_walk")
    return {"allocation": "ray walk along pixel-centre rays to min(d + eps, max range)",
            "value": r["updates"] / r["elapsed"], "unit": "voxel updates/s",
            "frames_per_s": steps / r["elapsed"], "ms_per_step": r["elapsed"] / steps * 1e3,
            "blocks_allocated": r["blocks"], "kernel_ms_mean": r["kernel_s"] * 1e3,
            "note": "kernel_ms_mean is GPU time per frame: the per-pixel walk and the integration kernel"}


def learned_leg(w, frames, poses, steps: int, warmup: int, full_gain: bool = True) -> dict:
    """Learned sensor-model weighting on the same frames (untrained model: the
    cost does not depend on the parameter values), and the training step time
    on one 640x480 room at 2 cm."""
    import torch
    from paper_2311_00626_amd import sensor_model as sm
    params = sm.init_params(0)
    r = timed_plain(w, frames, poses, "fp32", steps, warmup, 1 << 16, setup=lambda m: m.set_sensor_model(params),
                    weighting="learned")
    out = {"weighting": "learned sensor model (27-32-32-2 perceptron per pixel, bfloat16)",
           "value": r["updates"] / r["elapsed"], "unit": "voxel updates/s",
           "frames_per_s": steps / r["elapsed"], "ms_per_step": r["elapsed"] / steps * 1e3,
           "kernel_ms_mean": r["kernel_s"] * 1e3,
           "note": "kernel_ms_mean is GPU time per frame: the per-pixel inference pre-pass and the integration kernel"}
    vs = 0.02
    room = sm.prepare_room(1000, 24, synth_cam_640(), vs, window=8)
    n = 30
    sm.train([room], vs, steps=3, lr=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sm.train([room], vs, steps=n, lr=1e-3, log_every=n + 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    targets = sum(int(wd.target.numel()) for wd in room.windows) / len(room.windows)
    out["training"] = {"window_frames": 8, "target_voxels_per_window": targets, "steps": n,
                       "ms_per_step": dt / n * 1e3, "workload": "learning room 1000, 640x480, 2 cm"}
    if full_gain:
        log("leg: learned sensor model, full training configuration and held-out gain")
        g = sm.gain_run()
        out["gain_full_configuration"] = {
            "workload": "20 training rooms (seeds 1000-1019) x 100 corrupted 640x480 frames, 2 cm, windows of 8, "
                        "2400 Adam steps; held-out rooms 2000-2002 of 100 frames",
            "data_s": g["data_s"], "train_s": g["train_s"], "train_ms_per_step": g["train_s"] / g["steps"] * 1e3,
            "held_out_loss_before": g["held_out_loss_before"], "held_out_loss_after": g["held_out_loss_after"],
            "surface_error": g["surface_error"],
            "rms_gain_vs_linear_dropoff": {k: 1.0 - e["learned"]["rms_m"] / e["fallback"]["rms_m"]
                                           for k, e in g["surface_error"].items()}}
    return out


def synth_cam_640():
    from paper_2311_00626_amd import synth
    return synth.CAM_640


def rig_leg(n_steps: int, warmup: int):
    """Multi-sensor steps: 4 pinhole cameras (640x480, 848x480, 424x240,
    1280x720) and a 1024x64 spherical LiDAR (+-16 deg, 25 m, 2 cm range noise)
    on a rig moving through a 20 x 15 x 3 m room at 10 Hz, 5 cm voxels.  Each
    step is one replay of a captured hipGraph (argument upload + one batched
    integration launch); the launch shape is autotuned on the first steps
    before timing."""
    import torch
    from paper_2311_00626_amd import autotune, synth
    from paper_2311_00626_amd.tsdf import TsdfMap
    t0 = time.perf_counter()
    scene, steps = synth.rig_sequence(n_steps)
    L = synth.LidarModel(width=1024, height=64, max_range=25.0, interp_max_diff=0.2)
    params = synth.MapParams(0.05, 4.0, "linear_dropoff", max_range=5.0)
    rng = np.random.default_rng(11)
    data, pixels = [], 0
    for st in steps:
        views = [torch.as_tensor(synth.add_depth_noise(synth.render_depth(scene, c, T, device="cuda"), rng),
                                 device="cuda") for c, T in zip(st.cameras, st.poses)]
        views.append(torch.as_tensor(synth.add_range_noise(synth.render_range(scene, L, st.lidar_pose,
                                                                              device="cuda"), rng), device="cuda"))
        pixels += sum(v.numel() for v in views)
        data.append((views, [c.K for c in st.cameras] + [L], list(st.poses) + [st.lidar_pose]))
    log(f"rig: rendered {n_steps} steps in {time.perf_counter() - t0:.1f} s")

    def make_map():
        return TsdfMap.from_params(params, block_capacity=1 << 16)

    def make_runner(m):
        s = m.step(with_spherical=True)
        return (lambda k: s.run(*data[k])), s.close

    t0 = time.perf_counter()
    tune_steps = range(min(12, n_steps))
    choice, trials = autotune.tune("rig-4cam-lidar-5cm", make_map, None, tune_steps, make_runner=make_runner,
                                   rounds=2, refresh=True)
    log(f"rig: tuned {len(trials)} launch shapes in {time.perf_counter() - t0:.1f} s -> {choice}")
    m = make_map()
    choice.apply(m)
    step = m.step(with_spherical=True)
    for k in range(min(warmup, n_steps)):
        step.run(*data[k])
    torch.cuda.synchronize()
    st0 = m.full_stats()
    ev = region_events()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    timed = range(min(warmup, n_steps), n_steps)
    ev[0].record()
    for k in timed:
        step.run(*data[k])
    ev[1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t_start
    kms, kl = ev[0].elapsed_time(ev[1]), len(timed)
    st1 = m.full_stats()
    step.close()
    assert m.status() == 0, "map overflowed"
    n = len(timed)
    px = sum(sum(v.numel() for v in data[k][0]) for k in timed)
    alg = algorithmic_bytes(st1["voxel_writes"] - st0["voxel_writes"], st1["touched_blocks"] - st0["touched_blocks"],
                            st1["blocks"] - st0["blocks"], px, 1) / max(kl, 1)
    ks = kms / 1e3 / max(kl, 1)
    return {"steps": n, "views_per_step": 5, "pixels_per_step": pixels // n_steps,
            "value": (st1["voxel_updates"] - st0["voxel_updates"]) / el, "unit": "voxel updates/s",
            "steps_per_s": n / el, "ms_per_step": el / n * 1e3,
            "launch_config": asdict(choice),
            "tuning": [{"config": asdict(t.config), "kernel_ms": round(t.kernel_ms_per_launch, 4)} for t in trials[:5]]
            + [{"worst": asdict(trials[-1].config), "kernel_ms": round(trials[-1].kernel_ms_per_launch, 4)}],
            "blocks": st1["blocks"],
            "roofline": {"bound": "hbm", "achieved": alg / ks / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / ks / 1e9 / HBM_PEAK_GBS, "kernel": "integrate_views_kernel_dev (graph)",
                         "kernel_ms_mean": ks * 1e3, "algorithmic_bytes_per_launch": alg}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=290)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle time for the CPU baseline")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=16, help="views per launch of the batched leg (1 = skip it)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this size (PMC scaling)")
    ap.add_argument("--rig-steps", type=int, default=500,
                    help="steps of the multi-sensor rig leg (4 cameras + LiDAR, graph-replayed; 0 = skip it)")
    ap.add_argument("--legs", default="plain,fp16,batched,rig,precision,walk,learned",
                    help="comma-separated legs to run (plain is always run)")
    ap.add_argument("--skip-learned-gain", action="store_true",
                    help="learned leg: time inference and training only, without the full training run")
    ap.add_argument("--precision-voxels", default="0.01,0.02",
                    help="voxel sizes (m) of the box-room precision leg")
    ap.add_argument("--calibrate-only", action="store_true",
                    help="run only the PMC calibration kernels (--copy-calibration-mib, default 256) and exit")
    ap.add_argument("--partitions", type=int, default=0, choices=(0, 1, 8),
                    help="image bands (one per XCD) of the one-frame-per-launch legs; 0 = automatic")
    ap.add_argument("--chunk", type=int, default=0,
                    help="lattice blocks a wave culls per pass in lattice walks (0 = automatic)")
    ap.add_argument("--compaction", default="auto", choices=("auto", "never", "always"),
                    help="compacted launches of the one-frame-per-launch legs")
    ap.add_argument("--staging", default="auto", choices=("auto", "never", "always"),
                    help="LDS footprint staging of the one-frame-per-launch legs")
    args = ap.parse_args()
    global STAGING, PARTITIONS, CHUNK, COMPACTION
    STAGING = args.staging
    PARTITIONS = args.partitions
    CHUNK = args.chunk
    COMPACTION = args.compaction
    if args.calibrate_only:
        import torch
        calibration_kernels(args.copy_calibration_mib or 256, torch.device("cuda:0"))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path shards by space with no exchange; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_00626_amd import synth
    from paper_2311_00626_amd.tsdf import TsdfMap

    dev = torch.device("cuda:0")
    w = synth.cluttered_room_sequence(300)
    t0 = time.perf_counter()
    frames_host = w.frames(device="cuda")
    log(f"rendered {len(frames_host)} frames in {time.perf_counter() - t0:.1f} s")
    frames = torch.stack([torch.as_tensor(f) for f in frames_host]).to(dev).contiguous()
    n_frames = frames.shape[0]
    fl = list(frames.unbind(0))   # one view per frame, made before timing
    H, W = frames.shape[1], frames.shape[2]
    K = w.camera.K
    poses = [np.ascontiguousarray(p, dtype=np.float32) for p in w.poses]

    def plain_leg(storage: str):
        return timed_plain(w, frames, poses, storage, args.steps, args.warmup, 1 << 16,
                           per_frame=storage == "fp32")

    # ---- plain path, binary32 storage: the headline value ------------------
    p32 = plain_leg("fp32")
    elapsed, updates = p32["elapsed"], p32["updates"]
    touched, new_blocks = p32["touched"], p32["new_blocks"]
    alg_per_launch, mean_kernel_s, achieved = p32["alg_per_launch"], p32["kernel_s"], p32["achieved"]
    launches = p32["launches"]

    legs = set(args.legs.split(","))

    # ---- plain path, binary16 storage ---------------------------------------
    fp16 = None
    p16 = plain_leg("fp16") if "fp16" in legs else None
    if p16 is not None:
      fp16 = {"storage": "binary16 distance + binary16 weight, binary32 update arithmetic",
            "value": p16["updates"] / p16["elapsed"], "unit": "voxel updates/s",
            "frames_per_s": args.steps / p16["elapsed"], "ms_per_step": p16["elapsed"] / args.steps * 1e3,
            "roofline": {"bound": "hbm", "achieved": p16["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": p16["achieved"] / HBM_PEAK_GBS, "kernel": "integrate_depth_kernel<fp16>",
                         "kernel_ms_mean": p16["kernel_s"] * 1e3,
                         "algorithmic_bytes_per_launch": p16["alg_per_launch"]}}

    # ---- batched path: integrate_depth_views, several frames per launch ------
    batched = None
    if args.batch > 1 and "batched" in legs:
        B = args.batch
        mb = TsdfMap.from_params(w.params, block_capacity=1 << 16)
        first = n_frames % B or B           # warm-up batch, so that the rest splits evenly
        mb.integrate_depth_views(fl[:first], [K] * first, poses[:first])
        torch.cuda.synchronize()
        bb0, ub0, wb0, tb0 = counters(mb)
        ev = region_events()
        torch.cuda.synchronize()
        tb_start = time.perf_counter()
        ev[0].record()
        for a in range(first, n_frames, B):
            mb.integrate_depth_views(fl[a:a + B], [K] * B, poses[a:a + B])
        ev[1].record()
        torch.cuda.synchronize()
        tb_end = time.perf_counter()
        kms, kl = ev[0].elapsed_time(ev[1]), len(range(first, n_frames, B))
        bb1, ub1, wb1, tb1 = counters(mb)
        assert mb.status() == 0, "map overflowed"
        nfb = n_frames - first
        eb = tb_end - tb_start
        alg_b = algorithmic_bytes(wb1 - wb0, tb1 - tb0, bb1 - bb0, H * W, nfb) / max(kl, 1)
        kb = kms / 1e3 / max(kl, 1)
        batched = {"views_per_launch": B, "frames": nfb, "launches": kl,
                   "value": (ub1 - ub0) / eb, "unit": "voxel updates/s",
                   "frames_per_s": nfb / eb, "ms_per_launch": eb / kl * 1e3,
                   "voxel_updates": ub1 - ub0, "voxel_writes": wb1 - wb0,
                   "roofline": {"bound": "hbm", "achieved": alg_b / kb / 1e9, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": alg_b / kb / 1e9 / HBM_PEAK_GBS,
                                "kernel": "integrate_views_kernel", "kernel_ms_mean": kb * 1e3,
                                "algorithmic_bytes_per_launch": alg_b}}
        del mb

    rig = rig_leg(args.rig_steps, args.warmup) if args.rig_steps > 0 and "rig" in legs else None
    precision = ([precision_leg(float(vs), args.steps, args.warmup) for vs in args.precision_voxels.split(",")]
                 if "precision" in legs else None)
    walk = walk_leg(w, frames, poses, args.steps, args.warmup) if "walk" in legs else None
    if walk is not None:
        walk["blocks_allocated_exact_touch"] = p32["blocks"]
    learned = (learned_leg(w, frames, poses, args.steps, args.warmup, full_gain=not args.skip_learned_gain)
               if "learned" in legs else None)

    if args.copy_calibration_mib > 0:
        calibration_kernels(args.copy_calibration_mib, dev)

    result = {
        "metric": "voxel updates/s (frames/s and achieved HBM GB/s alongside)",
        "value": updates / elapsed,
        "unit": "voxel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "frames_per_s": args.steps / elapsed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded ray-cast room, rendered on device before timing)",
        "config": {"workload": w.name, "frames": n_frames, "width": W, "height": H,
                   "voxel_size_m": w.params.voxel_size, "truncation_vox": w.params.truncation_vox,
                   "weighting": w.params.weighting, "max_range_m": w.params.max_range,
                   "parallelism": "single GPU"},
        "voxel_updates": updates,
        "touched_blocks": touched,
        "candidate_blocks": p32["candidates"],
        "new_blocks": new_blocks,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(),
                     "kernel": "integrate_depth_kernel", "kernel_ms_mean": mean_kernel_s * 1e3,
                     "algorithmic_bytes_per_launch": alg_per_launch, "launches_timed": launches,
                     "frames_timed": p32["frames_timed"],
                     "block_granular_bytes_per_launch": p32["block_granular_per_launch"]},
        "per_frame": p32["per_frame"],
    }
    traffic = measured_traffic_record()
    if traffic is not None:
        result["roofline"]["traffic_profile"] = traffic
    if fp16 is not None:
        result["fp16"] = fp16
    if rig is not None:
        result["rig"] = rig
    if precision is not None:
        result["precision"] = precision
    if walk is not None:
        result["ray_walk"] = walk
    if learned is not None:
        result["learned"] = learned
    if batched is not None:
        result["batched"] = batched
    if not args.skip_cpu_baseline:
        cb = cpu_baseline(w, frames_host, args.cpu_budget)
        # the GPU's voxel updates/s over the oracle's (a baseline, not a measure of kernel quality)
        cb["gpu_speedup"] = {"vs_all_cores": result["value"] / cb["value"],
                             "vs_one_thread": result["value"] / cb["one_thread"]["value"]}
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
