"""Launch-shape autotuner for the integration kernels.

The kernels walk the block lattice of a frame (or of a batch of views) with a
persistent grid.  Five knobs shape that walk (tsdf_set_launch_config in the C
ABI): the number of workgroups per launch, the number of consecutive lattice
blocks a wave culls at once, one per lane (the chunk), whether workgroups are
banded over image columns (partitions), whether blocks are also culled
against a per-view pyramid of tile depth maxima (footprint), and whether a
cull pass first compacts the surviving blocks into a list that the waves then
share evenly (compaction; chunk and partitions do not apply to it).  None of
them changes a result: every configuration leaves a bit-identical map.  Which one
is fastest depends on the sensor sizes, the voxel size and the batch, so the
tuner measures the candidates on a few steps of the caller's own workload,
timing the integration launches with the library's HIP events, and keeps the
fastest.  Choices are cached per device and workload key, in memory and
optionally in a JSON file.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import torch

GROUPS = (256, 512, 1024, 2048)
CHUNKS = (0, 1, 4, 8)
PARTITIONS = (1, 8)
FOOTPRINTS = ("never", "always")


@dataclass(frozen=True)
class LaunchConfig:
    max_groups: int = 0      # 0 = library default
    partitions: int = 0      # 0 = library default (1)
    chunk: int = 0           # 0 = automatic from the lattice size
    footprint: str = "auto"  # footprint culling: auto, never, always
    compaction: str = "auto"  # compacted launch: auto, never, always

    def apply(self, m) -> None:
        m.set_launch_config(self.max_groups, self.partitions, self.chunk, self.footprint, self.compaction)


def default_candidates() -> List[LaunchConfig]:
    """The lattice-walk grid, then the compacted launches (grid size and
    footprint culling only)."""
    walk = [LaunchConfig(g, p, c, f, "never") for g in GROUPS for p in PARTITIONS for c in CHUNKS
            for f in FOOTPRINTS]
    return walk + [LaunchConfig(g, 1, 0, f, "always") for g in GROUPS for f in FOOTPRINTS]


@dataclass
class Trial:
    config: LaunchConfig
    kernel_ms_per_launch: float
    launches: int


_MEMO: Dict[str, LaunchConfig] = {}


def device_key() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def measure(make_map: Callable[[], object], run_step: Callable[[object, int], None], steps: Sequence[int],
            config: LaunchConfig, warmup: int = 2, make_runner: Optional[Callable] = None) -> Trial:
    """Kernel time per launch of `config` over `steps` on a fresh map.

    make_runner(m) -> (run, close), if given, is called after the launch shape is
    set (a graph step captures its grid size when it is created)."""
    m = make_map()
    config.apply(m)
    run, close = (make_runner(m) if make_runner else ((lambda k: run_step(m, k)), (lambda: None)))
    steps = list(steps)
    for k in steps[:warmup]:
        run(k)
    torch.cuda.synchronize()
    m.profile(True)
    for k in steps[warmup:]:
        run(k)
    torch.cuda.synchronize()
    ms, n = m.profile_read()
    m.profile(False)
    close()
    status = m.status()
    m.close()
    if status != 0:
        raise RuntimeError(f"map status {status} while tuning {config}")
    return Trial(config, ms / max(n, 1), n)


def tune(key: str, make_map: Callable[[], object], run_step: Callable[[object, int], None],
         steps: Sequence[int], candidates: Optional[Iterable[LaunchConfig]] = None,
         cache_path: Optional[str] = None, warmup: int = 2, rounds: int = 2,
         make_runner: Optional[Callable] = None, refresh: bool = False,
         device: Optional[str] = None) -> Tuple[LaunchConfig, List[Trial]]:
    """Fastest launch configuration for the workload `key` on this device.

    Every candidate runs `steps` (after `warmup` of them) on a fresh map,
    `rounds` times, interleaved; its time is the best round.  Returns the
    choice and the trials (empty if the choice came from a cache)."""
    full_key = f"{device if device is not None else device_key()}|{key}"
    if not refresh:
        if full_key in _MEMO:
            return _MEMO[full_key], []
        cached = _read_cache(cache_path).get(full_key)
        if cached is not None:
            cfg = LaunchConfig(**cached)
            _MEMO[full_key] = cfg
            return cfg, []
    cands = list(candidates) if candidates is not None else default_candidates()
    best: Dict[LaunchConfig, Trial] = {}
    for _ in range(max(rounds, 1)):
        for c in cands:
            t = measure(make_map, run_step, steps, c, warmup, make_runner)
            if c not in best or t.kernel_ms_per_launch < best[c].kernel_ms_per_launch:
                best[c] = t
    trials = sorted(best.values(), key=lambda t: t.kernel_ms_per_launch)
    choice = trials[0].config
    _MEMO[full_key] = choice
    if cache_path:
        data = _read_cache(cache_path)
        data[full_key] = asdict(choice)
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return choice, trials


def _read_cache(path: Optional[str]) -> dict:
    if not path:
        return {}
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}
