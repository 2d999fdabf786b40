"""Host logic of the launch-shape autotuner: the candidate grid, the choice of
the fastest trial and the per-device cache (no GPU calls)."""
import json

from paper_2311_00626_amd import autotune as at


class FakeMap:
    """Stands in for a TsdfMap: 'kernel time' is a function of the launch shape."""
    log = []

    def __init__(self):
        self.cfg = None
        self.n = 0

    def set_launch_config(self, g, p, c, f="auto", k="auto"):
        self.cfg = (g, p, c, f, k)

    def profile(self, on):
        self.n = 0

    def profile_read(self):
        g, p, c, f, k = self.cfg
        ms = 1.0 + abs(g - 1024) / 1024 + (p == 8) * 0.5 + abs(c - 4) * 0.01 + (f == "never") * 0.2
        ms += (k == "always") * 0.03
        return ms * self.n, self.n

    def status(self):
        return 0

    def close(self):
        FakeMap.log.append(self.cfg)


def test_candidates_cover_the_grid():
    c = at.default_candidates()
    walk = len(at.GROUPS) * len(at.CHUNKS) * len(at.PARTITIONS) * len(at.FOOTPRINTS)
    assert len(c) == walk + len(at.GROUPS) * len(at.FOOTPRINTS)
    assert len(set(c)) == len(c)
    assert all(x.partitions in (1, 8) and 0 <= x.chunk <= 64 for x in c)
    assert all(x.compaction == "never" for x in c[:walk])
    assert all(x.compaction == "always" and x.partitions == 1 for x in c[walk:])


def test_tune_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setattr(at.torch.cuda, "synchronize", lambda: None)
    at._MEMO.clear()
    cache = str(tmp_path / "launch.json")

    def run_step(m, k):
        m.n += 1

    choice, trials = at.tune("w1", FakeMap, run_step, range(6), cache_path=cache, device="devA")
    assert choice == at.LaunchConfig(1024, 1, 4, "always", "never")
    assert [t.kernel_ms_per_launch for t in trials] == sorted(t.kernel_ms_per_launch for t in trials)
    assert trials[0].launches == 4
    assert json.load(open(cache)) == {"devA|w1": {"max_groups": 1024, "partitions": 1, "chunk": 4,
                                                  "footprint": "always", "compaction": "never"}}
    # memoised, then from the file in a fresh process (memo cleared): no trials run
    FakeMap.log.clear()
    assert at.tune("w1", FakeMap, run_step, range(6), cache_path=cache, device="devA") == (choice, [])
    at._MEMO.clear()
    assert at.tune("w1", FakeMap, run_step, range(6), cache_path=cache, device="devA") == (choice, [])
    assert FakeMap.log == []
    # another device or workload is tuned afresh; refresh ignores the cache
    c2, t2 = at.tune("w1", FakeMap, run_step, range(6), cache_path=cache, device="devB",
                     candidates=[at.LaunchConfig(512, 1, 1), at.LaunchConfig(2048, 8, 8)])
    assert c2 == at.LaunchConfig(512, 1, 1) and len(t2) == 2
    assert set(json.load(open(cache))) == {"devA|w1", "devB|w1"}
    _, t3 = at.tune("w1", FakeMap, run_step, range(6), cache_path=cache, device="devA", refresh=True,
                    candidates=[at.LaunchConfig(256, 1, 0)])
    assert len(t3) == 1


def test_corrupt_cache_is_ignored(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert at._read_cache(str(p)) == {}
    assert at._read_cache(None) == {}


def test_cache_entry_without_compaction_loads(tmp_path):
    """An entry written before the compaction knob existed keeps the library's
    automatic choice for it."""
    at._MEMO.clear()
    p = tmp_path / "old.json"
    p.write_text(json.dumps({"devC|w2": {"max_groups": 512, "partitions": 1, "chunk": 8, "footprint": "never"}}))
    choice, trials = at.tune("w2", FakeMap, lambda m, k: None, range(4), cache_path=str(p), device="devC")
    assert trials == [] and choice == at.LaunchConfig(512, 1, 8, "never", "auto")
