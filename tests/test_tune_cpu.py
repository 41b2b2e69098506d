"""Autotuner logic on the CPU: cache keys, nearest lookup, JSON round trip,
and the sweep's choice with a fake timer (no GPU)."""
import json

import pytest

from paper_2204_04898_amd import tune


def test_key_buckets():
    assert tune.key_of(512, 4096, 98_969_504) == "A512-V4096-N134217728"
    assert tune.key_of(64, 4000, 10_000_000) == "A64-V4096-N8388608"
    assert tune.key_of(3, 1, 1) == "A16-V1-N1"        # activity bucket at least 16
    assert tune.key_of(513, 1, 1).startswith("A1024-")


def test_cache_roundtrip_and_nearest(tmp_path):
    path = str(tmp_path / "c.json")
    c = tune.Cache(path)
    assert c.lookup(512, 4096, 1e8) is None
    c.store(512, 4096, 98_969_504, {"tile_events": 2048, "emit_blocks": 512, "agg_blocks": 256, "ms": 1.0})
    c.store(512, 16, 1000, {"tile_events": 4096, "emit_blocks": 256, "agg_blocks": 256, "ms": 0.1})
    c.store(64, 4096, 98_969_504, {"tile_events": 4096, "emit_blocks": 1024, "agg_blocks": 1024, "ms": 2.0})
    with open(path) as fh:
        assert len(json.load(fh)) == 3
    c2 = tune.Cache(path)
    assert c2.lookup(512, 4096, 98_969_504)["tile_events"] == 2048   # exact
    assert c2.lookup(500, 3000, 90_000_000)["tile_events"] == 2048   # same buckets
    assert c2.lookup(512, 2048, 50_000_000)["tile_events"] == 2048   # nearest
    assert c2.lookup(512, 8, 2000)["tile_events"] == 4096            # nearest, small
    assert c2.lookup(64, 1, 1)["emit_blocks"] == 1024                # only A64 entry
    assert c2.lookup(4096, 4096, 98_969_504) is None                 # no entry with A4096


def test_cache_tolerates_bad_file(tmp_path):
    path = tmp_path / "bad.json"
    path.write_text("not json")
    assert tune.Cache(str(path)).lookup(16, 1, 1) is None


def test_sweep_picks_fastest_median():
    cost = {c: 1.0 + 0.01 * i for i, c in enumerate(tune.CANDIDATES)}
    fast = tune.CANDIDATES[7]
    cost[fast] = 0.5
    calls = []

    def run(c):
        calls.append(c)
        return cost[c]

    best, table = tune.sweep(run, reps=3)
    assert best == fast
    assert len(table) == len(tune.CANDIDATES)
    assert len(calls) == 4 * len(tune.CANDIDATES)       # one warm-up + 3 timed each
    assert min(table, key=lambda r: r["ms"])["ms"] == pytest.approx(500.0)


def test_sweep_median_ignores_one_outlier():
    seq = {(2048, 256, 256, 1): iter([9, 1.0, 50.0, 1.0]), (4096, 256, 256, 1): iter([9, 2.0, 2.0, 2.0])}
    best, _ = tune.sweep(lambda c: next(seq[c]), candidates=list(seq), reps=3)
    assert best == (2048, 256, 256, 1)


def test_sweep_rejects_empty():
    with pytest.raises(ValueError):
        tune.sweep(lambda c: 1.0, candidates=[])


def test_candidates_cover_both_launch_modes():
    """The sweep weighs the persistent launch (its grid sized by the library)
    against one launch per phase for every tile size."""
    modes = {(c[0], c[3]) for c in tune.CANDIDATES}
    assert modes == {(t, m) for t in tune.TILES for m in (0, 1)}
    assert all(c[1] == 0 and c[2] == 0 for c in tune.CANDIDATES if c[3] == 0)
