"""Launch-shape autotuner for the batched drill-down call.

Drill-down (Sec. 1) asks for many small views of one formatted log; the
batched call computes the DFGs of all of them in one pass, and its speed
depends on the launch shape: the events staged per block (tile_events), and
either the whole call as one persistent launch on a grid of resident blocks
(launch 0) or one launch per phase (launch 1) with the grid of the walks that
emit the per-view records (emit_blocks) and the grid of the per-view
aggregation (agg_blocks).  The best shape moves with the activity count, the
number of views and the log size, so it is measured, not guessed:

  sweep()   times every candidate shape with a caller-given runner, keeps the
            fastest (median of the repetitions), returns the whole table;
  Cache     a JSON file of the winners, keyed by (activity bucket, view-count
            bucket, event-count bucket); lookup() takes the exact key, else the
            nearest one with the same activity bucket;
  tune_batched()  runs the sweep on the GPU for one (log, views) workload and
            stores the winner.

pm4g.pm4g_dfg_batched consults the default cache when it is given no tuning.
The cache holds launch shapes only: capacities are sized per call.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import threading
import time
from typing import Callable, Iterable

TILES = (2048, 4096)
EMIT_BLOCKS = (256, 512, 1024, 2048)
AGG_BLOCKS = (256, 512, 1024)
# (tile_events, emit_blocks, agg_blocks, launch): the persistent launch sizes its own grid
CANDIDATES = tuple((t, 0, 0, 0) for t in TILES) + \
    tuple((t, e, a, 1) for t in TILES for e in EMIT_BLOCKS for a in AGG_BLOCKS)

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _pow2_bucket(x: int, lo: int = 1) -> int:
    x = max(int(x), lo)
    return 1 << int(round(math.log2(x)))


def key_of(n_activities: int, n_views: int, n_events: int) -> str:
    """Cache key: activity count rounded up to a power of two (the LDS table
    size follows it), view and event counts to the nearest power of two."""
    a = 1 << max(4, math.ceil(math.log2(max(int(n_activities), 1))))
    return f"A{a}-V{_pow2_bucket(n_views)}-N{_pow2_bucket(n_events)}"


def _parse(key: str) -> tuple[int, int, int]:
    a, v, n = key.split("-")
    return int(a[1:]), int(v[1:]), int(n[1:])


class Cache:
    """JSON file of {key: {"tile_events", "emit_blocks", "agg_blocks", "launch", "ms", ...}}."""

    def __init__(self, path: str | None = None):
        self.path = path or os.environ.get("PM4G_TUNE_CACHE", DEFAULT_PATH)
        self._lock = threading.Lock()
        self._data: dict | None = None

    def _load(self) -> dict:
        if self._data is None:
            try:
                with open(self.path) as fh:
                    d = json.load(fh)
                self._data = d if isinstance(d, dict) else {}
            except (OSError, ValueError):
                self._data = {}
        return self._data

    def entries(self) -> dict:
        with self._lock:
            return dict(self._load())

    def lookup(self, n_activities: int, n_views: int, n_events: int) -> dict | None:
        """Exact key, else the nearest entry (log distance in views and events)
        with the same activity bucket; None if there is none."""
        key = key_of(n_activities, n_views, n_events)
        with self._lock:
            d = self._load()
            if key in d:
                return dict(d[key])
            a, v, n = _parse(key)
            best, best_d = None, None
            for k, e in d.items():
                try:
                    ka, kv, kn = _parse(k)
                except ValueError:
                    continue
                if ka != a:
                    continue
                dist = abs(math.log2(kv) - math.log2(v)) + abs(math.log2(kn) - math.log2(n))
                if best_d is None or dist < best_d:
                    best, best_d = e, dist
            return dict(best) if best is not None else None

    def store(self, n_activities: int, n_views: int, n_events: int, entry: dict) -> str:
        key = key_of(n_activities, n_views, n_events)
        with self._lock:
            d = self._load()
            d[key] = dict(entry)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(d, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        return key


def sweep(run: Callable[[tuple], float], candidates: Iterable[tuple] = CANDIDATES,
          reps: int = 3) -> tuple[tuple, list[dict]]:
    """Times each candidate `reps` times with run(candidate) -> seconds (after
    one untimed call); returns the candidate with the smallest median and the
    table of medians.  Ties go to the earlier candidate."""
    table = []
    best, best_t = None, None
    for c in candidates:
        run(c)   # warm-up: capacities, code objects
        ts = [float(run(c)) for _ in range(max(1, reps))]
        med = statistics.median(ts)
        table.append({"tile_events": c[0], "emit_blocks": c[1], "agg_blocks": c[2],
                      "launch": c[3] if len(c) > 3 else 1, "ms": med * 1e3})
        if best_t is None or med < best_t:
            best, best_t = c, med
    if best is None:
        raise ValueError("no candidates to sweep")
    return best, table


def tune_batched(prep, views, masks, n_views: int, reps: int = 3, candidates=CANDIDATES,
                 cache: Cache | None = None, log: Callable[[str], None] | None = None) -> dict:
    """Sweeps the launch shape of pm4g_dfg_batched on this workload (device
    tensors as the call takes them), stores the winner in `cache` (the
    default cache if None) and returns it with the table."""
    import torch

    from . import pm4g

    out = pm4g.pm4g_dfg_batched(prep, views, masks, n_views, tuning=pm4g.BatchedTuning())
    req = [int(x) for x in out["required"].cpu().tolist()]
    caps = dict(pair_capacity=int(req[3] * 1.1) + 1024, record_capacity=int(req[1] * 1.1) + 1024,
                cell_capacity=int(req[4] * 1.1) + 1024)
    tunings: dict = {}

    def run(c):
        t = tunings.get(c)
        if t is None:
            t = pm4g.BatchedTuning(tile_events=c[0], emit_blocks=c[1], agg_blocks=c[2],
                                   launch=c[3] if len(c) > 3 else 1, **caps)
            # the pair count depends on the tile: let one call size it
            o = pm4g.pm4g_dfg_batched(prep, views, masks, n_views, tuning=t, out=out)
            r = [int(x) for x in o["required"].cpu().tolist()]
            t.pair_capacity = max(t.pair_capacity, int(r[3] * 1.1) + 1024)
            tunings[c] = t
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pm4g.pm4g_dfg_batched(prep, views, masks, n_views, tuning=t, out=out)
        return time.perf_counter() - t0

    best, table = sweep(run, candidates, reps)
    entry = {"tile_events": best[0], "emit_blocks": best[1], "agg_blocks": best[2],
             "launch": best[3] if len(best) > 3 else 1,
             "ms": min(r["ms"] for r in table), "n_activities": int(prep.n_activities),
             "n_views": int(n_views), "n_events": int(prep.n_events)}
    (cache or Cache()).store(prep.n_activities, n_views, prep.n_events, entry)
    if log:
        log(f"autotune: best tile {best[0]} emit {best[1]} agg {best[2]} launch {entry['launch']} "
            f"at {entry['ms']:.2f} ms")
    return {"best": entry, "table": table, "tuning": tunings[best]}


_default: Cache | None = None


def default_cache() -> Cache:
    global _default
    if _default is None:
        _default = Cache()
    return _default
