#!/usr/bin/env python3
"""Benchmark of the DFG hot path on one MI355X.

One step is the whole path over one synthetic log already resident in HBM:
format (range scan, case-key radix passes, per-case LDS ordering, case
table), the frequency/performance DFG with start/end/activity counts and the
FP64 mean, and the trace variants.  The default workload is the 100M-event
log (5M cases, lognormal lengths, 512 Zipf activities, ns timestamps,
shuffled rows).

Prints one JSON line: events/s for the whole step, the roofline of the
dominant kernel (the one with the most time per step: algorithmic bytes per
launch over its HIP-event-timed average duration on the launching stream;
the next kernel beside it), and the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published

WORKLOADS = {
    # name: (config index, description)
    "dfg-variants-100M": (3, "5M cases, ~99M events, lognormal lengths (median 12, max 2000), "
                             "512 activities (Zipf 1.1 Markov chain), int64 ns timestamps, shuffled rows"),
    "dfg-perf-10M": (2, "1M cases, ~10M events, geometric lengths (mean 10), 64 activities "
                        "(Zipf 1.1 Markov chain), int64 ms timestamps with 5% duplicates, shuffled rows"),
    "dfg-100k-presorted": (1, "10k cases, ~100k events, 16 activities, ms timestamps, rows presorted"),
}


def log_progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def packed_keys(log) -> bool:
    """Whether the library carries the activity inside the radix key: case-id
    bits plus activity bits fit in 32 (the rule of the formatting step)."""
    span = int(log.case.max()) - int(log.case.min()) if log.case.size else 0
    case_bits = span.bit_length()
    act_bits = max(log.n_activities - 1, 0).bit_length()
    return 0 < case_bits < 32 and case_bits + act_bits <= 32


def radix_passes(log) -> int:
    span = int(log.case.max()) - int(log.case.min()) if log.case.size else 0
    return max(1, (span.bit_length() + 7) // 8)


def kernel_bytes(stage: str, n: int, c: int, A: int, presorted: bool, packed: bool = False,
                 passes: int = 1) -> float | None:
    """Algorithmic HBM bytes one launch of a stage must move (reads + writes),
    averaged over the launches of one step where they differ."""
    e = n - c   # directly-follows pairs
    # radix scatter: the first pass reads the raw columns (case, act, ts = 16 B),
    # later passes the previous pass's elements; each writes one element.
    elem = 12.0 if packed else 16.0
    scatter_total = (16.0 + elem) * n + (passes - 1) * 2 * elem * n
    model = {
        "range_scan": 8.0 * n + (8.0 * n if presorted else 0.0),      # case + act (+ ts)
        "radix_hist": 4.0 * n,                                        # case key
        "radix_scan": None,
        "radix_scatter": scatter_total / passes,
        "segsort": (elem + 16.0) * n,                                 # sorted elements in, (case, act, ts) out
        "case_table": 8.0 * n + 12.0 * c,                             # case column twice, offsets + codes
        "dfg_count": 8.0 * n,                                         # case + act (A > 64)
        "dfg_main": 16.0 * n + (10.0 * e if A > 64 else 0.0),         # prepared log (+ bucketed edges)
        "dfg_agg": 10.0 * e,                                          # bucketed edges
        "variant_hash": 4.0 * n + 8.0 * c + 12.0 * c,                 # activities, offsets, hash + index
    }
    return model.get(stage)


def source_sha(files: list[str]) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


STAGE_SOURCES = {
    "radix_scatter": ["paper_2204_04898_amd/csrc/radix.hip", "paper_2204_04898_amd/csrc/common.hpp"],
    "radix_hist": ["paper_2204_04898_amd/csrc/radix.hip", "paper_2204_04898_amd/csrc/common.hpp"],
    "segsort": ["paper_2204_04898_amd/csrc/segsort.hip", "paper_2204_04898_amd/csrc/common.hpp"],
    "dfg_count": ["paper_2204_04898_amd/csrc/dfg.hip", "paper_2204_04898_amd/csrc/common.hpp"],
    "dfg_main": ["paper_2204_04898_amd/csrc/dfg.hip", "paper_2204_04898_amd/csrc/common.hpp"],
    "dfg_agg": ["paper_2204_04898_amd/csrc/dfg.hip", "paper_2204_04898_amd/csrc/common.hpp"],
}


# every source whose kernels run in one step of the DFG + variants path
STEP_SOURCES = ["paper_2204_04898_amd/csrc/" + f for f in (
    "range.hip", "radix.hip", "segsort.hip", "cases.hip", "dfg.hip", "variants.hip", "common.hpp", "devsort.hpp")]


def measured_step_traffic(workload: str) -> float | None:
    """HBM bytes of one whole step (all kernels) from the committed counter
    summary profiles/traffic_step_<workload>.txt, if its sources are current."""
    path = os.path.join(ROOT, "profiles", f"traffic_step_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_sha(STEP_SOURCES):
        return None
    try:
        return float(kv["bytes_per_step"])
    except (KeyError, ValueError):
        return None


def valu_issue_frac(stage: str, workload: str, per_launch_ms: float) -> float | None:
    """VALU instructions per launch (committed rocprofv3 SQ_INSTS_VALU summary)
    over the launch time, against one wave64 VALU instruction per CU per cycle;
    None when the stage is not in the summary or its sources changed since."""
    import re

    path = os.path.join(ROOT, "profiles", "valu_counters_step_views_100M.txt")
    if workload != "dfg-variants-100M" or stage not in ("segsort", "radix_scatter") or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(rf"{stage} = ([0-9a-f]+)", text)
    if not m or m.group(1) != source_sha(STAGE_SOURCES[stage]):
        return None
    insts = []
    for line in text.splitlines():
        cols = [c.strip() for c in line.split("|")]
        if len(cols) == 10 and cols[0].startswith("k_" + stage):
            insts.append((cols[0], float(cols[2])))
    if not insts:
        return None
    if stage == "radix_scatter":   # launches of one step: the first pass once, the others twice
        per_launch = sum(v * (1 if "true, true" in k else 2) for k, v in insts) / 3.0
    else:
        per_launch = insts[0][1]
    return per_launch / (per_launch_ms * 1e-3) / (256 * 2.4e9)


def measured_traffic(stage: str, workload: str) -> float | None:
    """HBM bytes per launch from the committed counter summary, if it is current.

    profiles/traffic_<stage>_<workload>.txt holds key=value lines written from
    two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch) and
    the copy-kernel calibration factor; it is ignored when the kernel's
    sources changed since (source_sha mismatch).
    """
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}.txt")
    if not os.path.exists(path) or stage not in STAGE_SOURCES:
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_sha(STAGE_SOURCES[stage]):
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _sample_cases(log, target_events: int):
    """Every event of the cases whose code is below a cut-off (codes are a
    random permutation, so it is a random subset of whole cases)."""
    import numpy as np

    C = int(log.lengths_by_code.shape[0])
    cum = np.cumsum(log.lengths_by_code)
    cut = min(int(np.searchsorted(cum, target_events, side="left")) + 1, C)
    keep = log.case < cut
    return cut, log.case[keep], log.act[keep], log.ts[keep]


def host_threads() -> int:
    """Host threads for the all-cores oracle row: the CPUs this process may run
    on, at most 16 (a GPU's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_all_cores(case, act, ts, A: int, threads: int) -> dict:
    """The oracle's DFG and variants of a log, computed on `threads` host
    threads: the cases are split into `threads` groups by case id (the
    directly-follows relation never crosses cases), each group runs the
    oracle's own functions (its C code releases the interpreter lock), and the
    groups' results are merged: cell counts and gap sums add (sums modulo
    2^64), minima and maxima combine, activity counts add; variants merge by
    exact sequence, counts add, the representative is the smallest, then the
    (count desc, representative asc) order."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    lo, hi = int(case.min()), int(case.max()) + 1
    edges = np.linspace(lo, hi, threads + 1).astype(np.int64)
    part = np.clip(np.searchsorted(edges, case, side="right") - 1, 0, threads - 1)
    order = np.argsort(part, kind="stable")
    bounds = np.searchsorted(part[order], np.arange(threads + 1))
    groups = [order[bounds[g]:bounds[g + 1]] for g in range(threads)]

    def run(idx):
        c, a, t = case[idx], act[idx], ts[idx]
        return oracle.dfg(c, a, t, A), oracle.variants(c, a, t, A)

    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(run, groups))
    d = {k: parts[0][0][k].copy() for k in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count",
                                             "act_count")}
    for pd, _ in parts[1:]:
        for k in ("count", "dt_sum", "start_count", "end_count", "act_count"):
            d[k] += pd[k]
        np.minimum(d["dt_min"], pd["dt_min"], out=d["dt_min"])
        np.maximum(d["dt_max"], pd["dt_max"], out=d["dt_max"])
    with np.errstate(invalid="ignore", divide="ignore"):
        d["dt_mean"] = np.where(d["count"] > 0, d["dt_sum"].astype(np.float64) / d["count"].astype(np.float64),
                                np.nan)
    d["n_cases"] = sum(pd["n_cases"] for pd, _ in parts)
    classes: dict = {}
    for _, pv in parts:
        off, acts = pv["var_off"], pv["var_acts"]
        for v in range(pv["n_variants"]):
            key = acts[off[v]:off[v + 1]].tobytes()
            n, rep = int(pv["var_count"][v]), int(pv["var_rep"][v])
            if key in classes:
                m, r = classes[key]
                classes[key] = (m + n, min(r, rep))
            else:
                classes[key] = (n, rep)
    ranked = sorted(classes.items(), key=lambda kv: (-kv[1][0], kv[1][1]))
    var = dict(n_variants=len(ranked), var_count=np.array([c for _, (c, _) in ranked], np.int64),
               var_rep=np.array([r for _, (_, r) in ranked], np.int64))
    return dict(dfg=d, variants=var)


def cpu_baseline(log, target_events: int) -> dict:
    """The oracle as it stands on a bounded sample of the same log: one host
    thread (the reported value), and all host threads (split by case, merged)."""
    import platform

    import oracle

    cut, case, act, ts = _sample_cases(log, target_events)
    A = log.n_activities
    t0 = time.perf_counter()
    oracle.dfg(case, act, ts, A)
    oracle.variants(case, act, ts, A)
    dt = time.perf_counter() - t0
    threads = host_threads()
    t1 = time.perf_counter()
    oracle_all_cores(case, act, ts, A, threads)
    dt_all = time.perf_counter() - t1
    return {"value": case.size / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"the {cut} cases with the lowest codes of the benchmark log ({case.size} events, "
                      f"rows in log order): DFG + variants, single thread, {dt:.2f} s",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "machine": platform.machine(),
            "all_cores": {"value": case.size / dt_all, "unit": "events/s", "cores": threads,
                          "how": "the oracle's DFG and variants on the sample's cases split into one group "
                                 "per host thread by case id, merged (counts and sums added, min/max "
                                 f"combined, variants merged by exact sequence); {dt_all:.2f} s"}}


def cpu_model() -> str | None:
    """The host CPU's model name (as lscpu prints it)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_views(log, prep, n_views: int, steps: int, per_view_sample: int, autotune: bool = True,
                compare_launch: bool = True) -> dict:
    """Batched drill-down views over the prepared log: one call for all views,
    against a loop of one-view calls of the same entry point."""
    import numpy as np
    import torch

    from paper_2204_04898_amd import pm4g, synth
    from paper_2204_04898_amd import tune as tuner

    views = synth.make_views(log, n_views, seed=synth.SEED_BASE + 4)
    visits = int(np.sum([log.lengths_by_code[views.case_lo[v]:views.case_hi[v]].sum() for v in range(n_views)]))
    vd, md = pm4g.views_to_device(views, prep.case_s.device)
    t0 = time.perf_counter()
    out = pm4g.pm4g_dfg_batched(prep, vd, md, n_views)          # sizes the capacities (retries)
    log_progress(f"views: first call (capacity sizing) {time.perf_counter() - t0:.2f} s")
    req = [int(x) for x in out["required"].cpu().tolist()]
    tuned = None
    if autotune:
        t0 = time.perf_counter()
        res = tuner.tune_batched(prep, vd, md, n_views, reps=2, log=log_progress)
        log_progress(f"views: autotune sweep {time.perf_counter() - t0:.1f} s")
        tune = res["tuning"]
        tuned = {k: res["best"][k] for k in ("tile_events", "emit_blocks", "agg_blocks", "launch")}
        tuned["sweep"] = len(res["table"])
    else:   # the cached launch shape (library defaults without a cache entry)
        tune = pm4g.BatchedTuning(pair_capacity=int(req[3] * 1.1) + 1024,
                                  record_capacity=int(req[1] * 1.1) + 1024,
                                  cell_capacity=int(req[4] * 1.1) + 1024)
        hit = tuner.default_cache().lookup(log.n_activities, n_views, prep.n_events)
        if hit is not None:
            tune.tile_events = int(hit["tile_events"])
            tune.emit_blocks = int(hit["emit_blocks"])
            tune.agg_blocks = int(hit["agg_blocks"])
            tune.launch = int(hit.get("launch", 1))
    out = pm4g.pm4g_dfg_batched(prep, vd, md, n_views, tuning=tune, out=out)
    torch.cuda.synchronize()
    pm4g.profile_enable(True)
    pm4g.profile_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        pm4g.pm4g_dfg_batched(prep, vd, md, n_views, tuning=tune, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    vprof = pm4g.profile_read()
    pm4g.profile_enable(False)
    view_stages = {name: tot / steps for name, (tot, cnt) in vprof.items() if cnt}
    # the other launch mode on the same calls: the whole call as one persistent
    # launch (launch 0) against one launch per phase (launch 1)
    other = pm4g.BatchedTuning.from_buffer_copy(tune)
    other.launch = 1 - tune.launch
    if other.launch == 1 and other.emit_blocks == 0:
        other.emit_blocks, other.agg_blocks = 2048, 256
    other_ms = None
    if compare_launch:
        pm4g.pm4g_dfg_batched(prep, vd, md, n_views, tuning=other, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pm4g.pm4g_dfg_batched(prep, vd, md, n_views, tuning=other, out=out)
        torch.cuda.synchronize()
        other_ms = (time.perf_counter() - t0) / steps * 1e3
    # per-view launches of the same entry point on a sample of the views
    # (one launch per phase: the faster form for one small view)
    idx = np.linspace(0, n_views - 1, per_view_sample).astype(int)
    one_t = pm4g.BatchedTuning(pair_capacity=int(req[3]) + 1024, record_capacity=int(req[1]) + 1024,
                               cell_capacity=int(req[4]) + 1024, launch=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for v in idx:
        pm4g.pm4g_dfg_batched(prep, vd[v * 24:(v + 1) * 24], md[v:v + 1], 1, tuning=one_t)
    torch.cuda.synchronize()
    per_view_s = (time.perf_counter() - t1) / len(idx)
    # the oracle beside it: a few views whose slices hold 0.2-2M events, each
    # given only its slice's cases (the view keeps nothing else)
    import oracle

    sizes = np.array([log.lengths_by_code[views.case_lo[v]:views.case_hi[v]].sum() for v in range(n_views)])
    pick = np.flatnonzero((sizes >= 200_000) & (sizes <= 2_000_000))[:4]
    o_visits, o_time = 0, 0.0
    for v in pick:
        sel = (log.case >= views.case_lo[v]) & (log.case < views.case_hi[v])
        c, a, t = log.case[sel], log.act[sel], log.ts[sel]
        t2 = time.perf_counter()
        oracle.view(c, a, t, log.n_activities, int(views.case_lo[v]), int(views.case_hi[v]), int(views.t_lo[v]),
                    int(views.t_hi[v]), views.masks[v])
        o_time += time.perf_counter() - t2
        o_visits += int(c.size)
    cpu_oracle = {"event_view_visits_per_s": o_visits / o_time if o_time else None, "cores": 1,
                  "sample": f"{len(pick)} views with 0.2-2M-event slices ({o_visits} event-view visits), "
                            "each on its slice's cases, single thread"}
    return {"views_per_s": n_views / dt, "ms_per_call": dt * 1e3, "n_views": n_views,
            "event_view_visits_per_s": visits / dt, "cpu_oracle": cpu_oracle,
            "event_view_visits": visits, "output_cells": req[0], "records": req[1],
            "run_places": req[2], "tile_view_pairs": req[3],
            "per_view_launch_views_per_s": 1.0 / per_view_s,
            "per_view_launch_sample": len(idx),
            "speedup_vs_per_view_launches": per_view_s * n_views / dt,
            "stages_ms_per_call": view_stages,
            "ms_per_call_by_launch": {("one persistent launch" if tune.launch == 0 else "one launch per phase"):
                                      dt * 1e3,
                                      ("one persistent launch" if other.launch == 0 else "one launch per phase"):
                                      other_ms},
            "tuning": tuned if tuned is not None else {"tile_events": tune.tile_events or 4096,
                                                       "emit_blocks": tune.emit_blocks or 2048,
                                                       "agg_blocks": tune.agg_blocks or 512,
                                                       "launch": tune.launch}}


def bench_cases(log, prep, steps: int = 5) -> dict:
    """Cases dataframe, case-level and directly-follows-level filters and
    sampling on the prepared log (whole-log calls)."""
    import numpy as np
    import torch

    from paper_2204_04898_amd import pm4g

    A = log.n_activities
    rng = np.random.default_rng(220404898 + 6)
    pm = np.zeros((A * A + 63) // 64, np.uint64)
    for b in rng.choice(A * A, A, replace=False):
        pm[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    pmd = torch.from_numpy(pm.view(np.int64)).to(prep.case_s.device)
    out = pm4g.Prepared.empty(prep.n_events, A, prep.case_s.device)
    # per-case variant ids of the same log (untimed), and the ten most frequent variants
    vo = pm4g.pm4g_variants_prepared(prep)
    torch.cuda.synchronize()
    nv = int(vo["n_variants"].item())
    vm = np.zeros((nv + 63) // 64 or 1, np.uint64)
    for b in range(min(nv, 10)):
        vm[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    vmd = torch.from_numpy(vm.view(np.int64)).to(prep.case_s.device)
    t_lo, t_hi = (int(x) for x in torch.quantile(prep.ts_s[::max(prep.n_events // 1000000, 1)].double(),
                                                  torch.tensor([0.3, 0.7], dtype=torch.float64,
                                                               device=prep.case_s.device)).cpu())
    C_all = int(prep.n_cases.item())
    res = {}
    for name, call in (("cases_dataframe", lambda: pm4g.pm4g_cases(prep)),
                       ("filter_events_5_40", lambda: pm4g.pm4g_filter_cases(prep, min_events=5, max_events=40,
                                                                             out=out)),
                       ("filter_drop_paths", lambda: pm4g.pm4g_filter_cases(prep, path_mask=pmd, path_keep=False,
                                                                            out=out)),
                       ("filter_contained_30_70pct", lambda: pm4g.pm4g_filter_cases(prep, contain_lo=t_lo,
                                                                                    contain_hi=t_hi, out=out)),
                       ("filter_top10_variants", lambda: pm4g.pm4g_filter_cases(
                           prep, case_variant=vo["case_variant"], variant_mask=vmd, n_variant_bits=nv,
                           variant_keep=True, out=out)),
                       ("sample_10pct_cases", lambda: pm4g.pm4g_sample(prep, C_all // 10, 7, False, out=out)),
                       ("sample_10pct_events", lambda: pm4g.pm4g_sample(prep, prep.n_events // 10, 7, True,
                                                                        out=out)),
                       ("df_events_keep_prev_pairs", lambda: pm4g.pm4g_filter_df_events(prep, pmd, 0, True, out=out)),
                       ("df_events_drop_prev_pairs", lambda: pm4g.pm4g_filter_df_events(prep, pmd, 0, False,
                                                                                       out=out))):
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        r = {"ms_per_call": dt * 1e3, "events_per_s": prep.n_events / dt}
        kept_e = kept_c = 0
        if name != "cases_dataframe":
            K = int(out.n_cases.item())
            kept_e, kept_c = int(out.case_off[K].item()), K
            r["kept_events"], r["kept_cases"] = kept_e, kept_c
        algo = filter_bytes(name, prep.n_events, C_all, kept_e, kept_c)
        if algo is not None:
            r["algorithmic_bytes"] = algo
            r["achieved_GBps"] = algo / dt / 1e9
            r["frac_of_hbm_peak"] = algo / dt / 1e9 / HBM_PEAK_GBS
        res[name] = r
    res["cpu_oracle"] = _cases_oracle_timing(log, pm)
    return res


def _cases_oracle_timing(log, path_mask, target_events: int = 2_000_000) -> dict:
    """The oracle's case filter, directly-follows filter and sampling on the
    cases with the lowest codes (about target_events events), single thread."""
    import numpy as np

    import oracle

    cum = np.cumsum(log.lengths_by_code)
    cut = min(int(np.searchsorted(cum, target_events, side="left")) + 1, int(cum.shape[0]))
    keep = log.case < cut
    c, a, t = log.case[keep], log.act[keep], log.ts[keep]
    A = log.n_activities
    out = {}
    for name, call in (("filter_events_5_40", lambda: oracle.filter_cases(c, a, t, A, min_events=5, max_events=40)),
                       ("filter_drop_paths", lambda: oracle.filter_cases(c, a, t, A, path_mask=path_mask,
                                                                         path_keep=False)),
                       ("df_events_drop_prev_pairs", lambda: oracle.filter_df_events(c, a, t, A, path_mask, 0,
                                                                                     False)),
                       ("sample_10pct_cases", lambda: oracle.sample(c, a, t, A, cut // 10, 7, False))):
        t0 = time.perf_counter()
        call()
        dt = time.perf_counter() - t0
        out[name] = {"events_per_s": c.size / dt}
    out["cores"] = 1
    out["sample"] = f"the {cut} cases with the lowest codes ({c.size} events), single thread"
    return out


def filter_bytes(name: str, n: int, c: int, kept_e: int, kept_c: int) -> int | None:
    """Algorithmic HBM bytes of one whole-log call of the cases section: n
    events, c cases, kept_e events and kept_c cases in the output.  A decision
    per case reads its offset pair and first and last timestamps (24 B) and
    writes its kept events and flag (8 B); the scans of those read 8 B and
    write 12 B per case; a kept event is read (16 B) and written (16 B); the
    output case table is 12 B per kept case.  Sampling by events computes its
    keys (no memory) and is reported without a byte count."""
    per_case = 24 + 8 + 8 + 12
    copy = 32 * kept_e + 12 * kept_c
    if name == "cases_dataframe":
        return c * (8 + 16 + 16)
    if name in ("filter_events_5_40", "filter_contained_30_70pct"):
        return c * per_case + copy
    if name == "filter_drop_paths":
        return n * 4 + c * 16 + c * per_case + copy                     # containment pass: act + offsets
    if name == "filter_top10_variants":
        return c * (per_case + 4) + copy                                # + the case's variant id
    if name == "sample_10pct_cases":
        return c * 4 * 8 + c * (8 + 8 + 8 + 12) + copy                  # 8 select passes over the codes
    if name.startswith("df_events_"):
        return 2 * n * 8 + copy                                         # count and emit read case + act
    return None


def bench_efg(log, prep, steps: int = 3, oracle_events: int = 1_000_000) -> dict:
    """Eventually-follows graph and temporal profile of a prepared log (whole-log
    calls), with the oracle timed on the cases of a bounded sample beside it."""
    import numpy as np
    import torch

    from paper_2204_04898_amd import pm4g

    o = pm4g.pm4g_efg(prep)
    torch.cuda.synchronize()
    ws = torch.empty(int(pm4g.load().pm4g_efg_workspace_bytes(prep.n_events, prep.n_activities)),
                     dtype=torch.uint8, device=prep.case_s.device)
    t0 = time.perf_counter()
    for _ in range(steps):
        pm4g.pm4g_efg(prep, out=o, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    pairs = int(o["n_pairs"].item())
    res = {"ms_per_call": dt * 1e3, "pairs": pairs, "pairs_per_s": pairs / dt, "events_per_s": prep.n_events / dt,
           "n_activities": prep.n_activities}
    import oracle

    cum = np.cumsum(log.lengths_by_code)
    cut = min(int(np.searchsorted(cum, oracle_events, side="left")) + 1, int(cum.shape[0]))
    keep = log.case < cut
    t1 = time.perf_counter()
    ob = oracle.efg(log.case[keep], log.act[keep], log.ts[keep], log.n_activities)
    odt = time.perf_counter() - t1
    res["cpu_oracle"] = {"pairs_per_s": ob["n_pairs"] / odt, "cores": 1,
                         "sample": f"the {cut} cases with the lowest codes ({int(keep.sum())} events, "
                                   f"{ob['n_pairs']} pairs), single thread, {odt:.2f} s"}
    return res


def bench_ingest(log, steps: int = 3) -> dict:
    """CSV ingestion of a log's text (ISO-8601 ms timestamps) already resident
    in device memory; the oracle's parse of a bounded sample timed beside it."""
    import torch

    import oracle
    from paper_2204_04898_amd import pm4g, synth

    text = synth.log_csv(log, "ms", True)
    t = torch.frombuffer(bytearray(text), dtype=torch.uint8).to("cuda")
    cap = log.n_events + 1
    pm4g.pm4g_ingest_csv(t, 0, 1, 2, ts_iso=True, ts_scale=3, capacity=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = pm4g.pm4g_ingest_csv(t, 0, 1, 2, ts_iso=True, ts_scale=3, capacity=cap)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    algo = len(text) + 16 * r["n_rows"]   # the text read once, codes and timestamps written
    res = {"ms_per_call": dt * 1e3, "bytes": len(text), "rows": r["n_rows"], "GB_per_s": len(text) / dt / 1e9,
           "rows_per_s": r["n_rows"] / dt, "n_cases": r["n_cases"], "n_acts": r["n_acts"],
           "algorithmic_bytes": algo, "achieved_GBps": algo / dt / 1e9,
           "frac_of_hbm_peak": algo / dt / 1e9 / HBM_PEAK_GBS,
           "note": "text resident in HBM; includes the workspace allocation of the binding"}
    cut = text.index(b"\n", 20_000_000) + 1
    t1 = time.perf_counter()
    o = oracle.ingest_csv(text[:cut], 0, 1, 2, ts_iso=True, ts_scale=3)
    odt = time.perf_counter() - t1
    res["cpu_oracle"] = {"GB_per_s": cut / odt / 1e9, "cores": 1,
                         "sample": f"the first {cut} bytes ({o['n_rows']} rows), single thread, {odt:.2f} s"}
    return res


def bench_parquet(log, steps: int = 3, oracle_rows: int = 2_000_000) -> dict:
    """Parquet ingestion of a log written by pyarrow with its defaults
    (dictionary-coded columns, 1 MiB data pages, no compression; string case
    and activity names, ms timestamps), the file resident in device memory; the
    oracle's reader timed on a file of the log's first rows beside it."""
    import io

    import numpy as np
    import pyarrow as pa
    import pyarrow.parquet as pq
    import torch

    import oracle
    from paper_2204_04898_amd import pm4g

    def parquet(lo, hi):
        names = np.array([f"Activity {k:04d}" for k in range(log.n_activities)], dtype=object)
        cases = np.char.add("case ", log.case[lo:hi].astype(str)).astype(object)
        t = pa.table({"case:concept:name": pa.array(list(cases)),
                      "concept:name": pa.array(list(names[log.act[lo:hi]])),
                      "time:timestamp": pa.array(log.ts[lo:hi], pa.timestamp("ms"))})
        buf = io.BytesIO()
        pq.write_table(t, buf, compression="NONE")
        return buf.getvalue()

    data = parquet(0, log.n_events)
    d = torch.frombuffer(bytearray(data), dtype=torch.uint8).to("cuda")
    cap = log.n_events
    r = pm4g.pm4g_ingest_parquet(d, 0, 1, 2, capacity=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = pm4g.pm4g_ingest_parquet(d, 0, 1, 2, capacity=cap)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    algo = len(data) + 16 * r["n_rows"]   # the file read once, codes and timestamps written
    res = {"ms_per_call": dt * 1e3, "bytes": len(data), "rows": r["n_rows"], "GB_per_s": len(data) / dt / 1e9,
           "rows_per_s": r["n_rows"] / dt, "n_cases": r["n_cases"], "n_acts": r["n_acts"],
           "algorithmic_bytes": algo, "achieved_GBps": algo / dt / 1e9,
           "frac_of_hbm_peak": algo / dt / 1e9 / HBM_PEAK_GBS,
           "layout": "pyarrow defaults without compression: dictionary pages (the case column falls back to "
                     "PLAIN once its dictionary passes 1 MiB), 1 MiB data pages, row groups of 1Mi rows",
           "note": "file resident in HBM; includes the footer read-back and the workspace allocation of the binding"}
    m = min(oracle_rows, log.n_events)
    small = parquet(0, m)
    t1 = time.perf_counter()
    o = oracle.ingest_parquet(small, 0, 1, 2)
    odt = time.perf_counter() - t1
    res["cpu_oracle"] = {"rows_per_s": o["n_rows"] / odt, "GB_per_s": len(small) / odt / 1e9, "cores": 1,
                         "sample": f"the log's first {m} rows written the same way ({len(small)} bytes), "
                                   f"single thread, {odt:.2f} s"}
    return res


def bench_serving(logs: dict, preps: dict, seconds: float, rate: float, workers: int = 4,
                  batch_work: int = 20_000_000, warmup_s: float = 5.0, stress_budget: int = 4 << 30,
                  side_seconds: float = 15.0) -> dict:
    """Open-loop Poisson mix of DFG / variants / filter queries on resident logs.

    A warm-up run of its own (warmup_s of arrivals, not reported), then the
    main run (`seconds` of arrivals, memory budget: 90 % of the HBM left free
    by the resident logs).  On the first side_seconds of the same arrivals: a
    stress run with a stress_budget-byte budget, where admission queues, and
    the one-request-per-launch baselines with 1 and with `workers` streams;
    the main run's figures over the same requests stand beside them."""
    import copy

    import numpy as np
    import torch

    from paper_2204_04898_amd import serve

    info = {k: serve.log_info(v) for k, v in logs.items()}
    A_of = {k: v.n_activities for k, v in logs.items()}
    reqs = serve.poisson_requests(np.random.default_rng(220404898 + 5), rate, seconds, info, A_of)
    warm = serve.poisson_requests(np.random.default_rng(220404898 + 6), rate, warmup_s, info, A_of)
    ex = serve.GpuExecutor(preps)
    torch.cuda.synchronize()
    free, _total = torch.cuda.mem_get_info()
    budget = int(free * 0.9)
    log_progress(f"serving: warm-up, {len(warm)} requests over {warmup_s} s")
    serve.Scheduler(ex, budget, max_batch=64, workers=workers, max_batch_work=batch_work).run(warm)
    log_progress(f"serving: main run, {len(reqs)} requests over {seconds} s")
    sch = serve.Scheduler(ex, budget, max_batch=64, workers=workers, max_batch_work=batch_work)
    ex.start_timeline()
    res = sch.run(copy.deepcopy(reqs), progress=log_progress)
    st = serve.latency_stats(res, sch)
    st["device_overlap"] = dict(ex.timeline(), how="HIP events on each worker's stream around each batch")
    st.update(offered_qps=rate, seconds=seconds, warmup_seconds=warmup_s, n_requests=len(reqs),
              max_batch_work=batch_work, budget="90% of the HBM free after the logs are resident",
              variants_answer=f"variant count + first {ex.variants_top} variants",
              admission="per-request estimate = the library's workspace-size query for the request's "
                        "capacities + the outputs it allocates")
    side = [r for r in reqs if r.arrival < side_seconds]
    ids = {r.rid for r in side}
    st["main_run_first_part"] = dict(serve.latency_stats([r for r in res if r.rid in ids]),
                                     seconds=side_seconds, workers=workers, max_batch=64)
    for sb in (stress_budget, stress_budget // 4):
        log_progress(f"serving: stress run, {sb >> 20} MiB budget, {len(side)} requests")
        stress = serve.Scheduler(ex, sb, max_batch=64, workers=workers, max_batch_work=batch_work)
        sres = stress.run(copy.deepcopy(side), progress=log_progress)
        st.setdefault("stress_budget", {})[f"{sb >> 20}MiB"] = dict(serve.latency_stats(sres, stress),
                                                                    seconds=side_seconds, budget_mib=sb >> 20)
    # a higher offered load on the same logs and mix: continuous batching
    # against one request per launch on as many streams
    hi_rate = 5 * rate
    hi = serve.poisson_requests(np.random.default_rng(220404898 + 7), hi_rate, 5.0, info, A_of)
    # a warm-up at this rate first (not reported): larger batches meet
    # buffer sizes the 200 queries/s runs never asked the allocator for
    hi_warm = serve.poisson_requests(np.random.default_rng(220404898 + 8), hi_rate, 2.0, info, A_of)
    for label, mb in (("continuous_batching", 64), ("one_request_per_launch", 1)):
        log_progress(f"serving: {hi_rate:.0f} queries/s, {label}")
        serve.Scheduler(ex, budget, max_batch=mb, workers=workers, max_batch_work=batch_work).run(
            copy.deepcopy(hi_warm))
        hs = serve.Scheduler(ex, budget, max_batch=mb, workers=workers, max_batch_work=batch_work)
        ex.start_timeline()
        hres = hs.run(copy.deepcopy(hi), progress=log_progress)
        st.setdefault("high_load", {})[label] = dict(serve.latency_stats(hres, hs), offered_qps=hi_rate, seconds=5.0,
                                                      max_batch=mb, n_requests=len(hi),
                                                      device_overlap=ex.timeline())
    for nw in sorted({1, workers}):
        log_progress(f"serving: one request per launch, {nw} stream(s)")
        base = serve.Scheduler(ex, budget, max_batch=1, workers=nw)
        bres = base.run(copy.deepcopy(side), progress=log_progress)
        st[f"one_request_per_launch_{nw}_streams"] = dict(serve.latency_stats(bres, base), seconds=side_seconds,
                                                         workers=nw, max_batch=1)
    return st


def kernel_overlap(trace_csv: str) -> dict:
    """From a rocprofv3 --kernel-trace CSV: the library's kernels grouped by the
    stream (queue) they ran on, and the share of their busy time during which
    kernels of two or more streams ran at once."""
    import csv

    spans = []
    with open(trace_csv) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name", "")
            if "pm4g::" not in name:
                continue
            q = row.get("Stream_Id") or row.get("Queue_Id") or "0"
            spans.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"]), q))
    if not spans:
        raise SystemExit("no library kernels in the trace")
    ev = []
    for a, b, q in spans:
        ev.append((a, 1, q))
        ev.append((b, -1, q))
    ev.sort(key=lambda e: (e[0], e[1]))
    active: dict = {}
    busy = multi = 0
    last = ev[0][0]
    for t, d, q in ev:
        if active:
            busy += t - last
            if len(active) >= 2:
                multi += t - last
        last = t
        active[q] = active.get(q, 0) + d
        if active[q] == 0:
            del active[q]
    streams = sorted({q for _, _, q in spans})
    return {"kernels": len(spans), "streams": len(streams), "busy_ms": busy / 1e6,
            "multi_stream_ms": multi / 1e6, "overlap_frac": multi / busy if busy else 0.0}


def calibrate_copy(gib: float = 1.0, reps: int = 3) -> None:
    """A plain streaming kernel of known traffic (reads gib GiB, writes gib GiB:
    an elementwise bitwise-not), for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    n = int(gib * (1 << 30))
    x = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.bitwise_not(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "reps": reps}))


def _counter_rows(path: str, kernel: str, counter: str) -> list[float]:
    import csv

    vals = []
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if kernel in row.get("Kernel_Name", "") and row.get("Counter_Name") == counter:
                vals.append(float(row["Counter_Value"]))
    return vals


def summarize_counters(a) -> None:
    """Writes profiles/traffic_<stage>_<workload>.txt from two rocprofv3 --pmc runs of the
    benchmark (FETCH_SIZE, WRITE_SIZE in KiB per dispatch) and of the copy calibration;
    with --stage step, the sum over every library kernel divided by the steps run
    (counted by the launches of the range scan's first kernel), into profiles/traffic_step_<workload>.txt."""
    cf = _counter_rows(a.copy_fetch_csv, a.copy_kernel, "FETCH_SIZE")
    cw = _counter_rows(a.copy_write_csv, a.copy_kernel, "WRITE_SIZE")
    copy_bytes = float(a.copy_bytes)
    if not (cf and cw):
        raise SystemExit("counter rows missing for the copy kernel")
    f_scale = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    w_scale = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    if a.stage == "step":
        fetch = _counter_rows(a.fetch_csv, "pm4g::", "FETCH_SIZE")
        write = _counter_rows(a.write_csv, "pm4g::", "WRITE_SIZE")
        steps = len(_counter_rows(a.fetch_csv, "k_range_init", "FETCH_SIZE"))
        if not (fetch and write and steps):
            raise SystemExit("counter rows missing for the step's kernels")
        fb = sum(fetch) * 1024.0 * f_scale / steps
        wb = sum(write) * 1024.0 * w_scale / steps
        path = os.path.join(ROOT, "profiles", f"traffic_step_{a.workload}.txt")
        with open(path, "w") as fh:
            fh.write(f"# HBM traffic of one whole step (every pm4g kernel) on the {a.workload} workload\n")
            fh.write("# from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of:\n")
            fh.write(f"#   {a.command}\n")
            fh.write("# scaled by the same counters on a plain copy of copy_bytes bytes "
                     "(python3 bench.py --calibrate-copy)\n")
            fh.write(f"steps = {steps}\nkernel_dispatches = {len(fetch)}\n")
            fh.write(f"fetch_bytes_per_step = {fb:.0f}\nwrite_bytes_per_step = {wb:.0f}\n")
            fh.write(f"copy_bytes = {int(copy_bytes)}\ncopy_fetch_scale = {f_scale:.4f}\n"
                     f"copy_write_scale = {w_scale:.4f}\n")
            fh.write(f"bytes_per_step = {fb + wb:.0f}\n")
            fh.write(f"source_sha = {source_sha(STEP_SOURCES)}\n")
        print(path)
        return
    fetch = _counter_rows(a.fetch_csv, a.kernel, "FETCH_SIZE")
    write = _counter_rows(a.write_csv, a.kernel, "WRITE_SIZE")
    if not (fetch and write):
        raise SystemExit("counter rows missing for the kernel")
    fb = sum(fetch) / len(fetch) * 1024.0 * f_scale
    wb = sum(write) / len(write) * 1024.0 * w_scale
    path = os.path.join(ROOT, "profiles", f"traffic_{a.stage}_{a.workload}.txt")
    with open(path, "w") as fh:
        fh.write(f"# HBM traffic of {a.kernel} (stage {a.stage}) on the {a.workload} workload, per launch\n")
        fh.write("# from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of:\n")
        fh.write(f"#   {a.command}\n")
        fh.write("# scaled by the same counters on a plain copy of copy_bytes bytes "
                 "(python3 bench.py --calibrate-copy)\n")
        fh.write(f"kernel = {a.kernel}\nstage = {a.stage}\n")
        fh.write(f"launches_fetch = {len(fetch)}\nlaunches_write = {len(write)}\n")
        fh.write(f"fetch_kib_per_launch = {sum(fetch) / len(fetch):.1f}\n")
        fh.write(f"write_kib_per_launch = {sum(write) / len(write):.1f}\n")
        fh.write(f"copy_bytes = {int(copy_bytes)}\ncopy_fetch_scale = {f_scale:.4f}\ncopy_write_scale = {w_scale:.4f}\n")
        fh.write(f"bytes_per_launch = {fb + wb:.0f}\n")
        fh.write(f"source_sha = {source_sha(STAGE_SOURCES[a.stage])}\n")
    print(path)


def kernel_table(stats_csv: str, match: str | None = None) -> str:
    """A markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv):
    the kernels (those whose name matches the regular expression, if given)
    with their calls, average and total time, by total time."""
    import csv
    import re

    rows = []
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            name = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "")
            name = re.sub(r"\(.*\)$", "", name).replace("pm4g::", "")
            if match and not re.search(match, name):
                continue
            rows.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
                         float(r["Percentage"])))
    rows.sort(key=lambda x: -x[3])
    out = ["| kernel | calls | avg us | total ms | % of the run's kernel time |", "|---|---:|---:|---:|---:|"]
    out += [f"| `{n}` | {c} | {a:.1f} | {t:.2f} | {p:.1f} |" for n, c, a, t, p in rows]
    out.append("")
    out.append(f"Sum of the listed kernels' time: {sum(r[3] for r in rows):.2f} ms over all calls.")
    return "\n".join(out)


def main() -> int:
    if "--kernel-table" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--kernel-table", required=True)
        sp.add_argument("--match", default=None, help="only kernels whose name matches this regular expression")
        a = sp.parse_args()
        print(kernel_table(a.kernel_table, a.match))
        return 0
    if "--calibrate-copy" in sys.argv:
        calibrate_copy()
        return 0
    if "--overlap-from" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--overlap-from", required=True)
        print(json.dumps(kernel_overlap(sp.parse_args().overlap_from)))
        return 0
    if "--summarize-counters" in sys.argv:
        sp = argparse.ArgumentParser()
        sp.add_argument("--summarize-counters", action="store_true")
        for k in ("fetch-csv", "write-csv", "copy-fetch-csv", "copy-write-csv", "kernel", "stage", "workload",
                  "command"):
            sp.add_argument("--" + k, required=True)
        sp.add_argument("--copy-kernel", default="bitwise_not")
        sp.add_argument("--copy-bytes", type=int, default=1 << 30)
        summarize_counters(sp.parse_args())
        return 0
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dfg-variants-100M", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample-events", type=int, default=40_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time prepare + DFG only")
    ap.add_argument("--views", type=int, default=4096, help="batched drill-down views (0: skip)")
    ap.add_argument("--view-steps", type=int, default=3)
    ap.add_argument("--per-view-sample", type=int, default=64)
    ap.add_argument("--no-launch-compare", action="store_true",
                    help="views: do not time the other launch mode (rocprofv3 --kernel-trace stops on "
                         "cooperative launches)")
    ap.add_argument("--no-autotune", action="store_true", help="batched views with the cached launch shape (no sweep)")
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (default: the package's)")
    ap.add_argument("--no-cases", action="store_true", help="skip the cases-dataframe and case-filter timing")
    ap.add_argument("--no-efg", action="store_true", help="skip the eventually-follows graph timing")
    ap.add_argument("--no-ingest", action="store_true", help="skip the CSV and Parquet ingestion timings")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="serving run length (0: skip)")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="serving warm-up run length")
    ap.add_argument("--serve-side-seconds", type=float, default=15.0,
                    help="arrivals replayed by the stress run and the one-request-per-launch baselines")
    ap.add_argument("--serve-stress-mib", type=int, default=4096, help="memory budget of the stress run")
    ap.add_argument("--serve-only", action="store_true", help="only the serving runs (for a kernel trace)")
    ap.add_argument("--overlap-from", default=None,
                    help="print the multi-stream overlap of a rocprofv3 kernel-trace CSV and exit")
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-workers", type=int, default=4, help="batches in flight (HIP streams)")
    ap.add_argument("--serve-batch-work", type=int, default=20_000_000,
                    help="events a batch may scan before it closes (a larger request runs alone)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (it would shard the log "
              "by case, each GPU running the whole path on its cases).", file=sys.stderr)
        return 2

    import torch

    from paper_2204_04898_amd import pm4g, synth

    k, desc = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    log = synth.config_log(k)
    N, A = log.n_events, log.n_activities
    log_progress(f"generated {args.workload}: {N} events, A={A} in {time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda:0")
    c = torch.from_numpy(log.case).to(dev)
    a = torch.from_numpy(log.act).to(dev)
    t = torch.from_numpy(log.ts).to(dev)
    prep = pm4g.Prepared.empty(N, A, dev)
    dout = pm4g._dfg_out(A, dev)
    vout = pm4g._var_out(N, dev)
    if args.serve_only:
        if k != 3:
            raise SystemExit("--serve-only serves the 99M- and 10M-event logs (the default workload)")
        pm4g.pm4g_prepare(c, a, t, A, out=prep)
        log2 = synth.config_log(2)
        c2, a2, t2 = (torch.from_numpy(x).to(dev) for x in (log2.case, log2.act, log2.ts))
        prep2 = pm4g.pm4g_prepare(c2, a2, t2, log2.n_activities)
        del c, a, t, c2, a2, t2, vout
        st = bench_serving({"dfg-perf-10M": log2, args.workload: log}, {"dfg-perf-10M": prep2, args.workload: prep},
                           args.serve_seconds, args.serve_qps, args.serve_workers, args.serve_batch_work,
                           args.serve_warmup, args.serve_stress_mib << 20, args.serve_side_seconds)
        print(json.dumps({"serving": st}), flush=True)
        return 0

    def step():
        pm4g.pm4g_prepare(c, a, t, A, presorted=log.presorted, out=prep)
        pm4g.pm4g_dfg_prepared(prep, out=dout)
        if not args.no_variants:
            pm4g.pm4g_variants_prepared(prep, out=vout)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log_progress(f"warmup done ({args.warmup} steps)")

    pm4g.profile_enable(True)
    pm4g.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pm4g.profile_read()
    pm4g.profile_enable(False)
    log_progress(f"timed {args.steps} steps in {t1 - t0:.3f} s")

    C = int(prep.n_cases.item())
    # validity of the last step: directly-follows pairs = events - cases, one start per case
    assert int(dout["count"].sum().item()) == N - C, "DFG invariant failed"
    assert int(dout["start_count"].sum().item()) == C, "start counts invariant failed"
    if not args.no_variants:
        assert int(vout["var_count"][: int(vout["n_variants"].item())].sum().item()) == C

    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = N * args.steps / (t1 - t0)

    stages = {name: {"ms_per_step": tot / args.steps, "launches_per_step": cnt / args.steps}
              for name, (tot, cnt) in prof.items() if cnt}
    packed, passes = packed_keys(log), radix_passes(log)
    kb = lambda name: kernel_bytes(name, N, C, A, log.presorted, packed, passes)
    # the kernel with the most time per step, and the next one (the radix
    # scatter's three launches and the per-case sort's one are close)
    ranked = sorted(((n, v) for n, v in prof.items() if kb(n) and v[1]), key=lambda kv: -kv[1][0])
    dname, (dms, dcnt) = ranked[0]
    per_launch_ms = dms / dcnt
    algo = kb(dname)
    achieved = algo / (per_launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(dname, args.workload)
    runner_up = None
    if len(ranked) > 1:
        rname, (rms, rcnt) = ranked[1]
        r_launch = rms / rcnt
        r_ach = kb(rname) / (r_launch * 1e-3) / 1e9
        runner_up = {"kernel": rname, "ms_per_step": rms / args.steps, "achieved": r_ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r_ach / HBM_PEAK_GBS,
                     "traffic": measured_traffic(rname, args.workload),
                     "algorithmic_bytes_per_launch": kb(rname), "avg_launch_ms": r_launch,
                     "valu_issue_frac": valu_issue_frac(rname, args.workload, r_launch)}

    out = {
        "metric": "DFG events/sec on 1 MI355X + % HBM roofline",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n_events": N, "n_cases": C,
                   "n_activities": A, "step": "prepare + dfg" + ("" if args.no_variants else " + variants")},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": algo, "avg_launch_ms": per_launch_ms,
                     "ms_per_step": dms / args.steps,
                     # instruction-bound kernels: the VALU issue rate reached (one
                     # wave64 instruction per CU per cycle is the peak)
                     "valu_issue_frac": valu_issue_frac(dname, args.workload, per_launch_ms),
                     "runner_up": runner_up},
        "stages": stages,
    }
    # the whole step against the HBM peak: measured traffic (all kernels of one
    # step, from the committed counter summary) and the compulsory floor of
    # 16 B/event (case, activity, timestamp read once)
    step_bytes = measured_step_traffic(args.workload)
    t_step = ms_per_step * 1e-3
    out["step_hbm"] = {"floor_bytes": 16 * N, "floor_frac": 16 * N / t_step / (HBM_PEAK_GBS * 1e9),
                       "measured_bytes": step_bytes,
                       "measured_frac": None if step_bytes is None else step_bytes / t_step / (HBM_PEAK_GBS * 1e9),
                       "measured_over_floor": None if step_bytes is None else step_bytes / (16 * N)}
    if args.views > 0 and k == 3:
        log_progress(f"batched views: {args.views} views")
        if args.tune_cache:
            os.environ["PM4G_TUNE_CACHE"] = args.tune_cache
        out["batched_views"] = bench_views(log, prep, args.views, args.view_steps, args.per_view_sample,
                                           autotune=not args.no_autotune,
                                           compare_launch=not args.no_launch_compare)
    if k == 3 and not args.no_cases:
        log_progress("cases dataframe and case filters")
        out["cases"] = bench_cases(log, prep)
    if k == 3 and not args.no_efg:
        log_progress("eventually-follows graph and temporal profile")
        out["efg"] = {args.workload: bench_efg(log, prep)}
    log2 = prep2 = None
    if k == 3 and (args.serve_seconds > 0 or not args.no_efg):
        log_progress("generating the 10M-event log")
        log2 = synth.config_log(2)
        c2, a2, t2 = (torch.from_numpy(x).to(dev) for x in (log2.case, log2.act, log2.ts))
        prep2 = pm4g.pm4g_prepare(c2, a2, t2, log2.n_activities)
    if k == 3 and not args.no_efg:
        log_progress("eventually-follows graph of the 10M-event log")
        out["efg"]["dfg-perf-10M"] = bench_efg(log2, prep2)
    if k == 3 and not args.no_ingest:
        if log2 is None:
            log2 = synth.config_log(2)
        log_progress("CSV ingestion of the 10M-event log")
        out["ingest_csv"] = {"dfg-perf-10M": bench_ingest(log2)}
        try:
            import pyarrow  # noqa: F401
        except ImportError:
            out["ingest_parquet"] = {"skipped": "pyarrow is not importable"}
        else:
            log_progress("Parquet ingestion of the 10M-event log")
            out["ingest_parquet"] = {"dfg-perf-10M": bench_parquet(log2)}
    if args.serve_seconds > 0 and k == 3:
        if prep2 is None:
            if log2 is None:
                log2 = synth.config_log(2)
            c2, a2, t2 = (torch.from_numpy(x).to(dev) for x in (log2.case, log2.act, log2.ts))
            prep2 = pm4g.pm4g_prepare(c2, a2, t2, log2.n_activities)
        log_progress(f"serving: {args.serve_seconds} s at {args.serve_qps} queries/s")
        out["serving"] = bench_serving({"dfg-perf-10M": log2, args.workload: log},
                                       {"dfg-perf-10M": prep2, args.workload: prep},
                                       args.serve_seconds, args.serve_qps, args.serve_workers,
                                       args.serve_batch_work, args.serve_warmup, args.serve_stress_mib << 20,
                                       args.serve_side_seconds)
    if not args.no_cpu_baseline:
        log_progress("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(log, args.cpu_sample_events)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
