"""Serving on the GPU: results of requests served in the continuous-batching
mix are bit-identical to the same requests served alone, and match the
oracle."""
import concurrent.futures as cf
import copy

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, serve, synth
from tests.gpu_util import cols, note, same_f64

pytestmark = pytest.mark.gpu

TOP = 40


def _prepare(log):
    c, a, t = cols(log.case, log.act, log.ts)
    p = pm4g.pm4g_prepare(c, a, t, log.n_activities)
    torch.cuda.synchronize()
    return p


def _same(x, y):
    if x is None or y is None:
        return x is y
    assert set(x) == set(y)
    for k in x:
        a, b = x[k], y[k]
        if isinstance(a, np.ndarray):
            if a.dtype == np.float64:
                assert same_f64(a, b), k
            else:
                assert np.array_equal(a, b), k
        else:
            assert a == b, k
    return True


def _kept_formatted(oprep, r):
    """The events a view keeps, from the oracle's formatted log (in order)."""
    code, off = oprep["case_code"], oprep["case_off"]
    j0 = int(np.searchsorted(code, r.case_lo, side="left"))
    j1 = int(np.searchsorted(code, r.case_hi, side="left")) if r.case_lo < r.case_hi else j0
    a, b = int(off[j0]), int(off[max(j1, j0)])
    c, act, ts = oprep["case_s"][a:b], oprep["act_s"][a:b], oprep["ts_s"][a:b]
    keep = ((ts >= r.t_lo) & (ts <= r.t_hi)
            & ((r.mask[act // 64] >> (act % 64).astype(np.uint64)) & np.uint64(1)).astype(bool))
    return c[keep], act[keep], ts[keep]


def _oracle_check(oprep, A, r, res):
    """Every field of a served answer against the oracle (the view by a scan
    of the oracle's formatted log; variants of the kept events)."""
    if r.kind in ("dfg", "filter"):
        ref = oracle.view_formatted(oprep, A, r.case_lo, r.case_hi, r.t_lo, r.t_hi, r.mask)
        assert res["n_events"] == ref["n_events"] and res["n_cases"] == ref["n_cases"], r.rid
        if r.kind == "dfg":
            nz = np.flatnonzero(ref["count"].ravel())
            assert np.array_equal(res["src"].astype(np.int64) * A + res["dst"], nz), r.rid
            for k in ("count", "dt_sum", "dt_min", "dt_max"):
                assert np.array_equal(res[k], ref[k].ravel()[nz]), (r.rid, k)
            assert same_f64(res["dt_mean"], ref["dt_mean"].ravel()[nz]), r.rid
            for k in ("start_count", "end_count", "act_count"):
                assert np.array_equal(res[k], ref[k]), (r.rid, k)
    else:
        c, a, t = _kept_formatted(oprep, r)
        ref = oracle.variants(c, a, t, A)
        assert res["n_variants"] == ref["n_variants"], r.rid
        assert res["n_events"] == c.size and res["n_cases"] == ref["n_cases"], r.rid
        K = min(res.get("top", TOP), ref["n_variants"])     # the answer carries the first variants
        for k in ("var_count", "var_len", "var_rep"):
            assert np.array_equal(res[k], ref[k][:K]), (r.rid, k)
        assert np.array_equal(res["var_off"], ref["var_off"][:K + 1]), r.rid
        assert np.array_equal(res["var_acts"], ref["var_acts"][:ref["var_off"][K]]), r.rid
    return r.kind


def test_mixed_requests_equal_alone_and_oracle():
    logs = {"small": synth.config_log(2, 0.01), "wide": synth.config_log(3, 0.004)}
    preps = {k: _prepare(v) for k, v in logs.items()}
    info = {k: serve.log_info(v) for k, v in logs.items()}
    A_of = {k: v.n_activities for k, v in logs.items()}
    rng = np.random.default_rng(2024)
    reqs = serve.poisson_requests(rng, rate=2000.0, seconds=0.03, logs=info, A_of=A_of,
                                  min_events=100, max_events=200_000)
    note(f"serving {len(reqs)} requests")
    ex = serve.GpuExecutor(preps, variants_top=TOP)
    sch = serve.Scheduler(ex, mem_budget=256 << 20, max_batch=16, workers=2)
    mixed = sch.run(copy.deepcopy(reqs))
    assert all(r.error is None for r in mixed), [r.error for r in mixed if r.error]
    assert max(len(b) for b in sch.batches) > 1        # batching happened
    opreps = {k: oracle.prepare(v.case, v.act, v.ts, v.n_activities) for k, v in logs.items()}
    for r0, rm in zip(reqs, mixed):
        alone = copy.deepcopy(r0)
        ex.run([alone])
        assert _same(alone.result, rm.result), rm.rid
        _oracle_check(opreps[rm.log], A_of[rm.log], rm, rm.result)
    st = serve.latency_stats(mixed)
    assert st["n"] == len(reqs)


def test_serving_full_size_logs_against_oracle():
    """At least 200 requests of the serving workload (slices log-uniform from
    1e4 events up to the whole log) over the resident 10M- and 99M-event logs,
    served in the continuous-batching mix; every field of every answer checked
    against the oracle."""
    logs = {"dfg-perf-10M": synth.config_log(2), "dfg-variants-100M": synth.config_log(3)}
    preps = {k: _prepare(v) for k, v in logs.items()}
    info = {k: serve.log_info(v) for k, v in logs.items()}
    A_of = {k: v.n_activities for k, v in logs.items()}
    reqs = serve.poisson_requests(np.random.default_rng(220404898 + 55), rate=200.0, seconds=1.15, logs=info,
                                  A_of=A_of)
    assert len(reqs) >= 200
    note(f"serving {len(reqs)} requests over the 10M- and 99M-event logs")
    ex = serve.GpuExecutor(preps, variants_top=TOP)
    free, _ = torch.cuda.mem_get_info()
    sch = serve.Scheduler(ex, mem_budget=int(free * 0.8), max_batch=64, workers=4, max_batch_work=20_000_000)
    done = sch.run(copy.deepcopy(reqs))
    assert all(r.error is None for r in done), [r.error for r in done if r.error][:3]
    del preps, ex
    note("oracle: formatted logs, then every answer")
    with cf.ThreadPoolExecutor(2) as pool:
        fut = {k: pool.submit(oracle.prepare, v.case, v.act, v.ts, v.n_activities) for k, v in logs.items()}
        opreps = {k: f.result() for k, f in fut.items()}
    with cf.ThreadPoolExecutor(8) as pool:
        kinds = list(pool.map(lambda r: _oracle_check(opreps[r.log], A_of[r.log], r, r.result), done))
    assert {"dfg", "filter", "variants"} <= set(kinds)
    note(f"checked {len(kinds)} answers")
