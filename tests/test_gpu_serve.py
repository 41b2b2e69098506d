"""Serving on the GPU: results of requests served in the continuous-batching
mix are bit-identical to the same requests served alone, and match the
oracle."""
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


def _oracle_check(log, r, res):
    A = log.n_activities
    if r.kind in ("dfg", "filter"):
        ref = oracle.view(log.case, log.act, log.ts, A, r.case_lo, r.case_hi, r.t_lo, r.t_hi, r.mask)
        assert res["n_events"] == ref["n_events"] and res["n_cases"] == ref["n_cases"]
        if r.kind == "dfg":
            nz = np.flatnonzero(ref["count"].ravel())
            assert np.array_equal(res["count"], ref["count"].ravel()[nz])
            assert np.array_equal(res["dt_sum"], ref["dt_sum"].ravel()[nz])
            assert np.array_equal(res["src"] * A + res["dst"], nz)
            assert np.array_equal(res["start_count"], ref["start_count"])
    else:
        keep = ((log.case >= r.case_lo) & (log.case < r.case_hi) & (log.ts >= r.t_lo) & (log.ts <= r.t_hi)
                & ((r.mask[log.act // 64] >> (log.act % 64).astype(np.uint64)) & np.uint64(1)).astype(bool))
        ref = oracle.variants(log.case[keep], log.act[keep], log.ts[keep], A)
        assert res["n_variants"] == ref["n_variants"]
        assert res["n_events"] == int(keep.sum())
        K = min(TOP, ref["n_variants"])     # the answer carries the first TOP variants
        for k in ("var_count", "var_len", "var_rep"):
            assert np.array_equal(res[k], ref[k][:K]), k
        assert np.array_equal(res["var_off"], ref["var_off"][:K + 1])
        assert np.array_equal(res["var_acts"], ref["var_acts"][:ref["var_off"][K]])


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
    for r0, rm in zip(reqs, mixed):
        alone = copy.deepcopy(r0)
        ex.run([alone])
        assert _same(alone.result, rm.result), rm.rid
        _oracle_check(logs[rm.log], rm, rm.result)
    st = serve.latency_stats(mixed)
    assert st["n"] == len(reqs)
