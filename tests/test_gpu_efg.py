"""Eventually-follows graph and temporal profile on the GPU against the oracle,
bit-exact: counts, the 128-bit gap and squared-gap sums, and the FP64 mean and
standard deviation, on one LDS table (A*A <= 4096) and on bucketed source
activities (A = 100, 512, 4096), with ns gaps whose squares need 128 bits, a
long case, multi-pass accumulation, and degenerate logs."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import cols, note, same_f64

pytestmark = pytest.mark.gpu


def _gpu_efg(case, act, ts, A):
    c, a, t = cols(case, act, ts)
    p = pm4g.pm4g_prepare(c, a, t, A)
    o = pm4g.pm4g_efg(p)
    torch.cuda.synchronize()
    return pm4g.efg_to_host(o, A)


def _check(case, act, ts, A):
    g = _gpu_efg(case, act, ts, A)
    o = oracle.efg(case, act, ts, A)
    assert g["status"] == 0
    assert g["n_pairs"] == o["n_pairs"]
    for k in ("count", "sum_lo", "sum_hi", "sq_lo", "sq_hi"):
        assert np.array_equal(g[k], o[k]), k
    for k in ("mean", "std"):
        assert same_f64(g[k], o[k]), k
    return g, o


def test_golden_road_fines():
    gd = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_road_fines.json")))
    r, A = gd["rows"], gd["A"]
    g, _ = _check(np.array(r["case"]), np.array(r["act"]), np.array(r["ts"]), A)
    assert g["n_pairs"] == gd["efg"]["n_pairs"]
    for x, y, n, s, q in gd["efg"]["cells"]:
        assert (g["count"][x, y], g["sum_lo"][x, y], g["sq_lo"][x, y]) == (n, s, q)


@pytest.mark.parametrize("k,scale", [(1, 0.3), (2, 0.01), (3, 0.002)])
def test_workloads(k, scale):
    log = synth.config_log(k, scale)
    note(f"efg: config {k} scale {scale}: N={log.n_events} A={log.n_activities}")
    _, o = _check(log.case, log.act, log.ts, log.n_activities)
    if k == 3:
        assert (o["sq_hi"] > 0).any()     # ns gaps: the squares use the high word


@pytest.mark.parametrize("A", [100, 4096])
def test_bucket_shapes(A):
    # A = 100: buckets of 40 source activities, the last one partial; A = 4096: one each
    rng = np.random.default_rng(A)
    n = 60_000
    case = rng.integers(0, 3000, n)
    act = rng.integers(0, A, n)
    ts = rng.integers(0, 10**6, n)
    _check(case, act, ts, A)


def test_long_case_and_multi_pass_accumulation():
    rng = np.random.default_rng(5)
    L = 3000                                          # 4.5M pairs in one case
    case = np.r_[np.zeros(L, np.int64), rng.integers(1, 500, 20_000)]
    act = rng.integers(0, 64, case.size)
    ts = rng.integers(-(2**40), 2**40, case.size)
    _check(case, act, ts, 64)
    old = pm4g.load().pm4g_debug_efg_pass_pairs(1000)  # many LDS passes per plan entry
    try:
        _check(case, act, ts, 64)
        log = synth.config_log(3, 0.001)
        _check(log.case, log.act, log.ts, log.n_activities)
    finally:
        pm4g.load().pm4g_debug_efg_pass_pairs(old)


def test_degenerate_logs():
    e = np.zeros(0, np.int64)
    g, _ = _check(e, e, e, 8)
    assert g["n_pairs"] == 0 and np.isnan(g["mean"]).all()
    n = 5000                                          # single-event cases: no pairs
    g, _ = _check(np.arange(n), np.arange(n) % 7, np.arange(n), 7)
    assert g["n_pairs"] == 0
    # one activity, equal gaps: std exactly 0 for gap-1 pairs... all gaps k: closed form
    L = 50
    g, _ = _check(np.zeros(L, np.int64), np.zeros(L, np.int64), 7 * np.arange(L), 1)
    assert g["count"][0, 0] == L * (L - 1) // 2 and g["sum_lo"][0, 0] == 7 * L * (L * L - 1) // 6


def test_wide_gaps_carry_into_high_words():
    # gaps up to about 2^63: the gap sums pass 2^64 and every square needs 128 bits
    rng = np.random.default_rng(17)
    n = 4000
    case = rng.integers(0, 40, n)
    act = rng.integers(0, 5, n)
    ts = rng.integers(-(2**62), 2**62, n)
    g, o = _check(case, act, ts, 5)
    assert (o["sum_hi"] > 0).any() and (o["sq_hi"] > 0).any()
    t = np.array([-(2**62), 0, 2**62 - 1, 2**62])
    _check(np.ones(4, np.int64), np.zeros(4, np.int64), t, 1)
