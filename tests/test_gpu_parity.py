"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, bit-exact (every output is an integer or a correctly
rounded FP64 function of identical integers)."""
import glob
import zlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import (assert_dfg_equal, check_dfg, check_prepare, check_variants, cols,
                            gpu_dfg, note)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INT64_MAX = np.iinfo(np.int64).max


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "worked_*.json"))),
                         ids=lambda p: os.path.basename(p))
def test_golden(path):
    g = json.load(open(path))
    r, A = g["rows"], g["A"]
    note(f"golden {os.path.basename(path)}")
    check_dfg(r["case"], r["act"], r["ts"], A)
    check_prepare(r["case"], r["act"], r["ts"], A)
    if "variants" in g["expected"]:
        check_variants(r["case"], r["act"], r["ts"], A)


@pytest.mark.parametrize("k,scale", [(1, 1.0), (2, 0.02), (3, 0.005), (3, 0.03)])
def test_workloads_scaled(k, scale):
    log = synth.config_log(k, scale)
    note(f"workload {k} scale {scale}: N={log.n_events} A={log.n_activities}")
    A = log.n_activities
    check_prepare(log.case, log.act, log.ts, A, presorted=log.presorted)
    check_dfg(log.case, log.act, log.ts, A, presorted=log.presorted)
    check_variants(log.case, log.act, log.ts, A, presorted=log.presorted)
    if log.presorted:   # same results without the promise
        check_dfg(log.case, log.act, log.ts, A, presorted=False)


def _rand_log(rng, n, A, case_pool, t_lo, t_hi):
    case = rng.choice(np.asarray(case_pool, np.int64), n).astype(np.int32)
    act = rng.integers(0, A, n).astype(np.int32)
    ts = rng.integers(t_lo, t_hi, n, dtype=np.int64)
    return case, act, ts


EDGE = {
    "empty": lambda r: (np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 3),
    "one": lambda r: (np.array([7], np.int32), np.array([2], np.int32), np.array([5], np.int64), 3),
    "A1": lambda r: (*_rand_log(r, 5000, 1, range(-50, 50), 0, 100), 1),
    "single_event_cases": lambda r: (r.permutation(20000).astype(np.int32) - 10000,
                                     r.integers(0, 9, 20000).astype(np.int32),
                                     r.integers(-10**15, 10**15, 20000, dtype=np.int64), 9),
    "equal_ts": lambda r: (*_rand_log(r, 30000, 6, range(-40, 40), 42, 43), 6),
    "sparse_extreme_ids": lambda r: (*_rand_log(r, 30000, 5, [-2**31, -2**31 + 1, -7, 0, 9, 2**20, 2**31 - 2, 2**31 - 1],
                                                -5, 5), 5),
    "ties_many": lambda r: (*_rand_log(r, 50000, 12, range(0, 3000), 0, 4), 12),
    "A65_partition": lambda r: (*_rand_log(r, 60000, 65, range(0, 5000), 0, 10**9), 65),
    "A4096": lambda r: (*_rand_log(r, 40000, 4096, range(0, 3000), 0, 10**12), 4096),
    "wide_ts_overflow": lambda r: (*_rand_log(r, 4000, 4, range(0, 10), -2**62, 2**62), 4),
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_cases(name):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    case, act, ts, A = EDGE[name](rng)
    note(f"edge case {name}: N={case.size} A={A}")
    g = check_dfg(case, act, ts, A)
    if name == "wide_ts_overflow":
        assert g["overflow"] == 1
    check_prepare(case, act, ts, A)
    check_variants(case, act, ts, A)


def test_long_cases_fallback():
    """Cases longer than the LDS window take the full-key sort."""
    rng = np.random.default_rng(5)
    lens = [1, 5000, 3, 2049, 2050, 10000, 7] + list(rng.integers(1, 30, 500))
    case = np.repeat(np.arange(len(lens), dtype=np.int32) * 3 - 700, lens)
    n = case.size
    act = rng.integers(0, 40, n).astype(np.int32)
    ts = rng.integers(0, 5000, n, dtype=np.int64)      # many ties inside the long cases
    perm = rng.permutation(n)
    note(f"long cases: N={n}")
    check_prepare(case[perm], act[perm], ts[perm], 40)
    check_dfg(case[perm], act[perm], ts[perm], 40)
    check_variants(case[perm], act[perm], ts[perm], 40)


def test_case_of_2049_events_stays_on_fast_path():
    rng = np.random.default_rng(6)
    lens = [2049] * 6 + list(rng.integers(1, 50, 300))
    case = np.repeat(np.arange(len(lens), dtype=np.int32), lens)
    act = rng.integers(0, 16, case.size).astype(np.int32)
    ts = rng.integers(0, 10**6, case.size, dtype=np.int64)
    perm = rng.permutation(case.size)
    check_prepare(case[perm], act[perm], ts[perm], 16)
    check_dfg(case[perm], act[perm], ts[perm], 16)


def test_activity_out_of_range_is_reported():
    case = np.array([0, 0, 1], np.int32)
    ts = np.array([1, 2, 3], np.int64)
    for bad in (3, -1):
        act = np.array([0, bad, 1], np.int32)
        c, a, t = cols(case, act, ts)
        with pytest.raises(pm4g.Pm4gError) as e:
            pm4g.pm4g_dfg(c, a, t, 3)
        assert e.value.code == pm4g.PM4G_E_RANGE
        out = pm4g._dfg_out(3, "cuda:0")
        with pytest.raises(pm4g.Pm4gError):
            pm4g.pm4g_dfg(c, a, t, 3, out=out)
        assert int(out["status"].item()) == pm4g.PM4G_E_RANGE


def test_false_presorted_claim_is_reported():
    log = synth.config_log(1, 0.05)
    perm = np.random.default_rng(1).permutation(log.n_events)
    c, a, t = cols(log.case[perm], log.act[perm], log.ts[perm])
    with pytest.raises(pm4g.Pm4gError) as e:
        pm4g.pm4g_dfg(c, a, t, 16, presorted=True)
    assert e.value.code == pm4g.PM4G_E_NOT_SORTED
    # equal (case, ts) pairs in row order are a valid claim
    case = np.array([1, 1, 1, 2], np.int32)
    ts = np.array([5, 5, 6, 0], np.int64)
    act = np.array([2, 0, 1, 1], np.int32)
    g = gpu_dfg(case, act, ts, 3, presorted=True)
    assert_dfg_equal(g, oracle.dfg(case, act, ts, 3), 3)


def test_forced_hash_collisions():
    """Truncated hashes put different sequences in one run; grouping stays exact."""
    log = synth.config_log(2, 0.01)
    for bits in (1, 3, 7):
        old = pm4g.debug_variant_hash_bits(bits)
        try:
            note(f"hash bits {bits}")
            check_variants(log.case, log.act, log.ts, log.n_activities)
        finally:
            pm4g.debug_variant_hash_bits(old)


def test_prepared_entry_points_and_determinism():
    log = synth.config_log(3, 0.01)
    A = log.n_activities
    c, a, t = cols(log.case, log.act, log.ts)
    p = pm4g.pm4g_prepare(c, a, t, A)
    d1 = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(p), A)
    d2 = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(p), A)
    o = oracle.dfg(log.case, log.act, log.ts, A)
    assert_dfg_equal(d1, o, A)
    for k in ("count", "dt_sum", "dt_min", "dt_max"):
        assert np.array_equal(d1[k], d2[k])
    v1 = pm4g.variants_to_host(pm4g.pm4g_variants_prepared(p), int(p.n_cases.item()))
    v2 = pm4g.variants_to_host(pm4g.pm4g_variants_prepared(p), int(p.n_cases.item()))
    for k in ("var_count", "var_acts", "case_variant"):
        assert np.array_equal(v1[k], v2[k])


def test_side_stream():
    log = synth.config_log(2, 0.005)
    s = torch.cuda.Stream()
    c, a, t = cols(log.case, log.act, log.ts)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        o = pm4g.pm4g_dfg(c, a, t, log.n_activities)
    s.synchronize()
    assert_dfg_equal(pm4g.dfg_to_host(o, log.n_activities),
                     oracle.dfg(log.case, log.act, log.ts, log.n_activities), log.n_activities)
