"""Pins of the CPU oracle against things other than itself.

- hand-worked examples (tests/golden/*.json), each citing the passage it follows;
- a literal brute force of the definitions on tiny random logs (hypothesis);
- invariants that hold at any size (I1-I7), special cases with closed forms
  (S1-S6), the paper's own replication relation (Sec. 4: replicating cases
  leaves variants and activities unchanged) and metamorphic relations;
- the sort cross-checked against numpy's stable lexsort on the same key.
"""
import glob
import json
import math
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2204_04898_amd import synth
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INT64_MAX = np.iinfo(np.int64).max
INT64_MIN = np.iinfo(np.int64).min


def _cells_dense(cells, A):
    cnt = np.zeros((A, A), np.int64)
    s = np.zeros((A, A), np.int64)
    mn = np.full((A, A), INT64_MAX, np.int64)
    mx = np.full((A, A), INT64_MIN, np.int64)
    mean = np.full((A, A), np.nan)
    for c in cells:
        x, y = c["src"], c["dst"]
        cnt[x, y], s[x, y], mn[x, y], mx[x, y], mean[x, y] = c["count"], c["sum"], c["min"], c["max"], c["mean"]
    return cnt, s, mn, mx, mean


def _same_float(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.array_equal(a.view(np.int64), b.view(np.int64)) or np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "worked_*.json"))),
                         ids=lambda p: os.path.basename(p))
def test_golden_worked_examples(path):
    g = json.load(open(path))
    A = g["A"]
    r = g["rows"]
    e = g["expected"]
    d = oracle.dfg(r["case"], r["act"], r["ts"], A, with_perm=True)
    cnt, s, mn, mx, mean = _cells_dense(e["cells"], A)
    assert d["perm"].tolist() == e["perm"]
    assert np.array_equal(d["count"], cnt)
    assert np.array_equal(d["dt_sum"], s)
    assert np.array_equal(d["dt_min"], mn)
    assert np.array_equal(d["dt_max"], mx)
    assert np.array_equal(d["dt_mean"], mean, equal_nan=True)
    assert d["act_count"].tolist() == e["act_count"]
    assert d["start_count"].tolist() == e["start_count"]
    assert d["end_count"].tolist() == e["end_count"]
    assert d["n_cases"] == e["n_cases"]
    assert d["overflow"] == e["overflow"]
    if "case_code" in e:
        p = oracle.prepare(r["case"], r["act"], r["ts"], A)
        assert p["case_code"].tolist() == e["case_code"]
        assert p["case_off"].tolist() == e["case_off"]
        assert p["row"].tolist() == e["perm"]
    if "variants" in e:
        v = oracle.variants(r["case"], r["act"], r["ts"], A)
        ev = e["variants"]
        for k in ("var_count", "var_len", "var_rep", "var_off", "var_acts", "case_variant"):
            assert v[k].tolist() == ev[k], k
        assert v["n_variants"] == ev["n_variants"]
    if "view" in g:
        w = g["view"]
        mask = np.zeros((A + 63) // 64, np.uint64)
        for a in w["subset"]:
            mask[a // 64] |= np.uint64(1) << np.uint64(a % 64)
        o = oracle.view(r["case"], r["act"], r["ts"], A, w["case_lo"], w["case_hi"], w["t_lo"], w["t_hi"], mask)
        ew = w["expected"]
        cnt, s, mn, mx, mean = _cells_dense(ew["cells"], A)
        assert np.array_equal(o["count"], cnt) and np.array_equal(o["dt_sum"], s)
        assert np.array_equal(o["dt_min"], mn) and np.array_equal(o["dt_max"], mx)
        assert np.array_equal(o["dt_mean"], mean, equal_nan=True)
        for k in ("act_count", "start_count", "end_count"):
            assert o[k].tolist() == ew[k], k
        assert o["n_events"] == ew["n_events"] and o["n_cases"] == ew["n_cases"]


# ---- brute force on tiny logs ---------------------------------------------

CASE_POOL = [-2**31, -7, -1, 0, 3, 4, 1000, 2**31 - 1]


@st.composite
def tiny_logs(draw, max_n=24):
    A = draw(st.integers(1, 5))
    n = draw(st.integers(0, max_n))
    codes = draw(st.lists(st.sampled_from(CASE_POOL), min_size=1, max_size=4, unique=True))
    wide = draw(st.booleans())
    if wide:
        tvals = st.integers(-2**62, 2**62)
    else:
        tvals = st.integers(-3, 3)    # many ties
    case = [draw(st.sampled_from(codes)) for _ in range(n)]
    act = [draw(st.integers(0, A - 1)) for _ in range(n)]
    ts = [draw(tvals) for _ in range(n)]
    return case, act, ts, A


def _check_dfg_against_bf(case, act, ts, A):
    d = oracle.dfg(case, act, ts, A)
    b = bf.dfg(case, act, ts, A)
    assert d["count"].tolist() == b["count"]
    assert d["dt_sum"].tolist() == b["dt_sum"]
    assert d["dt_min"].tolist() == b["dt_min"]
    assert d["dt_max"].tolist() == b["dt_max"]
    assert _same_float(d["dt_mean"], b["dt_mean"])
    assert d["act_count"].tolist() == b["act_count"]
    assert d["start_count"].tolist() == b["start_count"]
    assert d["end_count"].tolist() == b["end_count"]
    assert d["n_cases"] == b["n_cases"]
    assert d["overflow"] == b["overflow"]


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs())
def test_dfg_matches_bruteforce(log):
    _check_dfg_against_bf(*log)


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs())
def test_variants_match_bruteforce(log):
    case, act, ts, A = log
    v = oracle.variants(case, act, ts, A)
    b = bf.variants(case, act, ts)
    assert v["n_variants"] == b["n_variants"]
    assert v["var_count"].tolist() == b["var_count"]
    assert v["var_len"].tolist() == b["var_len"]
    assert v["var_rep"].tolist() == b["var_rep"]
    seqs = [v["var_acts"][v["var_off"][k]:v["var_off"][k + 1]].tolist() for k in range(v["n_variants"])]
    assert seqs == b["sequences"]
    assert v["case_code"].tolist() == b["case_code"]
    assert v["case_variant"].tolist() == b["case_variant"]


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs(), st.data())
def test_view_matches_bruteforce(log, data):
    case, act, ts, A = log
    lo = data.draw(st.sampled_from(CASE_POOL))
    hi = data.draw(st.sampled_from(CASE_POOL + [2**31 - 1]))
    t_lo = data.draw(st.integers(-2**62, 3))
    t_hi = data.draw(st.integers(-3, 2**62))
    subset = data.draw(st.sets(st.integers(0, A - 1)))
    mask = np.zeros((A + 63) // 64, np.uint64)
    for a in subset:
        mask[a // 64] |= np.uint64(1) << np.uint64(a % 64)
    b = bf.view(case, act, ts, A, lo, hi, t_lo, t_hi, subset)
    prep = oracle.prepare(case, act, ts, A)
    for o in (oracle.view(case, act, ts, A, lo, hi, t_lo, t_hi, mask),
              oracle.view_formatted(prep, A, lo, hi, t_lo, t_hi, mask)):
        for k in ("count", "dt_sum", "dt_min", "dt_max", "act_count", "start_count", "end_count"):
            assert o[k].tolist() == b[k], k
        assert _same_float(o["dt_mean"], b["dt_mean"])
        assert o["n_cases"] == b["n_cases"] and o["n_events"] == b["n_events"]
        assert o["overflow"] == b["overflow"]


@settings(max_examples=100, deadline=None)
@given(tiny_logs())
def test_prepare_order_is_definition(log):
    case, act, ts, A = log
    p = oracle.prepare(case, act, ts, A)
    n = len(case)
    # order: no later position precedes an earlier one (pairwise, by definition)
    rows = p["row"].tolist()
    for k in range(n - 1):
        assert bf.precedes(case, ts, rows[k], rows[k + 1])
    assert sorted(rows) == list(range(n))


def test_range_error():
    with pytest.raises(oracle.OracleError) as e:
        oracle.dfg([0, 0], [0, 3], [1, 2], 3)
    assert e.value.code == -2
    with pytest.raises(oracle.OracleError):
        oracle.dfg([0], [-1], [1], 3)


# ---- invariants at any size -------------------------------------------------

def check_invariants(log, d, v=None):
    A = log.n_activities
    N = log.n_events
    C = d["n_cases"]
    cnt = d["count"]
    assert cnt.sum() == N - C                                   # I1
    assert d["start_count"].sum() == C == d["end_count"].sum()  # I2
    assert np.array_equal(cnt.sum(axis=1) + d["end_count"], d["act_count"])    # I3
    assert np.array_equal(cnt.sum(axis=0) + d["start_count"], d["act_count"])  # I4
    assert d["act_count"].sum() == N                            # I5
    # I6 telescoping: the gap sums add up to the case spans (no overflow here)
    assert d["overflow"] == 0
    spans = 0
    ts = log.ts
    order = np.lexsort((np.arange(N), ts, log.case))
    cs = log.case[order]
    first = np.r_[True, cs[1:] != cs[:-1]] if N else np.zeros(0, bool)
    last = np.r_[cs[1:] != cs[:-1], True] if N else np.zeros(0, bool)
    spans = int(ts[order][last].astype(object).sum() - ts[order][first].astype(object).sum()) if N else 0
    assert int(d["dt_sum"].astype(object).sum()) == spans
    # I7
    nz = cnt > 0
    assert np.all(d["dt_min"][nz] >= 0)
    assert np.all(d["dt_min"][nz] <= d["dt_max"][nz])
    assert np.all(d["dt_min"][nz].astype(object) * cnt[nz] <= d["dt_sum"][nz].astype(object))
    assert np.all(d["dt_sum"][nz].astype(object) <= d["dt_max"][nz].astype(object) * cnt[nz])
    assert np.all(cnt[~nz] == 0) and np.all(d["dt_sum"][~nz] == 0)
    assert np.all(d["dt_min"][~nz] == INT64_MAX) and np.all(d["dt_max"][~nz] == INT64_MIN)
    assert np.all(np.isnan(d["dt_mean"][~nz]))
    if v is not None:
        assert v["var_count"].sum() == C                                           # I8
        assert int((v["var_count"] * v["var_len"]).sum()) == N
        # I9: DFG and endpoints rebuilt from (sequence, count) equal the DFG's
        cnt2 = np.zeros((A, A), np.int64)
        st_ = np.zeros(A, np.int64)
        en_ = np.zeros(A, np.int64)
        for k in range(v["n_variants"]):
            seq = v["var_acts"][v["var_off"][k]:v["var_off"][k + 1]]
            n_k = v["var_count"][k]
            st_[seq[0]] += n_k
            en_[seq[-1]] += n_k
            np.add.at(cnt2, (seq[:-1], seq[1:]), n_k)
        assert np.array_equal(cnt2, cnt)
        assert np.array_equal(st_, d["start_count"]) and np.array_equal(en_, d["end_count"])
        # I10: order (count desc, rep asc) and case_variant[rep] = v
        key = list(zip((-v["var_count"]).tolist(), v["var_rep"].tolist()))
        assert key == sorted(key) and len(set(v["var_rep"].tolist())) == v["n_variants"]
        pos = {c: j for j, c in enumerate(v["case_code"].tolist())}
        for k in range(v["n_variants"]):
            assert v["case_variant"][pos[int(v["var_rep"][k])]] == k


@pytest.mark.parametrize("k,scale", [(1, 1.0), (2, 0.01), (3, 0.002)])
def test_invariants_on_workloads(k, scale):
    log = synth.config_log(k, scale)
    d = oracle.dfg(log.case, log.act, log.ts, log.n_activities)
    v = oracle.variants(log.case, log.act, log.ts, log.n_activities)
    check_invariants(log, d, v)


def test_sort_matches_numpy_lexsort():
    log = synth.config_log(2, 0.005)    # 5% duplicate timestamps: row tie-break matters
    d = oracle.dfg(log.case, log.act, log.ts, log.n_activities, with_perm=True)
    ref = np.lexsort((np.arange(log.n_events), log.ts, log.case))
    assert np.array_equal(d["perm"], ref)


# ---- special cases ------------------------------------------------------------

def test_s1_single_event_cases():
    rng = np.random.default_rng(1)
    n, A = 500, 7
    case = rng.permutation(n).astype(np.int32) - 250
    act = rng.integers(0, A, n).astype(np.int32)
    ts = rng.integers(-10**12, 10**12, n)
    d = oracle.dfg(case, act, ts, A)
    assert d["count"].sum() == 0
    assert np.array_equal(d["start_count"], d["act_count"])
    assert np.array_equal(d["end_count"], d["act_count"])
    assert d["n_cases"] == n


def test_s2_chain():
    A = 9
    rng = np.random.default_rng(2)
    rows = rng.permutation(A)
    case = np.zeros(A, np.int32)
    act = np.arange(A, dtype=np.int32)[rows]
    ts = (np.arange(A, dtype=np.int64) * 10 + 5)[rows]
    d = oracle.dfg(case, act, ts, A)
    expect = np.zeros((A, A), np.int64)
    expect[np.arange(A - 1), np.arange(1, A)] = 1
    assert np.array_equal(d["count"], expect)
    assert np.array_equal(d["dt_sum"][expect == 1], np.full(A - 1, 10))


def test_s3_same_sequence():
    seq = [2, 0, 0, 1, 2]
    C = 37
    case = np.repeat(np.arange(C, dtype=np.int32) * 3 - 40, len(seq))
    act = np.tile(np.array(seq, np.int32), C)
    ts = np.tile(np.arange(len(seq), dtype=np.int64), C) + np.repeat(np.arange(C) * 1000, len(seq))
    perm = np.random.default_rng(3).permutation(case.size)
    v = oracle.variants(case[perm], act[perm], ts[perm], 3)
    assert v["n_variants"] == 1 and v["var_count"].tolist() == [C]
    assert v["var_acts"].tolist() == seq and v["var_rep"].tolist() == [-40]


def test_s4_constant_gap():
    log = synth.config_log(1, 0.05)
    g = 777
    # rebuild the timestamps as case start + g * position, positions in row order
    ts = np.zeros(log.n_events, np.int64)
    pos = {}
    for i, c in enumerate(log.case.tolist()):
        pos[c] = pos.get(c, -1) + 1
        ts[i] = 10**9 + g * pos[c]
    d = oracle.dfg(log.case, log.act, ts, log.n_activities)
    nz = d["count"] > 0
    assert np.array_equal(d["dt_sum"][nz], g * d["count"][nz])
    assert np.all(d["dt_min"][nz] == g) and np.all(d["dt_max"][nz] == g)
    assert np.all(d["dt_mean"][nz] == float(g))


def test_s5_all_equal_timestamps_row_order():
    rng = np.random.default_rng(5)
    n = 300
    case = rng.integers(-5, 5, n).astype(np.int32)
    act = rng.integers(0, 4, n).astype(np.int32)
    ts = np.full(n, 42, np.int64)
    d = oracle.dfg(case, act, ts, 4, with_perm=True)
    assert np.array_equal(d["perm"], np.argsort(case, kind="stable"))


def test_s6_empty_and_tiny():
    d = oracle.dfg([], [], [], 3)
    assert d["n_cases"] == 0 and d["count"].sum() == 0 and d["overflow"] == 0
    assert np.all(d["dt_min"] == INT64_MAX) and np.all(d["dt_max"] == INT64_MIN)
    v = oracle.variants([], [], [], 3)
    assert v["n_variants"] == 0 and v["n_cases"] == 0
    d = oracle.dfg([5], [2], [7], 3)
    assert d["n_cases"] == 1 and d["start_count"].tolist() == [0, 0, 1] == d["end_count"].tolist()


def test_overflow_flag_exact_boundary():
    # total span exactly INT64_MAX: no overflow; one more: overflow
    half = INT64_MAX // 2
    d = oracle.dfg([0, 0, 1, 1], [0, 0, 0, 0], [0, half, 0, INT64_MAX - half], 1)
    assert d["overflow"] == 0 and int(d["dt_sum"][0, 0]) == INT64_MAX
    d = oracle.dfg([0, 0, 1, 1], [0, 0, 0, 0], [0, half, 0, INT64_MAX - half + 1], 1)
    assert d["overflow"] == 1 and int(d["dt_sum"][0, 0]) == INT64_MIN


# ---- replication (Sec. 4) and metamorphic relations -------------------------------

def test_replication_relation():
    log = synth.config_log(3, 0.0004)
    A = log.n_activities
    k = 3
    C = int(log.case.max()) + 1
    case = np.concatenate([log.case + j * C for j in range(k)]).astype(np.int32)
    act = np.tile(log.act, k)
    ts = np.tile(log.ts, k)
    d1 = oracle.dfg(log.case, log.act, log.ts, A)
    dk = oracle.dfg(case, act, ts, A)
    for key in ("count", "dt_sum", "start_count", "end_count", "act_count"):
        assert np.array_equal(dk[key], k * d1[key]), key
    assert np.array_equal(dk["dt_min"], d1["dt_min"]) and np.array_equal(dk["dt_max"], d1["dt_max"])
    v1 = oracle.variants(log.case, log.act, log.ts, A)
    vk = oracle.variants(case, act, ts, A)
    assert vk["n_variants"] == v1["n_variants"]
    assert np.array_equal(vk["var_count"], k * v1["var_count"])
    for key in ("var_len", "var_rep", "var_off", "var_acts"):
        assert np.array_equal(vk[key], v1[key]), key


def test_metamorphic_relabel_shift_permute():
    log = synth.config_log(3, 0.0004)     # ns gaps: no timestamp ties within a case
    A = log.n_activities
    d = oracle.dfg(log.case, log.act, log.ts, A)
    rng = np.random.default_rng(11)
    pi = rng.permutation(A)
    dr = oracle.dfg(log.case, pi[log.act].astype(np.int32), log.ts, A)
    inv = np.argsort(pi)
    for key in ("count", "dt_sum", "dt_min", "dt_max"):
        assert np.array_equal(dr[key][np.ix_(pi, pi)], d[key]), key
    assert np.array_equal(dr["start_count"][pi], d["start_count"])
    assert np.array_equal(inv[pi], np.arange(A))
    ds = oracle.dfg(log.case, log.act, log.ts - 123456789, A)
    for key in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
        assert np.array_equal(ds[key], d[key]), key
    perm = rng.permutation(log.n_events)
    dp = oracle.dfg(log.case[perm], log.act[perm], log.ts[perm], A)
    for key in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
        assert np.array_equal(dp[key], d[key]), key


def test_view_unfiltered_equals_plain_and_additivity():
    log = synth.config_log(2, 0.002)
    A = log.n_activities
    W = (A + 63) // 64
    full = np.full(W, np.uint64(0xFFFFFFFFFFFFFFFF))
    d = oracle.dfg(log.case, log.act, log.ts, A)
    o = oracle.view(log.case, log.act, log.ts, A, -2**31, 2**31 - 1, INT64_MIN, INT64_MAX, full)
    for key in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
        assert np.array_equal(o[key], d[key]), key
    assert o["n_events"] == log.n_events
    C = int(log.case.max()) + 1
    mid = C // 3
    a = oracle.view(log.case, log.act, log.ts, A, 0, mid, INT64_MIN, INT64_MAX, full)
    b = oracle.view(log.case, log.act, log.ts, A, mid, C, INT64_MIN, INT64_MAX, full)
    assert np.array_equal(a["count"] + b["count"], d["count"])
    assert np.array_equal(a["dt_sum"] + b["dt_sum"], d["dt_sum"])
    assert np.array_equal(np.minimum(a["dt_min"], b["dt_min"]), d["dt_min"])
    assert np.array_equal(np.maximum(a["dt_max"], b["dt_max"]), d["dt_max"])
    assert a["n_cases"] + b["n_cases"] == d["n_cases"]



def test_view_formatted_equals_view_on_workload_views():
    """The scan of the formatted log gives the same view as filtering the raw
    log and formatting the kept events from scratch, on workload-shaped views
    (including empty ranges, a full range and a sign-bit case range)."""
    log = synth.config_log(3, 0.002)
    A = log.n_activities
    prep = oracle.prepare(log.case, log.act, log.ts, A)
    views = synth.make_views(log, 40, seed=7, min_events=10, max_events=20_000)
    W = (A + 63) // 64
    full = np.full(W, np.uint64(0xFFFFFFFFFFFFFFFF))
    extra = [(0, 0, INT64_MIN, INT64_MAX, full), (5, 3, INT64_MIN, INT64_MAX, full),
             (-2**31, 2**31 - 1, INT64_MIN, INT64_MAX, full), (-2**31, 100, INT64_MIN, INT64_MAX, full),
             (int(log.case.max()), 2**31 - 1, INT64_MIN, INT64_MAX, full)]
    cases = [(int(views.case_lo[v]), int(views.case_hi[v]), int(views.t_lo[v]), int(views.t_hi[v]),
              views.masks[v]) for v in range(views.n_views)] + extra
    for lo, hi, t_lo, t_hi, mask in cases:
        a = oracle.view(log.case, log.act, log.ts, A, lo, hi, t_lo, t_hi, mask)
        b = oracle.view_formatted(prep, A, lo, hi, t_lo, t_hi, mask)
        for key in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
            assert np.array_equal(a[key], b[key]), (lo, hi, key)
        assert _same_float(a["dt_mean"], b["dt_mean"])
        assert (a["n_events"], a["n_cases"], a["overflow"]) == (b["n_events"], b["n_cases"], b["overflow"])
    d = oracle.dfg(log.case, log.act, log.ts, A)
    u = oracle.view_formatted(prep, A, -2**31, 2**31 - 1, INT64_MIN, INT64_MAX, full)
    for key in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
        assert np.array_equal(u[key], d[key]), key
    with pytest.raises(oracle.OracleError):
        bad = dict(prep)
        bad["act_s"] = prep["act_s"].copy()
        bad["act_s"][0] = A
        oracle.view_formatted(bad, A, -2**31, 2**31 - 1, INT64_MIN, INT64_MAX, full)


def test_oracle_calls_from_concurrent_threads_match_sequential_calls():
    """The oracle's functions give the same results when several host threads
    call them at once (the variant sort's comparator context is per thread)."""
    import concurrent.futures as cf
    logs = [synth.config_log(3, 0.001 * (k + 1)) for k in range(6)]
    seq = [oracle.variants(g.case, g.act, g.ts, g.n_activities) for g in logs]
    with cf.ThreadPoolExecutor(6) as ex:
        par = list(ex.map(lambda g: oracle.variants(g.case, g.act, g.ts, g.n_activities), logs * 2))
    for k, p in enumerate(par):
        s = seq[k % len(logs)]
        for key in ("var_count", "var_len", "var_rep", "var_off", "var_acts", "case_variant"):
            assert np.array_equal(p[key], s[key]), (k, key)

def test_generators_are_seeded_and_shaped():
    a = synth.config_log(2, 0.01)
    b = synth.config_log(2, 0.01)
    assert np.array_equal(a.case, b.case) and np.array_equal(a.act, b.act) and np.array_equal(a.ts, b.ts)
    assert abs(a.n_events / 10_000 - 10.0) < 0.5               # geometric mean 10
    c = synth.config_log(3, 0.002)
    assert 16.0 < c.n_events / 10_000 < 23.5                    # lognormal(ln 12, 1) mean ~19.8
    assert int(c.lengths_by_code.max()) <= 2000
    one = synth.config_log(1, 1.0)
    assert 95_000 < one.n_events < 105_000 and one.presorted


def test_generator_markov_chain_frequencies():
    """The sampled sequences follow pi0 and P (alias sampling), within 5 sigma."""
    rng = np.random.default_rng(123)
    A = 6
    pi0, P = synth.markov_chain(A, "zipf", rng)
    lengths = rng.geometric(0.2, size=60_000).astype(np.int64)
    acts = synth.markov_sequences(lengths, pi0, P, rng)
    off = np.zeros(lengths.size + 1, np.int64)
    np.cumsum(lengths, out=off[1:])
    first = acts[off[:-1]]
    f0 = np.bincount(first, minlength=A) / first.size
    assert np.all(np.abs(f0 - pi0) < 5 * np.sqrt(pi0 * (1 - pi0) / first.size) + 1e-9)
    nonfirst = np.ones(acts.size, bool)
    nonfirst[off[:-1]] = False
    idx = np.flatnonzero(nonfirst)
    prev, nxt = acts[idx - 1], acts[idx]
    T = np.zeros((A, A))
    np.add.at(T, (prev, nxt), 1)
    rows = T.sum(axis=1, keepdims=True)
    emp = T / rows
    sd = np.sqrt(P * (1 - P) / rows)
    assert np.all(np.abs(emp - P) < 5 * sd + 1e-9)
    for r in range(A):
        pr, al = synth.alias_table(P[r])
        q = pr / A
        np.add.at(q, al, (1 - pr) / A)
        assert np.allclose(q, P[r], atol=1e-12)


# ---- cases dataframe and case-level filters --------------------------------

def _mask(bits, nbits):
    m = np.zeros((nbits + 63) // 64, np.uint64)
    for b in bits:
        m[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    return m


def _golden_window_kw(f, A, n_variants):
    """Keywords of the time-window, start/end activity and variant filters of a
    golden filter entry."""
    kw = {}
    if "contain" in f:
        kw["contain_lo"], kw["contain_hi"] = f["contain"]
    if "meet" in f:
        kw["meet_lo"], kw["meet_hi"] = f["meet"]
    if "start_acts" in f:
        kw["start_mask"] = _mask(f["start_acts"], A)
    if "end_acts" in f:
        kw["end_mask"] = _mask(f["end_acts"], A)
    if "variants" in f:
        kw["variant_mask"] = _mask(f["variants"], n_variants)
        kw["n_variant_bits"] = n_variants
        kw["variant_keep"] = f["variant_keep"]
    return kw


def test_cases_golden():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_road_fines.json")))
    r, A = g["rows"], g["A"]
    o = oracle.cases(r["case"], r["act"], r["ts"], A)
    for k, v in g["cases"]["expected"].items():
        assert o[k].tolist() == v, k
    for f in g["cases"]["filters"]:
        kw = {k: f[k] for k in ("min_events", "max_events", "min_thr", "max_thr") if k in f}
        if "activities" in f:
            kw["act_mask"] = _mask(f["activities"], A)
        if "paths" in f:
            kw["path_mask"] = _mask([x * A + y for x, y in f["paths"]], A * A)
            kw["path_keep"] = f["path_keep"]
        kw.update(_golden_window_kw(f, A, len(g["expected"]["variants"]["var_count"])))
        o = oracle.filter_cases(r["case"], r["act"], r["ts"], A, **kw)
        got = list(zip(o["case_s"].tolist(), o["act_s"].tolist(), o["ts_s"].tolist()))
        assert got == [tuple(e) for e in f["events"]], f["name"]
        assert o["n_cases"] == len(f["kept_cases"]), f["name"]
        assert sorted(set(o["case_s"].tolist())) == f["kept_cases"], f["name"]


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs())
def test_cases_match_bruteforce(log):
    case, act, ts, A = log
    o = oracle.cases(case, act, ts, A)
    b = bf.cases(case, act, ts)
    assert o["case_code"].tolist() == b["case_code"]
    assert o["n_events"].tolist() == b["n_events"]
    assert o["throughput"].tolist() == b["throughput"]


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs(), st.data())
def test_filter_cases_match_bruteforce(log, data):
    case, act, ts, A = log
    lo_e = data.draw(st.integers(0, 4))
    hi_e = data.draw(st.integers(lo_e, 30))
    lo_t = data.draw(st.sampled_from([oracle.I64_MIN, -5, 0, 1, 2**40]))
    hi_t = data.draw(st.sampled_from([oracle.I64_MAX, 0, 3, 2**61]))
    acts = data.draw(st.none() | st.sets(st.integers(0, A - 1)))
    paths = data.draw(st.none() | st.sets(st.tuples(st.integers(0, A - 1), st.integers(0, A - 1))))
    keep = data.draw(st.booleans())
    kw = dict(min_events=lo_e, max_events=hi_e, min_thr=lo_t, max_thr=hi_t, path_keep=keep)
    if acts is not None:
        kw["act_mask"] = _mask(acts, A)
    if paths is not None:
        kw["path_mask"] = _mask([x * A + y for x, y in paths], A * A)
    o = oracle.filter_cases(case, act, ts, A, **kw)
    ev, nc = bf.filter_cases(case, act, ts, lo_e, hi_e, lo_t, hi_t, acts, paths, keep)
    got = list(zip(o["case_s"].tolist(), o["act_s"].tolist(), o["ts_s"].tolist()))
    assert got == ev
    assert o["n_cases"] == nc and o["n_events"] == len(ev)


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs(), st.data())
def test_window_start_end_variant_filters_match_bruteforce(log, data):
    case, act, ts, A = log
    tv = sorted(set(int(x) for x in ts)) or [0]
    bound = st.sampled_from(tv) | st.integers(-2**62, 2**62)
    contain = data.draw(st.none() | st.tuples(bound, bound))
    meet = data.draw(st.none() | st.tuples(bound, bound))
    starts = data.draw(st.none() | st.sets(st.integers(0, A - 1)))
    ends = data.draw(st.none() | st.sets(st.integers(0, A - 1)))
    nv = oracle.variants(case, act, ts, A)["n_variants"]
    vbits = data.draw(st.integers(0, nv + 2))                # ids at or above it are outside the set
    vset = data.draw(st.none() | st.sets(st.integers(0, max(vbits - 1, 0))))
    if vset is not None:
        vset = {v for v in vset if v < vbits}
    vkeep = data.draw(st.booleans())
    kw = {}
    if contain is not None:
        kw["contain_lo"], kw["contain_hi"] = contain
    if meet is not None:
        kw["meet_lo"], kw["meet_hi"] = meet
    if starts is not None:
        kw["start_mask"] = _mask(starts, A)
    if ends is not None:
        kw["end_mask"] = _mask(ends, A)
    if vset is not None:
        kw.update(variant_mask=_mask(vset, max(vbits, 1)), n_variant_bits=vbits, variant_keep=vkeep)
    o = oracle.filter_cases(case, act, ts, A, **kw)
    ev, nc = bf.filter_cases(case, act, ts, 0, oracle.I64_MAX, oracle.I64_MIN, oracle.I64_MAX, contain=contain,
                             meet=meet, start_set=starts, end_set=ends, variant_set=vset, variant_keep=vkeep)
    got = list(zip(o["case_s"].tolist(), o["act_s"].tolist(), o["ts_s"].tolist()))
    assert got == ev
    assert o["n_cases"] == nc and o["n_events"] == len(ev)


def test_cases_invariants_on_workload():
    log = synth.config_log(2, 0.01)
    o = oracle.cases(log.case, log.act, log.ts, log.n_activities)
    assert o["n_events"].sum() == log.n_events
    assert (o["throughput"] >= 0).all()                    # timestamps ordered inside a case
    d = oracle.dfg(log.case, log.act, log.ts, log.n_activities)
    assert o["n_cases"] == d["n_cases"]
    # the whole log passes an unrestricted filter; a path set of every cell keeps the cases
    # with at least two events, and its complement keeps the single-event ones
    A = log.n_activities
    allp = _mask(range(A * A), A * A)
    f = oracle.filter_cases(log.case, log.act, log.ts, A)
    assert f["n_events"] == log.n_events and f["n_cases"] == o["n_cases"]
    k = oracle.filter_cases(log.case, log.act, log.ts, A, path_mask=allp, path_keep=True)
    d2 = oracle.filter_cases(log.case, log.act, log.ts, A, path_mask=allp, path_keep=False)
    assert k["n_cases"] == int((o["n_events"] >= 2).sum()) and d2["n_cases"] == int((o["n_events"] == 1).sum())
    assert k["n_events"] + d2["n_events"] == log.n_events

    # a variant set and its complement split the cases; keeping every variant keeps all
    v = oracle.variants(log.case, log.act, log.ts, A)
    nv = v["n_variants"]
    half = _mask(range(0, nv, 2), nv)
    kv = oracle.filter_cases(log.case, log.act, log.ts, A, variant_mask=half, n_variant_bits=nv, variant_keep=True)
    dv = oracle.filter_cases(log.case, log.act, log.ts, A, variant_mask=half, n_variant_bits=nv, variant_keep=False)
    assert kv["n_cases"] == int(v["var_count"][0::2].sum()) and kv["n_cases"] + dv["n_cases"] == o["n_cases"]
    assert kv["n_events"] == int((v["var_count"] * v["var_len"])[0::2].sum())
    # every case is contained in [min ts, max ts]; the start sets of all activities keep everything
    every = _mask(range(A), A)
    w = oracle.filter_cases(log.case, log.act, log.ts, A, contain_lo=int(log.ts.min()), contain_hi=int(log.ts.max()),
                            start_mask=every, end_mask=every)
    assert w["n_events"] == log.n_events
    # a case intersects a window iff it is not wholly before or wholly after it
    lo, hi = np.percentile(log.ts, [40, 60]).astype(np.int64).tolist()
    m = oracle.filter_cases(log.case, log.act, log.ts, A, meet_lo=lo, meet_hi=hi)
    before = oracle.filter_cases(log.case, log.act, log.ts, A, contain_hi=lo - 1)
    after = oracle.filter_cases(log.case, log.act, log.ts, A, contain_lo=hi + 1)
    assert m["n_cases"] + before["n_cases"] + after["n_cases"] == o["n_cases"]


# ---- directly-follows-level event filter ---------------------------------------

def _pairs_of(spec, A):
    return [(x, y) for x in range(A) for y in range(A)] if spec == "all" else [tuple(p) for p in spec]


def test_df_events_golden():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_road_fines.json")))
    r, A = g["rows"], g["A"]
    for f in g["df_events"]["filters"]:
        pm = _mask([x * A + y for x, y in _pairs_of(f["pairs"], A)], A * A)
        o = oracle.filter_df_events(r["case"], r["act"], r["ts"], A, pm, f["side"], f["keep"])
        got = list(zip(o["case_s"].tolist(), o["act_s"].tolist(), o["ts_s"].tolist()))
        assert got == [tuple(e) for e in f["events"]], f["name"]
        assert o["n_cases"] == f["n_cases"], f["name"]


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs(), st.data())
def test_df_events_match_bruteforce(log, data):
    case, act, ts, A = log
    pairs = data.draw(st.sets(st.tuples(st.integers(0, A - 1), st.integers(0, A - 1))))
    side = data.draw(st.sampled_from([0, 1]))
    keep = data.draw(st.booleans())
    o = oracle.filter_df_events(case, act, ts, A, _mask([x * A + y for x, y in pairs], A * A), side, keep)
    ev, nc = bf.filter_df_events(case, act, ts, pairs, side, keep)
    got = list(zip(o["case_s"].tolist(), o["act_s"].tolist(), o["ts_s"].tolist()))
    assert got == ev
    assert o["n_events"] == len(ev) and o["n_cases"] == nc


def test_df_events_invariants_on_workload():
    log = synth.config_log(2, 0.01)
    A = log.n_activities
    d = oracle.dfg(log.case, log.act, log.ts, A)
    rng = np.random.default_rng(7)
    cells = rng.choice(A * A, A, replace=False)
    pm = _mask(cells, A * A)
    # the events matched on either side number the DFG counts of the chosen cells
    expect = int(d["count"].reshape(-1)[cells].sum())
    for side in (0, 1):
        k = oracle.filter_df_events(log.case, log.act, log.ts, A, pm, side, True)
        dr = oracle.filter_df_events(log.case, log.act, log.ts, A, pm, side, False)
        assert k["n_events"] == expect
        assert k["n_events"] + dr["n_events"] == log.n_events
    # with every pair chosen, side 0 drops all but each case's first event and side 1
    # all but its last: the start and end activity counts
    allp = _mask(range(A * A), A * A)
    first = oracle.filter_df_events(log.case, log.act, log.ts, A, allp, 0, False)
    last = oracle.filter_df_events(log.case, log.act, log.ts, A, allp, 1, False)
    assert np.array_equal(np.bincount(first["act_s"], minlength=A), d["start_count"])
    assert np.array_equal(np.bincount(last["act_s"], minlength=A), d["end_count"])
    assert first["n_cases"] == last["n_cases"] == d["n_cases"]


# ---- eventually-follows graph and temporal profile -----------------------------

def _u128(lo, hi):
    return int(lo) + (int(hi) << 64)


def _efg_exact_stats(n, S, Q):
    """Mean and sample std of a cell from its exact sums, by exact rationals."""
    from fractions import Fraction
    if n == 0:
        return math.nan, math.nan
    mean = float(Fraction(S, n))
    if n == 1:
        return mean, 0.0
    return mean, math.sqrt(float(Fraction(n * Q - S * S, n * (n - 1))))


def _check_efg_stats(o, n, S, Q, x, y):
    em, es = _efg_exact_stats(n, S, Q)
    m, sd = float(o["mean"][x, y]), float(o["std"][x, y])
    if n == 0:
        assert math.isnan(m) and math.isnan(sd)
        return
    assert math.isclose(m, em, rel_tol=1e-15, abs_tol=0.0), (x, y, m, em)
    assert math.isclose(sd, es, rel_tol=1e-13, abs_tol=1e-300), (x, y, sd, es)


def test_efg_golden():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_road_fines.json")))
    r, A, e = g["rows"], g["A"], g["efg"]
    o = oracle.efg(r["case"], r["act"], r["ts"], A)
    assert o["n_pairs"] == e["n_pairs"]
    want = {(x, y): (n, s, q) for x, y, n, s, q in e["cells"]}
    for x in range(A):
        for y in range(A):
            n, s, q = want.get((x, y), (0, 0, 0))
            assert int(o["count"][x, y]) == n, (x, y)
            assert _u128(o["sum_lo"][x, y], o["sum_hi"][x, y]) == s, (x, y)
            assert _u128(o["sq_lo"][x, y], o["sq_hi"][x, y]) == q, (x, y)
            _check_efg_stats(o, n, s, q, x, y)
    cf = e["create_fine_to_payment"]
    assert math.isclose(o["mean"][0, 4], cf["mean"], rel_tol=1e-15)
    assert math.isclose(o["std"][0, 4], cf["std"], rel_tol=1e-15)


@settings(max_examples=250, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs())
def test_efg_match_bruteforce(log):
    case, act, ts, A = log
    o = oracle.efg(case, act, ts, A)
    b = bf.efg(case, act, ts, A)
    assert o["n_pairs"] == b["n_pairs"]
    for x in range(A):
        for y in range(A):
            n, S, Q = b["count"][x][y], b["S"][x][y], b["Q"][x][y]
            assert int(o["count"][x, y]) == n
            assert _u128(o["sum_lo"][x, y], o["sum_hi"][x, y]) == S
            assert _u128(o["sq_lo"][x, y], o["sq_hi"][x, y]) == Q % 2**128     # kept modulo 2^128
            if Q < 2**128:
                _check_efg_stats(o, n, S, Q, x, y)


@pytest.mark.parametrize("L,k", [(2, 1), (7, 3), (40, 1000), (200, 10**9)])
def test_efg_closed_form_one_activity(L, k):
    """One case of L events of one activity at 0, k, 2k, ...: the gap g*k occurs
    L - g times, so n = L(L-1)/2, S = k L(L^2-1)/6, Q = k^2 L^2(L^2-1)/12 and
    the mean is k(L+1)/3."""
    o = oracle.efg([5] * L, [0] * L, [k * i for i in range(L)], 1)
    n, S, Q = L * (L - 1) // 2, k * L * (L * L - 1) // 6, k * k * L * L * (L * L - 1) // 12
    assert int(o["count"][0, 0]) == n and o["n_pairs"] == n
    assert _u128(o["sum_lo"][0, 0], o["sum_hi"][0, 0]) == S
    assert _u128(o["sq_lo"][0, 0], o["sq_hi"][0, 0]) == Q
    assert math.isclose(o["mean"][0, 0], k * (L + 1) / 3, rel_tol=1e-15)
    _check_efg_stats(o, n, S, Q, 0, 0)


def test_efg_wide_gaps_carry_into_high_words():
    # gaps near 2^62: the gap sum passes 2^64 and every square needs 128 bits
    t = [-(2**62), 0, 2**62 - 1, 2**62]
    o = oracle.efg([1] * 4, [0, 0, 0, 0], t, 1)
    gaps = [t[j] - t[i] for i in range(4) for j in range(i + 1, 4)]
    assert _u128(o["sum_lo"][0, 0], o["sum_hi"][0, 0]) == sum(gaps) > 2**64
    assert _u128(o["sq_lo"][0, 0], o["sq_hi"][0, 0]) == sum(d * d for d in gaps)
    _check_efg_stats(o, 6, sum(gaps), sum(d * d for d in gaps), 0, 0)


def test_efg_invariants_on_workload():
    log = synth.config_log(2, 0.005)
    A = log.n_activities
    o = oracle.efg(log.case, log.act, log.ts, A)
    d = oracle.dfg(log.case, log.act, log.ts, A)
    L = log.lengths_by_code.astype(np.int64)
    assert o["n_pairs"] == int(o["count"].sum()) == int((L * (L - 1) // 2).sum())
    assert (o["count"] >= d["count"]).all()               # every directly-follows pair is one
    # cases of exactly two events: the EFG is their DFG
    codes = np.flatnonzero(L == 2)
    keep = np.isin(log.case, codes)
    two = oracle.efg(log.case[keep], log.act[keep], log.ts[keep], A)
    d2 = oracle.dfg(log.case[keep], log.act[keep], log.ts[keep], A)
    assert np.array_equal(two["count"], d2["count"])
    assert np.array_equal(two["sum_lo"].view(np.int64), d2["dt_sum"])
    # replicating every case (new case ids) doubles the counts and sums, keeps the mean,
    # and scales the sample variance by 2(n-1)/(2n-1)
    off = int(log.case.max()) + 1
    rc = np.concatenate([log.case, log.case + off])
    ra, rt = np.concatenate([log.act, log.act]), np.concatenate([log.ts, log.ts])
    o2 = oracle.efg(rc, ra, rt, A)
    assert np.array_equal(o2["count"], 2 * o["count"])
    S1 = [_u128(a, b) for a, b in zip(o["sum_lo"].ravel(), o["sum_hi"].ravel())]
    S2 = [_u128(a, b) for a, b in zip(o2["sum_lo"].ravel(), o2["sum_hi"].ravel())]
    assert S2 == [2 * x for x in S1]
    nz = o["count"] > 0
    assert np.allclose(o2["mean"][nz], o["mean"][nz], rtol=1e-15, atol=0)
    m = o["count"] > 1
    n = o["count"][m].astype(np.float64)
    assert np.allclose(o2["std"][m] ** 2 * (2 * n - 1), o["std"][m] ** 2 * 2 * (n - 1), rtol=1e-12, atol=0)


# ---- sampling ------------------------------------------------------------------

def test_splitmix_published_sequence():
    # the first outputs of SplitMix64 from state 0, as its reference implementation prints them
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [oracle.splitmix(0, x) for x in range(4)] == want


def _splitmix_at(seed: int, x: int) -> int:
    """The x-th output from state seed: the stream after x + 1 steps, its state
    reached by adding the increment x times in one product (the stream's
    state after x steps is seed + x * increment modulo 2^64)."""
    g = _SplitMix64Stream((seed + x * 0x9E3779B97F4A7C15) & _SplitMix64Stream.M)
    return g.next()


class _SplitMix64Stream:
    """SplitMix64 as a stateful stream (Steele, Lea and Flood, OOPSLA 2014):
    each call adds the odd increment 0x9E3779B97F4A7C15 to the 64-bit state,
    then passes the new state through the variant-13 mixer."""

    M = 2**64 - 1

    def __init__(self, state: int):
        self.state = state & self.M

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.M
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.M
        return z ^ (z >> 31)


def test_splitmix_stream_matches_published_sequence():
    g = _SplitMix64Stream(0)
    assert [g.next() for _ in range(4)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_splitmix_nonzero_seeds_follow_the_stream():
    # the oracle's x-th output from state `seed` equals the stream's (x+1)-th
    # step from that state, for seeds whose high and low bits are both set
    # (a slip such as (seed + x + 1) * increment agrees with this only at seed 0)
    rng = np.random.default_rng(20140414)
    seeds = [1, 2**63, 2**64 - 1, 0x0123456789ABCDEF] + [int(s) for s in rng.integers(1, 2**63, 12)]
    for seed in seeds:
        g = _SplitMix64Stream(seed)
        want = [g.next() for _ in range(80)]
        assert [oracle.splitmix(seed, x) for x in range(80)] == want
        assert [_splitmix_at(seed, x) for x in range(80)] == want


def _sample_triples(o):
    return list(zip(o["case_s"].tolist(), o["act_s"].tolist(), o["ts_s"].tolist()))


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_logs(), st.integers(0, 30), st.integers(0, 2**64 - 1), st.booleans())
def test_sample_match_bruteforce(log, k, seed, by_events):
    case, act, ts, A = log
    o = oracle.sample(case, act, ts, A, k, seed, by_events)
    f = oracle.prepare(case, act, ts, A)
    if by_events:
        n = len(case)
        g = _SplitMix64Stream(seed)
        keys = [g.next() for _ in range(n)]
        keep = set(sorted(range(n), key=lambda u: keys[u])[:k])
        want = [(f["case_s"][u], f["act_s"][u], f["ts_s"][u]) for u in range(n) if u in keep]
    else:
        codes = sorted(set(case))
        chosen = set(sorted(codes, key=lambda c: _splitmix_at(seed, c & 0xFFFFFFFF))[:k])
        want = [(c, a, t) for c, a, t in zip(f["case_s"], f["act_s"], f["ts_s"]) if c in chosen]
    assert _sample_triples(o) == [tuple(int(x) for x in w) for w in want]
    assert o["n_cases"] == len({w[0] for w in want})


def test_sample_sizes_nesting_and_uniformity():
    from collections import Counter

    log = synth.config_log(2, 0.002)
    A = log.n_activities
    C = int(np.unique(log.case).size)
    for by_events, total in ((False, C), (True, log.n_events)):
        assert oracle.sample(log.case, log.act, log.ts, A, 0, 7, by_events)["n_events"] == 0
        whole = oracle.sample(log.case, log.act, log.ts, A, total + 5, 7, by_events)
        assert whole["n_events"] == log.n_events
        prev = Counter()
        for k in (1, 10, 100, total // 2):
            o = oracle.sample(log.case, log.act, log.ts, A, k, 7, by_events)
            if by_events:
                assert o["n_events"] == k
            else:
                assert o["n_cases"] == k == len(set(o["case_s"].tolist()))
            units = Counter(_sample_triples(o))
            assert not (prev - units)                       # a smaller sample is a sub-multiset
            prev = units
    # one case out of four, many seeds: each case about equally often
    case, act, ts = np.array([1, 2, 3, 4]), np.zeros(4, np.int64), np.zeros(4, np.int64)
    hits = np.zeros(5, np.int64)
    for seed in range(4000):
        hits[int(oracle.sample(case, act, ts, 1, 1, seed)["case_s"][0])] += 1
    chi2 = float((((hits[1:] - 1000) ** 2) / 1000).sum())
    assert chi2 < 16.3                                      # chi-square, 3 dof, p = 0.001


# ---- CSV ingestion ---------------------------------------------------------------

GOLDEN_DIR = os.path.join(os.path.dirname(__file__), "golden")


def _csv_values(text, offs, lens):
    return [oracle.csv_value(text[o:o + n]).decode() for o, n in zip(offs, lens)]


def test_csv_golden_road_fines():
    g = json.load(open(os.path.join(GOLDEN_DIR, "worked_road_fines.json")))["csv"]
    text = open(os.path.join(GOLDEN_DIR, g["file"]), "rb").read()
    o = oracle.ingest_csv(text, g["case_col"], g["act_col"], g["ts_col"])
    assert o["n_rows"] == g["n_rows"]
    assert o["case"].tolist() == g["case"] and o["act"].tolist() == g["act"] and o["ts"].tolist() == g["ts"]
    assert _csv_values(text, o["case_off"], o["case_len"]) == g["case_values"]
    assert _csv_values(text, o["act_off"], o["act_len"]) == g["act_values"]


_FIELD_CHARS = st.sampled_from(list("ab Z,\"'\t;") + ["é", "中"])


def _iso(draw, aware):
    """An ISO-8601 date-time; aware ones always carry a time and an offset
    (pandas reads a naive value after an offset one with that offset)."""
    y = draw(st.integers(1700, 2250))
    mo = draw(st.integers(1, 12))
    import calendar
    d = draw(st.integers(1, calendar.monthrange(y, mo)[1]))
    s = f"{y:04d}-{mo:02d}-{d:02d}"
    if aware or draw(st.booleans()):
        s += draw(st.sampled_from(["T", " "])) + f"{draw(st.integers(0, 23)):02d}:{draw(st.integers(0, 59)):02d}"
        if draw(st.booleans()):
            s += f":{draw(st.integers(0, 59)):02d}"
            if draw(st.booleans()):
                s += "." + "".join(str(draw(st.integers(0, 9))) for _ in range(draw(st.integers(1, 9))))
        if aware:
            s += draw(st.sampled_from(["Z", "+01:00", "-05:30", "+0200", "-03"]))
    return s


@st.composite
def csv_tables(draw):
    rows = draw(st.integers(0, 12))
    ncol = draw(st.integers(3, 5))
    cols = draw(st.permutations(range(ncol)))[:3]
    iso = draw(st.booleans())
    aware = draw(st.booleans())
    pool_c = draw(st.lists(st.text(_FIELD_CHARS, min_size=1, max_size=6), min_size=1, max_size=4))
    pool_a = draw(st.lists(st.text(_FIELD_CHARS, min_size=1, max_size=6), min_size=1, max_size=4))
    table = []
    for _ in range(rows):
        row = [draw(st.text(_FIELD_CHARS, max_size=4)) for _ in range(ncol)]
        row[cols[0]] = draw(st.sampled_from(pool_c))
        row[cols[1]] = draw(st.sampled_from(pool_a))
        row[cols[2]] = _iso(draw, aware) if iso else str(draw(st.integers(-(2**62), 2**62)))
        table.append(row)
    crlf = draw(st.booleans())
    blank = draw(st.booleans())
    return table, cols, iso, crlf, blank, ncol


def _to_csv(table, ncol, crlf, blank, quote_all):
    nl = "\r\n" if crlf else "\n"

    def q(v):
        if quote_all or any(ch in v for ch in ",\"\r\n") or v == "":
            return '"' + v.replace('"', '""') + '"'
        return v
    lines = [",".join(f"h{k}" for k in range(ncol))]
    for i, r in enumerate(table):
        lines.append(",".join(q(v) for v in r))
        if blank and i == 0:
            lines.append("")
    return (nl.join(lines) + nl).encode()


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(csv_tables(), st.booleans(), st.sampled_from([3, 6, 9]))
def test_csv_matches_pandas(tab, quote_all, scale):
    import io

    import pandas as pd
    table, cols, iso, crlf, blank, ncol = tab
    text = _to_csv(table, ncol, crlf, blank, quote_all)
    o = oracle.ingest_csv(text, cols[0], cols[1], cols[2], ts_iso=iso, ts_scale=scale)
    df = pd.read_csv(io.BytesIO(text), dtype=str, keep_default_na=False, skip_blank_lines=True, encoding="utf-8")
    assert o["n_rows"] == len(table) == len(df)
    if not table:
        return
    for col, key, off, ln in ((cols[0], "case", "case_off", "case_len"), (cols[1], "act", "act_off", "act_len")):
        codes, uniques = pd.factorize(df.iloc[:, col], sort=False)
        assert o[key].tolist() == codes.tolist()
        assert [v.encode() for v in uniques] == [oracle.csv_value(text[a:a + n]) for a, n in zip(o[off], o[ln])]
    tcol = df.iloc[:, cols[2]]
    if iso:
        ns = pd.to_datetime(tcol, format="ISO8601", utc=True).astype("int64")
        want = [int(v) // 10 ** (9 - scale) for v in ns]
    else:
        want = [int(v) for v in tcol]
    assert o["ts"].tolist() == want


def test_csv_timestamps_against_datetime():
    import datetime as dt
    rng = np.random.default_rng(11)
    epoch = dt.datetime(1970, 1, 1, tzinfo=dt.timezone.utc)
    lines = ["c,a,t"]
    want = []
    for _ in range(2000):
        x = epoch + dt.timedelta(microseconds=int(rng.integers(-(2**52), 2**52)))
        off = int(rng.integers(-14 * 60, 14 * 60 + 1))
        tz = dt.timezone(dt.timedelta(minutes=off))
        loc = x.astimezone(tz)
        s = loc.strftime("%Y-%m-%dT%H:%M:%S.%f") + ("+" if off >= 0 else "-") + f"{abs(off) // 60:02d}:{abs(off) % 60:02d}"
        lines.append(f"1,a,{s}")
        want.append((x - epoch) // dt.timedelta(microseconds=1))
    o = oracle.ingest_csv(("\n".join(lines) + "\n").encode(), 0, 1, 2, ts_iso=True, ts_scale=6)
    assert o["ts"].tolist() == want


@pytest.mark.parametrize("text,iso,row", [
    (b"c,a,t\n1,x,5\n2,y\n3,z,7\n", False, 1),                      # too few fields
    (b"c,a,t\n1,x,2006-02-28\n2,y,2006-02-30\n", True, 1),          # no such day
    (b"c,a,t\n1,x,2006-01-01 24:00\n", True, 0),                     # hour out of range
    (b"c,a,t\n1,x,2006-01-01T10:00+01:00x\n", True, 0),              # trailing bytes
    (b"c,a,t\n1,x,12a\n", False, 0),                                 # not an integer
    (b"c,a,t\n1,x,9223372036854775808\n", False, 0),                 # beyond int64
    (b"c,a,t\n1,x,5\n2,\"y,6\n", False, 1),                         # quoted run open at the end
])
def test_csv_parse_errors(text, iso, row):
    with pytest.raises(oracle.CsvParseError) as e:
        oracle.ingest_csv(text, 0, 1, 2, ts_iso=iso)
    assert e.value.row == row
