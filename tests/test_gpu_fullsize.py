"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times, element by element against the oracle: the 10M-event workload; the
99M-event workload (formatted log, every DFG table, every variants array);
every one of the 4096 batched views over it (each answered by the oracle's
scan of its own formatted log).  Invariants that hold at any size are
checked beside them.  The oracle's independent calls run in host threads
(its C functions release the interpreter lock)."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import assert_dfg_equal, assert_variants_equal, note, same_f64

pytestmark = pytest.mark.gpu
_ROWS = {}   # the 99M-event log's row permutation from the GPU, until it is checked


def _dev(log):
    return (torch.from_numpy(log.case).cuda(), torch.from_numpy(log.act).cuda(), torch.from_numpy(log.ts).cuda())


def test_full_10M_against_oracle():
    log = synth.config_log(2)
    note(f"10M workload: N={log.n_events}")
    A = log.n_activities
    c, a, t = _dev(log)
    prep = pm4g.pm4g_prepare(c, a, t, A)
    d = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(prep), A)
    C = int(prep.n_cases.item())
    v = pm4g.variants_to_host(pm4g.pm4g_variants_prepared(prep), C)
    note("oracle on 10M events")
    assert_dfg_equal(d, oracle.dfg(log.case, log.act, log.ts, A), A)
    assert_variants_equal(v, oracle.variants(log.case, log.act, log.ts, A))
    p = oracle.prepare(log.case, log.act, log.ts, A)
    h = pm4g.prepared_to_host(prep)
    for k in ("case_s", "act_s", "ts_s", "case_off", "case_code"):
        assert np.array_equal(h[k], p[k]), k
    hr = pm4g.prepared_to_host(pm4g.pm4g_prepare(c, a, t, A, rows=True))
    for k in ("row", "case_s", "act_s", "ts_s", "case_off", "case_code"):
        assert np.array_equal(hr[k], p[k]), ("with rows", k)


@pytest.fixture(scope="module")
def big():
    log = synth.config_log(3)
    note(f"99M workload: N={log.n_events}")
    c, a, t = _dev(log)
    prep = pm4g.pm4g_prepare(c, a, t, log.n_activities)
    # the same log formatted with its row permutation (the sort's other variant)
    rows = pm4g.pm4g_prepare(c, a, t, log.n_activities, rows=True).row
    del c, a, t
    torch.cuda.synchronize()
    _ROWS["99M"] = rows
    return log, prep


@pytest.fixture(scope="module")
def big_oracle(big):
    """The oracle's formatted log, DFG and variants of the 99M-event log, run concurrently."""
    log, _ = big
    A = log.n_activities
    note("oracle: prepare, dfg, variants and eventually-follows graph of 99M events (four host threads)")
    with cf.ThreadPoolExecutor(4) as ex:
        fp = ex.submit(oracle.prepare, log.case, log.act, log.ts, A)
        fd = ex.submit(oracle.dfg, log.case, log.act, log.ts, A)
        fv = ex.submit(oracle.variants, log.case, log.act, log.ts, A)
        fe = ex.submit(oracle.efg, log.case, log.act, log.ts, A)
        out = dict(prep=fp.result(), dfg=fd.result(), variants=fv.result(), efg=fe.result())
    note("oracle done")
    return out


def test_full_99M_against_oracle(big, big_oracle):
    log, prep = big
    A = log.n_activities
    N = log.n_events
    d = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(prep), A)
    C = int(prep.n_cases.item())
    v = pm4g.variants_to_host(pm4g.pm4g_variants_prepared(prep), C)
    h = pm4g.prepared_to_host(prep)
    o = big_oracle
    assert h["status"] == 0 and h["n_cases"] == o["prep"]["n_cases"]
    for k in ("case_s", "act_s", "ts_s", "case_off", "case_code"):
        assert np.array_equal(h[k], o["prep"][k]), k
    assert np.array_equal(_ROWS.pop("99M").cpu().numpy(), o["prep"]["row"]), "row"
    assert_dfg_equal(d, o["dfg"], A)
    assert_variants_equal(v, o["variants"])
    # invariants, independent of the oracle
    cnt = d["count"]
    assert C == log.lengths_by_code.shape[0] and cnt.sum() == N - C
    assert d["start_count"].sum() == C == d["end_count"].sum()
    assert np.array_equal(cnt.sum(axis=1) + d["end_count"], d["act_count"])
    assert np.array_equal(cnt.sum(axis=0) + d["start_count"], d["act_count"])
    assert np.array_equal(d["act_count"], np.bincount(log.act, minlength=A))
    assert d["overflow"] == 0
    first = np.full(C, np.iinfo(np.int64).max)
    last = np.full(C, np.iinfo(np.int64).min)
    np.minimum.at(first, log.case, log.ts)
    np.maximum.at(last, log.case, log.ts)
    assert int(d["dt_sum"].astype(object).sum()) == int((last - first).astype(object).sum())
    assert v["var_count"].sum() == C and int((v["var_count"] * v["var_len"]).sum()) == N


def test_full_4096_views(big, big_oracle):
    """All 4096 views of the batched benchmark call, each against the oracle's
    scan of the case-range slice of its formatted log."""
    log, prep = big
    A = log.n_activities
    views = synth.make_views(log, 4096, seed=synth.SEED_BASE + 4)
    vd, md = pm4g.views_to_device(views, "cuda:0")
    o = pm4g.pm4g_dfg_batched(prep, vd, md, views.n_views)
    res = pm4g.batched_to_host(o, views.n_views, A)
    oprep = big_oracle["prep"]
    note("oracle: 4096 views")

    def check(v):
        r = res[v]
        cols = np.bincount(r["dst"], weights=r["count"], minlength=A).astype(np.int64)
        rows = np.bincount(r["src"], weights=r["count"], minlength=A).astype(np.int64)
        assert np.array_equal(r["act_count"], r["start_count"] + cols), v
        assert np.array_equal(r["end_count"], r["act_count"] - rows), v
        assert np.all(np.diff(r["src"].astype(np.int64) * A + r["dst"]) > 0), v
        ref = oracle.view_formatted(oprep, A, int(views.case_lo[v]), int(views.case_hi[v]),
                                    int(views.t_lo[v]), int(views.t_hi[v]), views.masks[v])
        nzc = np.flatnonzero(ref["count"].ravel())
        assert np.array_equal(r["src"].astype(np.int64) * A + r["dst"], nzc), v
        for k in ("count", "dt_sum", "dt_min", "dt_max"):
            assert np.array_equal(r[k], ref[k].ravel()[nzc]), (v, k)
        assert same_f64(r["dt_mean"], ref["dt_mean"].ravel()[nzc]), v
        for k in ("start_count", "end_count", "act_count"):
            assert np.array_equal(r[k], ref[k]), (v, k)
        assert r["n_events"] == ref["n_events"] and r["n_cases"] == ref["n_cases"], v
        return ref["n_events"]

    with cf.ThreadPoolExecutor(8) as ex:
        kept = list(ex.map(check, range(views.n_views)))
    note(f"4096 views checked: {sum(kept)} kept events")

    # the other launch mode gives the same bytes: the whole call as one
    # persistent launch and one launch per phase
    for launch in (0, 1):
        t = pm4g.BatchedTuning(tile_events=4096, launch=launch)
        o2 = pm4g.pm4g_dfg_batched(prep, vd, md, views.n_views, tuning=t)
        note(f"launch mode {launch}: compared with the checked call")
        for k in ("edge_off", "src", "dst", "count", "dt_sum", "dt_min", "dt_max", "start_count",
                  "end_count", "act_count", "n_events", "n_cases"):
            m = int(o["edge_off"][views.n_views].item()) if k in ("src", "dst", "count", "dt_sum", "dt_min",
                                                                  "dt_max") else None
            a, b = (o[k], o2[k]) if m is None else (o[k][:m], o2[k][:m])
            assert torch.equal(a, b), (launch, k)


def _u128(lo, hi):
    return [int(a) + (int(b) << 64) for a, b in zip(lo.ravel(), hi.ravel())]


def test_full_99M_efg(big, big_oracle):
    """The eventually-follows graph of the 99M-event log (2.6e9 pairs): every
    cell against the oracle; total pairs, per-activity row and column counts,
    and per-activity gap sums, each computed on the host from the formatted log."""
    log, prep = big
    A = log.n_activities
    h = pm4g.prepared_to_host(prep)
    e = pm4g.efg_to_host(pm4g.pm4g_efg(prep), A)
    oe = big_oracle["efg"]
    for k in ("count", "sum_lo", "sum_hi", "sq_lo", "sq_hi"):
        assert np.array_equal(e[k], oe[k]), k
    assert same_f64(e["mean"], oe["mean"]) and same_f64(e["std"], oe["std"])
    assert e["n_pairs"] == oe["n_pairs"]
    L = log.lengths_by_code.astype(np.int64)
    assert e["status"] == 0 and e["n_pairs"] == int((L * (L - 1) // 2).sum()) == int(e["count"].sum())
    off, act, ts = h["case_off"], h["act_s"], h["ts_s"]
    lens = np.diff(off)
    pos = np.arange(act.size, dtype=np.int64) - np.repeat(off[:-1], lens)     # index within the case
    tail = np.repeat(lens, lens) - pos - 1                                       # later events of the case
    assert np.array_equal(e["count"].sum(axis=1), np.bincount(act, weights=tail, minlength=A).astype(np.int64))
    assert np.array_equal(e["count"].sum(axis=0), np.bincount(act, weights=pos, minlength=A).astype(np.int64))
    # gap sums: event i contributes sum over later j of (t_j - t_i), from suffix sums of
    # the times relative to the case start (all within int64)
    rel = ts - np.repeat(ts[off[:-1]], lens)
    csum = np.cumsum(rel)
    case_total = np.add.reduceat(rel, off[:-1]) if rel.size else rel
    before = csum - np.repeat(csum[off[:-1]] - rel[off[:-1]], lens)             # inclusive prefix within case
    later = np.repeat(case_total, lens) - before                                 # sum of later rel times
    contrib = later - tail * rel
    assert (contrib >= 0).all()
    assert contrib.max() < 2**60
    # three 20-bit pieces: each per-activity sum stays below 2^53, so the float bins are exact
    pieces = [np.bincount(act, weights=((contrib >> (20 * k)) & 0xFFFFF).astype(np.float64), minlength=A)
              for k in range(3)]
    assert max(p.max() for p in pieces) < 2**53
    want = [sum(int(pieces[k][a]) << (20 * k) for k in range(3)) for a in range(A)]
    S = np.array(_u128(e["sum_lo"], e["sum_hi"]), dtype=object).reshape(A, A)
    assert [int(x) for x in S.sum(axis=1)] == want
    nz = e["count"] > 0
    assert np.isnan(e["mean"][~nz]).all() and np.isfinite(e["mean"][nz]).all() and (e["std"][nz] >= 0).all()


def test_full_99M_filters_and_sampling(big):
    log, prep = big
    A = log.n_activities
    N, C = log.n_events, int(prep.n_cases.item())
    L = log.lengths_by_code.astype(np.int64)                  # case codes are dense 0..C-1
    c = pm4g.pm4g_cases(prep)
    assert np.array_equal(c["n_events"][:C].cpu().numpy(), L)

    def kept(f):
        torch.cuda.synchronize()
        K = int(f.n_cases.item())
        assert int(f.status.item()) == 0
        return K, int(f.case_off[K].item()), f.case_code[:K].cpu().numpy()

    K, M, codes = kept(pm4g.pm4g_filter_cases(prep, min_events=5, max_events=40))
    sel = (L >= 5) & (L <= 40)
    assert K == int(sel.sum()) and M == int(L[sel].sum()) and np.array_equal(codes, np.flatnonzero(sel))
    # sampling: exactly k cases (whole) or k events; a smaller sample is a subset
    K1, M1, c1 = kept(pm4g.pm4g_sample(prep, C // 10, 5, False))
    K2, M2, c2 = kept(pm4g.pm4g_sample(prep, C // 20, 5, False))
    assert K1 == C // 10 and M1 == int(L[c1].sum()) and K2 == C // 20 and np.isin(c2, c1).all()
    _, M3, _ = kept(pm4g.pm4g_sample(prep, N // 10, 5, True))
    assert M3 == N // 10
    # directly-follows filter: dropping every event that has a previous one keeps each case's first
    allp = torch.from_numpy(np.full((A * A + 63) // 64, -1, np.int64)).cuda()
    f = pm4g.pm4g_filter_df_events(prep, allp, 0, False)
    K4, M4, _ = kept(f)
    d = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(prep), A)
    assert K4 == C == M4
    assert np.array_equal(np.bincount(f.act_s[:M4].cpu().numpy(), minlength=A), d["start_count"])
    # variant filter: the ten most frequent variants keep exactly their cases
    v = pm4g.pm4g_variants_prepared(prep)
    torch.cuda.synchronize()
    nv = int(v["n_variants"].item())
    vm = np.zeros((nv + 63) // 64, np.uint64)
    vm[0] = np.uint64((1 << 10) - 1)
    K5, _, _ = kept(pm4g.pm4g_filter_cases(prep, case_variant=v["case_variant"], n_variant_bits=nv,
                                           variant_mask=torch.from_numpy(vm.view(np.int64)).cuda()))
    assert K5 == int(v["var_count"][:10].sum().item())


def test_full_10M_csv_roundtrip():
    """CSV ingestion of the 10M-event log's text (509 MB): the timestamps come back
    exactly and the codes follow the first appearance of each case and activity."""
    log = synth.config_log(2)
    text = synth.log_csv(log, "ms", True)
    note(f"csv: {len(text)} bytes")
    t = torch.frombuffer(bytearray(text), dtype=torch.uint8).cuda()
    r = pm4g.pm4g_ingest_csv(t, 0, 1, 2, ts_iso=True, ts_scale=3, capacity=log.n_events + 1)
    assert r["n_rows"] == log.n_events
    assert np.array_equal(r["ts"].cpu().numpy(), log.ts)
    for col, key, n in ((log.case, "case_code", "n_cases"), (log.act, "act_code", "n_acts")):
        uniq, first = np.unique(col, return_index=True)
        rank = np.empty(uniq.size, np.int64)
        rank[np.argsort(first)] = np.arange(uniq.size)
        assert r[n] == uniq.size
        assert np.array_equal(r[key].cpu().numpy(), rank[np.searchsorted(uniq, col)])
    off, ln = r["case_dict_off"].cpu().numpy(), r["case_dict_len"].cpu().numpy()
    for code in (0, 1, r["n_cases"] - 1):
        value = int(text[off[code]:off[code] + ln[code]][1:]) - 2**31
        assert value == log.case[np.flatnonzero(r["case_code"].cpu().numpy() == code)[0]]
