"""Cases dataframe and case-level filters on the GPU against the oracle:
events and throughput per case, and the kept cases' events (order and case
table) for range, activity, path, time-window, start/end activity and variant
predicates, bit-exact."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import cols, dev, note

pytestmark = pytest.mark.gpu

I64_MIN, I64_MAX = pm4g.I64_MIN, pm4g.I64_MAX


def _prep(case, act, ts, A):
    c, a, t = cols(case, act, ts)
    p = pm4g.pm4g_prepare(c, a, t, A)
    torch.cuda.synchronize()
    return p


def _mask(bits, nbits):
    m = np.zeros(max((nbits + 63) // 64, 1), np.uint64)
    for b in bits:
        m[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    return m


def _gpu_cases(p):
    o = pm4g.pm4g_cases(p)
    torch.cuda.synchronize()
    C = int(p.n_cases.item())
    return {k: v[:C].cpu().numpy() for k, v in o.items()}, p.case_code[:C].cpu().numpy()


MASKS = ("act_mask", "path_mask", "start_mask", "end_mask", "variant_mask")


def _case_variant(p):
    v = pm4g.pm4g_variants_prepared(p)
    torch.cuda.synchronize()
    return v["case_variant"], int(v["n_variants"].item())


def _gpu_filter(p, case_variant=None, **kw):
    A = p.n_activities
    for k in MASKS:
        if k in kw:
            kw[k] = dev(kw[k].view(np.int64), np.int64)
    if "variant_mask" in kw:
        kw["case_variant"] = case_variant
    f = pm4g.pm4g_filter_cases(p, **kw)
    torch.cuda.synchronize()
    assert int(f.status.item()) == 0
    K = int(f.n_cases.item())
    off = f.case_off[:K + 1].cpu().numpy()
    m = int(off[K])
    return dict(case_s=f.case_s[:m].cpu().numpy(), act_s=f.act_s[:m].cpu().numpy(),
                ts_s=f.ts_s[:m].cpu().numpy(), case_off=off, case_code=f.case_code[:K].cpu().numpy(),
                n_cases=K, n_events=m), A


def _check_filter(case, act, ts, A, p, case_variant=None, **kw):
    """GPU filter with the binding's keywords against the oracle (its names for
    the throughput bounds), plus the output case table's consistency."""
    g, _ = _gpu_filter(p, case_variant, **dict(kw))
    okw = {k: v for k, v in kw.items() if k not in ("min_throughput", "max_throughput")}
    if "min_throughput" in kw:
        okw["min_thr"] = kw["min_throughput"]
    if "max_throughput" in kw:
        okw["max_thr"] = kw["max_throughput"]
    o = oracle.filter_cases(case, act, ts, A, **okw)
    assert g["n_events"] == o["n_events"] and g["n_cases"] == o["n_cases"], (kw, g["n_events"], o["n_events"])
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(g[k], o[k]), (k, kw)
    if g["n_events"]:
        starts = np.flatnonzero(np.r_[True, g["case_s"][1:] != g["case_s"][:-1]])
        assert np.array_equal(g["case_off"][:-1], starts)
        assert np.array_equal(g["case_code"], g["case_s"][starts])
    return g


def test_golden_road_fines():
    gd = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_road_fines.json")))
    r, A = gd["rows"], gd["A"]
    case, act, ts = (np.array(r[k]) for k in ("case", "act", "ts"))
    p = _prep(case, act, ts, A)
    c, codes = _gpu_cases(p)
    exp = gd["cases"]["expected"]
    assert codes.tolist() == exp["case_code"]
    assert c["n_events"].tolist() == exp["n_events"]
    assert c["throughput"].tolist() == exp["throughput"]
    cv, nv = _case_variant(p)
    assert cv[:4].cpu().tolist() == gd["expected"]["variants"]["case_variant"]
    for f in gd["cases"]["filters"]:
        kw = {k: f[k] for k in ("min_events", "max_events") if k in f}
        if "min_thr" in f:
            kw["min_throughput"], kw["max_throughput"] = f["min_thr"], f["max_thr"]
        if "activities" in f:
            kw["act_mask"] = _mask(f["activities"], A)
        if "paths" in f:
            kw["path_mask"] = _mask([x * A + y for x, y in f["paths"]], A * A)
            kw["path_keep"] = f["path_keep"]
        if "contain" in f:
            kw["contain_lo"], kw["contain_hi"] = f["contain"]
        if "meet" in f:
            kw["meet_lo"], kw["meet_hi"] = f["meet"]
        if "start_acts" in f:
            kw["start_mask"] = _mask(f["start_acts"], A)
        if "end_acts" in f:
            kw["end_mask"] = _mask(f["end_acts"], A)
        if "variants" in f:
            kw["variant_mask"] = _mask(f["variants"], nv)
            kw["n_variant_bits"], kw["variant_keep"] = nv, f["variant_keep"]
        g, _ = _gpu_filter(p, cv, **kw)
        got = list(zip(g["case_s"].tolist(), g["act_s"].tolist(), g["ts_s"].tolist()))
        assert got == [tuple(e) for e in f["events"]], f["name"]
        assert g["case_code"].tolist() == f["kept_cases"], f["name"]


@pytest.mark.parametrize("k,scale", [(2, 0.02), (3, 0.005)])
def test_workloads(k, scale):
    log = synth.config_log(k, scale)
    A = log.n_activities
    note(f"cases dataframe: config {k} scale {scale}: N={log.n_events}")
    p = _prep(log.case, log.act, log.ts, A)
    c, codes = _gpu_cases(p)
    o = oracle.cases(log.case, log.act, log.ts, A)
    assert np.array_equal(codes, o["case_code"])
    assert np.array_equal(c["n_events"], o["n_events"])
    assert np.array_equal(c["throughput"], o["throughput"])
    rng = np.random.default_rng(100 + k)
    med_thr = int(np.median(o["throughput"]))
    filters = [
        dict(),
        dict(min_events=5, max_events=40),
        dict(min_throughput=med_thr // 2, max_throughput=med_thr * 3),
        dict(act_mask=_mask(rng.choice(A, 3, replace=False).tolist(), A)),
        dict(path_mask=_mask(rng.choice(A * A, A, replace=False).tolist(), A * A), path_keep=True),
        dict(path_mask=_mask(rng.choice(A * A, A, replace=False).tolist(), A * A), path_keep=False,
             min_events=3),
        dict(min_events=10**9),                                     # nothing kept
    ]
    for f in filters:
        _check_filter(log.case, log.act, log.ts, A, p, **f)


@pytest.mark.parametrize("k,scale", [(2, 0.02), (3, 0.005)])
def test_window_start_end_variant_filters(k, scale):
    log = synth.config_log(k, scale)
    A = log.n_activities
    note(f"window/start/end/variant filters: config {k} scale {scale}: N={log.n_events}")
    p = _prep(log.case, log.act, log.ts, A)
    cv, nv = _case_variant(p)
    rng = np.random.default_rng(200 + k)
    lo, mid, hi = (int(x) for x in np.percentile(log.ts, [30, 50, 70]))
    top = list(range(min(nv, 5)))
    filters = [
        dict(contain_lo=lo, contain_hi=hi),
        dict(meet_lo=mid, meet_hi=mid),                             # cases running at one instant
        dict(meet_lo=lo, meet_hi=hi, min_events=3),
        dict(contain_hi=lo),                                        # wholly before a time
        dict(start_mask=_mask(rng.choice(A, 2, replace=False).tolist(), A)),
        dict(end_mask=_mask(rng.choice(A, 3, replace=False).tolist(), A),
             start_mask=_mask(range(A // 2), A)),
        dict(variant_mask=_mask(top, nv), n_variant_bits=nv, variant_keep=True),
        dict(variant_mask=_mask(top, nv), n_variant_bits=nv, variant_keep=False),
        dict(variant_mask=_mask(range(1, nv, 3), nv), n_variant_bits=nv, variant_keep=True,
             contain_lo=lo),
        # a set narrower than the ids: the ids at or above n_variant_bits are outside it
        dict(variant_mask=_mask([0], 1), n_variant_bits=1, variant_keep=False),
        dict(contain_lo=hi, contain_hi=lo),                         # empty window: nothing kept
    ]
    for f in filters:
        _check_filter(log.case, log.act, log.ts, A, p, case_variant=cv, **f)


def test_variant_filter_invalid_arguments():
    log = synth.config_log(2, 0.002)
    A = log.n_activities
    p = _prep(log.case, log.act, log.ts, A)
    vm = dev(_mask([0], 1).view(np.int64), np.int64)
    with pytest.raises(pm4g.Pm4gError):
        pm4g.pm4g_filter_cases(p, variant_mask=vm, n_variant_bits=1)    # no case_variant
    cv, _ = _case_variant(p)
    with pytest.raises(pm4g.Pm4gError):
        pm4g.pm4g_filter_cases(p, variant_mask=vm, case_variant=cv, n_variant_bits=-1)


def test_filtered_log_composes_with_dfg_and_variants():
    log = synth.config_log(2, 0.01)
    A = log.n_activities
    p = _prep(log.case, log.act, log.ts, A)
    pm = _mask(list(range(0, A * A, 7)), A * A)
    f = pm4g.pm4g_filter_cases(p, min_events=4, path_mask=dev(pm.view(np.int64), np.int64), path_keep=False)
    torch.cuda.synchronize()
    K = int(f.n_cases.item())
    m = int(f.case_off[K].item())
    # the DFG walks every event of its input: give it exactly the kept ones
    sub = pm4g.Prepared(f.case_s[:m], f.act_s[:m], f.ts_s[:m], f.case_off, f.case_code, f.n_cases, f.status, A)
    d = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(sub), A)
    v = pm4g.variants_to_host(pm4g.pm4g_variants_prepared(f))
    ref = oracle.filter_cases(log.case, log.act, log.ts, A, min_events=4, path_mask=pm, path_keep=False)
    od = oracle.dfg(ref["case_s"], ref["act_s"], ref["ts_s"], A)
    ov = oracle.variants(ref["case_s"], ref["act_s"], ref["ts_s"], A)
    for k in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
        assert np.array_equal(d[k], od[k]), k
    for k in ("var_count", "var_len", "var_rep", "var_off", "var_acts"):
        assert np.array_equal(v[k], ov[k]), k


def test_capacity_and_empty():
    log = synth.config_log(2, 0.002)
    A = log.n_activities
    p = _prep(log.case, log.act, log.ts, A)
    small = pm4g.Prepared.empty(10, A, p.case_s.device)
    f = pm4g.pm4g_filter_cases(p, out=small)
    torch.cuda.synchronize()
    assert int(f.status.item()) == pm4g.PM4G_E_CAPACITY
    assert int(f.n_cases.item()) == 0 and int(f.case_off[0].item()) == 0
    e = _prep(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), A)
    c, codes = _gpu_cases(e)
    assert codes.size == 0
    g, _ = _gpu_filter(e)
    assert g["n_events"] == 0 and g["n_cases"] == 0
