"""Event-level filters on the GPU against the oracle, bit-exact: the
directly-follows-level filter (previous- and next-event pair, keep and drop;
the DFG of the filtered log; capacity and argument errors) and one drill-down
view materialised as a log (kept events of the oracle's formatted log)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import cols, dev, note

pytestmark = pytest.mark.gpu


def _prep(case, act, ts, A):
    c, a, t = cols(case, act, ts)
    p = pm4g.pm4g_prepare(c, a, t, A)
    torch.cuda.synchronize()
    return p


def _mask(cells, nbits):
    m = np.zeros(max((nbits + 63) // 64, 1), np.uint64)
    for b in cells:
        m[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    return m


def _run(p, pm, side, keep, out=None):
    f = pm4g.pm4g_filter_df_events(p, dev(pm.view(np.int64), np.int64), side, keep, out=out)
    torch.cuda.synchronize()
    K = int(f.n_cases.item())
    off = f.case_off[:K + 1].cpu().numpy()
    m = int(off[K])
    return f, dict(case_s=f.case_s[:m].cpu().numpy(), act_s=f.act_s[:m].cpu().numpy(),
                   ts_s=f.ts_s[:m].cpu().numpy(), case_off=off, case_code=f.case_code[:K].cpu().numpy(),
                   n_cases=K, n_events=m, status=int(f.status.item()))


def _check(case, act, ts, A, p, pm, side, keep):
    f, g = _run(p, pm, side, keep)
    assert g["status"] == 0
    o = oracle.filter_df_events(case, act, ts, A, pm, side, keep)
    assert g["n_events"] == o["n_events"] and g["n_cases"] == o["n_cases"], (side, keep)
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(g[k], o[k]), (k, side, keep)
    if g["n_events"]:
        starts = np.flatnonzero(np.r_[True, g["case_s"][1:] != g["case_s"][:-1]])
        assert np.array_equal(g["case_off"][:-1], starts)
        assert np.array_equal(g["case_code"], g["case_s"][starts])
    return f, g, o


def test_golden_road_fines():
    gd = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_road_fines.json")))
    r, A = gd["rows"], gd["A"]
    case, act, ts = (np.array(r[k]) for k in ("case", "act", "ts"))
    p = _prep(case, act, ts, A)
    for f in gd["df_events"]["filters"]:
        pairs = ([(x, y) for x in range(A) for y in range(A)] if f["pairs"] == "all"
                 else [tuple(q) for q in f["pairs"]])
        _, g = _run(p, _mask([x * A + y for x, y in pairs], A * A), f["side"], f["keep"])
        got = list(zip(g["case_s"].tolist(), g["act_s"].tolist(), g["ts_s"].tolist()))
        assert got == [tuple(e) for e in f["events"]], f["name"]
        assert g["n_cases"] == f["n_cases"], f["name"]


@pytest.mark.parametrize("k,scale", [(2, 0.02), (3, 0.005)])
def test_workloads(k, scale):
    log = synth.config_log(k, scale)
    A = log.n_activities
    note(f"df-level filter: config {k} scale {scale}: N={log.n_events}")
    p = _prep(log.case, log.act, log.ts, A)
    rng = np.random.default_rng(300 + k)
    sets = [rng.choice(A * A, A, replace=False).tolist(), rng.choice(A * A, A * A // 3, replace=False).tolist(),
            [], list(range(A * A))]
    for cells in sets:
        pm = _mask(cells, A * A)
        for side in (0, 1):
            for keep in (True, False):
                _check(log.case, log.act, log.ts, A, p, pm, side, keep)


def test_filtered_log_composes_with_dfg():
    log = synth.config_log(2, 0.01)
    A = log.n_activities
    p = _prep(log.case, log.act, log.ts, A)
    pm = _mask(list(range(1, A * A, 5)), A * A)
    f, g, o = _check(log.case, log.act, log.ts, A, p, pm, 0, False)
    m = g["n_events"]
    sub = pm4g.Prepared(f.case_s[:m], f.act_s[:m], f.ts_s[:m], f.case_off, f.case_code, f.n_cases, f.status, A)
    d = pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(sub), A)
    od = oracle.dfg(o["case_s"], o["act_s"], o["ts_s"], A)
    for key in ("count", "dt_sum", "dt_min", "dt_max", "start_count", "end_count", "act_count"):
        assert np.array_equal(d[key], od[key]), key


def test_capacity_empty_and_arguments():
    log = synth.config_log(2, 0.002)
    A = log.n_activities
    p = _prep(log.case, log.act, log.ts, A)
    pm = _mask(range(A * A), A * A)
    small = pm4g.Prepared.empty(10, A, p.case_s.device)
    _, g = _run(p, pm, 0, False, out=small)                  # one event per case: more than 10
    assert g["status"] == pm4g.PM4G_E_CAPACITY and g["n_events"] == 0 and g["n_cases"] == 0
    # the same output buffers serve a call that fits
    one = np.array([3, 3, 3]), np.array([0, 1, 2]), np.array([5, 6, 7])
    q = _prep(*one, A)
    _, g = _run(q, _mask([0 * A + 1], A * A), 0, True, out=small)
    assert g["status"] == 0 and g["act_s"].tolist() == [1] and g["case_code"].tolist() == [3]
    e = _prep(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), A)
    for side in (0, 1):
        _, g = _run(e, pm, side, False)
        assert g["n_events"] == 0 and g["n_cases"] == 0 and g["status"] == 0
    pmd = dev(pm.view(np.int64), np.int64)
    with pytest.raises(pm4g.Pm4gError):
        pm4g.pm4g_filter_df_events(p, pmd, side=2)


@pytest.mark.parametrize("k,scale", [(2, 0.02), (3, 0.005)])
def test_view_filter_matches_formatted_log(k, scale):
    log = synth.config_log(k, scale)
    A = log.n_activities
    note(f"view filter: config {k} scale {scale}: N={log.n_events}")
    p = _prep(log.case, log.act, log.ts, A)
    o = oracle.prepare(log.case, log.act, log.ts, A)
    views = synth.make_views(log, 6, seed=400 + k, min_events=1, max_events=log.n_events)
    rec = views.packed()
    W = (A + 63) // 64
    for v in range(views.n_views):
        vd = torch.from_numpy(rec[v:v + 1].view(np.uint8).copy()).to(p.case_s.device)
        md = dev(views.masks[v].view(np.int64), np.int64)
        f = pm4g.pm4g_filter_view(p, vd, md)
        torch.cuda.synchronize()
        K = int(f.n_cases.item())
        m = int(f.case_off[K].item())
        assert int(f.status.item()) == 0
        # a view keeps an event iff its case is in [lo, hi), its timestamp in
        # [t_lo, t_hi] and its activity in the mask; the order is the formatted log's
        bits = (views.masks[v][o["act_s"] // 64] >> (o["act_s"] % 64).astype(np.uint64)) & np.uint64(1)
        sel = ((o["case_s"] >= views.case_lo[v]) & (o["case_s"] < views.case_hi[v]) & (o["ts_s"] >= views.t_lo[v])
               & (o["ts_s"] <= views.t_hi[v]) & (bits == 1))
        assert m == int(sel.sum()), v
        assert np.array_equal(f.case_s[:m].cpu().numpy(), o["case_s"][sel])
        assert np.array_equal(f.act_s[:m].cpu().numpy(), o["act_s"][sel])
        assert np.array_equal(f.ts_s[:m].cpu().numpy(), o["ts_s"][sel])
        codes, starts = np.unique(o["case_s"][sel], return_index=True)
        assert K == codes.size
        assert np.array_equal(f.case_code[:K].cpu().numpy(), codes)
        assert np.array_equal(f.case_off[:K].cpu().numpy(), starts)
    assert W == views.masks.shape[1]
