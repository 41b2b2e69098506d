"""GPU parity of the batched drill-down views against the oracle's view
function (filter, then re-discover), view by view, bit-exact."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import cols, note, same_f64

pytestmark = pytest.mark.gpu
INT64_MIN = np.iinfo(np.int64).min
INT64_MAX = np.iinfo(np.int64).max


def dense_to_sparse(o, A):
    nz = np.flatnonzero(o["count"].ravel())
    return dict(src=(nz // A).astype(np.int32), dst=(nz % A).astype(np.int32),
                count=o["count"].ravel()[nz], dt_sum=o["dt_sum"].ravel()[nz],
                dt_min=o["dt_min"].ravel()[nz], dt_max=o["dt_max"].ravel()[nz],
                dt_mean=o["dt_mean"].ravel()[nz])


def check_views(log, views, tuning=None, sample=None):
    A = log.n_activities
    c, a, t = cols(log.case, log.act, log.ts)
    prep = pm4g.pm4g_prepare(c, a, t, A, presorted=log.presorted)
    vd, md = pm4g.views_to_device(views, "cuda:0")
    V = views.n_views
    o = pm4g.pm4g_dfg_batched(prep, vd, md, V, tuning=tuning)
    res = pm4g.batched_to_host(o, V, A)
    idx = range(V) if sample is None else sample
    for v in idx:
        ref = oracle.view(log.case, log.act, log.ts, A, int(views.case_lo[v]), int(views.case_hi[v]),
                          int(views.t_lo[v]), int(views.t_hi[v]), views.masks[v])
        sp = dense_to_sparse(ref, A)
        g = res[v]
        for k in ("src", "dst", "count", "dt_sum", "dt_min", "dt_max"):
            assert np.array_equal(g[k], sp[k]), (v, k)
        assert same_f64(g["dt_mean"], sp["dt_mean"]), v
        for k in ("start_count", "end_count", "act_count"):
            assert np.array_equal(g[k], ref[k]), (v, k)
        assert g["n_events"] == ref["n_events"] and g["n_cases"] == ref["n_cases"], v
    return res


@pytest.mark.parametrize("launch", [0, 1])
@pytest.mark.parametrize("tile", [2048, 4096])
def test_views_scaled_workload(tile, launch):
    """Both launch modes: the whole call as one persistent launch (0) and one
    launch per phase (1)."""
    log = synth.config_log(3, 0.004)          # ~400k events, 512 activities
    views = synth.make_views(log, 48, seed=7, min_events=50, max_events=300_000)
    note(f"views: N={log.n_events} V={views.n_views} tile={tile} launch={launch}")
    t = pm4g.BatchedTuning(tile_events=tile, launch=launch)
    check_views(log, views, tuning=t)


def test_views_small_activity_set_and_edge_views():
    log = synth.config_log(2, 0.01)           # ~100k events, 64 activities, 5% tied timestamps
    A = log.n_activities
    base = synth.make_views(log, 20, seed=3, min_events=10, max_events=50_000)
    C = int(log.case.max()) + 1
    full = np.full((1, 1), np.uint64(0xFFFFFFFFFFFFFFFF))
    extra_lo = np.array([0, 5, 10, 0, 3, -7], np.int32)
    extra_hi = np.array([C, 5, 4, C, 4, C + 10], np.int32)       # full, empty, reversed, ...
    extra_tl = np.array([INT64_MIN, INT64_MIN, INT64_MIN, 0, INT64_MIN, INT64_MIN], np.int64)
    extra_th = np.array([INT64_MAX, INT64_MAX, INT64_MAX, -1, INT64_MAX, INT64_MAX], np.int64)
    extra_m = np.repeat(full, 6, axis=0)
    extra_m[4] = 0                                                # empty activity set
    extra_m[5] = np.uint64(0x5555555555555555)
    views = synth.Views(case_lo=np.concatenate([base.case_lo, extra_lo]),
                        case_hi=np.concatenate([base.case_hi, extra_hi]),
                        t_lo=np.concatenate([base.t_lo, extra_tl]), t_hi=np.concatenate([base.t_hi, extra_th]),
                        masks=np.concatenate([base.masks, extra_m]))
    res = check_views(log, views)
    # the unfiltered view equals the plain DFG
    d = oracle.dfg(log.case, log.act, log.ts, A)
    assert int(res[base.n_views]["count"].sum()) == int(d["count"].sum())
    assert res[base.n_views + 1]["n_events"] == 0


@pytest.mark.parametrize("launch", [0, 1])
def test_views_long_cases_cross_tiles(launch):
    """Cases longer than a tile: the previous kept event comes from an earlier tile."""
    rng = np.random.default_rng(9)
    lens = [9000, 3, 5000, 1, 2500] + list(rng.integers(1, 40, 400))
    case = np.repeat(np.arange(len(lens), dtype=np.int32), lens)
    n = case.size
    A = 16
    act = rng.integers(0, A, n).astype(np.int32)
    ts = rng.integers(0, 10**6, n, dtype=np.int64)
    perm = rng.permutation(n)
    log = synth.Log(case=case[perm], act=act[perm], ts=ts[perm], n_activities=A, presorted=False,
                    lengths_by_code=np.asarray(lens, np.int64))
    V = 12
    lo = rng.integers(0, 3, V).astype(np.int32)
    hi = (lo + rng.integers(1, len(lens), V)).astype(np.int32)
    tl = rng.integers(0, 300_000, V)
    th = tl + rng.integers(100_000, 10**6, V)
    masks = np.zeros((V, 1), np.uint64)
    for v in range(V):
        for x in rng.choice(A, rng.integers(1, A + 1), replace=False):
            masks[v, 0] |= np.uint64(1) << np.uint64(x)
    views = synth.Views(case_lo=lo, case_hi=hi, t_lo=tl, t_hi=th, masks=masks)
    check_views(log, views, tuning=pm4g.BatchedTuning(tile_events=2048, launch=launch))


@pytest.mark.parametrize("launch", [0, 1])
def test_views_capacity_retry(launch):
    """Tiny capacities force the PM4G_E_CAPACITY path; the binding retries with what was required."""
    log = synth.config_log(3, 0.002)
    views = synth.make_views(log, 16, seed=11, min_events=100, max_events=100_000)
    t = pm4g.BatchedTuning(pair_capacity=8, record_capacity=64, cell_capacity=16, launch=launch)
    check_views(log, views, tuning=t)


@pytest.mark.parametrize("span", [(1 << 52) - 1, 1 << 52, 1 << 62])
def test_views_record_layouts(span):
    """Longest case lasting just under, exactly and far over 2^52 time units:
    below that every record packs its cell and gap into one word, otherwise the
    cell is kept apart.  Both layouts give the oracle's tables."""
    rng = np.random.default_rng(21)
    lens = [2, 3] + list(rng.integers(1, 30, 600))
    case = np.repeat(np.arange(len(lens), dtype=np.int32), lens)
    n = case.size
    A = 24
    act = rng.integers(0, A, n).astype(np.int32)
    ts = rng.integers(-(1 << 40), 1 << 40, n, dtype=np.int64)
    b = -(1 << 61)
    ts[0:2] = [b, b + span]                           # case 0 lasts exactly `span`
    ts[2:5] = [b, b + span // 2, b + span]            # case 1 too, in two gaps
    perm = rng.permutation(n)
    log = synth.Log(case=case[perm], act=act[perm], ts=ts[perm], n_activities=A, presorted=False,
                    lengths_by_code=np.asarray(lens, np.int64))
    V = 10
    lo = rng.integers(0, 4, V).astype(np.int32)
    hi = (lo + rng.integers(1, len(lens), V)).astype(np.int32)
    tl = np.full(V, INT64_MIN, np.int64)
    th = np.full(V, INT64_MAX, np.int64)
    tl[5:] = rng.integers(-(1 << 40), 0, V - 5)
    th[5:] = tl[5:] + rng.integers(1 << 39, 1 << 41, V - 5)
    masks = np.full((V, 1), np.uint64((1 << A) - 1))
    masks[3, 0] = np.uint64(0xAAAAAA)
    lo[0], hi[0] = 0, len(lens)                        # the whole log
    views = synth.Views(case_lo=lo, case_hi=hi, t_lo=tl, t_hi=th, masks=masks)
    note(f"views: record layouts, longest case {span}")
    res = check_views(log, views)
    assert int(res[0]["dt_max"].max()) == span


def test_batched_call_does_not_wait_and_reports_capacity_on_the_device():
    """The C call enqueues and returns while earlier work on its stream is still
    running (a bounded spin kernel queued first); a short record capacity then
    shows up in the device status word with the required sizes, and a second
    call with those sizes gives the oracle's tables."""
    log = synth.config_log(3, 0.002)
    A = log.n_activities
    c, a, t = cols(log.case, log.act, log.ts)
    prep = pm4g.pm4g_prepare(c, a, t, A)
    views = synth.make_views(log, 12, seed=5, min_events=100, max_events=50_000)
    vd, md = pm4g.views_to_device(views, "cuda:0")
    V = views.n_views
    L = pm4g.load()
    s = torch.cuda.Stream()
    tun = pm4g.BatchedTuning(record_capacity=64)
    need = int(L.pm4g_batched_workspace_bytes(prep.n_events, A, V, ctypes.byref(tun)))
    with torch.cuda.stream(s):
        ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        o = pm4g._batched_out(V, A, 1 << 20, "cuda:0")
    s.synchronize()
    with torch.cuda.stream(s):
        torch.cuda._sleep(300_000_000)           # about 0.15 s on the stream, bounded
    p = prep._struct()
    st = pm4g._batched_struct(o)
    rc = L.pm4g_dfg_batched(ctypes.byref(p), pm4g._ptr(vd), pm4g._ptr(md), V, ctypes.byref(st),
                            ctypes.byref(tun), pm4g._ptr(ws), need, ctypes.c_void_p(s.cuda_stream))
    assert rc == 0
    assert not s.query(), "the call waited for its stream"
    s.synchronize()
    assert int(o["status"].item()) == pm4g.PM4G_E_CAPACITY
    req = o["required"].cpu().numpy()
    assert req[1] > 64 and req[3] > 0
    tun.record_capacity = int(req[1])
    for _ in range(3):   # the cell counts become known once the records fit
        need = int(L.pm4g_batched_workspace_bytes(prep.n_events, A, V, ctypes.byref(tun)))
        with torch.cuda.stream(s):
            ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        rc = L.pm4g_dfg_batched(ctypes.byref(p), pm4g._ptr(vd), pm4g._ptr(md), V, ctypes.byref(st),
                                ctypes.byref(tun), pm4g._ptr(ws), need, ctypes.c_void_p(s.cuda_stream))
        assert rc == 0
        s.synchronize()
        if int(o["status"].item()) == 0:
            break
        req = o["required"].cpu().numpy()
        assert int(o["status"].item()) == pm4g.PM4G_E_CAPACITY and req[0] <= (1 << 20) and req[4] > 0
        tun.cell_capacity = int(req[4])
    assert int(o["status"].item()) == 0
    res = pm4g.batched_to_host(o, V, A)
    for v in range(V):
        ref = oracle.view(log.case, log.act, log.ts, A, int(views.case_lo[v]), int(views.case_hi[v]),
                          int(views.t_lo[v]), int(views.t_hi[v]), views.masks[v])
        sp = dense_to_sparse(ref, A)
        for k in ("src", "dst", "count", "dt_sum", "dt_min", "dt_max"):
            assert np.array_equal(res[v][k], sp[k]), (v, k)
        assert res[v]["n_events"] == ref["n_events"], v


@pytest.mark.parametrize("n_events,n_views", [(1, 1), (1, 0), (5000, 0), (5000, 1), (70_000, 3)])
def test_launch_modes_on_small_and_empty_calls(n_events, n_views):
    """One event, no views, one view: the persistent launch (every phase on a
    grid of resident blocks, most of them idle) and the per-phase launches give
    the oracle's tables."""
    rng = np.random.default_rng(n_events + 7 * n_views)
    A = 20
    C = max(1, n_events // 9)
    case = np.sort(rng.integers(0, C, n_events)).astype(np.int32)
    case[0] = 0
    _, case = np.unique(case, return_inverse=True)
    case = case.astype(np.int32)
    act = rng.integers(0, A, n_events).astype(np.int32)
    ts = rng.integers(0, 10**9, n_events, dtype=np.int64)
    perm = rng.permutation(n_events)
    lens = np.bincount(case).astype(np.int64)
    log = synth.Log(case=case[perm], act=act[perm], ts=ts[perm], n_activities=A, presorted=False,
                    lengths_by_code=lens)
    nc = int(case.max()) + 1
    lo = rng.integers(0, nc, n_views).astype(np.int32)
    hi = np.minimum(lo + rng.integers(1, nc + 1, n_views), nc).astype(np.int32)
    views = synth.Views(case_lo=lo, case_hi=hi, t_lo=np.full(n_views, 10**8, np.int64),
                        t_hi=np.full(n_views, 9 * 10**8, np.int64),
                        masks=np.full((n_views, 1), np.uint64((1 << A) - 1 - 6)))
    for launch in (0, 1):
        note(f"launch {launch}: N={n_events} V={n_views}")
        res = check_views(log, views, tuning=pm4g.BatchedTuning(tile_events=4096, launch=launch))
        assert len(res) == n_views
