"""Sampling on the GPU against the oracle, bit-exact: k cases or k events by
SplitMix64 keys, for several seeds and sizes (k = 0, 1, a fraction, all and
more than all), capacity, an empty log, and case ids with the sign bit set."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import cols, note

pytestmark = pytest.mark.gpu


def _prep(case, act, ts, A):
    c, a, t = cols(case, act, ts)
    p = pm4g.pm4g_prepare(c, a, t, A)
    torch.cuda.synchronize()
    return p


def _run(p, k, seed, by_events, out=None):
    f = pm4g.pm4g_sample(p, k, seed, by_events, out=out)
    torch.cuda.synchronize()
    K = int(f.n_cases.item())
    off = f.case_off[:K + 1].cpu().numpy()
    m = int(off[K])
    return dict(case_s=f.case_s[:m].cpu().numpy(), act_s=f.act_s[:m].cpu().numpy(), ts_s=f.ts_s[:m].cpu().numpy(),
                case_off=off, case_code=f.case_code[:K].cpu().numpy(), n_cases=K, n_events=m,
                status=int(f.status.item()))


def _check(log_cols, A, p, k, seed, by_events):
    g = _run(p, k, seed, by_events)
    o = oracle.sample(*log_cols, A, k, seed, by_events)
    assert g["status"] == 0
    assert g["n_events"] == o["n_events"] and g["n_cases"] == o["n_cases"], (k, seed, by_events)
    for key in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(g[key], o[key]), (key, k, seed, by_events)
    if g["n_events"]:
        starts = np.flatnonzero(np.r_[True, g["case_s"][1:] != g["case_s"][:-1]])
        assert np.array_equal(g["case_off"][:-1], starts)
        assert np.array_equal(g["case_code"], g["case_s"][starts])
    return g


@pytest.mark.parametrize("k_cfg,scale", [(2, 0.02), (3, 0.005)])
def test_workloads(k_cfg, scale):
    log = synth.config_log(k_cfg, scale)
    A = log.n_activities
    note(f"sampling: config {k_cfg} scale {scale}: N={log.n_events}")
    p = _prep(log.case, log.act, log.ts, A)
    C = int(p.n_cases.item())
    lc = (log.case, log.act, log.ts)
    for by_events, total in ((False, C), (True, log.n_events)):
        for k in (0, 1, 37, total // 10, total - 1, total, total + 3):
            for seed in (0, 12345, 2**64 - 1):
                _check(lc, A, p, k, seed, by_events)


def test_nested_samples_and_capacity():
    log = synth.config_log(2, 0.01)
    A = log.n_activities
    p = _prep(log.case, log.act, log.ts, A)
    small = _run(p, 100, 9, False)
    large = _run(p, 1000, 9, False)
    assert set(small["case_code"].tolist()) <= set(large["case_code"].tolist())
    out = pm4g.Prepared.empty(50, A, p.case_s.device)
    g = _run(p, 1000, 9, False, out=out)              # 1000 cases hold more than 50 events
    assert g["status"] == pm4g.PM4G_E_CAPACITY and g["n_events"] == 0
    g = _run(p, 50, 9, True, out=out)                 # exactly 50 events fit
    assert g["status"] == 0 and g["n_events"] == 50


def test_empty_and_negative_case_ids():
    A = 4
    e = _prep(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), A)
    for by_events in (False, True):
        g = _run(e, 5, 1, by_events)
        assert g["n_events"] == 0 and g["n_cases"] == 0 and g["status"] == 0
    rng = np.random.default_rng(3)
    case = rng.integers(-(2**31), 2**31 - 1, 5000)
    act = rng.integers(0, A, case.size)
    ts = rng.integers(0, 100, case.size)
    p = _prep(case, act, ts, A)
    for by_events in (False, True):
        _check((case, act, ts), A, p, 777, 2024, by_events)
    with pytest.raises(pm4g.Pm4gError):
        pm4g.pm4g_sample(p, -1, 0)
