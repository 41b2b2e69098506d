"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it element by element with the CPU oracle."""
import sys

import numpy as np
import torch

import oracle
from paper_2204_04898_amd import pm4g

DEV = "cuda:0"


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(DEV)


def cols(case, act, ts):
    return dev(case, np.int32), dev(act, np.int32), dev(ts, np.int64)


def same_f64(a, b) -> bool:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    return np.array_equal(a.view(np.int64), b.view(np.int64))


def assert_dfg_equal(g: dict, o: dict, A: int):
    for k in ("count", "dt_sum", "dt_min", "dt_max"):
        if not np.array_equal(g[k], o[k]):
            bad = np.argwhere(g[k] != o[k])[:5]
            raise AssertionError(f"{k} differs at {bad.tolist()}: gpu {[g[k][tuple(i)] for i in bad]} "
                                 f"oracle {[o[k][tuple(i)] for i in bad]}")
    assert same_f64(g["dt_mean"], o["dt_mean"]), "dt_mean differs"
    for k in ("act_count", "start_count", "end_count"):
        assert np.array_equal(g[k], o[k]), k
    assert g["n_cases"] == o["n_cases"], (g["n_cases"], o["n_cases"])
    assert g["overflow"] == o["overflow"]
    assert g["status"] == 0


def gpu_dfg(case, act, ts, A, presorted=False):
    c, a, t = cols(case, act, ts)
    o = pm4g.pm4g_dfg(c, a, t, A, presorted=presorted)
    torch.cuda.synchronize()
    return pm4g.dfg_to_host(o, A)


def check_dfg(case, act, ts, A, presorted=False):
    g = gpu_dfg(case, act, ts, A, presorted)
    o = oracle.dfg(case, act, ts, A)
    assert_dfg_equal(g, o, A)
    return g


def check_prepare(case, act, ts, A, presorted=False):
    """The formatted log against the oracle's, without and with the row
    permutation (the two sort variants), the rows element by element."""
    c, a, t = cols(case, act, ts)
    o = oracle.prepare(case, act, ts, A)
    for rows in (False, True):
        p = pm4g.pm4g_prepare(c, a, t, A, presorted=presorted, rows=rows)
        torch.cuda.synchronize()
        h = pm4g.prepared_to_host(p)
        assert h["status"] == 0
        assert h["n_cases"] == o["n_cases"]
        assert np.array_equal(h["case_s"], o["case_s"]), "case_s"
        assert np.array_equal(h["act_s"], o["act_s"]), "act_s"
        assert np.array_equal(h["ts_s"], o["ts_s"]), "ts_s"
        assert np.array_equal(h["case_off"], o["case_off"]), "case_off"
        assert np.array_equal(h["case_code"], o["case_code"]), "case_code"
        if rows:
            assert np.array_equal(h["row"], o["row"]), "row"
    return p


def assert_variants_equal(g: dict, o: dict):
    assert g["status"] == 0
    assert g["n_variants"] == o["n_variants"], (g["n_variants"], o["n_variants"])
    for k in ("var_count", "var_len", "var_rep", "var_off", "var_acts", "case_variant"):
        if not np.array_equal(g[k], o[k]):
            bad = np.flatnonzero(g[k] != o[k])[:5]
            raise AssertionError(f"{k} differs at {bad.tolist()}")


def check_variants(case, act, ts, A, presorted=False):
    c, a, t = cols(case, act, ts)
    v = pm4g.pm4g_variants(c, a, t, A, presorted=presorted)
    torch.cuda.synchronize()
    o = oracle.variants(case, act, ts, A)
    g = pm4g.variants_to_host(v, o["n_cases"])
    assert_variants_equal(g, o)
    return g
