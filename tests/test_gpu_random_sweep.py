"""A seeded sweep of small random logs of varied shape through every entry
point, each against the oracle bit-exactly: activity counts from 1 to 600
(one LDS table and bucketed paths), case ids over the whole int32 range,
timestamps with ties, negatives and wide gaps, rows shuffled or presorted,
and random predicates for the filters and sampling."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g
from tests.gpu_util import assert_dfg_equal, assert_variants_equal, cols, dev, note, same_f64

pytestmark = pytest.mark.gpu


def _random_log(rng):
    A = int(rng.choice([1, 2, 7, 64, 65, 300, 600]))
    C = int(rng.integers(1, 3000))
    law = rng.integers(0, 3)
    if law == 0:
        L = rng.integers(1, 4, C)
    elif law == 1:
        L = rng.geometric(0.08, C)
    else:
        L = np.clip(rng.lognormal(2.0, 1.2, C).astype(np.int64), 1, 600)
    codes = rng.choice(np.arange(-(2**31), 2**31 - 1, 9973, dtype=np.int64), C, replace=False).astype(np.int32)
    case = np.repeat(codes, L)
    n = case.size
    act = rng.integers(0, A, n).astype(np.int32)
    ts_kind = rng.integers(0, 3)
    if ts_kind == 0:
        ts = rng.integers(-5, 5, n)                                   # many ties
    elif ts_kind == 1:
        ts = rng.integers(0, 10**13, n)
    else:
        ts = rng.integers(-(2**61), 2**61, n)                         # wide gaps
    presorted = bool(rng.integers(0, 2)) and ts_kind != 0
    if presorted:
        order = np.lexsort((np.arange(n), ts, case))
    else:
        order = rng.permutation(n)
    return case[order], act[order], ts[order].astype(np.int64), A, presorted


def _mask(bits, nbits):
    m = np.zeros(max((nbits + 63) // 64, 1), np.uint64)
    for b in bits:
        m[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    return m


def _prepared_events(f):
    K = int(f.n_cases.item())
    m = int(f.case_off[K].item())
    return f.case_s[:m].cpu().numpy(), f.act_s[:m].cpu().numpy(), f.ts_s[:m].cpu().numpy()


@pytest.mark.parametrize("seed", range(24))
def test_sweep(seed):
    rng = np.random.default_rng(7000 + seed)
    case, act, ts, A, presorted = _random_log(rng)
    note(f"sweep seed {seed}: N={case.size} A={A} presorted={presorted}")
    c, a, t = cols(case, act, ts)
    p = pm4g.pm4g_prepare(c, a, t, A, presorted=presorted)
    torch.cuda.synchronize()
    assert int(p.status.item()) == 0
    assert_dfg_equal(pm4g.dfg_to_host(pm4g.pm4g_dfg_prepared(p), A), oracle.dfg(case, act, ts, A), A)
    C = int(p.n_cases.item())
    v = pm4g.pm4g_variants_prepared(p)
    assert_variants_equal(pm4g.variants_to_host(v, C), oracle.variants(case, act, ts, A))
    # cases dataframe and a random case filter
    cd = pm4g.pm4g_cases(p)
    oc = oracle.cases(case, act, ts, A)
    assert np.array_equal(cd["n_events"][:C].cpu().numpy(), oc["n_events"])
    assert np.array_equal(cd["throughput"][:C].cpu().numpy(), oc["throughput"])
    nv = int(v["n_variants"].item())
    kw = dict(min_events=int(rng.integers(0, 3)), max_events=int(rng.integers(3, 50)),
              contain_lo=int(np.percentile(ts, 10)), meet_hi=int(np.percentile(ts, 90)),
              start_mask=_mask(rng.choice(A, max(1, A // 2), replace=False), A),
              path_mask=_mask(rng.choice(A * A, max(1, A * A // 3), replace=False), A * A),
              path_keep=bool(rng.integers(0, 2)),
              variant_mask=_mask(range(0, nv, 2), nv), n_variant_bits=nv, variant_keep=bool(rng.integers(0, 2)))
    gkw = dict(kw)
    for k in ("start_mask", "path_mask", "variant_mask"):
        gkw[k] = dev(kw[k].view(np.int64), np.int64)
    f = pm4g.pm4g_filter_cases(p, case_variant=v["case_variant"], **gkw)
    torch.cuda.synchronize()
    of = oracle.filter_cases(case, act, ts, A, **kw)
    g = _prepared_events(f)
    for x, k in zip(g, ("case_s", "act_s", "ts_s")):
        assert np.array_equal(x, of[k]), k
    # directly-follows event filter, both sides
    pm = _mask(rng.choice(A * A, max(1, A * A // 4), replace=False), A * A)
    for side in (0, 1):
        keep = bool(rng.integers(0, 2))
        f = pm4g.pm4g_filter_df_events(p, dev(pm.view(np.int64), np.int64), side, keep)
        torch.cuda.synchronize()
        od = oracle.filter_df_events(case, act, ts, A, pm, side, keep)
        for x, k in zip(_prepared_events(f), ("case_s", "act_s", "ts_s")):
            assert np.array_equal(x, od[k]), (side, k)
    # sampling
    for by_events in (False, True):
        total = case.size if by_events else C
        k = int(rng.integers(0, total + 2))
        sd = int(rng.integers(0, 2**63))
        f = pm4g.pm4g_sample(p, k, sd, by_events)
        torch.cuda.synchronize()
        osm = oracle.sample(case, act, ts, A, k, sd, by_events)
        for x, kk in zip(_prepared_events(f), ("case_s", "act_s", "ts_s")):
            assert np.array_equal(x, osm[kk]), (by_events, kk)
    # eventually-follows graph
    e = pm4g.efg_to_host(pm4g.pm4g_efg(p), A)
    oe = oracle.efg(case, act, ts, A)
    assert e["n_pairs"] == oe["n_pairs"]
    for k in ("count", "sum_lo", "sum_hi", "sq_lo", "sq_hi"):
        assert np.array_equal(e[k], oe[k]), k
    assert same_f64(e["mean"], oe["mean"]) and same_f64(e["std"], oe["std"])
