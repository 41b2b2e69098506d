"""Every binding wrapper called on a stream that is not torch's current one.

The side stream is held back by a spin kernel queued first, so the library's
kernels run after the current stream has already allocated and overwritten
fresh memory.  If a wrapper allocated an output or a workspace on the current
stream and dropped it before its kernels ran, the caching allocator would hand
that memory to the current stream's writes and the results would differ from
the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import DEV, assert_dfg_equal, cols, note, same_f64

pytestmark = pytest.mark.gpu

SPIN_CYCLES = 200_000_000     # about 0.1 s at 2.4 GHz, bounded


def _clobber():
    """Allocates and overwrites a few hundred MB on the current stream."""
    junk = [torch.full((1 << 24,), -7, dtype=torch.int64, device=DEV) for _ in range(4)]
    for j in junk:
        j.add_(3)
    return junk


def _host_prepared(p):
    K = int(p.n_cases.item())
    off = p.case_off[:K + 1].cpu().numpy()
    m = int(off[K])
    return dict(case_s=p.case_s[:m].cpu().numpy(), act_s=p.act_s[:m].cpu().numpy(),
                ts_s=p.ts_s[:m].cpu().numpy(), n_cases=K)


def test_wrappers_on_a_side_stream():
    log = synth.config_log(2, 0.01)
    A = log.n_activities
    note(f"streams: N={log.n_events} A={A}")
    c, a, t = cols(log.case, log.act, log.ts)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()

    side_results = {}
    with torch.cuda.stream(side):
        torch.cuda._sleep(SPIN_CYCLES)
    # every call below is queued on `side` behind the spin, from the current stream's context
    p = pm4g.pm4g_prepare(c, a, t, A, stream=side)
    with torch.cuda.stream(side):
        torch.cuda._sleep(SPIN_CYCLES)
    side_results["dfg"] = pm4g.pm4g_dfg(c, a, t, A, stream=side)
    junk1 = _clobber()
    side_results["dfg_prep"] = pm4g.pm4g_dfg_prepared(p, stream=side)
    side_results["var"] = pm4g.pm4g_variants_prepared(p, stream=side)
    junk2 = _clobber()
    lo, hi = int(log.case.min()), int(log.case.max()) + 1
    t_lo, t_hi = int(np.quantile(log.ts, 0.2)), int(np.quantile(log.ts, 0.8))
    mask_words = np.zeros((A + 63) // 64, np.uint64)
    mask_words[0] = np.uint64(0x5555_5555_5555_5555)
    rec = np.zeros(1, dtype=np.dtype([("lo", "<i4"), ("hi", "<i4"), ("t_lo", "<i8"), ("t_hi", "<i8")]))
    rec["lo"], rec["hi"], rec["t_lo"], rec["t_hi"] = lo, hi, t_lo, t_hi
    vdev = torch.from_numpy(rec.view(np.uint8).copy()).to(DEV)
    mdev = torch.from_numpy(mask_words.view(np.int64).copy()).to(DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(SPIN_CYCLES)
    side_results["view"] = pm4g.pm4g_filter_view(p, vdev, mdev, stream=side)
    side_results["sample"] = pm4g.pm4g_sample(p, 1000, 99, stream=side)
    pair_mask = torch.zeros((A * A + 63) // 64, dtype=torch.int64, device=DEV)
    pair_mask[:4] = 0x0F0F_0F0F
    side_results["dfev"] = pm4g.pm4g_filter_df_events(p, pair_mask, stream=side)
    side_results["cases"] = pm4g.pm4g_cases(p, stream=side)
    side_results["fcases"] = pm4g.pm4g_filter_cases(p, min_events=3, max_events=20, stream=side)
    side_results["efg"] = pm4g.pm4g_efg(p, stream=side)
    junk3 = _clobber()
    side.synchronize()
    torch.cuda.synchronize()
    del junk1, junk2, junk3

    lc = (log.case, log.act, log.ts)
    od = oracle.dfg(*lc, A)
    for k in ("dfg", "dfg_prep"):
        assert_dfg_equal(pm4g.dfg_to_host(side_results[k], A), od, A)
    ov = oracle.variants(*lc, A)
    h = pm4g.variants_to_host(side_results["var"], ov["n_cases"])
    for k in ("var_count", "var_rep", "var_acts", "case_variant"):
        assert np.array_equal(h[k], ov[k]), k
    op = oracle.prepare(*lc, A)
    hp = _host_prepared(p)
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(hp[k], op[k]), k

    keep = (log.case >= lo) & (log.case < hi) & (log.ts >= t_lo) & (log.ts <= t_hi)
    keep &= ((mask_words[log.act // 64] >> (log.act % 64).astype(np.uint64)) & np.uint64(1)).astype(bool)
    ref = oracle.prepare(log.case[keep], log.act[keep], log.ts[keep], A)
    hv = _host_prepared(side_results["view"])
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(hv[k], ref[k]), ("view", k)

    osm = oracle.sample(*lc, A, 1000, 99, False)
    hs = _host_prepared(side_results["sample"])
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(hs[k], osm[k]), ("sample", k)

    pm_host = pair_mask.cpu().numpy().view(np.uint64)
    ode = oracle.filter_df_events(*lc, A, pm_host, 0, True)
    hd = _host_prepared(side_results["dfev"])
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(hd[k], ode[k]), ("df events", k)

    oc = oracle.cases(*lc, A)
    C = oc["n_cases"]
    assert np.array_equal(side_results["cases"]["n_events"][:C].cpu().numpy(), oc["n_events"])
    assert np.array_equal(side_results["cases"]["throughput"][:C].cpu().numpy(), oc["throughput"])

    ofc = oracle.filter_cases(*lc, A, min_events=3, max_events=20)
    hf = _host_prepared(side_results["fcases"])
    for k in ("case_s", "act_s", "ts_s"):
        assert np.array_equal(hf[k], ofc[k]), ("case filter", k)

    oe = oracle.efg(*lc, A)
    he = pm4g.efg_to_host(side_results["efg"], A)
    assert np.array_equal(he["count"], oe["count"])
    assert same_f64(he["mean"], oe["mean"]) and same_f64(he["std"], oe["std"])
