"""Parquet ingestion on the GPU against the oracle's reader, element by
element: the road-fines fixtures, pyarrow-written files in every covered
layout (dictionary or PLAIN values, data pages v1 and v2, required and
optional columns, many row groups and pages, integer and string columns), a
10M-event log, forced value-hash collisions, nulls, and unsupported or
malformed files."""
import io
import os

import numpy as np
import pyarrow as pa
import pyarrow.parquet as pq
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import note

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dev(data: bytes):
    return torch.frombuffer(bytearray(data), dtype=torch.uint8).to("cuda:0")


def _write(table, **kw):
    buf = io.BytesIO()
    pq.write_table(table, buf, compression="NONE", **kw)
    return buf.getvalue()


def _check(data: bytes, cols=(0, 1, 2)):
    g = pm4g.pm4g_ingest_parquet(_dev(data), *cols)
    o = oracle.ingest_parquet(data, *cols)
    assert g["n_rows"] == o["n_rows"] and g["n_cases"] == o["n_cases"] and g["n_acts"] == o["n_acts"]
    assert np.array_equal(g["case_code"].cpu().numpy(), o["case"])
    assert np.array_equal(g["act_code"].cpu().numpy(), o["act"])
    assert np.array_equal(g["ts"].cpu().numpy(), o["ts"])
    for k in ("case", "act"):
        assert np.array_equal(g[k + "_dict_off"].cpu().numpy(), o[k + "_off"]), k
        assert np.array_equal(g[k + "_dict_len"].cpu().numpy(), o[k + "_len"]), k
    return g


@pytest.mark.parametrize("name", ["road_fines_dict_v1.parquet", "road_fines_plain_v2.parquet"])
def test_golden(name):
    note(f"parquet golden {name}")
    _check(open(os.path.join(GOLDEN, name), "rb").read())


def _table(rng, n, case_kind="int64", act_kind="string", ts_kind="int64", n_cases=300, n_acts=40):
    case = rng.integers(-2**31, 2**31, n_cases)[rng.integers(0, n_cases, n)]
    acts = np.array([f"activity {k} " + "x" * int(rng.integers(0, 30)) for k in range(n_acts)], dtype=object)
    act = rng.integers(0, n_acts, n)
    ts = rng.integers(-2**62, 2**62, n)
    return pa.table({
        "case": {"int64": pa.array(case.astype(np.int64)), "int32": pa.array(case.astype(np.int32)),
                 "string": pa.array([f"c{x}" for x in case])}[case_kind],
        "activity": {"string": pa.array(list(acts[act])), "int32": pa.array(act.astype(np.int32)),
                     "int64": pa.array((act.astype(np.int64) << 40) - 7)}[act_kind],
        "time": {"int64": pa.array(ts), "int32": pa.array((ts >> 40).astype(np.int32)),
                 "ts_ns": pa.array(ts, pa.timestamp("ns")), "ts_ms": pa.array(ts >> 20, pa.timestamp("ms"))}[ts_kind],
    })


LAYOUTS = [dict(use_dictionary=d, data_page_version=v) for d in (True, False) for v in ("1.0", "2.0")]


@pytest.mark.parametrize("layout", LAYOUTS, ids=lambda l: f"dict{int(l['use_dictionary'])}-v{l['data_page_version']}")
@pytest.mark.parametrize("kinds", [("int64", "string", "int64"), ("int32", "int32", "ts_ns"),
                                   ("string", "string", "ts_ms"), ("int64", "int64", "int32")])
def test_layouts(layout, kinds):
    rng = np.random.default_rng(abs(hash((kinds, str(layout)))) % 2**32)
    note(f"parquet layout {layout} {kinds}")
    _check(_write(_table(rng, 20_000, *kinds), row_group_size=7_000, data_page_size=4096, **layout))


def test_required_columns_dictionary_fallback_and_column_order():
    rng = np.random.default_rng(3)
    t = _table(rng, 30_000)
    t = t.cast(pa.schema([pa.field(f.name, f.type, nullable=False) for f in t.schema]))
    for layout in LAYOUTS:
        _check(_write(t, row_group_size=2_500, data_page_size=1024, **layout))
    n = 60_000
    t2 = pa.table({"case": pa.array([f"case-{x:012d}" for x in rng.permutation(n)]),
                   "activity": pa.array([f"a{x}" for x in rng.integers(0, 50, n)]),
                   "time": pa.array(rng.integers(0, 2**40, n))})
    _check(_write(t2, dictionary_pagesize_limit=16_384, data_page_size=8192))
    t3 = pa.table({"time": t.column(2), "other": pa.array(rng.random(t.num_rows)), "activity": t.column(1),
                   "case": t.column(0)})
    _check(_write(t3), cols=(3, 2, 0))
    _check(_write(_table(rng, 0)))


def test_event_log_of_10M_events():
    """The 10M-event log with string activities and ms timestamps, as pyarrow
    writes it by default (dictionary pages, 1 MiB data pages) but uncompressed."""
    log = synth.config_log(2)
    names = np.array([f"Activity {k:04d}" for k in range(log.n_activities)], dtype=object)
    t = pa.table({"case:concept:name": pa.array(log.case), "concept:name": pa.array(list(names[log.act])),
                  "time:timestamp": pa.array(log.ts, pa.timestamp("ms"))})
    data = _write(t)
    note(f"parquet 10M: {len(data)} bytes")
    g = _check(data)
    assert g["n_rows"] == log.n_events


def test_hash_collisions_are_resolved():
    rng = np.random.default_rng(9)
    data = _write(_table(rng, 5000, "string", "string", "int64", n_cases=2000), data_page_size=2048)
    old = pm4g.load().pm4g_debug_csv_hash_bits(3)
    try:
        _check(data)
    finally:
        pm4g.load().pm4g_debug_csv_hash_bits(old)


@pytest.mark.parametrize("col", [0, 1, 2])
def test_null_reported_at_its_row(col):
    rng = np.random.default_rng(7 + col)
    t = _table(rng, 9000)
    arrs = [t.column(k).to_pylist() for k in range(3)]
    arrs[col][4321] = None
    arrs[(col + 1) % 3][8000] = None
    t2 = pa.table({nm: pa.array(a, t.schema.field(k).type) for k, (nm, a) in enumerate(zip(t.column_names, arrs))})
    data = _write(t2, row_group_size=3000, data_page_size=2048)
    with pytest.raises(pm4g.Pm4gError) as e:
        pm4g.pm4g_ingest_parquet(_dev(data), 0, 1, 2)
    assert e.value.code == pm4g.PM4G_E_PARSE and "4321" in str(e.value)


def test_unsupported_and_malformed():
    rng = np.random.default_rng(8)
    t = _table(rng, 3000)
    buf = io.BytesIO()
    pq.write_table(t, buf, compression="SNAPPY")
    with pytest.raises(pm4g.Pm4gError) as e:
        pm4g.pm4g_ingest_parquet(_dev(buf.getvalue()), 0, 1, 2)
    assert e.value.code == pm4g.PM4G_E_UNSUPPORTED
    good = _write(t)
    for bad in (good[:-1], b"PAR1" + good[4:-4] + b"XXXX", good[:4] + bytes(26) + good[30:]):
        with pytest.raises(pm4g.Pm4gError) as e:
            pm4g.pm4g_ingest_parquet(_dev(bad), 0, 1, 2, capacity=3000)
        assert e.value.code in (pm4g.PM4G_E_PARSE, pm4g.PM4G_E_INVALID)
    with pytest.raises(pm4g.Pm4gError) as e:
        pm4g.pm4g_ingest_parquet(_dev(good), 0, 1, 7)
    assert e.value.code == pm4g.PM4G_E_INVALID
    with pytest.raises(pm4g.Pm4gError) as e:
        pm4g.pm4g_ingest_parquet(_dev(good), 0, 1, 2, capacity=10)
    assert e.value.code == pm4g.PM4G_E_CAPACITY


def test_pages_of_few_values_and_long_byte_arrays():
    """Pages of a few values each (more than the page table reserves, so the
    decode walks the headers again) and byte arrays longer than the chain
    walk's candidate window (entries found by walking a segment directly)."""
    rng = np.random.default_rng(21)
    t = _table(rng, 3_000, "string", "string", "int64", n_cases=900)
    _check(_write(t, data_page_size=64, write_batch_size=4))
    _check(_write(t, data_page_size=64, write_batch_size=4, use_dictionary=False, data_page_version="2.0"))
    n = 4_000
    long_case = pa.array(["case " + "y" * int(rng.integers(0, 900)) + str(x) for x in rng.integers(0, 700, n)])
    t2 = pa.table({"case": long_case, "activity": pa.array([f"a{x}" for x in rng.integers(0, 30, n)]),
                   "time": pa.array(rng.integers(0, 2**40, n))})
    _check(_write(t2, use_dictionary=False))
    _check(_write(t2, dictionary_pagesize_limit=100_000))
