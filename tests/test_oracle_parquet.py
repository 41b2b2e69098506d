"""Pins of the oracle's Parquet reader against things other than itself:
the hand-worked road-fines log (tests/golden/road_fines.csv as Parquet, codes
by first appearance worked out by hand), and pyarrow (an independent
implementation of the format) with pandas.factorize on files that pyarrow
writes in every covered layout: dictionary-coded or PLAIN values, data pages
of version 1 and 2, required and optional columns, several row groups and
many pages, integer and string columns."""
import io
import os

import numpy as np
import pandas as pd
import pyarrow as pa
import pyarrow.parquet as pq
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# the ten data rows of road_fines.csv in order; codes by first appearance, by hand
RF_CASE_CODES = [0, 1, 0, 2, 1, 0, 2, 0, 0, 3]             # 7, -3, 12, 5
RF_ACT_CODES = [0, 1, 1, 1, 2, 3, 2, 4, 2, 2]              # Send Fine, Create Fine, Payment, Insert ..., Add penalty
RF_TS = [100, 50, 40, 10, 50, 160, 25, 160, 300, 70]
RF_ACTS = [b"Send Fine", b"Create Fine", b"Payment", b"Insert Fine Notification", b"Add penalty"]


@pytest.mark.parametrize("name", ["road_fines_dict_v1.parquet", "road_fines_plain_v2.parquet"])
def test_golden_road_fines(name):
    data = open(os.path.join(GOLDEN, name), "rb").read()
    o = oracle.ingest_parquet(data, 0, 1, 2)
    assert o["case"].tolist() == RF_CASE_CODES
    assert o["act"].tolist() == RF_ACT_CODES
    assert o["ts"].tolist() == RF_TS
    assert [data[a:a + b] for a, b in zip(o["act_off"], o["act_len"])] == RF_ACTS
    if "plain" in name:   # string case ids: the bytes at the first row
        assert [data[a:a + b] for a, b in zip(o["case_off"], o["case_len"])] == [b"7", b"-3", b"12", b"5"]
    else:                 # integer case ids: the value itself
        assert o["case_off"].tolist() == [7, -3, 12, 5] and o["case_len"].tolist() == [-1] * 4


def _write(table, **kw):
    buf = io.BytesIO()
    pq.write_table(table, buf, compression="NONE", **kw)
    return buf.getvalue()


def _expect(data, cols=(0, 1, 2)):
    t = pq.read_table(io.BytesIO(data))
    c = [t.column(k).to_numpy(zero_copy_only=False) for k in cols]
    ts = c[2]
    if np.issubdtype(ts.dtype, np.datetime64):
        ts = ts.view(np.int64)
    return pd.factorize(c[0])[0], pd.factorize(c[1])[0], ts.astype(np.int64), c


def _check(data, cols=(0, 1, 2)):
    o = oracle.ingest_parquet(data, *cols)
    cc, ac, ts, raw = _expect(data, cols)
    assert np.array_equal(o["case"], cc)
    assert np.array_equal(o["act"], ac)
    assert np.array_equal(o["ts"], ts)
    # the per-code values are the values at each code's first row
    for key, k in (("case", 0), ("act", 1)):
        first = np.array([np.flatnonzero(o[key] == code)[0] for code in range(int(o[key].max()) + 1)]) \
            if o["n_rows"] else np.zeros(0, np.int64)
        offs, lens = o[key + "_off"], o[key + "_len"]
        for code, row in enumerate(first):
            v = raw[k][row]
            if isinstance(v, str):
                assert data[offs[code]:offs[code] + lens[code]] == v.encode()
            else:
                assert lens[code] == -1 and offs[code] == int(v)
    return o


def _table(rng, n, case_kind="int64", act_kind="string", ts_kind="int64", n_cases=300, n_acts=40):
    case = rng.integers(-2**31, 2**31, n_cases)[rng.integers(0, n_cases, n)]
    acts = np.array([f"activity {k} " + "x" * int(rng.integers(0, 30)) for k in range(n_acts)], dtype=object)
    act = rng.integers(0, n_acts, n)
    ts = rng.integers(-2**62, 2**62, n)
    cols = {
        "case": {"int64": pa.array(case.astype(np.int64)), "int32": pa.array(case.astype(np.int32)),
                 "string": pa.array([f"c{x}" for x in case])}[case_kind],
        "activity": {"string": pa.array(list(acts[act])), "int32": pa.array(act.astype(np.int32)),
                     "int64": pa.array((act.astype(np.int64) << 40) - 7)}[act_kind],
        "time": {"int64": pa.array(ts), "int32": pa.array((ts >> 40).astype(np.int32)),
                 "ts_ns": pa.array(ts, pa.timestamp("ns")), "ts_ms": pa.array(ts >> 20, pa.timestamp("ms"))}[ts_kind],
    }
    return pa.table(cols)


LAYOUTS = [dict(use_dictionary=d, data_page_version=v) for d in (True, False) for v in ("1.0", "2.0")]


@pytest.mark.parametrize("layout", LAYOUTS, ids=lambda l: f"dict{int(l['use_dictionary'])}-v{l['data_page_version']}")
@pytest.mark.parametrize("kinds", [("int64", "string", "int64"), ("int32", "int32", "ts_ns"),
                                   ("string", "string", "ts_ms"), ("int64", "int64", "int32")])
def test_against_pyarrow(layout, kinds):
    rng = np.random.default_rng(hash((kinds, layout["data_page_version"], layout["use_dictionary"])) % 2**32)
    t = _table(rng, 20_000, *kinds)
    _check(_write(t, row_group_size=7_000, data_page_size=4096, **layout))


def test_required_columns_many_row_groups_and_pages():
    rng = np.random.default_rng(3)
    t = _table(rng, 30_000)
    t = t.cast(pa.schema([pa.field(f.name, f.type, nullable=False) for f in t.schema]))
    for layout in LAYOUTS:
        _check(_write(t, row_group_size=2_500, data_page_size=1024, **layout))


def test_large_dictionary_falls_back_to_plain_pages():
    """pyarrow stops dictionary coding a chunk when its dictionary grows past
    a limit and writes the rest of the chunk PLAIN: both kinds of data page in
    one chunk."""
    rng = np.random.default_rng(4)
    n = 60_000
    t = pa.table({"case": pa.array([f"case-{x:012d}" for x in rng.permutation(n)]),
                  "activity": pa.array([f"a{x}" for x in rng.integers(0, 50, n)]),
                  "time": pa.array(rng.integers(0, 2**40, n))})
    _check(_write(t, dictionary_pagesize_limit=16_384, data_page_size=8192))


def test_column_order_and_extra_columns():
    rng = np.random.default_rng(5)
    t = _table(rng, 5000)
    t = pa.table({"time": t.column(2), "other": pa.array(rng.random(5000)), "activity": t.column(1),
                  "case": t.column(0)})
    _check(_write(t), cols=(3, 2, 0))


def test_empty_table():
    t = _table(np.random.default_rng(6), 0)
    o = _check(_write(t))
    assert o["n_rows"] == 0 and o["n_cases"] == 0


@pytest.mark.parametrize("col", [0, 1, 2])
def test_null_is_a_parse_error_at_its_row(col):
    rng = np.random.default_rng(7 + col)
    t = _table(rng, 9000)
    arrs = [t.column(k).to_pylist() for k in range(3)]
    arrs[col][4321] = None
    arrs[(col + 1) % 3][8000] = None
    t2 = pa.table({n: pa.array(a, t.schema.field(k).type) for k, (n, a) in enumerate(zip(t.column_names, arrs))})
    data = _write(t2, row_group_size=3000, data_page_size=2048)
    with pytest.raises(oracle.CsvParseError) as e:
        oracle.ingest_parquet(data, 0, 1, 2)
    assert e.value.row == 4321


def test_unsupported_and_malformed():
    rng = np.random.default_rng(8)
    t = _table(rng, 3000)
    buf = io.BytesIO()
    pq.write_table(t, buf, compression="SNAPPY")
    with pytest.raises(oracle.ParquetUnsupported):
        oracle.ingest_parquet(buf.getvalue(), 0, 1, 2)
    nested = pa.table({"case": pa.array([[1, 2], [3]]), "activity": pa.array(["a", "b"]),
                       "time": pa.array([1, 2])})
    with pytest.raises(oracle.ParquetUnsupported):
        oracle.ingest_parquet(_write(nested), 0, 1, 2)
    good = _write(t)
    for bad in (good[:-1], good[:100], b"PAR1" + good[4:-4] + b"XXXX", good[:4] + bytes(26) + good[30:]):
        with pytest.raises(oracle.OracleError):
            oracle.ingest_parquet(bad, 0, 1, 2)
    with pytest.raises(oracle.OracleError):
        oracle.ingest_parquet(good, 0, 1, 7)          # no such column
    with pytest.raises(oracle.OracleError):
        oracle.ingest_parquet(good, 0, 1, 2, max_rows=10)
    dbl = pa.table({"case": pa.array([1.5]), "activity": pa.array(["a"]), "time": pa.array([1])})
    with pytest.raises(oracle.ParquetUnsupported):
        oracle.ingest_parquet(_write(dbl), 0, 1, 2)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.data())
def test_hypothesis_tables(data):
    n = data.draw(st.integers(0, 300))
    strs = st.text(alphabet=st.characters(min_codepoint=32, max_codepoint=0x2FF), max_size=12)
    case = data.draw(st.lists(st.sampled_from(data.draw(st.lists(strs, min_size=1, max_size=8))), min_size=n, max_size=n))
    act = data.draw(st.lists(st.integers(-2**31, 2**31 - 1), min_size=n, max_size=n))
    ts = data.draw(st.lists(st.integers(-2**63, 2**63 - 1), min_size=n, max_size=n))
    layout = data.draw(st.sampled_from(LAYOUTS))
    t = pa.table({"case": pa.array(case, pa.string()), "activity": pa.array(act, pa.int32()),
                  "time": pa.array(ts, pa.int64())})
    _check(_write(t, data_page_size=data.draw(st.sampled_from([64, 512, 1 << 20])),
                  row_group_size=data.draw(st.sampled_from([7, 100, 10_000])), **layout))
