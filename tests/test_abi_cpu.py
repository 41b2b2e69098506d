"""The C-ABI library on the CPU: it loads, exports what include/pm4g.h
declares, sizes workspaces, and rejects bad arguments before any device work.
No call here reaches a HIP runtime function (no GPU is needed)."""
import ctypes
import os
import re

import pytest

from paper_2204_04898_amd import pm4g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pm4g.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pm4g_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = pm4g.load()
    names = declared_functions()
    assert "pm4g_dfg" in names and "pm4g_variants" in names and "pm4g_prepare" in names
    for n in names:
        assert hasattr(lib, n), n
    assert lib.pm4g_abi_version() == 2


def test_workspace_sizes():
    lib = pm4g.load()
    for op in (pm4g.OP_PREPARE, pm4g.OP_DFG, pm4g.OP_DFG_PREPARED, pm4g.OP_VARIANTS,
               pm4g.OP_VARIANTS_PREPARED):
        for n, A in ((0, 1), (1, 16), (100_000, 64), (10_000_000, 512), (1000, 4096)):
            assert lib.pm4g_workspace_bytes(op, n, A, 0) > 0
    assert lib.pm4g_workspace_bytes(pm4g.OP_DFG, -1, 16, 0) == 0
    assert lib.pm4g_workspace_bytes(pm4g.OP_DFG, 10, 0, 0) == 0
    assert lib.pm4g_workspace_bytes(pm4g.OP_DFG, 10, 4097, 0) == 0
    assert lib.pm4g_workspace_bytes(pm4g.OP_DFG, 2**31, 16, 0) == 0
    assert lib.pm4g_workspace_bytes(99, 10, 16, 0) == 0
    # the raw-log DFG needs the formatted log on top of the aggregation space
    assert lib.pm4g_workspace_bytes(pm4g.OP_DFG, 10**6, 64, 0) > lib.pm4g_workspace_bytes(
        pm4g.OP_DFG_PREPARED, 10**6, 64, 0)


def _fake(n):   # non-NULL host addresses: validation never dereferences them
    return ctypes.c_void_p(0x1000)


def test_validation_before_any_device_work():
    lib = pm4g.load()
    out = pm4g._DfgOut(*[_fake(0)] * 11)
    ws = ctypes.c_void_p(0x1000)
    # NULL log
    assert lib.pm4g_dfg(None, ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    assert b"NULL" in lib.pm4g_last_error()
    log = pm4g._Log(_fake(0), _fake(0), _fake(0), 10, 0, 0)          # A = 0
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    log = pm4g._Log(_fake(0), _fake(0), _fake(0), 10, 4097, 0)       # A too large
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    log = pm4g._Log(_fake(0), _fake(0), _fake(0), -5, 16, 0)         # n < 0
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    log = pm4g._Log(_fake(0), _fake(0), _fake(0), 10, 16, 0x8)       # unknown flag
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    log = pm4g._Log(None, _fake(0), _fake(0), 10, 16, 0)             # NULL column
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    log = pm4g._Log(_fake(0), _fake(0), _fake(0), 10, 16, 0)
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(out), ws, 16, None) == pm4g.PM4G_E_WORKSPACE
    assert b"workspace" in lib.pm4g_last_error()
    bad = pm4g._DfgOut(*([_fake(0)] * 10 + [None]))                   # NULL status
    assert lib.pm4g_dfg(ctypes.byref(log), ctypes.byref(bad), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    vout = pm4g._VarOut(*([None] * 8))
    assert lib.pm4g_variants(ctypes.byref(log), ctypes.byref(vout), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    prep = pm4g._Prepared(_fake(0), _fake(0), _fake(0), None, None, None, None, 10, 16)
    vout = pm4g._VarOut(*([_fake(0)] * 8))
    assert lib.pm4g_variants_prepared(ctypes.byref(prep), ctypes.byref(vout), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    p2 = pm4g._Prepared(_fake(0), _fake(0), _fake(0), _fake(0), _fake(0), _fake(0), _fake(0), 10, 16)
    assert lib.pm4g_prepare(ctypes.byref(log), ctypes.byref(pm4g._Prepared(*([_fake(0)] * 7), 11, 16)),
                            ws, 1 << 40, None) == pm4g.PM4G_E_INVALID   # n differs
    assert p2.n_events == 10


def test_status_strings():
    lib = pm4g.load()
    for code in range(-6, 1):
        assert lib.pm4g_status_string(code)
    assert lib.pm4g_status_string(-99) == b"unknown status"


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(pm4g, "_lib", None)
    monkeypatch.setattr(pm4g, "LIB_PATH", "/nonexistent/libpm4g.so")
    with pytest.raises(RuntimeError, match="missing"):
        pm4g.load()


def test_batched_and_filter_validation():
    lib = pm4g.load()
    ws = ctypes.c_void_p(0x1000)
    prep = pm4g._Prepared(*([_fake(0)] * 7), 100, 2000)        # A above the batched limit
    out = pm4g._BatchedOut(*([_fake(0)] * 13), 10, _fake(0), _fake(0))
    assert lib.pm4g_dfg_batched(ctypes.byref(prep), _fake(0), _fake(0), 4, ctypes.byref(out), None, ws,
                                1 << 40, None) == pm4g.PM4G_E_INVALID
    prep = pm4g._Prepared(*([_fake(0)] * 7), 100, 16)
    assert lib.pm4g_dfg_batched(ctypes.byref(prep), None, None, 4, ctypes.byref(out), None, ws,
                                1 << 40, None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_dfg_batched(ctypes.byref(prep), _fake(0), _fake(0), -1, ctypes.byref(out), None, ws,
                                1 << 40, None) == pm4g.PM4G_E_INVALID
    bad_t = pm4g.BatchedTuning(tile_events=1000)
    assert lib.pm4g_dfg_batched(ctypes.byref(prep), _fake(0), _fake(0), 4, ctypes.byref(out),
                                ctypes.byref(bad_t), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_dfg_batched(ctypes.byref(prep), _fake(0), _fake(0), 4, ctypes.byref(out), None, ws,
                                16, None) == pm4g.PM4G_E_WORKSPACE
    assert lib.pm4g_batched_workspace_bytes(100, 16, 4, None) > 0
    assert lib.pm4g_batched_workspace_bytes(100, 2000, 4, None) == 0
    # (view, cell bucket) pairs at and past 2^32: A = 1024 has 257 buckets
    big = pm4g._Prepared(*([_fake(0)] * 7), 100, 1024)
    v_ok, v_over = (2**32 - 1) // 257, (2**32 - 1) // 257 + 1
    assert lib.pm4g_batched_workspace_bytes(100, 1024, v_over, None) == 0
    assert lib.pm4g_dfg_batched(ctypes.byref(big), _fake(0), _fake(0), v_over, ctypes.byref(out), None, ws,
                                1 << 40, None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_batched_workspace_bytes(100, 1024, v_ok, None) > 0
    t = pm4g.BatchedTuning(record_capacity=10**6)
    assert lib.pm4g_batched_workspace_bytes(100, 16, 4, ctypes.byref(t)) > lib.pm4g_batched_workspace_bytes(
        100, 16, 4, None)
    fo = pm4g._Prepared(*([_fake(0)] * 7), 100, 8)                 # A differs
    assert lib.pm4g_filter_view(ctypes.byref(prep), _fake(0), _fake(0), ctypes.byref(fo), ws, 1 << 40,
                                None) == pm4g.PM4G_E_INVALID
    fo = pm4g._Prepared(*([_fake(0)] * 7), 100, 16)
    assert lib.pm4g_filter_view(ctypes.byref(prep), None, _fake(0), ctypes.byref(fo), ws, 1 << 40,
                                None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_filter_view(ctypes.byref(prep), _fake(0), _fake(0), ctypes.byref(fo), ws, 8,
                                None) == pm4g.PM4G_E_WORKSPACE


def test_later_workspace_sizes_and_limits():
    lib = pm4g.load()
    for n in (0, 1, 10**6):
        assert lib.pm4g_filter_cases_workspace_bytes(n) > 0
        assert lib.pm4g_sample_workspace_bytes(n) > 0
        assert lib.pm4g_efg_workspace_bytes(n, 512) > 0
        assert lib.pm4g_ingest_csv_workspace_bytes(n * 40, n) > 0
    assert lib.pm4g_efg_workspace_bytes(10, 4096) > 0
    assert lib.pm4g_efg_workspace_bytes(10, 4097) == 0
    assert lib.pm4g_efg_workspace_bytes(10, 0) == 0
    assert lib.pm4g_efg_workspace_bytes(2**31, 16) == 0
    assert lib.pm4g_sample_workspace_bytes(2**31) == 0
    assert lib.pm4g_filter_cases_workspace_bytes(-1) == 0
    assert lib.pm4g_ingest_csv_workspace_bytes(100, 2**31) == 0
    assert lib.pm4g_ingest_csv_workspace_bytes(-1, 10) == 0


def test_later_entry_points_validate_before_any_device_work():
    lib = pm4g.load()
    f = _fake(0)
    ws = ctypes.c_void_p(0x1000)
    prep = pm4g._Prepared(f, f, f, f, f, f, f, 10, 8)
    out = pm4g._Prepared(f, f, f, f, f, f, f, 10, 8)
    # sampling: k < 0, by_events outside {0, 1}
    assert lib.pm4g_sample(ctypes.byref(prep), -1, 0, 0, ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_sample(ctypes.byref(prep), 1, 0, 2, ctypes.byref(out), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    # directly-follows filter: side and keep are 0 or 1, the pair set is required
    assert lib.pm4g_filter_df_events(ctypes.byref(prep), f, 2, 1, ctypes.byref(out), ws, 1 << 40,
                                     None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_filter_df_events(ctypes.byref(prep), None, 0, 1, ctypes.byref(out), ws, 1 << 40,
                                     None) == pm4g.PM4G_E_INVALID
    # case filter: path_keep / variant_keep are 0 or 1; a variant set needs case_variant
    cf = pm4g.CaseFilter(0, pm4g.I64_MAX, pm4g.I64_MIN, pm4g.I64_MAX, None, None, 2, 1, pm4g.I64_MIN,
                         pm4g.I64_MAX, pm4g.I64_MIN, pm4g.I64_MAX, None, None, None, None, 0)
    assert lib.pm4g_filter_cases(ctypes.byref(prep), ctypes.byref(cf), ctypes.byref(out), ws, 1 << 40,
                                 None) == pm4g.PM4G_E_INVALID
    cf.path_keep = 1
    cf.variant_mask = f
    assert lib.pm4g_filter_cases(ctypes.byref(prep), ctypes.byref(cf), ctypes.byref(out), ws, 1 << 40,
                                 None) == pm4g.PM4G_E_INVALID
    assert b"case_variant" in lib.pm4g_last_error()
    # the EFG above its activity limit (the prepared log itself allows 4096)
    big = pm4g._Prepared(f, f, f, f, f, f, f, 10, 4097)
    eo = pm4g._EfgOut(*[f] * 9)
    assert lib.pm4g_efg(ctypes.byref(big), ctypes.byref(eo), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    # CSV: separator, timestamp scale and workspace
    sc = pm4g.CsvSchema(0, 1, 2, 1, 1, 3, b'"', b"\0" * 7)
    co = pm4g._CsvOut(f, f, f, 10, f, f, f, f, f, f, f, f, f)
    assert lib.pm4g_ingest_csv(f, 100, ctypes.byref(sc), ctypes.byref(co), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    sc.sep, sc.ts_scale = b",", 10
    assert lib.pm4g_ingest_csv(f, 100, ctypes.byref(sc), ctypes.byref(co), ws, 1 << 40, None) == pm4g.PM4G_E_INVALID
    sc.ts_scale = 3
    assert lib.pm4g_ingest_csv(f, 100, ctypes.byref(sc), ctypes.byref(co), ws, 16, None) == pm4g.PM4G_E_WORKSPACE


def test_noalloc_rejects_oversized_logs_before_device_work():
    # the size check precedes the scratch lookup, so it runs without a GPU
    lib = pm4g.load()
    A, n = 512, 20_000_000
    assert lib.pm4g_workspace_bytes(pm4g.OP_DFG_PREPARED, n, A, 0) > pm4g.PM4G_NOALLOC_SCRATCH_BYTES
    p = pm4g._Prepared(_fake(0), _fake(0), _fake(0), _fake(0), _fake(0), _fake(0), _fake(0), n, A)
    out = pm4g._DfgOut(*[_fake(0)] * 11)
    assert lib.pm4g_dfg_prepared_noalloc(ctypes.byref(p), ctypes.byref(out), None) == pm4g.PM4G_E_WORKSPACE
    assert b"scratch" in lib.pm4g_last_error()
    # every log of at most 64 activities fits
    for n in (0, 1, 10**6, 2**31 - 1):
        assert lib.pm4g_workspace_bytes(pm4g.OP_DFG_PREPARED, n, 64, 0) <= pm4g.PM4G_NOALLOC_SCRATCH_BYTES
    bad = pm4g._Prepared(_fake(0), _fake(0), _fake(0), _fake(0), _fake(0), _fake(0), _fake(0), 10, 0)
    assert lib.pm4g_dfg_prepared_noalloc(ctypes.byref(bad), ctypes.byref(out), None) == pm4g.PM4G_E_INVALID
    assert lib.pm4g_dfg_prepared_noalloc(None, ctypes.byref(out), None) == pm4g.PM4G_E_INVALID
