"""CPU oracle for DFG discovery (test infrastructure only).

Loads ``libpm4g_oracle.so`` built from ``pm4g_oracle.c`` in this directory
(building it with gcc if it is missing) and wraps each function for numpy
arrays.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark import this package; the HIP library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pm4g_oracle.c")
_LIB = os.path.join(_HERE, "libpm4g_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, plain C11)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.orc_prepare.argtypes = [i64, P, P, P, i32, P, P, P, P, P, P, P]
        L.orc_dfg.argtypes = [i64, P, P, P, i32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_variants.argtypes = [i64, P, P, P, i32, P, P, P, P, P, P, P, P, P]
        L.orc_view.argtypes = [i64, P, P, P, i32, i32, i32, i64, i64, P,
                               P, P, P, P, P, P, P, P, P, P, P]
        L.orc_view_formatted.argtypes = [i64, P, P, P, i64, P, P, i32, i32, i32, i64, i64, P,
                                         P, P, P, P, P, P, P, P, P, P, P]
        L.orc_cases.argtypes = [i64, P, P, P, i32, P, P, P, P]
        L.orc_filter_cases.argtypes = [i64, P, P, P, i32, P, P, P, i32, P, P, P, i64, i32, P, P, P, P, P]
        L.orc_filter_df_events.argtypes = [i64, P, P, P, i32, P, i32, i32, P, P, P, P, P]
        L.orc_efg.argtypes = [i64, P, P, P, i32, P, P, P, P, P, P, P, P]
        L.orc_sample.argtypes = [i64, P, P, P, i32, i64, ctypes.c_uint64, i32, P, P, P, P, P]
        L.orc_ingest_csv.argtypes = [ctypes.c_char_p, i64, i32, i32, i32, ctypes.c_char, i32, i32, i32, i64,
                                     P, P, P, P, P, P, P, P, P, P, P]
        L.orc_ingest_parquet.argtypes = [ctypes.c_char_p, i64, i32, i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_splitmix.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_splitmix.restype = ctypes.c_uint64
        for f in (L.orc_prepare, L.orc_dfg, L.orc_variants, L.orc_view, L.orc_view_formatted, L.orc_cases, L.orc_filter_cases,
                  L.orc_filter_df_events, L.orc_efg, L.orc_sample, L.orc_ingest_csv, L.orc_ingest_parquet):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({-1: "invalid argument", -2: "activity out of range"}.get(code, str(code)))
        self.code = code


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cols(case, act, ts):
    case = np.ascontiguousarray(case, dtype=np.int32)
    act = np.ascontiguousarray(act, dtype=np.int32)
    ts = np.ascontiguousarray(ts, dtype=np.int64)
    if not (case.shape == act.shape == ts.shape and case.ndim == 1):
        raise ValueError("case, act, ts must be 1-D and of equal length")
    return case, act, ts


def prepare(case, act, ts, A: int) -> dict:
    """The formatted log: rows in (case, ts, row) order plus the case table."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    m = max(n, 1)
    out = dict(row=np.empty(m, np.int64), case_s=np.empty(m, np.int32), act_s=np.empty(m, np.int32),
               ts_s=np.empty(m, np.int64), case_off=np.empty(m + 1, np.int64),
               case_code=np.empty(m, np.int32))
    C = np.zeros(1, np.int64)
    rc = _load().orc_prepare(n, _p(case), _p(act), _p(ts), A, _p(out["row"]), _p(out["case_s"]),
                             _p(out["act_s"]), _p(out["ts_s"]), _p(out["case_off"]),
                             _p(out["case_code"]), _p(C))
    if rc:
        raise OracleError(rc)
    c = int(C[0])
    for k in ("row", "case_s", "act_s", "ts_s"):
        out[k] = out[k][:n]
    out["case_off"] = out["case_off"][:c + 1]
    out["case_code"] = out["case_code"][:c]
    out["n_cases"] = c
    return out


def dfg(case, act, ts, A: int, with_perm: bool = False) -> dict:
    """Frequency/performance DFG with start/end/activity counts (dense A x A)."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    cells = A * A
    o = dict(count=np.empty(cells, np.int64), dt_sum=np.empty(cells, np.int64),
             dt_min=np.empty(cells, np.int64), dt_max=np.empty(cells, np.int64),
             dt_mean=np.empty(cells, np.float64), start_count=np.empty(A, np.int64),
             end_count=np.empty(A, np.int64), act_count=np.empty(A, np.int64))
    perm = np.empty(max(n, 1), np.int64) if with_perm else None
    C = np.zeros(1, np.int64)
    ov = np.zeros(1, np.int32)
    rc = _load().orc_dfg(n, _p(case), _p(act), _p(ts), A, _p(perm) if perm is not None else None,
                         _p(o["count"]), _p(o["dt_sum"]), _p(o["dt_min"]), _p(o["dt_max"]),
                         _p(o["dt_mean"]), _p(o["start_count"]), _p(o["end_count"]),
                         _p(o["act_count"]), _p(C), _p(ov))
    if rc:
        raise OracleError(rc)
    for k in ("count", "dt_sum", "dt_min", "dt_max", "dt_mean"):
        o[k] = o[k].reshape(A, A)
    o["n_cases"] = int(C[0])
    o["overflow"] = int(ov[0])
    if perm is not None:
        o["perm"] = perm[:n]
    return o


def variants(case, act, ts, A: int) -> dict:
    """Exact trace variants, ids in (count desc, representative asc) order."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    m = max(n, 1)
    o = dict(var_count=np.empty(m, np.int64), var_len=np.empty(m, np.int32),
             var_rep=np.empty(m, np.int32), var_off=np.empty(m + 1, np.int64),
             var_acts=np.empty(m, np.int32), case_code=np.empty(m, np.int32),
             case_variant=np.empty(m, np.int32))
    V = np.zeros(1, np.int64)
    C = np.zeros(1, np.int64)
    rc = _load().orc_variants(n, _p(case), _p(act), _p(ts), A, _p(V), _p(o["var_count"]),
                              _p(o["var_len"]), _p(o["var_rep"]), _p(o["var_off"]),
                              _p(o["var_acts"]), _p(o["case_code"]), _p(o["case_variant"]), _p(C))
    if rc:
        raise OracleError(rc)
    v, c = int(V[0]), int(C[0])
    for k in ("var_count", "var_len", "var_rep"):
        o[k] = o[k][:v]
    o["var_off"] = o["var_off"][:v + 1]
    o["var_acts"] = o["var_acts"][:int(o["var_off"][v])]
    o["case_code"] = o["case_code"][:c]
    o["case_variant"] = o["case_variant"][:c]
    o["n_variants"] = v
    o["n_cases"] = c
    return o


def view(case, act, ts, A: int, case_lo: int, case_hi: int, t_lo: int, t_hi: int,
         mask) -> dict:
    """DFG of the events retained by one drill-down view (dense A x A)."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    W = (A + 63) // 64
    mask = np.ascontiguousarray(mask, dtype=np.uint64)
    if mask.shape != (W,):
        raise ValueError("mask must have ceil(A/64) words")
    cells = A * A
    o = dict(count=np.empty(cells, np.int64), dt_sum=np.empty(cells, np.int64),
             dt_min=np.empty(cells, np.int64), dt_max=np.empty(cells, np.int64),
             dt_mean=np.empty(cells, np.float64), start_count=np.empty(A, np.int64),
             end_count=np.empty(A, np.int64), act_count=np.empty(A, np.int64))
    C = np.zeros(1, np.int64)
    ov = np.zeros(1, np.int32)
    ne = np.zeros(1, np.int64)
    rc = _load().orc_view(n, _p(case), _p(act), _p(ts), A, int(case_lo), int(case_hi), int(t_lo),
                          int(t_hi), _p(mask), _p(o["count"]), _p(o["dt_sum"]), _p(o["dt_min"]),
                          _p(o["dt_max"]), _p(o["dt_mean"]), _p(o["start_count"]),
                          _p(o["end_count"]), _p(o["act_count"]), _p(C), _p(ov), _p(ne))
    if rc:
        raise OracleError(rc)
    for k in ("count", "dt_sum", "dt_min", "dt_max", "dt_mean"):
        o[k] = o[k].reshape(A, A)
    o["n_cases"] = int(C[0])
    o["overflow"] = int(ov[0])
    o["n_events"] = int(ne[0])
    return o



def view_formatted(prep: dict, A: int, case_lo: int, case_hi: int, t_lo: int, t_hi: int, mask) -> dict:
    """One drill-down view answered by a scan of the formatted log `prep`
    (the dict prepare() returns): same outputs as view()."""
    case_s = np.ascontiguousarray(prep["case_s"], dtype=np.int32)
    act_s = np.ascontiguousarray(prep["act_s"], dtype=np.int32)
    ts_s = np.ascontiguousarray(prep["ts_s"], dtype=np.int64)
    off = np.ascontiguousarray(prep["case_off"], dtype=np.int64)
    code = np.ascontiguousarray(prep["case_code"], dtype=np.int32)
    n, C = case_s.shape[0], code.shape[0]
    if off.shape != (C + 1,) or act_s.shape != (n,) or ts_s.shape != (n,):
        raise ValueError("prep is not a formatted log")
    W = (A + 63) // 64
    mask = np.ascontiguousarray(mask, dtype=np.uint64)
    if mask.shape != (W,):
        raise ValueError("mask must have ceil(A/64) words")
    cells = A * A
    o = dict(count=np.empty(cells, np.int64), dt_sum=np.empty(cells, np.int64),
             dt_min=np.empty(cells, np.int64), dt_max=np.empty(cells, np.int64),
             dt_mean=np.empty(cells, np.float64), start_count=np.empty(A, np.int64),
             end_count=np.empty(A, np.int64), act_count=np.empty(A, np.int64))
    nc = np.zeros(1, np.int64)
    ov = np.zeros(1, np.int32)
    ne = np.zeros(1, np.int64)
    rc = _load().orc_view_formatted(n, _p(case_s), _p(act_s), _p(ts_s), C, _p(off), _p(code), A,
                                    int(case_lo), int(case_hi), int(t_lo), int(t_hi), _p(mask),
                                    _p(o["count"]), _p(o["dt_sum"]), _p(o["dt_min"]), _p(o["dt_max"]),
                                    _p(o["dt_mean"]), _p(o["start_count"]), _p(o["end_count"]),
                                    _p(o["act_count"]), _p(nc), _p(ov), _p(ne))
    if rc:
        raise OracleError(rc)
    for k in ("count", "dt_sum", "dt_min", "dt_max", "dt_mean"):
        o[k] = o[k].reshape(A, A)
    o["n_cases"] = int(nc[0])
    o["overflow"] = int(ov[0])
    o["n_events"] = int(ne[0])
    return o

def cases(case, act, ts, A: int) -> dict:
    """The cases dataframe: per case (ascending code) its events and throughput time."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    m = max(n, 1)
    out = dict(case_code=np.empty(m, np.int32), n_events=np.empty(m, np.int64),
               throughput=np.empty(m, np.int64))
    C = np.zeros(1, np.int64)
    rc = _load().orc_cases(n, _p(case), _p(act), _p(ts), A, _p(out["case_code"]), _p(out["n_events"]),
                           _p(out["throughput"]), _p(C))
    if rc:
        raise OracleError(rc)
    c = int(C[0])
    return {k: v[:c] for k, v in out.items()} | {"n_cases": c}


I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def filter_cases(case, act, ts, A: int, min_events: int = 0, max_events: int = I64_MAX,
                 min_thr: int = I64_MIN, max_thr: int = I64_MAX, act_mask=None, path_mask=None,
                 path_keep: bool = True, contain_lo: int = I64_MIN, contain_hi: int = I64_MAX,
                 meet_lo: int = I64_MIN, meet_hi: int = I64_MAX, start_mask=None, end_mask=None,
                 variant_mask=None, n_variant_bits: int = 0, variant_keep: bool = True) -> dict:
    """Events (in order) of the cases passing the case-level filters."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    m = max(n, 1)
    out = dict(case_s=np.empty(m, np.int32), act_s=np.empty(m, np.int32), ts_s=np.empty(m, np.int64))
    no, nc = np.zeros(1, np.int64), np.zeros(1, np.int64)
    bounds = np.array([min_events, max_events, min_thr, max_thr, contain_lo, contain_hi, meet_lo, meet_hi],
                      dtype=np.int64)
    masks = [None if x is None else np.ascontiguousarray(x, dtype=np.uint64)
             for x in (act_mask, path_mask, start_mask, end_mask, variant_mask)]
    ptr = [None if x is None else _p(x) for x in masks]
    rc = _load().orc_filter_cases(n, _p(case), _p(act), _p(ts), A, _p(bounds), ptr[0], ptr[1],
                                  1 if path_keep else 0, ptr[2], ptr[3], ptr[4], int(n_variant_bits),
                                  1 if variant_keep else 0, _p(out["case_s"]), _p(out["act_s"]),
                                  _p(out["ts_s"]), _p(no), _p(nc))
    if rc:
        raise OracleError(rc)
    k = int(no[0])
    return {key: v[:k] for key, v in out.items()} | {"n_events": k, "n_cases": int(nc[0])}


def filter_df_events(case, act, ts, A: int, path_mask, side: int = 0, keep: bool = True) -> dict:
    """Events kept by the directly-follows-level filter: side 0 pairs an event
    with the previous event of its case, side 1 with the next one."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    m = max(n, 1)
    out = dict(case_s=np.empty(m, np.int32), act_s=np.empty(m, np.int32), ts_s=np.empty(m, np.int64))
    no, nc = np.zeros(1, np.int64), np.zeros(1, np.int64)
    pm = np.ascontiguousarray(path_mask, dtype=np.uint64)
    rc = _load().orc_filter_df_events(n, _p(case), _p(act), _p(ts), A, _p(pm), int(side), 1 if keep else 0,
                                      _p(out["case_s"]), _p(out["act_s"]), _p(out["ts_s"]), _p(no), _p(nc))
    if rc:
        raise OracleError(rc)
    k = int(no[0])
    return {key: v[:k] for key, v in out.items()} | {"n_events": k, "n_cases": int(nc[0])}


def efg(case, act, ts, A: int) -> dict:
    """Eventually-follows graph and temporal profile, [A, A] arrays: count,
    the exact 128-bit gap sum and squared-gap sum as (lo, hi) uint64 words,
    mean and sample std (FP64); n_pairs."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    cells = A * A
    out = dict(count=np.empty(cells, np.int64), sum_lo=np.empty(cells, np.uint64), sum_hi=np.empty(cells, np.uint64),
               sq_lo=np.empty(cells, np.uint64), sq_hi=np.empty(cells, np.uint64), mean=np.empty(cells, np.float64),
               std=np.empty(cells, np.float64))
    npairs = np.zeros(1, np.int64)
    rc = _load().orc_efg(n, _p(case), _p(act), _p(ts), A, _p(out["count"]), _p(out["sum_lo"]), _p(out["sum_hi"]),
                         _p(out["sq_lo"]), _p(out["sq_hi"]), _p(out["mean"]), _p(out["std"]), _p(npairs))
    if rc:
        raise OracleError(rc)
    out = {k: v.reshape(A, A) for k, v in out.items()}
    out["n_pairs"] = int(npairs[0])
    return out


def splitmix(seed: int, x: int) -> int:
    """The x-th output of SplitMix64 started from state seed."""
    return int(_load().orc_splitmix(seed & (2**64 - 1), x & (2**64 - 1)))


def sample(case, act, ts, A: int, k: int, seed: int, by_events: bool = False) -> dict:
    """A sample of k cases (whole) or k events of the formatted log, in order."""
    case, act, ts = _cols(case, act, ts)
    n = case.shape[0]
    m = max(n, 1)
    out = dict(case_s=np.empty(m, np.int32), act_s=np.empty(m, np.int32), ts_s=np.empty(m, np.int64))
    no, nc = np.zeros(1, np.int64), np.zeros(1, np.int64)
    rc = _load().orc_sample(n, _p(case), _p(act), _p(ts), A, int(k), seed & (2**64 - 1), 1 if by_events else 0,
                            _p(out["case_s"]), _p(out["act_s"]), _p(out["ts_s"]), _p(no), _p(nc))
    if rc:
        raise OracleError(rc)
    kk = int(no[0])
    return {key: v[:kk] for key, v in out.items()} | {"n_events": kk, "n_cases": int(nc[0])}


class CsvParseError(OracleError):
    def __init__(self, row: int):
        RuntimeError.__init__(self, f"CSV parse error at data row {row}")
        self.code = -3
        self.row = row


def ingest_csv(text: bytes, case_col: int, act_col: int, ts_col: int, sep: bytes = b",", has_header: bool = True,
               ts_iso: bool = False, ts_scale: int = 3, max_rows: int | None = None) -> dict:
    """Columns of a CSV text: case and activity codes (first-appearance order),
    timestamps, and per code the raw byte range of its first field."""
    n = len(text)
    cap = max_rows if max_rows is not None else n + 1
    m = max(cap, 1)
    out = dict(case=np.empty(m, np.int32), act=np.empty(m, np.int32), ts=np.empty(m, np.int64),
               case_off=np.empty(m, np.int64), case_len=np.empty(m, np.int32), act_off=np.empty(m, np.int64),
               act_len=np.empty(m, np.int32))
    nr, nc, na, bad = (np.zeros(1, np.int64) for _ in range(4))
    rc = _load().orc_ingest_csv(text, n, case_col, act_col, ts_col, sep, 1 if has_header else 0, 1 if ts_iso else 0,
                                ts_scale, cap, _p(out["case"]), _p(out["act"]), _p(out["ts"]), _p(nr),
                                _p(out["case_off"]), _p(out["case_len"]), _p(nc), _p(out["act_off"]),
                                _p(out["act_len"]), _p(na), _p(bad))
    if rc == -3:
        raise CsvParseError(int(bad[0]))
    if rc:
        raise OracleError(rc)
    r, c, a = int(nr[0]), int(nc[0]), int(na[0])
    res = {k: out[k][:r] for k in ("case", "act", "ts")}
    res.update(case_off=out["case_off"][:c], case_len=out["case_len"][:c], act_off=out["act_off"][:a],
               act_len=out["act_len"][:a], n_rows=r, n_cases=c, n_acts=a)
    return res



class ParquetUnsupported(OracleError):
    def __init__(self):
        RuntimeError.__init__(self, "Parquet feature outside the covered subset")
        self.code = -4


def ingest_parquet(data: bytes, case_col: int, act_col: int, ts_col: int, max_rows: int | None = None) -> dict:
    """Columns of a Parquet file (leaf columns case_col, act_col, ts_col): case
    and activity codes (first-appearance order), timestamps, and per code the
    byte range of its value at its first row (integer columns: the value, -1)."""
    n = len(data)
    cap = max_rows if max_rows is not None else n
    m = max(cap, 1)
    out = dict(case=np.empty(m, np.int32), act=np.empty(m, np.int32), ts=np.empty(m, np.int64),
               case_off=np.empty(m, np.int64), case_len=np.empty(m, np.int32), act_off=np.empty(m, np.int64),
               act_len=np.empty(m, np.int32))
    nr, nc, na, bad = (np.zeros(1, np.int64) for _ in range(4))
    rc = _load().orc_ingest_parquet(data, n, case_col, act_col, ts_col, cap, _p(out["case"]), _p(out["act"]),
                                    _p(out["ts"]), _p(nr), _p(out["case_off"]), _p(out["case_len"]), _p(nc),
                                    _p(out["act_off"]), _p(out["act_len"]), _p(na), _p(bad))
    if rc == -3:
        raise CsvParseError(int(bad[0]))
    if rc == -4:
        raise ParquetUnsupported()
    if rc:
        raise OracleError(rc)
    r, c, a = int(nr[0]), int(nc[0]), int(na[0])
    res = {k: out[k][:r] for k in ("case", "act", "ts")}
    res.update(case_off=out["case_off"][:c], case_len=out["case_len"][:c], act_off=out["act_off"][:a],
               act_len=out["act_len"][:a], n_rows=r, n_cases=c, n_acts=a)
    return res

def csv_value(raw: bytes) -> bytes:
    """The value of a raw CSV field (quoted runs unwrapped, doubled quotes single)."""
    out = bytearray()
    inq = False
    i = 0
    while i < len(raw):
        ch = raw[i:i + 1]
        if ch == b'"':
            if inq and raw[i + 1:i + 2] == b'"':
                out += b'"'
                i += 1
            else:
                inq = not inq
        else:
            out += ch
        i += 1
    return bytes(out)
