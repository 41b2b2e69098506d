"""Thin Python binding of libpm4g (the C ABI in include/pm4g.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  The library is loaded from this package directory; if it is
missing, every call raises (there is no fallback path).

Entry points mirror the C names: pm4g_prepare, pm4g_dfg, pm4g_dfg_prepared,
pm4g_variants, pm4g_variants_prepared, pm4g_dfg_batched.
"""
from __future__ import annotations

import ctypes
import dataclasses
import functools
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PM4G_LIBRARY names another build of the same library
LIB_PATH = os.environ.get("PM4G_LIBRARY") or os.path.join(_HERE, "libpm4g.so")

PM4G_OK = 0
PM4G_E_INVALID = -1
PM4G_E_RANGE = -2
PM4G_E_NOT_SORTED = -3
PM4G_E_CAPACITY = -4
PM4G_E_WORKSPACE = -5
PM4G_E_DEVICE = -6
PM4G_E_PARSE = -7
PM4G_E_UNSUPPORTED = -8
PM4G_PRESORTED = 1
PM4G_MAX_ACTIVITIES = 4096

OP_PREPARE, OP_DFG, OP_DFG_PREPARED, OP_VARIANTS, OP_VARIANTS_PREPARED, OP_DFG_BATCHED = 1, 2, 3, 4, 5, 6

_P = ctypes.c_void_p


class _Log(ctypes.Structure):
    _fields_ = [("case_id", _P), ("activity", _P), ("timestamp", _P), ("n_events", ctypes.c_int64),
                ("n_activities", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class _Prepared(ctypes.Structure):
    _fields_ = [("case_s", _P), ("act_s", _P), ("ts_s", _P), ("case_off", _P), ("case_code", _P),
                ("n_cases", _P), ("status", _P), ("n_events", ctypes.c_int64),
                ("n_activities", ctypes.c_int32), ("row", _P)]


class _DfgOut(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("count", "dt_sum", "dt_min", "dt_max", "dt_mean", "start_count",
                                  "end_count", "act_count", "n_cases", "overflow", "status")]


class _VarOut(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("n_variants", "var_count", "var_len", "var_rep", "var_off",
                                  "var_acts", "case_variant", "status")]


class _BatchedOut(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("edge_off", "src", "dst", "count", "dt_sum", "dt_min", "dt_max", "dt_mean",
                                  "start_count", "end_count", "act_count", "n_events", "n_cases")] + \
               [("cap_edges", ctypes.c_int64), ("required", _P), ("status", _P)]


class BatchedTuning(ctypes.Structure):
    """Launch shape and capacities of pm4g_dfg_batched (zero fields: library defaults)."""

    _fields_ = [("tile_events", ctypes.c_int32), ("emit_blocks", ctypes.c_int32),
                ("agg_blocks", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("pair_capacity", ctypes.c_int64), ("record_capacity", ctypes.c_int64),
                ("descriptor_capacity", ctypes.c_int64), ("cell_capacity", ctypes.c_int64)]


class CaseFilter(ctypes.Structure):
    """Case-level filter (host struct; the masks are device pointers)."""

    _fields_ = [("min_events", ctypes.c_int64), ("max_events", ctypes.c_int64),
                ("min_throughput", ctypes.c_int64), ("max_throughput", ctypes.c_int64),
                ("act_mask", _P), ("path_mask", _P), ("path_keep", ctypes.c_int32),
                ("variant_keep", ctypes.c_int32), ("contain_lo", ctypes.c_int64), ("contain_hi", ctypes.c_int64),
                ("meet_lo", ctypes.c_int64), ("meet_hi", ctypes.c_int64), ("start_mask", _P),
                ("end_mask", _P), ("case_variant", _P), ("variant_mask", _P),
                ("n_variant_bits", ctypes.c_int64)]


class _EfgOut(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("count", "sum_lo", "sum_hi", "sq_lo", "sq_hi", "mean", "std", "n_pairs",
                                  "status")]


class CsvSchema(ctypes.Structure):
    _fields_ = [("case_col", ctypes.c_int32), ("act_col", ctypes.c_int32), ("ts_col", ctypes.c_int32),
                ("has_header", ctypes.c_int32), ("ts_iso", ctypes.c_int32), ("ts_scale", ctypes.c_int32),
                ("sep", ctypes.c_char), ("reserved", ctypes.c_char * 7)]


class ParquetSchema(ctypes.Structure):
    _fields_ = [("case_col", ctypes.c_int32), ("act_col", ctypes.c_int32), ("ts_col", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _CsvOut(ctypes.Structure):
    _fields_ = [("case_code", _P), ("act_code", _P), ("ts", _P), ("capacity", ctypes.c_int64), ("n_rows", _P),
                ("case_dict_off", _P), ("case_dict_len", _P), ("n_cases", _P), ("act_dict_off", _P),
                ("act_dict_len", _P), ("n_acts", _P), ("status", _P), ("bad_row", _P)]


class Pm4gError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pm4g error {code}: {msg}")
        self.code = code


_lib = None
_lock = threading.Lock()


def load():
    """Loads libpm4g.so (built in-tree by paper_2204_04898_amd.build)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_04898_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            L.pm4g_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
            L.pm4g_workspace_bytes.restype = ctypes.c_size_t
            for name, argt in (("pm4g_prepare", [ctypes.POINTER(_Log), ctypes.POINTER(_Prepared)]),
                               ("pm4g_dfg", [ctypes.POINTER(_Log), ctypes.POINTER(_DfgOut)]),
                               ("pm4g_dfg_prepared", [ctypes.POINTER(_Prepared), ctypes.POINTER(_DfgOut)]),
                               ("pm4g_variants", [ctypes.POINTER(_Log), ctypes.POINTER(_VarOut)]),
                               ("pm4g_variants_prepared", [ctypes.POINTER(_Prepared), ctypes.POINTER(_VarOut)])):
                f = getattr(L, name)
                f.argtypes = argt + [_P, ctypes.c_size_t, _P]
                f.restype = ctypes.c_int
            L.pm4g_dfg_prepared_noalloc.argtypes = [ctypes.POINTER(_Prepared), ctypes.POINTER(_DfgOut), _P]
            L.pm4g_dfg_prepared_noalloc.restype = ctypes.c_int
            L.pm4g_status_string.argtypes = [ctypes.c_int]
            L.pm4g_status_string.restype = ctypes.c_char_p
            L.pm4g_last_error.argtypes = []
            L.pm4g_last_error.restype = ctypes.c_char_p
            L.pm4g_abi_version.restype = ctypes.c_int
            L.pm4g_batched_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.POINTER(BatchedTuning)]
            L.pm4g_batched_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_dfg_batched.argtypes = [ctypes.POINTER(_Prepared), _P, _P, ctypes.c_int32,
                                           ctypes.POINTER(_BatchedOut), ctypes.POINTER(BatchedTuning),
                                           _P, ctypes.c_size_t, _P]
            L.pm4g_dfg_batched.restype = ctypes.c_int
            L.pm4g_filter_workspace_bytes.argtypes = [ctypes.c_int64]
            L.pm4g_filter_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_filter_view.argtypes = [ctypes.POINTER(_Prepared), _P, _P, ctypes.POINTER(_Prepared), _P,
                                           ctypes.c_size_t, _P]
            L.pm4g_filter_view.restype = ctypes.c_int
            L.pm4g_filter_df_events.argtypes = [ctypes.POINTER(_Prepared), _P, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(_Prepared), _P, ctypes.c_size_t, _P]
            L.pm4g_filter_df_events.restype = ctypes.c_int
            L.pm4g_efg_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
            L.pm4g_efg_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_efg.argtypes = [ctypes.POINTER(_Prepared), ctypes.POINTER(_EfgOut), _P, ctypes.c_size_t, _P]
            L.pm4g_efg.restype = ctypes.c_int
            L.pm4g_sample_workspace_bytes.argtypes = [ctypes.c_int64]
            L.pm4g_sample_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_sample.argtypes = [ctypes.POINTER(_Prepared), ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.POINTER(_Prepared), _P, ctypes.c_size_t, _P]
            L.pm4g_sample.restype = ctypes.c_int
            L.pm4g_ingest_csv_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
            L.pm4g_ingest_csv_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_ingest_csv.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(CsvSchema), ctypes.POINTER(_CsvOut), _P,
                                          ctypes.c_size_t, _P]
            L.pm4g_ingest_csv.restype = ctypes.c_int
            L.pm4g_parquet_rows.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _P]
            L.pm4g_parquet_rows.restype = ctypes.c_int
            L.pm4g_ingest_parquet_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
            L.pm4g_ingest_parquet_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_ingest_parquet.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(ParquetSchema), ctypes.POINTER(_CsvOut),
                                              _P, ctypes.c_size_t, _P]
            L.pm4g_ingest_parquet.restype = ctypes.c_int
            L.pm4g_cases.argtypes = [ctypes.POINTER(_Prepared), _P, _P, _P]
            L.pm4g_cases.restype = ctypes.c_int
            L.pm4g_filter_cases_workspace_bytes.argtypes = [ctypes.c_int64]
            L.pm4g_filter_cases_workspace_bytes.restype = ctypes.c_size_t
            L.pm4g_filter_cases.argtypes = [ctypes.POINTER(_Prepared), ctypes.POINTER(CaseFilter),
                                            ctypes.POINTER(_Prepared), _P, ctypes.c_size_t, _P]
            L.pm4g_filter_cases.restype = ctypes.c_int
            L.pm4g_profile_enable.argtypes = [ctypes.c_int]
            L.pm4g_profile_enable.restype = ctypes.c_int
            L.pm4g_profile_read.argtypes = [_P, _P, ctypes.c_int]
            L.pm4g_profile_read.restype = ctypes.c_int
            L.pm4g_profile_stage_name.argtypes = [ctypes.c_int]
            L.pm4g_profile_stage_name.restype = ctypes.c_char_p
            L.pm4g_profile_stage_count.restype = ctypes.c_int
            L.pm4g_debug_csv_hash_bits.argtypes = [ctypes.c_int]
            L.pm4g_debug_csv_hash_bits.restype = ctypes.c_int
            L.pm4g_debug_efg_pass_pairs.argtypes = [ctypes.c_int64]
            L.pm4g_debug_efg_pass_pairs.restype = ctypes.c_int64
            if hasattr(L, "pm4g_debug_variant_hash_bits"):
                L.pm4g_debug_variant_hash_bits.argtypes = [ctypes.c_int]
                L.pm4g_debug_variant_hash_bits.restype = ctypes.c_int
            _lib = L
    return _lib


def _check(rc: int):
    if rc != PM4G_OK:
        L = load()
        raise Pm4gError(rc, L.pm4g_last_error().decode() or L.pm4g_status_string(rc).decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(fn):
    """Runs a wrapper with its `stream` argument as torch's current stream, so
    that every tensor it allocates (outputs, workspaces) belongs to the stream
    its kernels run on: the caching allocator then never hands that memory to
    work queued on another stream while the kernels may still use it."""

    @functools.wraps(fn)
    def wrapped(*args, stream=None, **kw):
        if stream is None:
            return fn(*args, **kw)
        with torch.cuda.stream(stream):
            return fn(*args, stream=stream, **kw)

    return wrapped


# One growing workspace per (device, stream): keeps allocation out of repeated calls.
_ws_cache: dict = {}


def workspace(op: int, n_events: int, n_activities: int, device, stream=None, n_views: int = 0):
    need = int(load().pm4g_workspace_bytes(op, n_events, n_activities, n_views))
    if need == 0:
        raise Pm4gError(PM4G_E_INVALID, "invalid sizes for the workspace query")
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (torch.device(device).index, s.cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < need:
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf, need


def _cols(case, act, ts):
    for t, dt in ((case, torch.int32), (act, torch.int32), (ts, torch.int64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous() or t.dim() != 1:
            raise ValueError("case/act must be contiguous 1-D int32 and ts int64 CUDA tensors")
    if not (case.numel() == act.numel() == ts.numel()):
        raise ValueError("case, act and ts differ in length")


def _log(case, act, ts, A: int, presorted: bool) -> _Log:
    _cols(case, act, ts)
    return _Log(_ptr(case), _ptr(act), _ptr(ts), case.numel(), int(A), PM4G_PRESORTED if presorted else 0)


@dataclasses.dataclass
class Prepared:
    """A prepared (formatted) log in device memory, Sec. 3 formatting steps."""

    case_s: torch.Tensor
    act_s: torch.Tensor
    ts_s: torch.Tensor
    case_off: torch.Tensor
    case_code: torch.Tensor
    n_cases: torch.Tensor     # int64 [1]
    status: torch.Tensor      # int32 [1]
    n_activities: int
    row: torch.Tensor | None = None   # int32 [n]: raw row of each position (pm4g_prepare with rows)

    @property
    def n_events(self) -> int:
        return int(self.case_s.numel())

    def _struct(self) -> _Prepared:
        return _Prepared(_ptr(self.case_s), _ptr(self.act_s), _ptr(self.ts_s), _ptr(self.case_off),
                         _ptr(self.case_code), _ptr(self.n_cases), _ptr(self.status), self.n_events,
                         self.n_activities, _ptr(self.row))

    @staticmethod
    def empty(n: int, A: int, device, rows: bool = False) -> "Prepared":
        m = max(n, 1)
        return Prepared(case_s=torch.empty(n, dtype=torch.int32, device=device),
                        act_s=torch.empty(n, dtype=torch.int32, device=device),
                        ts_s=torch.empty(n, dtype=torch.int64, device=device),
                        case_off=torch.empty(m + 1, dtype=torch.int64, device=device),
                        case_code=torch.empty(m, dtype=torch.int32, device=device),
                        n_cases=torch.zeros(1, dtype=torch.int64, device=device),
                        status=torch.zeros(1, dtype=torch.int32, device=device), n_activities=A,
                        row=torch.empty(n, dtype=torch.int32, device=device) if rows else None)


@_on_stream
def pm4g_prepare(case, act, ts, A: int, presorted: bool = False, out: Prepared | None = None,
                 rows: bool = False, stream=None) -> Prepared:
    """Formats a raw log on the GPU (order, per-case table; with `rows`, also
    the raw row of each position).  Synchronises the stream."""
    log = _log(case, act, ts, A, presorted)
    if out is None:
        out = Prepared.empty(case.numel(), A, case.device, rows=rows)
    ws, need = workspace(OP_PREPARE, case.numel(), A, case.device, stream)
    p = out._struct()
    _check(load().pm4g_prepare(ctypes.byref(log), ctypes.byref(p), _ptr(ws), need, _stream(stream)))
    return out


def _dfg_out(A: int, device) -> dict:
    cells = A * A
    o = dict(count=torch.empty(cells, dtype=torch.int64, device=device),
             dt_sum=torch.empty(cells, dtype=torch.int64, device=device),
             dt_min=torch.empty(cells, dtype=torch.int64, device=device),
             dt_max=torch.empty(cells, dtype=torch.int64, device=device),
             dt_mean=torch.empty(cells, dtype=torch.float64, device=device),
             start_count=torch.empty(A, dtype=torch.int64, device=device),
             end_count=torch.empty(A, dtype=torch.int64, device=device),
             act_count=torch.empty(A, dtype=torch.int64, device=device),
             n_cases=torch.zeros(1, dtype=torch.int64, device=device),
             overflow=torch.zeros(1, dtype=torch.int32, device=device),
             status=torch.zeros(1, dtype=torch.int32, device=device))
    return o


def _dfg_struct(o: dict) -> _DfgOut:
    return _DfgOut(*[_ptr(o.get(k)) for k in ("count", "dt_sum", "dt_min", "dt_max", "dt_mean",
                                               "start_count", "end_count", "act_count", "n_cases",
                                               "overflow", "status")])


@_on_stream
def pm4g_dfg(case, act, ts, A: int, presorted: bool = False, out: dict | None = None,
             stream=None) -> dict:
    """DFG of a raw log (formats it in the workspace first).  Synchronises once or twice."""
    log = _log(case, act, ts, A, presorted)
    o = out if out is not None else _dfg_out(A, case.device)
    ws, need = workspace(OP_DFG, case.numel(), A, case.device, stream)
    s = _dfg_struct(o)
    _check(load().pm4g_dfg(ctypes.byref(log), ctypes.byref(s), _ptr(ws), need, _stream(stream)))
    return o


@_on_stream
def pm4g_dfg_prepared(prep: Prepared, out: dict | None = None, stream=None) -> dict:
    """DFG of a prepared log.  Asynchronous on the stream."""
    o = out if out is not None else _dfg_out(prep.n_activities, prep.case_s.device)
    ws, need = workspace(OP_DFG_PREPARED, prep.n_events, prep.n_activities, prep.case_s.device, stream)
    p = prep._struct()
    s = _dfg_struct(o)
    _check(load().pm4g_dfg_prepared(ctypes.byref(p), ctypes.byref(s), _ptr(ws), need, _stream(stream)))
    return o


PM4G_NOALLOC_SCRATCH_BYTES = 128 << 20


@_on_stream
def pm4g_dfg_prepared_noalloc(prep: Prepared, out: dict, stream=None) -> dict:
    """DFG of a prepared log into caller-allocated outputs, with the workspace
    in the library's own per-GPU scratch array: the C call allocates nothing.
    Calls overlapping in time on one GPU race on that array.  Asynchronous."""
    p = prep._struct()
    s = _dfg_struct(out)
    _check(load().pm4g_dfg_prepared_noalloc(ctypes.byref(p), ctypes.byref(s), _stream(stream)))
    return out


def _var_out(n: int, device, with_cases: bool = True) -> dict:
    m = max(n, 1)
    return dict(n_variants=torch.zeros(1, dtype=torch.int64, device=device),
                var_count=torch.empty(m, dtype=torch.int64, device=device),
                var_len=torch.empty(m, dtype=torch.int32, device=device),
                var_rep=torch.empty(m, dtype=torch.int32, device=device),
                var_off=torch.empty(m + 1, dtype=torch.int64, device=device),
                var_acts=torch.empty(m, dtype=torch.int32, device=device),
                case_variant=torch.empty(m, dtype=torch.int32, device=device) if with_cases else None,
                status=torch.zeros(1, dtype=torch.int32, device=device))


def _var_struct(o: dict) -> _VarOut:
    return _VarOut(*[_ptr(o.get(k)) for k in ("n_variants", "var_count", "var_len", "var_rep",
                                               "var_off", "var_acts", "case_variant", "status")])


@_on_stream
def pm4g_variants(case, act, ts, A: int, presorted: bool = False, out: dict | None = None,
                  stream=None) -> dict:
    """Trace variants of a raw log.  Synchronises once or twice."""
    log = _log(case, act, ts, A, presorted)
    o = out if out is not None else _var_out(case.numel(), case.device)
    ws, need = workspace(OP_VARIANTS, case.numel(), A, case.device, stream)
    s = _var_struct(o)
    _check(load().pm4g_variants(ctypes.byref(log), ctypes.byref(s), _ptr(ws), need, _stream(stream)))
    return o


@_on_stream
def pm4g_variants_prepared(prep: Prepared, out: dict | None = None, ws: torch.Tensor | None = None,
                           stream=None) -> dict:
    """Trace variants of a prepared log.  Asynchronous on the stream.  `ws`: a
    workspace of at least variants_workspace_bytes(...) bytes (default: the
    binding's growing per-stream workspace)."""
    o = out if out is not None else _var_out(prep.n_events, prep.case_s.device)
    need = variants_workspace_bytes(prep.n_events, prep.n_activities)
    if ws is None or ws.numel() < need:
        ws, need = workspace(OP_VARIANTS_PREPARED, prep.n_events, prep.n_activities, prep.case_s.device, stream)
    p = prep._struct()
    s = _var_struct(o)
    _check(load().pm4g_variants_prepared(ctypes.byref(p), ctypes.byref(s), _ptr(ws), need, _stream(stream)))
    return o


def variants_workspace_bytes(n_events: int, A: int) -> int:
    """Workspace bytes of pm4g_variants_prepared on a prepared log of n_events."""
    return int(load().pm4g_workspace_bytes(OP_VARIANTS_PREPARED, int(n_events), int(A), 0))


def batched_workspace_bytes(n_events: int, A: int, n_views: int, tuning: "BatchedTuning | None" = None) -> int:
    """Workspace bytes of pm4g_dfg_batched (0: invalid sizes or tuning)."""
    return int(load().pm4g_batched_workspace_bytes(int(n_events), int(A), int(n_views),
                                                   ctypes.byref(tuning) if tuning is not None else None))


def filter_workspace_bytes(n_events: int) -> int:
    """Workspace bytes of pm4g_filter_view / pm4g_filter_df_events on a log of n_events."""
    return int(load().pm4g_filter_workspace_bytes(int(n_events)))


def batched_out_bytes(n_views: int, A: int, cap_edges: int) -> int:
    """Device bytes of the outputs _batched_out allocates."""
    cap = max(int(cap_edges), 1)
    return 8 * (n_views + 1) + cap * (4 + 4 + 8 * 5) + 3 * 8 * max(n_views * A, 1) + 2 * 8 * max(n_views, 1) + 44


def prepared_bytes(n: int, rows: bool = False) -> int:
    """Device bytes of Prepared.empty(n, ...)."""
    m = max(int(n), 1)
    return int(n) * (4 + 4 + 8 + (4 if rows else 0)) + 8 * (m + 1) + 4 * m + 12


def variants_out_bytes(n: int, with_cases: bool = True) -> int:
    """Device bytes of the variants outputs sized for n events."""
    m = max(int(n), 1)
    return 8 + m * (8 + 4 + 4 + 4 + (4 if with_cases else 0)) + 8 * (m + 1) + 4


PM4G_BATCHED_MAX_ACTIVITIES = 1024


def views_to_device(views, device) -> tuple[torch.Tensor, torch.Tensor]:
    """Packs synth.Views (or any object with case_lo/case_hi/t_lo/t_hi/masks) for the library."""
    import numpy as np
    rec = np.zeros(len(views.case_lo), dtype=np.dtype([("lo", "<i4"), ("hi", "<i4"), ("t_lo", "<i8"),
                                                        ("t_hi", "<i8")]))
    rec["lo"], rec["hi"], rec["t_lo"], rec["t_hi"] = views.case_lo, views.case_hi, views.t_lo, views.t_hi
    v = torch.from_numpy(rec.view(np.uint8).copy()).to(device)
    m = torch.from_numpy(np.ascontiguousarray(views.masks).view(np.int64).copy()).to(device)
    return v, m


def _batched_out(V: int, A: int, cap_edges: int, device) -> dict:
    cap = max(int(cap_edges), 1)
    i64 = dict(dtype=torch.int64, device=device)
    return dict(edge_off=torch.empty(V + 1, **i64),
                src=torch.empty(cap, dtype=torch.int32, device=device),
                dst=torch.empty(cap, dtype=torch.int32, device=device),
                count=torch.empty(cap, **i64), dt_sum=torch.empty(cap, **i64),
                dt_min=torch.empty(cap, **i64), dt_max=torch.empty(cap, **i64),
                dt_mean=torch.empty(cap, dtype=torch.float64, device=device),
                start_count=torch.empty(max(V * A, 1), **i64), end_count=torch.empty(max(V * A, 1), **i64),
                act_count=torch.empty(max(V * A, 1), **i64), n_events=torch.empty(max(V, 1), **i64),
                n_cases=torch.empty(max(V, 1), **i64), required=torch.zeros(5, **i64),
                status=torch.zeros(1, dtype=torch.int32, device=device), cap_edges=cap)


def _batched_struct(o: dict) -> _BatchedOut:
    return _BatchedOut(*[_ptr(o[k]) for k in ("edge_off", "src", "dst", "count", "dt_sum", "dt_min", "dt_max",
                                               "dt_mean", "start_count", "end_count", "act_count",
                                               "n_events", "n_cases")],
                       o["cap_edges"], _ptr(o["required"]), _ptr(o["status"]))


@_on_stream
def pm4g_dfg_batched(prep: Prepared, views: torch.Tensor, masks: torch.Tensor, n_views: int,
                     tuning: BatchedTuning | None = None, cap_edges: int | None = None,
                     out: dict | None = None, stream=None, retry: bool = True,
                     keep_workspace: bool = True) -> dict:
    """DFGs of n_views drill-down views in one pass (Sec. 1 drill-down, Sec. 3 filters).

    views: device uint8 tensor of n_views packed pm4g_view records; masks: device
    int64 tensor [n_views, ceil(A/64)].  With no `tuning`, the launch shape
    comes from the autotune cache (tune.py).  The library call does not wait;
    this wrapper synchronises the stream once to read the device status.  With
    `retry`, capacities found too small are raised to what the call reported
    and the call is repeated.  keep_workspace=False allocates the workspace for
    this call only (on the stream) instead of growing the per-stream one.
    """
    L = load()
    A = prep.n_activities
    dev = prep.case_s.device
    t = BatchedTuning() if tuning is None else BatchedTuning.from_buffer_copy(tuning)
    if t.tile_events == 0 and t.emit_blocks == 0 and t.agg_blocks == 0 and t.launch == 0:
        # launch shape from the autotune cache (capacities: the tuning's or the library's)
        from . import tune
        hit = tune.default_cache().lookup(A, n_views, prep.n_events)
        if hit is not None:
            t.tile_events = int(hit["tile_events"])
            t.emit_blocks = int(hit["emit_blocks"])
            t.agg_blocks = int(hit["agg_blocks"])
            t.launch = int(hit.get("launch", 1))
    # output cells: at most A*A per view and one per kept event
    cap = int(cap_edges) if cap_edges is not None else \
        max(1024, min(int(n_views) * A * A, prep.n_events, 1 << 24))
    o = out if out is not None else _batched_out(n_views, A, cap, dev)
    for _ in range(6):
        need = int(L.pm4g_batched_workspace_bytes(prep.n_events, A, n_views, ctypes.byref(t)))
        if need == 0:
            raise Pm4gError(PM4G_E_INVALID, "invalid sizes or tuning for the batched workspace")
        ws = _batched_ws(dev, need, stream) if keep_workspace else torch.empty(need, dtype=torch.uint8, device=dev)
        p = prep._struct()
        s = _batched_struct(o)
        rc = L.pm4g_dfg_batched(ctypes.byref(p), _ptr(views), _ptr(masks), int(n_views), ctypes.byref(s),
                                ctypes.byref(t), _ptr(ws), need, _stream(stream))
        if rc == PM4G_OK:
            (torch.cuda.current_stream() if stream is None else stream).synchronize()
            status = int(o["status"].item())
            if status == PM4G_OK:
                return o
            if status != PM4G_E_CAPACITY or not retry:
                raise Pm4gError(status, L.pm4g_status_string(status).decode())
        elif rc != PM4G_E_CAPACITY or not retry:
            _check(rc)
        req = [int(x) for x in o["required"].cpu().tolist()]
        grow = lambda cur, r: max(int(cur), int(r * 1.25) + 1024)
        if req[3] > 0:
            t.pair_capacity = grow(t.pair_capacity, req[3])
        if req[1] > 0:
            t.record_capacity = grow(t.record_capacity, req[1])
        if req[4] > 0:
            t.cell_capacity = grow(t.cell_capacity, req[4])
        if req[0] > o["cap_edges"]:
            o = _batched_out(n_views, A, int(req[0] * 1.1) + 1024, dev)
    raise Pm4gError(PM4G_E_CAPACITY, "capacities still short after retries")


@_on_stream
def pm4g_filter_view(prep: Prepared, view: torch.Tensor, mask: torch.Tensor, out: Prepared | None = None,
                     ws: torch.Tensor | None = None, stream=None) -> Prepared:
    """The kept events of one view as a prepared log (device record `view`, device `mask` words).

    Asynchronous; out's kept count is out.case_off[out.n_cases] on the device.
    """
    L = load()
    dev = prep.case_s.device
    o = out if out is not None else Prepared.empty(prep.n_events, prep.n_activities, dev)
    need = int(L.pm4g_filter_workspace_bytes(prep.n_events))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    p = prep._struct()
    q = o._struct()
    _check(L.pm4g_filter_view(ctypes.byref(p), _ptr(view), _ptr(mask), ctypes.byref(q), _ptr(ws), need,
                              _stream(stream)))
    return o


@_on_stream
def pm4g_filter_df_events(prep: Prepared, pair_mask: torch.Tensor, side: int = 0, keep: bool = True,
                          out: Prepared | None = None, ws: torch.Tensor | None = None, stream=None) -> Prepared:
    """Events kept by the directly-follows-level filter, as a prepared log.

    pair_mask: device int64 tensor of ceil(A*A/64) words, bit src*A + dst;
    side 0 pairs an event with the previous event of its case, side 1 with the
    next one.  Asynchronous; the kept count is out.case_off[out.n_cases]."""
    L = load()
    dev = prep.case_s.device
    o = out if out is not None else Prepared.empty(prep.n_events, prep.n_activities, dev)
    need = int(L.pm4g_filter_workspace_bytes(prep.n_events))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    p = prep._struct()
    q = o._struct()
    _check(L.pm4g_filter_df_events(ctypes.byref(p), _ptr(pair_mask), int(side), 1 if keep else 0,
                                   ctypes.byref(q), _ptr(ws), need, _stream(stream)))
    return o


@_on_stream
def pm4g_sample(prep: Prepared, k: int, seed: int, by_events: bool = False, out: Prepared | None = None,
                ws: torch.Tensor | None = None, stream=None) -> Prepared:
    """A sample of k cases (whole) or k events of a prepared log, as a
    prepared log.  Asynchronous; the kept count is out.case_off[out.n_cases]."""
    L = load()
    dev = prep.case_s.device
    o = out if out is not None else Prepared.empty(prep.n_events, prep.n_activities, dev)
    need = int(L.pm4g_sample_workspace_bytes(prep.n_events))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    p = prep._struct()
    q = o._struct()
    _check(L.pm4g_sample(ctypes.byref(p), int(k), int(seed) & (2**64 - 1), 1 if by_events else 0,
                         ctypes.byref(q), _ptr(ws), need, _stream(stream)))
    return o


@_on_stream
def pm4g_ingest_csv(text: torch.Tensor, case_col: int, act_col: int, ts_col: int, sep: bytes = b",",
                    has_header: bool = True, ts_iso: bool = False, ts_scale: int = 3, capacity: int | None = None,
                    stream=None) -> dict:
    """Columns of a CSV text held in a device uint8 tensor: case_code and
    act_code (int32, first-appearance order), ts (int64), and per code the raw
    byte range of its first field; counts as host ints.  Raises Pm4gError on a
    parse error (its message names the row) or when the rows exceed capacity
    (default: an upper bound from the text's newlines)."""
    L = load()
    dev = text.device
    n = int(text.numel())
    if capacity is None:
        capacity = int((text == 10).sum().item()) + 1
    cap = max(int(capacity), 1)
    i32 = dict(dtype=torch.int32, device=dev)
    i64 = dict(dtype=torch.int64, device=dev)
    o = dict(case_code=torch.empty(cap, **i32), act_code=torch.empty(cap, **i32), ts=torch.empty(cap, **i64),
             n_rows=torch.zeros(1, **i64), case_dict_off=torch.empty(cap, **i64), case_dict_len=torch.empty(cap, **i32),
             n_cases=torch.zeros(1, **i64), act_dict_off=torch.empty(cap, **i64), act_dict_len=torch.empty(cap, **i32),
             n_acts=torch.zeros(1, **i64), status=torch.zeros(1, **i32), bad_row=torch.zeros(1, **i64))
    need = int(L.pm4g_ingest_csv_workspace_bytes(n, int(capacity)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    sc = CsvSchema(int(case_col), int(act_col), int(ts_col), 1 if has_header else 0, 1 if ts_iso else 0,
                   int(ts_scale), sep, b"\0" * 7)
    q = _CsvOut(_ptr(o["case_code"]), _ptr(o["act_code"]), _ptr(o["ts"]), int(capacity), _ptr(o["n_rows"]),
                _ptr(o["case_dict_off"]), _ptr(o["case_dict_len"]), _ptr(o["n_cases"]), _ptr(o["act_dict_off"]),
                _ptr(o["act_dict_len"]), _ptr(o["n_acts"]), _ptr(o["status"]), _ptr(o["bad_row"]))
    _check(L.pm4g_ingest_csv(_ptr(text), n, ctypes.byref(sc), ctypes.byref(q), _ptr(ws), need, _stream(stream)))
    r, c, a = int(o["n_rows"].item()), int(o["n_cases"].item()), int(o["n_acts"].item())
    res = {k: o[k][:r] for k in ("case_code", "act_code", "ts")}
    res.update(case_dict_off=o["case_dict_off"][:c], case_dict_len=o["case_dict_len"][:c],
               act_dict_off=o["act_dict_off"][:a], act_dict_len=o["act_dict_len"][:a], n_rows=r, n_cases=c,
               n_acts=a)
    return res


@_on_stream
def pm4g_ingest_parquet(data: torch.Tensor, case_col: int, act_col: int, ts_col: int, capacity: int | None = None,
                        stream=None) -> dict:
    """Columns of a Parquet file held in a device uint8 tensor (leaf columns
    case_col, act_col, ts_col): case_code and act_code (int32, first-appearance
    order), ts (int64), and per code *_dict_off / *_dict_len (the byte range of
    the value at the code's first row; for integer columns the value and -1);
    counts as host ints.  Raises Pm4gError on a parse error (its message names
    the row of a null), on a feature outside the covered subset, or when the
    rows exceed capacity (default: the footer's row count)."""
    L = load()
    dev = data.device
    n = int(data.numel())
    s = _stream(stream)
    if capacity is None:
        rows = ctypes.c_int64(0)
        _check(L.pm4g_parquet_rows(_ptr(data), n, ctypes.byref(rows), s))
        capacity = int(rows.value)
    cap = max(int(capacity), 1)
    i32 = dict(dtype=torch.int32, device=dev)
    i64 = dict(dtype=torch.int64, device=dev)
    o = dict(case_code=torch.empty(cap, **i32), act_code=torch.empty(cap, **i32), ts=torch.empty(cap, **i64),
             n_rows=torch.zeros(1, **i64), case_dict_off=torch.empty(cap, **i64), case_dict_len=torch.empty(cap, **i32),
             n_cases=torch.zeros(1, **i64), act_dict_off=torch.empty(cap, **i64), act_dict_len=torch.empty(cap, **i32),
             n_acts=torch.zeros(1, **i64), status=torch.zeros(1, **i32), bad_row=torch.zeros(1, **i64))
    need = int(L.pm4g_ingest_parquet_workspace_bytes(n, int(capacity)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    sc = ParquetSchema(int(case_col), int(act_col), int(ts_col), 0)
    q = _CsvOut(_ptr(o["case_code"]), _ptr(o["act_code"]), _ptr(o["ts"]), int(capacity), _ptr(o["n_rows"]),
                _ptr(o["case_dict_off"]), _ptr(o["case_dict_len"]), _ptr(o["n_cases"]), _ptr(o["act_dict_off"]),
                _ptr(o["act_dict_len"]), _ptr(o["n_acts"]), _ptr(o["status"]), _ptr(o["bad_row"]))
    _check(L.pm4g_ingest_parquet(_ptr(data), n, ctypes.byref(sc), ctypes.byref(q), _ptr(ws), need, s))
    r, c, a = int(o["n_rows"].item()), int(o["n_cases"].item()), int(o["n_acts"].item())
    res = {k: o[k][:r] for k in ("case_code", "act_code", "ts")}
    res.update(case_dict_off=o["case_dict_off"][:c], case_dict_len=o["case_dict_len"][:c],
               act_dict_off=o["act_dict_off"][:a], act_dict_len=o["act_dict_len"][:a], n_rows=r, n_cases=c,
               n_acts=a)
    return res


PM4G_EFG_MAX_ACTIVITIES = 4096


@_on_stream
def pm4g_efg(prep: Prepared, out: dict | None = None, ws: torch.Tensor | None = None, stream=None) -> dict:
    """Eventually-follows graph and temporal profile of a prepared log: device
    [A*A] count (int64), sum_lo/sum_hi and sq_lo/sq_hi (exact gap sums as
    int64-typed uint64 words), mean and std (float64); n_pairs, status.
    Asynchronous."""
    L = load()
    dev = prep.case_s.device
    A = prep.n_activities
    cells = A * A
    if out is None:
        i64 = dict(dtype=torch.int64, device=dev)
        out = dict(count=torch.empty(cells, **i64), sum_lo=torch.empty(cells, **i64), sum_hi=torch.empty(cells, **i64),
                   sq_lo=torch.empty(cells, **i64), sq_hi=torch.empty(cells, **i64),
                   mean=torch.empty(cells, dtype=torch.float64, device=dev),
                   std=torch.empty(cells, dtype=torch.float64, device=dev), n_pairs=torch.zeros(1, **i64),
                   status=torch.zeros(1, dtype=torch.int32, device=dev))
    need = int(L.pm4g_efg_workspace_bytes(prep.n_events, A))
    if need == 0:
        raise Pm4gError(PM4G_E_INVALID, f"no EFG workspace size for n={prep.n_events}, A={A}")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    s = _EfgOut(*[_ptr(out.get(k)) for k in ("count", "sum_lo", "sum_hi", "sq_lo", "sq_hi", "mean", "std",
                                              "n_pairs", "status")])
    p = prep._struct()
    _check(L.pm4g_efg(ctypes.byref(p), ctypes.byref(s), _ptr(ws), need, _stream(stream)))
    return out


def efg_to_host(o: dict, A: int) -> dict:
    """The EFG outputs as [A, A] numpy arrays (sum/sq words as uint64)."""
    import numpy as np
    h = {}
    for k in ("count", "sum_lo", "sum_hi", "sq_lo", "sq_hi", "mean", "std"):
        v = o[k].cpu().numpy()
        if k in ("sum_lo", "sum_hi", "sq_lo", "sq_hi"):
            v = v.view(np.uint64)
        h[k] = v.reshape(A, A)
    h["n_pairs"] = int(o["n_pairs"].item())
    h["status"] = int(o["status"].item())
    return h


I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


@_on_stream
def pm4g_cases(prep: Prepared, stream=None) -> dict:
    """Cases dataframe: per case (case-table order) its events and throughput time.

    Device int64 tensors of prep.n_events entries; the first *prep.n_cases are set.
    Asynchronous on the stream."""
    dev = prep.case_s.device
    m = max(prep.n_events, 1)
    o = dict(n_events=torch.empty(m, dtype=torch.int64, device=dev),
             throughput=torch.empty(m, dtype=torch.int64, device=dev))
    p = prep._struct()
    _check(load().pm4g_cases(ctypes.byref(p), _ptr(o["n_events"]), _ptr(o["throughput"]), _stream(stream)))
    return o


@_on_stream
def pm4g_filter_cases(prep: Prepared, min_events: int = 0, max_events: int = I64_MAX,
                      min_throughput: int = I64_MIN, max_throughput: int = I64_MAX,
                      act_mask: torch.Tensor | None = None, path_mask: torch.Tensor | None = None,
                      path_keep: bool = True, contain_lo: int = I64_MIN, contain_hi: int = I64_MAX,
                      meet_lo: int = I64_MIN, meet_hi: int = I64_MAX, start_mask: torch.Tensor | None = None,
                      end_mask: torch.Tensor | None = None, case_variant: torch.Tensor | None = None,
                      variant_mask: torch.Tensor | None = None, n_variant_bits: int = 0,
                      variant_keep: bool = True, out: Prepared | None = None, ws: torch.Tensor | None = None,
                      stream=None) -> Prepared:
    """Events of the cases passing the case-level filters, as a prepared log.

    act_mask / start_mask / end_mask: device int64 tensors of ceil(A/64)
    words; path_mask: ceil(A*A/64) words with bit src*A + dst; variant_mask:
    ceil(n_variant_bits/64) words over the ids in case_variant (the int32
    per-case variant ids pm4g_variants_prepared writes for the same log).
    Asynchronous; the kept count is out.case_off[out.n_cases] on the device."""
    L = load()
    dev = prep.case_s.device
    o = out if out is not None else Prepared.empty(prep.n_events, prep.n_activities, dev)
    need = int(L.pm4g_filter_cases_workspace_bytes(prep.n_events))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def opt(t):
        return _ptr(t) if t is not None else None

    f = CaseFilter(int(min_events), int(max_events), int(min_throughput), int(max_throughput), opt(act_mask),
                   opt(path_mask), 1 if path_keep else 0, 1 if variant_keep else 0, int(contain_lo),
                   int(contain_hi), int(meet_lo), int(meet_hi), opt(start_mask), opt(end_mask), opt(case_variant),
                   opt(variant_mask), int(n_variant_bits))
    p = prep._struct()
    q = o._struct()
    _check(L.pm4g_filter_cases(ctypes.byref(p), ctypes.byref(f), ctypes.byref(q), _ptr(ws), need,
                               _stream(stream)))
    return o


_bws_cache: dict = {}


def _batched_ws(device, need: int, stream=None) -> torch.Tensor:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (torch.device(device).index, s.cuda_stream)
    buf = _bws_cache.get(key)
    if buf is None or buf.numel() < need:
        _bws_cache.pop(key, None)
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        _bws_cache[key] = buf
    return buf


def batched_to_host(o: dict, n_views: int, A: int) -> dict:
    """Per-view results on the host: list of dicts with sparse cells and counts."""
    off = o["edge_off"][:n_views + 1].cpu().numpy()
    E = int(off[-1]) if n_views > 0 else 0
    cols = {k: o[k][:E].cpu().numpy() for k in ("src", "dst", "count", "dt_sum", "dt_min", "dt_max", "dt_mean")}
    st = o["start_count"][:n_views * A].cpu().numpy().reshape(n_views, A)
    en = o["end_count"][:n_views * A].cpu().numpy().reshape(n_views, A)
    ac = o["act_count"][:n_views * A].cpu().numpy().reshape(n_views, A)
    ne = o["n_events"][:n_views].cpu().numpy()
    nc = o["n_cases"][:n_views].cpu().numpy()
    res = []
    for v in range(n_views):
        a, b = int(off[v]), int(off[v + 1])
        d = {k: c[a:b] for k, c in cols.items()}
        d.update(start_count=st[v], end_count=en[v], act_count=ac[v], n_events=int(ne[v]), n_cases=int(nc[v]))
        res.append(d)
    return res


def debug_variant_hash_bits(bits: int) -> int:
    """Test hook: truncate the variant hash of this thread's calls to `bits` bits (0 = full)."""
    return load().pm4g_debug_variant_hash_bits(int(bits))


def profile_enable(on: bool) -> bool:
    """Turns the library's per-stage HIP-event timing on or off."""
    return bool(load().pm4g_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{stage name: (total ms, launches)} since the last read; waits for the events."""
    L = load()
    n = L.pm4g_profile_stage_count()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(L.pm4g_profile_read(ctypes.cast(ms, _P), ctypes.cast(cnt, _P), n))
    return {L.pm4g_profile_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}


# ---- host views of results (copies to host; for tests and reporting) ------------

def dfg_to_host(o: dict, A: int) -> dict:
    h = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
    for k in ("count", "dt_sum", "dt_min", "dt_max", "dt_mean"):
        h[k] = h[k].reshape(A, A)
    for k in ("n_cases", "overflow", "status"):
        h[k] = int(h[k][0])
    return h


def variants_to_host(o: dict, n_cases: int | None = None, top: int | None = None) -> dict:
    """Variants on the host; with `top`, only the first `top` variants of the
    order (count desc, representative asc) and their sequences (n_variants
    still counts all)."""
    V = int(o["n_variants"].item())
    h = dict(n_variants=V, status=int(o["status"].item()))
    K = V if top is None else min(V, int(top))
    for k in ("var_count", "var_len", "var_rep"):
        h[k] = o[k][:K].cpu().numpy()
    h["var_off"] = o["var_off"][:K + 1].cpu().numpy()
    h["var_acts"] = o["var_acts"][:int(h["var_off"][K])].cpu().numpy()
    if o.get("case_variant") is not None and n_cases is not None:
        h["case_variant"] = o["case_variant"][:n_cases].cpu().numpy()
    return h


def prepared_to_host(p: Prepared) -> dict:
    C = int(p.n_cases.item())
    h = dict(case_s=p.case_s.cpu().numpy(), act_s=p.act_s.cpu().numpy(), ts_s=p.ts_s.cpu().numpy(),
             case_off=p.case_off[:C + 1].cpu().numpy(), case_code=p.case_code[:C].cpu().numpy(),
             n_cases=C, status=int(p.status.item()))
    if p.row is not None:
        h["row"] = p.row.cpu().numpy()
    return h
