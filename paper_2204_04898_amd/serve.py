"""Continuous-batching query server over event logs resident in HBM.

The paper names the responsiveness of the tool and drill-down into smaller
views as what users need (Sec. 1); this module serves DFG, variant and
filter queries on such views while the prepared logs (Sec. 3 formatting,
done once) stay on the GPU.

Scheduling (host side, independent of the executor):
  - requests carry a scheduled arrival time (open loop); latency is measured
    from it, not from dispatch;
  - admission by memory: each request has a device-memory estimate (for the
    GPU executor: the library's own workspace-size queries plus the outputs
    the request allocates); a batch is formed from the head of the FIFO queue
    while the estimates fit in the budget left by the batches in flight; the
    head never gets skipped, so no request starves; a request larger than the
    whole budget is rejected;
  - a batch also stops at a work cap (events to scan), so a large request
    runs alone instead of holding small ones back;
  - continuous batching: `workers` persistent worker threads, each with its
    own HIP stream, run up to `workers` batches at once, so requests that
    arrive while a batch runs join the next batch and its work overlaps on
    the device with the running one.

GpuExecutor runs a batch with the library: all DFG and FILTER views of one
log in one pm4g_dfg_batched launch, each VARIANTS view as pm4g_filter_view +
pm4g_variants_prepared; a variants answer carries the variant count and the
first `variants_top` variants (count desc, representative asc) with their
sequences.  Every device buffer a batch uses (workspaces, outputs) is
allocated for that batch, sized by its requests, on the worker's stream, and
is what the requests' estimates charge; the executor keeps nothing else but
the resident logs and one stream per worker.
"""
from __future__ import annotations

import dataclasses
import queue as _queue
import threading
import time
from typing import Callable

import numpy as np

KINDS = ("dfg", "variants", "filter")


@dataclasses.dataclass
class Request:
    rid: int
    log: str
    kind: str                 # "dfg" | "variants" | "filter"
    case_lo: int
    case_hi: int
    t_lo: int
    t_hi: int
    mask: np.ndarray          # uint64 words, bit a selects activity a
    arrival: float            # scheduled arrival, seconds on the server clock
    est_bytes: int = 0
    est_work: int = 0
    dispatched: float = float("nan")
    done: float = float("nan")
    result: dict | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """FIFO admission by memory estimate, up to `workers` batches in flight."""

    def __init__(self, executor, mem_budget: int, max_batch: int = 256, workers: int = 2,
                 clock: Callable[[], float] = time.monotonic, max_batch_work: int | None = None):
        self.ex = executor
        self.budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.workers = int(workers)
        # work cap of one batch (the executor's work units, e.g. events scanned);
        # a request above it runs in a batch of its own, so small requests do not
        # wait behind it
        self.max_batch_work = max_batch_work
        self.clock = clock
        self._lock = threading.Condition()
        self._in_flight_bytes = 0
        self._in_flight = 0
        self.max_in_flight_bytes = 0
        self.batches: list[list[int]] = []
        self.max_queue = 0          # longest the waiting queue has been
        self.memory_blocked = 0     # batch formations that stopped because the head did not fit in memory

    def form_batch(self, queue: list[Request]) -> list[Request]:
        """Head-of-queue batch that fits the memory left; removes it from `queue`."""
        batch: list[Request] = []
        room = self.budget - self._in_flight_bytes
        work = 0
        cap = self.max_batch_work
        batchable = getattr(self.ex, "batchable", None)
        while queue and len(batch) < self.max_batch:
            r = queue[0]
            if r.est_bytes > room:
                if not batch:
                    self.memory_blocked += 1
                break
            if cap is not None and batch and work + r.est_work > cap:
                break
            # a request the executor cannot share a launch with runs in a batch
            # of its own: it would only lengthen the batch of the others
            if batchable is not None and batch and not (batchable(r) and batchable(batch[0])):
                break
            room -= r.est_bytes
            work += r.est_work
            batch.append(queue.pop(0))
        return batch

    def run(self, requests: list[Request], t0: float | None = None,
            progress: Callable[[str], None] | None = None) -> list[Request]:
        """Serves `requests` (arrival times relative to t0); returns them completed.

        `workers` persistent threads take the formed batches (each keeps its
        own stream and buffers in the executor); the calling thread admits
        arrivals and forms a batch whenever a worker is free."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            r.est_bytes = int(self.ex.estimate(r))
            r.est_work = int(self.ex.work(r)) if hasattr(self.ex, "work") else 0
        t0 = self.clock() if t0 is None else t0
        waiting: list[Request] = []
        done: list[Request] = []
        work: _queue.Queue = _queue.Queue()

        def worker(k: int):
            while True:
                batch = work.get()
                if batch is None:
                    return
                self._serve(batch, t0, done, k)

        threads = [threading.Thread(target=worker, args=(k,), daemon=True) for k in range(self.workers)]
        for th in threads:
            th.start()
        i = 0
        last_note = self.clock()
        while True:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                i += 1
                if r.est_bytes > self.budget:
                    r.error = "request exceeds the memory budget"
                    r.dispatched = r.done = now
                    with self._lock:
                        done.append(r)
                else:
                    waiting.append(r)
            self.max_queue = max(self.max_queue, len(waiting))
            batch: list[Request] = []
            with self._lock:
                if self._in_flight < self.workers:
                    batch = self.form_batch(waiting)
                if batch:
                    self._in_flight += 1
                    self._in_flight_bytes += sum(r.est_bytes for r in batch)
                    self.max_in_flight_bytes = max(self.max_in_flight_bytes, self._in_flight_bytes)
                    self.batches.append([r.rid for r in batch])
                elif i == len(pending) and not waiting and self._in_flight == 0:
                    break
                else:
                    # sleep until the next arrival or a completion (notified), at most 5 ms
                    nxt = pending[i].arrival - now if i < len(pending) else 0.005
                    self._lock.wait(timeout=min(max(nxt, 0.0), 0.005))
            if batch:
                for r in batch:
                    r.dispatched = now
                work.put(batch)
            if progress is not None and self.clock() - last_note > 2.0:
                last_note = self.clock()
                progress(f"serving: {len(done)}/{len(pending)} done, {len(waiting)} waiting at t={now:.1f} s")
        for _ in threads:
            work.put(None)
        for th in threads:
            th.join()
        return sorted(done, key=lambda r: r.rid)

    def _serve(self, batch: list[Request], t0: float, done: list[Request], worker: int = 0):
        try:
            self.ex.run(batch, worker)
        except Exception as e:  # reported per request; the server keeps going
            for r in batch:
                r.error = f"{type(e).__name__}: {e}"
        end = self.clock() - t0
        with self._lock:
            for r in batch:
                r.done = end
                done.append(r)
            self._in_flight -= 1
            self._in_flight_bytes -= sum(r.est_bytes for r in batch)
            self._lock.notify_all()


def latency_stats(reqs: list[Request], sched: "Scheduler | None" = None) -> dict:
    """Latency (completion - scheduled arrival) percentiles, completed queries
    per second, and the admission wait (dispatch - arrival); with the
    scheduler, its queue statistics."""
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    if lat.size == 0:
        return dict(n=0, rejected=len(reqs))
    wait = np.array([r.dispatched - r.arrival for r in ok]) * 1e3
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    st = dict(n=len(ok), rejected=len(reqs) - len(ok), p50_ms=float(np.percentile(lat, 50)),
              p99_ms=float(np.percentile(lat, 99)), max_ms=float(lat.max()),
              qps=len(ok) / span if span > 0 else float("nan"),
              wait_p50_ms=float(np.percentile(wait, 50)), wait_p99_ms=float(np.percentile(wait, 99)))
    if sched is not None:
        st.update(max_queue=sched.max_queue, memory_blocked=sched.memory_blocked,
                  max_in_flight_bytes=sched.max_in_flight_bytes, budget_bytes=sched.budget,
                  batches=len(sched.batches), workers=sched.workers)
    return st


def log_info(log) -> dict:
    """What the request generator needs of a synthetic log (a synth.Log)."""
    cum = np.zeros(log.lengths_by_code.shape[0] + 1, np.int64)
    np.cumsum(log.lengths_by_code, out=cum[1:])
    return dict(lengths_by_code=log.lengths_by_code, cum=cum, t_min=int(log.ts.min()), t_max=int(log.ts.max()))


def poisson_requests(rng: np.random.Generator, rate: float, seconds: float, logs: dict, A_of: dict,
                     mix=(("dfg", 0.4), ("variants", 0.3), ("filter", 0.3)),
                     min_events: float = 1e4, max_events: float = 1e8) -> list[Request]:
    """Open-loop Poisson arrivals: log chosen uniformly, kind by `mix`, view with
    a log-uniform slice size in [min_events, max_events] (capped at the log),
    a time window and an activity subset as in the batched-view workload."""
    names = sorted(logs)
    kinds = [k for k, _ in mix]
    probs = np.array([p for _, p in mix], float)
    probs /= probs.sum()
    out = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        name = names[int(rng.integers(0, len(names)))]
        lg = logs[name]
        lengths = lg["lengths_by_code"]
        cum = lg["cum"]
        C = lengths.shape[0]
        N = int(cum[-1])
        A = A_of[name]
        hi_cap = min(max_events, N)
        lo_cap = min(min_events, hi_cap)
        S = int(round(np.exp(rng.uniform(np.log(lo_cap), np.log(max(hi_cap, lo_cap))))))
        p = int(rng.integers(0, C))
        h = int(np.searchsorted(cum, cum[p] + S, side="left"))
        h = min(max(h, p + 1), C)
        if cum[h] - cum[p] < S:
            p = max(int(np.searchsorted(cum, cum[h] - S, side="right")) - 1, 0)
        f = rng.uniform(0.05, 1.0)
        span = lg["t_max"] - lg["t_min"]
        w = int(f * span)
        tl = lg["t_min"] + int(rng.integers(0, max(1, span - w + 1)))
        k = int(rng.integers(min(8, A), A + 1))
        mask = np.zeros((A + 63) // 64, np.uint64)
        for a in rng.choice(A, size=k, replace=False):
            mask[a // 64] |= np.uint64(1) << np.uint64(a % 64)
        kind = kinds[int(rng.choice(len(kinds), p=probs))]
        out.append(Request(rid=rid, log=name, kind=kind, case_lo=p, case_hi=h, t_lo=tl, t_hi=tl + w,
                           mask=mask, arrival=t))
        rid += 1
    return out


class GpuExecutor:
    """Runs batches with libpm4g, one HIP stream per worker thread.  A batch's
    device buffers are allocated for it on the worker's stream and sized by
    its requests; estimate() charges each request what it makes the batch
    allocate, from the library's size queries."""

    def __init__(self, logs: dict, device="cuda:0", variants_top: int = 1000):
        import torch

        from . import pm4g
        self.torch = torch
        self.pm4g = pm4g
        self.device = torch.device(device)
        self.variants_top = int(variants_top)
        self.logs = {}
        for name, prep in logs.items():
            C = int(prep.n_cases.item())
            off = prep.case_off[:C + 1].cpu().numpy()
            # int64, as the view bounds are: a search with a wider key would
            # convert the whole array on every call
            codes = prep.case_code[:C].cpu().numpy().astype(np.int64)
            self.logs[name] = dict(prep=prep, off=off, codes=codes)
        self._streams: list = []   # one per worker index, kept across runs (and their memory pools)
        self._streams_lock = threading.Lock()

    def slice_events(self, r: Request) -> int:
        lg = self.logs[r.log]
        a = int(np.searchsorted(lg["codes"], np.int64(r.case_lo), side="left"))
        b = int(np.searchsorted(lg["codes"], np.int64(r.case_hi), side="left"))
        return int(lg["off"][b] - lg["off"][a]) if b > a else 0

    def batchable(self, r: Request) -> bool:
        """DFG and FILTER views of a batch share one batched launch; a VARIANTS
        view runs its own filter and variants calls."""
        return r.kind != "variants"

    def work(self, r: Request) -> int:
        """Work estimate: events of the view's case slice (variants cost about
        four passes over them)."""
        S = self.slice_events(r)
        return 4 * S if r.kind == "variants" else S

    # capacities of one view in a batched call: one record per kept event
    # (at most the slice's events), the (tile, view) pairs its slice spans
    # (the library keeps a run place per pair and cell bucket), cells and
    # output cells at most one per kept event and A*A (+A start cells) per view
    _TILE = 2048   # the smaller tile: its pair count bounds the larger one's

    def _caps(self, r: Request) -> tuple[int, int, int, int]:
        A = self.logs[r.log]["prep"].n_activities
        S = self.slice_events(r)
        pairs = S // self._TILE + 2
        return (S + 1, pairs, min(S, A * (A + 1)) + 1, min(S, A * A) + 1)

    def _batched_tuning(self, rs: list[Request]):
        caps = [self._caps(r) for r in rs]
        t = self.pm4g.BatchedTuning()
        # one launch per phase: the workers' batches interleave on the device
        # (a persistent launch holds every CU until it ends)
        t.launch = 1
        t.record_capacity = sum(c[0] for c in caps)
        t.pair_capacity = sum(c[1] for c in caps)
        t.cell_capacity = sum(c[2] for c in caps)
        return t, sum(c[3] for c in caps)

    def estimate(self, r: Request) -> int:
        """Device bytes the request makes its batch allocate: the library's
        workspace size for the request's capacities plus its outputs."""
        pm4g = self.pm4g
        prep = self.logs[r.log]["prep"]
        A, N = prep.n_activities, prep.n_events
        if r.kind == "variants":
            S = self.slice_events(r)
            return (pm4g.filter_workspace_bytes(N) + pm4g.prepared_bytes(S)
                    + pm4g.variants_workspace_bytes(S, A) + pm4g.variants_out_bytes(S, with_cases=False)
                    + 256 * 4)
        t, edges = self._batched_tuning([r])
        return pm4g.batched_workspace_bytes(N, A, 1, t) + pm4g.batched_out_bytes(1, A, edges) + 256 * 2

    def _stream(self, worker: int):
        """The HIP stream of worker `worker`: the same stream for that index in
        every run, so the buffers its batches free stay cached for it."""
        with self._streams_lock:
            while len(self._streams) <= worker:
                self._streams.append(self.torch.cuda.Stream(device=self.device))
            return self._streams[worker]

    def start_timeline(self) -> None:
        """Records, from now on, each batch's device-side span: a HIP event on
        its worker's stream before its first launch and after its last one,
        against a reference event on the current stream."""
        torch = self.torch
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref.record()
        self._spans = []

    def timeline(self) -> dict:
        """Device-side overlap of the recorded batches: the time during which
        batches of two or more workers were in progress on the GPU, over the
        time during which any was."""
        torch = self.torch
        torch.cuda.synchronize()
        ev = []
        for w, a, b in self._spans:
            t0, t1 = self._ref.elapsed_time(a), self._ref.elapsed_time(b)
            ev.append((t0, 1, w))
            ev.append((t1, -1, w))
        ev.sort(key=lambda e: (e[0], e[1]))
        open_: dict = {}
        busy = multi = 0.0
        last = ev[0][0] if ev else 0.0
        for t, d, w in ev:
            if open_:
                busy += t - last
                if len(open_) >= 2:
                    multi += t - last
            last = t
            open_[w] = open_.get(w, 0) + d
            if open_[w] == 0:
                del open_[w]
        self._spans = None
        return {"batches": len(ev) // 2, "busy_ms": busy, "multi_worker_ms": multi,
                "overlap_frac": multi / busy if busy else 0.0}

    def run(self, batch: list[Request], worker: int = 0) -> None:
        torch = self.torch
        pm4g = self.pm4g
        s = self._stream(worker)
        spans = getattr(self, "_spans", None)
        if spans is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
        with torch.cuda.stream(s):
            by_log: dict[str, list[Request]] = {}
            for r in batch:
                if r.kind in ("dfg", "filter"):
                    by_log.setdefault(r.log, []).append(r)
            for name, rs in by_log.items():
                prep = self.logs[name]["prep"]
                A = prep.n_activities
                rec = np.zeros(len(rs), dtype=np.dtype([("lo", "<i4"), ("hi", "<i4"), ("t_lo", "<i8"),
                                                       ("t_hi", "<i8")]))
                rec["lo"] = [r.case_lo for r in rs]
                rec["hi"] = [r.case_hi for r in rs]
                rec["t_lo"] = [r.t_lo for r in rs]
                rec["t_hi"] = [r.t_hi for r in rs]
                masks = np.stack([r.mask for r in rs]).view(np.int64)
                vd = torch.from_numpy(rec.view(np.uint8).copy()).to(self.device, non_blocking=False)
                md = torch.from_numpy(np.ascontiguousarray(masks)).to(self.device)
                t, edges = self._batched_tuning(rs)
                o = pm4g.pm4g_dfg_batched(prep, vd, md, len(rs), tuning=t, cap_edges=edges, stream=s,
                                          keep_workspace=False)
                res = pm4g.batched_to_host(o, len(rs), A)
                for r, d in zip(rs, res):
                    if r.kind == "filter":
                        r.result = dict(n_events=d["n_events"], n_cases=d["n_cases"])
                    else:
                        r.result = d
            for r in batch:
                if r.kind != "variants":
                    continue
                prep = self.logs[r.log]["prep"]
                A = prep.n_activities
                rec = np.zeros(1, dtype=np.dtype([("lo", "<i4"), ("hi", "<i4"), ("t_lo", "<i8"),
                                                  ("t_hi", "<i8")]))
                rec["lo"], rec["hi"], rec["t_lo"], rec["t_hi"] = r.case_lo, r.case_hi, r.t_lo, r.t_hi
                vd = torch.from_numpy(rec.view(np.uint8).copy()).to(self.device)
                md = torch.from_numpy(np.ascontiguousarray(r.mask).view(np.int64).copy()).to(self.device)
                S = max(self.slice_events(r), 1)
                fws = torch.empty(max(pm4g.filter_workspace_bytes(prep.n_events), 1), dtype=torch.uint8,
                                  device=self.device)
                sub = pm4g.pm4g_filter_view(prep, vd, md, out=pm4g.Prepared.empty(S, A, self.device), ws=fws,
                                            stream=s)
                vws = torch.empty(max(pm4g.variants_workspace_bytes(S, A), 1), dtype=torch.uint8,
                                  device=self.device)
                v = pm4g.pm4g_variants_prepared(sub, out=pm4g._var_out(S, self.device, with_cases=False),
                                                ws=vws, stream=s)
                s.synchronize()
                C = int(sub.n_cases.item())
                h = pm4g.variants_to_host(v, top=self.variants_top)
                h["n_events"] = int(sub.case_off[C].item())
                h["n_cases"] = C
                r.result = h
        if spans is not None:
            e1.record(s)
            spans.append((worker, e0, e1))
        s.synchronize()
