"""Scheduler logic of the serving loop on the CPU: a fake executor with
known memory estimates and service times (no GPU)."""
import threading
import time

import numpy as np
import pytest

from paper_2204_04898_amd.serve import Request, Scheduler, latency_stats


class FakeExecutor:
    def __init__(self, est, service_s=0.002, fail_rids=()):
        self.est = est
        self.service_s = service_s
        self.fail = set(fail_rids)
        self.lock = threading.Lock()
        self.concurrent = 0
        self.max_concurrent = 0
        self.batches = []

    def estimate(self, r):
        return self.est(r)

    def run(self, batch, worker=0):
        with self.lock:
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
            self.batches.append([r.rid for r in batch])
        time.sleep(self.service_s)
        for r in batch:
            if r.rid in self.fail:
                raise RuntimeError("executor failure")
            r.result = {"rid": r.rid}
        with self.lock:
            self.concurrent -= 1


def reqs(n, gap=0.0005, kind="dfg"):
    return [Request(rid=i, log="L", kind=kind, case_lo=0, case_hi=1, t_lo=0, t_hi=1,
                    mask=np.zeros(1, np.uint64), arrival=i * gap) for i in range(n)]


def test_every_request_completes_fifo_within_budget():
    ex = FakeExecutor(est=lambda r: 100 + 10 * (r.rid % 7))
    sch = Scheduler(ex, mem_budget=600, max_batch=8, workers=2)
    out = sch.run(reqs(60))
    assert [r.rid for r in out] == list(range(60))
    assert all(r.error is None and r.result == {"rid": r.rid} for r in out)
    assert sch.max_in_flight_bytes <= 600
    assert ex.max_concurrent <= 2
    # FIFO: batches are contiguous runs in arrival order
    flat = [rid for b in sch.batches for rid in b]
    assert flat == sorted(flat)
    assert all(len(b) <= 8 for b in sch.batches)
    # latency is measured from the scheduled arrival
    assert all(r.done >= r.arrival and r.dispatched >= r.arrival - 1e-9 for r in out)


def test_requests_arriving_during_a_batch_join_a_later_batch():
    ex = FakeExecutor(est=lambda r: 1, service_s=0.02)
    sch = Scheduler(ex, mem_budget=10**9, max_batch=1000, workers=1)
    out = sch.run(reqs(20, gap=0.003))
    assert len(sch.batches) >= 2 and len(sch.batches[0]) < 20
    assert all(r.error is None for r in out)


def test_oversized_request_rejected_others_served():
    ex = FakeExecutor(est=lambda r: 10**6 if r.rid == 3 else 10)
    sch = Scheduler(ex, mem_budget=1000, max_batch=4, workers=2)
    out = sch.run(reqs(10))
    assert out[3].error == "request exceeds the memory budget" and out[3].result is None
    assert all(r.error is None for r in out if r.rid != 3)
    st = latency_stats(out)
    assert st["n"] == 9 and st["rejected"] == 1


def test_head_is_never_skipped():
    # a big request waits for memory; smaller ones behind it do not overtake it
    ex = FakeExecutor(est=lambda r: 900 if r.rid == 1 else 200, service_s=0.01)
    sch = Scheduler(ex, mem_budget=1000, max_batch=10, workers=2)
    out = sch.run(reqs(6, gap=0.0))
    order = [rid for b in sch.batches for rid in b]
    assert order == sorted(order)
    assert all(r.error is None for r in out)


def test_executor_failure_is_reported_per_request():
    ex = FakeExecutor(est=lambda r: 1, fail_rids={5})
    sch = Scheduler(ex, mem_budget=100, max_batch=1, workers=2)
    out = sch.run(reqs(8))
    assert out[5].error and "executor failure" in out[5].error
    assert all(r.error is None for r in out if r.rid != 5)


def test_work_cap_closes_batches_and_large_requests_run_alone():
    class WorkExecutor(FakeExecutor):
        def work(self, r):
            return 1000 if r.rid % 10 == 3 else 10

    ex = WorkExecutor(est=lambda r: 1, service_s=0.002)
    sch = Scheduler(ex, mem_budget=10**6, max_batch=64, workers=1, max_batch_work=100)
    out = sch.run(reqs(40, gap=0.0))   # all arrive at once
    assert all(r.error is None for r in out)
    for b in sch.batches:
        big = [rid for rid in b if rid % 10 == 3]
        if big:
            # a request above the cap forms a batch only when it heads the queue, and alone
            assert b == big
        else:
            assert 10 * len(b) <= 100
    # FIFO order is kept
    flat = [rid for b in sch.batches for rid in b]
    assert flat == sorted(flat)


def test_tight_budget_queues_requests_by_memory():
    """With a budget that holds two requests at a time and four workers, the
    third concurrent request waits for memory, not for a worker: the queue
    builds, admission waits grow, and the bytes in flight never exceed the budget."""
    ex = FakeExecutor(est=lambda r: 400, service_s=0.02)
    sch = Scheduler(ex, mem_budget=1000, max_batch=1, workers=4)
    out = sch.run(reqs(24, gap=0.001))
    assert all(r.error is None for r in out)
    assert sch.max_in_flight_bytes <= 1000
    assert ex.max_concurrent <= 2              # memory, not the four workers, bounds the overlap
    assert sch.memory_blocked > 0 and sch.max_queue > 2
    st = latency_stats(out, sch)
    assert st["wait_p99_ms"] > 20.0 and st["max_queue"] == sch.max_queue
    assert st["budget_bytes"] == 1000 and st["memory_blocked"] == sch.memory_blocked


def test_unbatchable_requests_run_alone():
    """Requests the executor cannot share a launch with form batches of their own."""
    class Ex(FakeExecutor):
        def batchable(self, r):
            return r.kind != "variants"
    ex = Ex(est=lambda r: 1, service_s=0.02)
    rs = reqs(30, gap=0.0)
    for r in rs[::3]:
        r.kind = "variants"
    sch = Scheduler(ex, mem_budget=10**9, max_batch=64, workers=1)
    out = sch.run(rs)
    assert all(r.error is None for r in out)
    kind = {r.rid: r.kind for r in rs}
    for b in sch.batches:
        if any(kind[i] == "variants" for i in b):
            assert len(b) == 1, b
    assert max(len(b) for b in sch.batches) > 1
