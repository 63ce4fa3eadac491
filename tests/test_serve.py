"""Scheduler of the serving loop, on the CPU with a fake executor."""
import dataclasses
import threading
import time

import pytest

from paper_1606_09218_amd.serve import Executor, Server, summarize


@dataclasses.dataclass
class Req:
    idx: int
    arrival_s: float
    dur: float
    mem: int
    fail: bool = False


class FakeExecutor(Executor):
    def __init__(self):
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.starts = []

    def footprint(self, req):
        return req.mem

    def run(self, req, slot):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.starts.append(req.idx)
        time.sleep(req.dur)
        with self.lock:
            self.running -= 1
        if req.fail:
            raise RuntimeError("poisoned request")
        return {"idx": req.idx, "slot": slot}


def trace(n=24, gap=0.004, dur=0.02, mem=10):
    return [Req(i, i * gap, dur * (1 + (i % 3)), mem * (1 + (i % 4))) for i in range(n)]


def test_all_complete_fifo_and_latency_bounds():
    ex = FakeExecutor()
    reqs = trace()
    srv = Server(ex, n_slots=3, hbm_budget=1000)
    recs = srv.run_trace(reqs)
    assert all(r.error is None for r in recs)
    # admitted in arrival order (the scheduler admits on one thread; the slot
    # workers may start two back-to-back admissions in either order)
    assert [r.idx for r in sorted(recs, key=lambda r: r.admitted)] == list(range(len(reqs)))
    for r, q in zip(recs, reqs):
        assert r.result["idx"] == q.idx
        assert r.latency >= q.dur - 1e-3
        assert r.admitted >= r.arrival - 1e-3
    assert ex.max_running <= 3
    assert srv.peak_concurrency <= 3
    s = summarize(recs)
    assert s["completed"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_limits_concurrency_and_blocks_in_order():
    ex = FakeExecutor()
    reqs = [Req(i, 0.0, 0.03, 60) for i in range(6)]
    srv = Server(ex, n_slots=6, hbm_budget=130)    # only two fit at once
    recs = srv.run_trace(reqs)
    assert all(r.error is None for r in recs)
    assert srv.peak_bytes <= 130
    assert ex.max_running <= 2
    assert [r.idx for r in sorted(recs, key=lambda r: r.admitted)] == list(range(6))


def test_oversized_request_rejected_others_served():
    ex = FakeExecutor()
    reqs = [Req(0, 0.0, 0.01, 10), Req(1, 0.0, 0.01, 5000), Req(2, 0.0, 0.01, 10)]
    recs = Server(ex, n_slots=2, hbm_budget=100).run_trace(reqs)
    assert recs[1].error and "exceeds" in recs[1].error
    assert recs[0].error is None and recs[2].error is None


def test_failing_request_fails_alone():
    ex = FakeExecutor()
    reqs = trace(8)
    reqs[3].fail = True
    recs = Server(ex, n_slots=2, hbm_budget=1000).run_trace(reqs)
    assert recs[3].error and "poisoned" in recs[3].error
    assert all(r.error is None for i, r in enumerate(recs) if i != 3)


def test_continuous_batching_overlaps_arrivals():
    """A request that arrives while an earlier one runs starts before that one
    finishes (it is not held back until a batch drains)."""
    ex = FakeExecutor()
    reqs = [Req(0, 0.0, 0.2, 10), Req(1, 0.05, 0.02, 10), Req(2, 0.06, 0.02, 10)]
    recs = Server(ex, n_slots=2, hbm_budget=100).run_trace(reqs)
    assert recs[1].admitted < recs[0].done
    assert recs[1].done < recs[0].done


def test_one_worker_thread_per_slot():
    """Every request of a replay runs on one of n_slots long-lived threads,
    and none of them is left when run_trace returns."""
    seen = set()

    class ThreadRecorder(FakeExecutor):
        def run(self, req, slot):
            seen.add(threading.get_ident())
            return super().run(req, slot)

    before = threading.active_count()
    Server(ThreadRecorder(), n_slots=3, hbm_budget=1000).run_trace(trace(30, gap=0.001, dur=0.002))
    assert 1 <= len(seen) <= 3
    assert threading.active_count() == before


def test_time_scale_and_empty_trace():
    ex = FakeExecutor()
    assert Server(ex).run_trace([]) == []
    reqs = trace(5, gap=0.1, dur=0.001)
    t0 = time.perf_counter()
    Server(ex, n_slots=1).run_trace(reqs, time_scale=0.1)
    assert time.perf_counter() - t0 < 0.3
