"""Continuous-batching server for RS assemblies on one GPU.

Requests (particle systems of different N and n) arrive over time.  Each is
admitted as soon as a slot is free and its device-memory footprint fits in
the remaining HBM budget; admitted requests run concurrently on their slot's
HIP stream, so work of different requests overlaps on the device.  Admission
is first-come first-served: a request that does not fit yet blocks the ones
behind it, so large requests cannot starve.  Latency is measured from the
request's arrival to the completion of its result (energy, ranks; the grid
stays on the device until the request is retired).

The scheduler is executor-agnostic: GpuExecutor drives librs.so; tests use a
CPU executor to exercise admission, ordering and accounting without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import queue
import sys
import threading
import time
from typing import Any, Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Record:
    idx: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    footprint: int = 0
    result: Any = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Executor:
    """Interface: footprint(req) -> bytes; make_slot(i) -> slot; run(req, slot) -> result."""

    def footprint(self, req) -> int:  # pragma: no cover - interface
        raise NotImplementedError

    def make_slot(self, i: int):  # pragma: no cover - interface
        return i

    def run(self, req, slot):  # pragma: no cover - interface
        raise NotImplementedError

    def close(self):
        """Release what the executor holds (device memory, handles)."""


class Server:
    """Continuous batching over `n_slots` slots.  Each slot has one worker
    thread for the whole replay (started by run_trace and joined before it
    returns), so the number of host threads that call into the GPU runtime
    is the number of slots, not the number of requests."""

    def __init__(self, executor: Executor, n_slots: int = 4, hbm_budget: int = 1 << 40,
                 clock: Callable[[], float] = time.perf_counter):
        if n_slots < 1:
            raise ValueError("n_slots must be >= 1")
        self.ex = executor
        self.n_slots = n_slots
        self.budget = int(hbm_budget)
        self.clock = clock
        self._cv = threading.Condition()
        self._slots = [executor.make_slot(i) for i in range(n_slots)]
        self._free_slots = collections.deque(range(n_slots))
        self._in_use = 0
        self.peak_bytes = 0
        self.peak_concurrency = 0
        self._concurrency = 0

    # -- worker: one per slot -------------------------------------------------
    def _worker(self, i: int, inbox: "queue.Queue"):
        slot = self._slots[i]
        while True:
            item = inbox.get()
            if item is None:
                return
            req, rec = item
            try:
                rec.result = self.ex.run(req, slot)
            except Exception as e:  # a failing request fails alone
                rec.error = f"{type(e).__name__}: {e}"
            with self._cv:
                rec.done = self.clock()
                self._in_use -= rec.footprint
                self._free_slots.append(i)
                self._concurrency -= 1
                self._cv.notify_all()

    # -- replay of an arrival trace ------------------------------------------
    def run_trace(self, requests: List[Any], arrival_of: Callable[[Any], float] = lambda r: r.arrival_s,
                  time_scale: float = 1.0, progress_every: int = 0) -> List[Record]:
        """Replay `requests` with their arrival offsets (seconds, scaled by
        time_scale) in real time and return one Record per request.  With
        progress_every > 0 a line goes to stderr each time that many more
        requests have finished."""
        order = sorted(range(len(requests)), key=lambda i: arrival_of(requests[i]))
        t0 = self.clock()
        recs = [Record(i, t0 + arrival_of(requests[i]) * time_scale) for i in range(len(requests))]
        pending: collections.deque = collections.deque()
        nxt = 0
        reported = 0
        for i, r in enumerate(requests):
            recs[i].footprint = int(self.ex.footprint(r))
            if recs[i].footprint > self.budget:
                recs[i].error = "rejected: footprint exceeds the HBM budget"
        inboxes = [queue.Queue() for _ in range(self.n_slots)]
        workers = [threading.Thread(target=self._worker, args=(i, inboxes[i]), daemon=True)
                   for i in range(self.n_slots)]
        for th in workers:
            th.start()
        try:
            with self._cv:
                while nxt < len(order) or pending or self._concurrency > 0:
                    now = self.clock()
                    while nxt < len(order) and recs[order[nxt]].arrival <= now:
                        i = order[nxt]
                        nxt += 1
                        if recs[i].error is None:
                            pending.append(i)
                        else:
                            recs[i].admitted = recs[i].done = now
                    # admit in arrival order while a slot and the memory are free
                    while pending and self._free_slots and \
                            self._in_use + recs[pending[0]].footprint <= self.budget:
                        i = pending.popleft()
                        rec = recs[i]
                        slot = self._free_slots.popleft()
                        self._in_use += rec.footprint
                        self._concurrency += 1
                        self.peak_bytes = max(self.peak_bytes, self._in_use)
                        self.peak_concurrency = max(self.peak_concurrency, self._concurrency)
                        rec.admitted = self.clock()
                        inboxes[slot].put((requests[i], rec))
                    wait = None
                    if nxt < len(order):
                        wait = max(0.0, recs[order[nxt]].arrival - self.clock())
                    if nxt < len(order) or pending or self._concurrency > 0:
                        self._cv.wait(timeout=wait if wait is not None else 1.0)
                    if progress_every > 0:
                        done = sum(1 for r in recs if r.done == r.done)   # done is NaN until set
                        if done >= reported + progress_every:
                            reported = done - done % progress_every
                            print(f"serving: {done} of {len(recs)} requests done", file=sys.stderr,
                                  flush=True)
        finally:
            for q in inboxes:
                q.put(None)
            for th in workers:
                th.join()
        return recs


def summarize(recs: List[Record]) -> Dict[str, Any]:
    ok = [r for r in recs if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(0)
    if not ok:
        return {"completed": 0, "failed": len(recs)}
    span = max(r.done for r in ok) - min(r.arrival for r in recs)
    return {
        "completed": len(ok),
        "failed": len(recs) - len(ok),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "throughput_per_s": len(ok) / span if span > 0 else float("inf"),
        "makespan_s": span,
    }


class GpuExecutor(Executor):
    """Runs one request = RS assembly (+ grid on the device) + energy on the
    slot's own HIP stream through librs.so."""

    def __init__(self, device: int = 0, prec: str = "mixed_fp16", with_grid: bool = True,
                 eps_tucker: float = 1e-6, r_max: int = 384, digest: bool = False):
        import torch

        from . import _lib
        self.torch = torch
        self.lib = _lib
        self.ctx = _lib.Context(device)
        self.device = torch.device(f"cuda:{device}")
        self.prec = prec
        self.with_grid = with_grid
        self.eps = eps_tucker
        self.r_max = r_max
        self.digest = digest
        self._factors: Dict[tuple, Any] = {}
        self._lock = threading.Lock()

    def factors(self, sysm):
        key = (sysm.b, sysm.n, sysm.R, sysm.R_l, sysm.n_s, sysm.kernel, sysm.lam)
        with self._lock:
            f = self._factors.get(key)
            if f is None:
                f = self.lib.Factors(self.ctx, sysm.b, sysm.n, sysm.R, sysm.R_l,
                                     sysm.n_s if sysm.n_s else -1, kernel=sysm.kernel, lam=sysm.lam,
                                     delta_rel=sysm.delta_rel)
                self._factors[key] = f
        return f

    def close(self):
        """Wait for the device, then free the quadrature tables and the
        context (rather than leaving them to the garbage collector)."""
        if self.ctx is None:
            return
        self.torch.cuda.synchronize(self.device)
        with self._lock:
            for f in self._factors.values():
                f.close()
            self._factors.clear()
        self.ctx.close()
        self.ctx = None

    def footprint(self, req) -> int:
        sysm = req.system() if hasattr(req, "system") else req
        f = self.factors(sysm)
        r_max = min(self.r_max, sysm.n)
        grid_bytes = sysm.n ** 3 * (8 if self.prec == "fp64" else 4) if self.with_grid else 0
        return self.lib.footprint_bytes(f, sysm.N, r_max, self.prec) + grid_bytes

    def make_slot(self, i: int):
        return self.torch.cuda.Stream(device=self.device)

    def run(self, req, slot):
        torch = self.torch
        sysm = req.system() if hasattr(req, "system") else req
        f = self.factors(sysm)
        with torch.cuda.stream(slot):
            pos = torch.tensor(sysm.pos, dtype=torch.float64).to(self.device, non_blocking=False)
            q = torch.tensor(sysm.q, dtype=torch.float64).to(self.device, non_blocking=False)
            grid = None
            if self.with_grid:
                dt = torch.float64 if self.prec == "fp64" else torch.float32
                grid = torch.empty(sysm.n ** 3, dtype=dt, device=self.device)
            opts = self.lib.make_aopts(self.eps, r_max=min(self.r_max, sysm.n), prec=self.prec)
            T = self.lib.assemble(self.ctx, f, pos, q, grid, opts, stream=slot)
            E = torch.empty(1, dtype=torch.float64, device=self.device)
            self.lib.energy(T, E, stream=slot)
            slot.synchronize()
            inf = T.info()
            out = {"energy": E.item(), "ranks": list(inf.ranks), "N": sysm.N, "n": sysm.n,
                   "status": T.status}
            if self.digest and grid is not None:
                out["grid_digest"] = grid_digest(grid)
            T.free()
            del grid
        return out


def grid_digest(grid) -> tuple:
    """A few exact reductions of a device grid (sum in FP64, max |value|,
    and every 9973rd value), computed on the device: two results with the
    same digest agree bitwise on all sampled values and almost surely
    everywhere."""
    g = grid.double()
    return (float(g.sum().item()), float(g.abs().max().item()),
            tuple(float(v) for v in g[::9973][:256].cpu().tolist()))
