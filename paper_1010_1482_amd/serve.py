"""Serving form: continuous batching of N-body evaluations of uneven size.

Requests (positions and masses of one particle set, an expansion order and a
method) arrive over time.  The server keeps a fixed set of slots, each a
worker thread with its own HIP stream; a request is admitted when a slot is
free and its device footprint (arena + inputs + outputs) fits the remaining
HBM budget, in arrival order.  Admitted requests run concurrently on their
slots' streams (the library calls release the GIL), so the work of several
requests overlaps on the device; a finished request frees its slot and its
budget, and the next waiting request is admitted immediately.

Per request the server records the scheduled arrival, admission, start and
finish times; latency = finish - scheduled arrival.  Each request's tree and
expansions live in its own arena until the request completes.  When the
arena estimate falls short (clustered data), the executor asks the server
for the extra bytes (Request.grow) before it allocates them: the budget
counts what the device actually holds, a growth waits while other requests
run and fails the request when it can never fit.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    p: int
    t_arrive: float                      # scheduled arrival, seconds from start
    make_inputs: Callable[[], tuple]     # -> host (x, y, z, m) float64 arrays
    method: str = "fmm"
    precision: str = "fp32"
    leaf_max: int = 64
    theta: float = 0.5
    keep_output: bool = False
    # filled by the server
    status: str = "pending"
    error: str = ""
    t_admit: float = float("nan")
    t_start: float = float("nan")
    t_finish: float = float("nan")
    footprint: int = 0
    output: Optional[tuple] = None
    grow: Optional[Callable[[int], None]] = None  # set by the server at admission

    @property
    def latency(self) -> float:
        return self.t_finish - self.t_arrive


class Server:
    """Continuous-batching request loop over `slots` concurrent streams.

    executor(request, slot) -> output tuple runs one request on a slot; the
    default runs the HIP library (see hip_executor).  footprint(request) ->
    bytes is the admission size."""

    def __init__(self, budget_bytes: int, slots: int = 4,
                 executor: Optional[Callable] = None,
                 footprint: Optional[Callable[[Request], int]] = None):
        self.budget = int(budget_bytes)
        self.nslots = int(slots)
        self.executor = executor
        self.footprint = footprint
        self.in_use = 0
        self.cv = threading.Condition()
        self.free_slots = collections.deque(range(self.nslots))
        self.jobs = [collections.deque() for _ in range(self.nslots)]
        self.job_cv = [threading.Condition() for _ in range(self.nslots)]
        self.stop = False
        self.t0 = 0.0
        self.done = []
        self.running = 0   # admitted and not finished
        self.growing = 0   # of those, waiting for budget to grow their arena
        self.max_in_use = 0

    def grow(self, req: Request, extra: int) -> None:
        """Charge `extra` more bytes to a running request (called from its
        worker before it allocates them).  Waits while other running
        requests may still free budget; raises MemoryError when the request
        alone would exceed the budget or nothing else can free any.  New
        admissions wait while a growth is pending."""
        extra = int(extra)
        if extra <= 0:
            return
        with self.cv:
            self.growing += 1
            try:
                while self.in_use + extra > self.budget:
                    if req.footprint + extra > self.budget or self.running - self.growing <= 0:
                        raise MemoryError(f"arena growth by {extra} bytes does not fit the "
                                          f"HBM budget {self.budget}")
                    self.cv.wait(timeout=0.05)
                self.in_use += extra
                self.max_in_use = max(self.max_in_use, self.in_use)
                req.footprint += extra
            finally:
                self.growing -= 1
                self.cv.notify_all()

    def _now(self) -> float:
        return time.perf_counter() - self.t0

    def _worker(self, slot: int):
        while True:
            with self.job_cv[slot]:
                while not self.jobs[slot] and not self.stop:
                    self.job_cv[slot].wait()
                if not self.jobs[slot]:
                    return
                req = self.jobs[slot].popleft()
            req.t_start = self._now()
            try:
                out = self.executor(req, slot)
                req.status = "ok"
                if req.keep_output:
                    req.output = out
            except Exception as e:  # a failed request frees its slot and budget
                req.status = "failed"
                req.error = f"{type(e).__name__}: {e}"
            req.t_finish = self._now()
            with self.cv:
                self.in_use -= req.footprint
                self.running -= 1
                self.free_slots.append(slot)
                self.done.append(req)
                self.cv.notify_all()

    def run(self, requests, realtime: bool = True):
        """Serve `requests` (sorted by t_arrive).  realtime=False submits all
        at t = 0 (closed loop).  Returns the requests with their timings."""
        reqs = sorted(requests, key=lambda r: r.t_arrive)
        for r in reqs:
            r.footprint = int(self.footprint(r)) if self.footprint else 0
        threads = [threading.Thread(target=self._worker, args=(k,), daemon=True)
                   for k in range(self.nslots)]
        for th in threads:
            th.start()
        self.t0 = time.perf_counter()
        pending = collections.deque()
        i = 0
        with self.cv:
            while i < len(reqs) or pending or len(self.done) < len(reqs):
                now = self._now()
                while i < len(reqs) and (not realtime or reqs[i].t_arrive <= now):
                    r = reqs[i]
                    i += 1
                    if r.footprint > self.budget:
                        r.status = "rejected"
                        r.error = f"footprint {r.footprint} exceeds budget {self.budget}"
                        r.t_admit = r.t_start = r.t_finish = now
                        self.done.append(r)
                        continue
                    pending.append(r)
                # admission in arrival order: a slot and the budget must be free
                while pending and self.free_slots and not self.growing and \
                        self.in_use + pending[0].footprint <= self.budget:
                    r = pending.popleft()
                    slot = self.free_slots.popleft()
                    self.in_use += r.footprint
                    self.max_in_use = max(self.max_in_use, self.in_use)
                    self.running += 1
                    r.grow = (lambda extra, r=r: self.grow(r, extra))
                    r.t_admit = self._now()
                    with self.job_cv[slot]:
                        self.jobs[slot].append(r)
                        self.job_cv[slot].notify()
                if len(self.done) == len(reqs):
                    break
                wait = None
                if i < len(reqs) and realtime:
                    wait = max(0.0, reqs[i].t_arrive - self._now())
                self.cv.wait(timeout=wait if wait is not None else 0.05)
        self.stop = True
        for k in range(self.nslots):
            with self.job_cv[k]:
                self.job_cv[k].notify_all()
        for th in threads:
            th.join()
        return reqs


def summarize(reqs, wall: Optional[float] = None) -> dict:
    ok = [r for r in reqs if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    span = wall if wall is not None else (max(r.t_finish for r in ok) if ok else 0.0)
    parts = sum(r.n for r in ok)
    return {"requests": len(reqs), "ok": len(ok),
            "failed": sum(r.status == "failed" for r in reqs),
            "rejected": sum(r.status == "rejected" for r in reqs),
            "makespan_s": span, "particles": parts,
            "particles_per_s": parts / span if span > 0 else 0.0,
            "requests_per_s": len(ok) / span if span > 0 else 0.0,
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                           "p99": float(np.percentile(lat, 99) * 1e3),
                           "mean": float(lat.mean() * 1e3),
                           "max": float(lat.max() * 1e3)}}


# ---------------------------------------------------------------------------
# HIP executor
# ---------------------------------------------------------------------------
def hip_footprint(req: Request) -> int:
    from . import hfmm
    meth = hfmm.METHODS[req.method]
    prec = hfmm.PRECISIONS[req.precision]
    arena = hfmm.arena_bytes(req.n, 0, req.leaf_max, req.p, meth, prec)
    out_b = 8 if prec == hfmm.FP64 else 4
    return int(arena + req.n * (4 * 8 + 4 * out_b))


class HipExecutor:
    """Runs a request on its slot's stream: H2D of the inputs (pinned host
    buffers), build + upward + evaluate in the request's own arena, D2H of
    the outputs.  Everything for one request is enqueued on one stream."""

    def __init__(self, slots: int, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]

    def __call__(self, req: Request, slot: int):
        torch = self.torch
        from . import hfmm
        x, y, z, m = req.make_inputs()
        s = self.streams[slot]
        host_in = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
                   for a in (x, y, z, m)]
        prec = hfmm.PRECISIONS[req.precision]
        meth = hfmm.METHODS[req.method]
        nbytes = hfmm.arena_bytes(req.n, 0, req.leaf_max, req.p, meth, prec)
        with torch.cuda.stream(s):
            dev = [h.to(self.device, non_blocking=True) for h in host_in]
            for _ in range(4):
                # the arena the footprint charged; a larger one only once the
                # server has charged the difference
                arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                try:
                    out = hfmm.solve(*dev, p=req.p, method=meth, precision=prec,
                                     leaf_max=req.leaf_max, theta=req.theta, arena=arena,
                                     stream=s)
                    break
                except hfmm.HfmmError as e:
                    if e.code != hfmm.E_NOMEM:
                        raise
                    need = int(hfmm._lib().hfmm_last_required_bytes() * 1.25)
                    del arena
                    if req.grow is not None:
                        req.grow(need - nbytes)
                    nbytes = need
            else:
                raise MemoryError("arena did not suffice after growing")
            host_out = [torch.empty(o.shape, dtype=o.dtype, pin_memory=True) for o in out]
            for h, o in zip(host_out, out):
                h.copy_(o, non_blocking=True)
        s.synchronize()
        return tuple(h.numpy() for h in host_out)


def trace_requests(trace, precision="fp32", leaf_max=64, keep=()):
    """Request objects for workloads.request_trace entries."""
    from . import workloads as W
    out = []
    for e in trace:
        def mk(e=e):
            return W.make(e["dist"], e["n"], e["seed"])
        out.append(Request(rid=e["i"], n=e["n"], p=e["p"], t_arrive=e["t_arrive"],
                           make_inputs=mk, precision=precision, leaf_max=leaf_max,
                           keep_output=e["i"] in keep))
    return out
