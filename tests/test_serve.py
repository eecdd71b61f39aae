"""Serving-loop scheduling on the CPU with a test double in place of the HIP
executor: admission order, HBM-budget accounting, oversize rejection, a
failing request, concurrency and latency bookkeeping."""
import threading
import time

import numpy as np

from paper_1010_1482_amd.serve import Request, Server, summarize


class FakeExecutor:
    """Sleeps n microseconds per request; records concurrency and budget."""

    def __init__(self, server_ref, fail_ids=()):
        self.server_ref = server_ref
        self.fail_ids = set(fail_ids)
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.max_in_use = 0
        self.order = []

    def __call__(self, req, slot):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.max_in_use = max(self.max_in_use, self.server_ref[0].in_use)
            self.order.append(req.rid)
        try:
            time.sleep(req.n * 1e-6)
            if req.rid in self.fail_ids:
                raise RuntimeError("injected failure")
            return (req.rid,)
        finally:
            with self.lock:
                self.running -= 1


def make(n_req, sizes, arrivals):
    return [Request(rid=i, n=int(sizes[i]), p=6, t_arrive=float(arrivals[i]),
                    make_inputs=lambda: None) for i in range(n_req)]


def test_budget_is_never_exceeded_and_slots_overlap():
    ref = [None]
    ex = FakeExecutor(ref)
    srv = Server(budget_bytes=3000, slots=4, executor=ex, footprint=lambda r: r.n)
    ref[0] = srv
    reqs = make(40, [1000] * 40, np.zeros(40))
    srv.run(reqs, realtime=False)
    assert all(r.status == "ok" for r in reqs)
    assert ex.max_in_use <= 3000
    assert ex.max_running == 3          # budget, not slots, limits concurrency
    assert srv.in_use == 0 and len(srv.free_slots) == 4


def test_admission_in_arrival_order():
    ref = [None]
    ex = FakeExecutor(ref)
    srv = Server(budget_bytes=10 ** 9, slots=1, executor=ex, footprint=lambda r: r.n)
    ref[0] = srv
    arr = np.linspace(0, 0.02, 10)
    reqs = make(10, [500] * 10, arr[::-1])   # ids arrive in reverse
    srv.run(reqs)
    assert ex.order == list(range(9, -1, -1))
    for r in reqs:
        assert r.t_admit >= r.t_arrive - 1e-3
        assert r.t_finish >= r.t_start >= r.t_admit


def test_oversize_rejected_and_failure_isolated():
    ref = [None]
    ex = FakeExecutor(ref, fail_ids={3})
    srv = Server(budget_bytes=5000, slots=2, executor=ex, footprint=lambda r: r.n)
    ref[0] = srv
    sizes = [1000] * 8
    sizes[5] = 6000
    reqs = make(8, sizes, np.zeros(8))
    srv.run(reqs, realtime=False)
    st = {r.rid: r.status for r in reqs}
    assert st[5] == "rejected" and st[3] == "failed"
    assert all(st[i] == "ok" for i in (0, 1, 2, 4, 6, 7))
    assert "injected" in reqs[3].error
    assert srv.in_use == 0 and len(srv.free_slots) == 2
    s = summarize(reqs)
    assert s["ok"] == 6 and s["failed"] == 1 and s["rejected"] == 1


def test_latency_includes_queueing():
    ref = [None]
    ex = FakeExecutor(ref)
    srv = Server(budget_bytes=10 ** 9, slots=1, executor=ex, footprint=lambda r: 1)
    ref[0] = srv
    reqs = make(5, [20000] * 5, np.zeros(5))   # 20 ms each, one slot
    srv.run(reqs, realtime=False)
    lat = sorted(r.latency for r in reqs)
    assert lat[-1] > 4 * 0.02 * 0.9        # the last one waited for four others
    s = summarize(reqs)
    assert s["latency_ms"]["p99"] >= s["latency_ms"]["p50"] > 0
