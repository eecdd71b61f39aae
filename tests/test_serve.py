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


class GrowingExecutor(FakeExecutor):
    """Asks the server for `extra[rid]` more bytes before it runs."""

    def __init__(self, server_ref, extra):
        super().__init__(server_ref)
        self.extra = extra

    def __call__(self, req, slot):
        if self.extra.get(req.rid):
            req.grow(self.extra[req.rid])
        with self.lock:
            self.max_in_use = max(self.max_in_use, self.server_ref[0].in_use)
        return super().__call__(req, slot)


def test_arena_growth_is_charged_to_the_budget():
    ref = [None]
    ex = GrowingExecutor(ref, {i: 500 for i in range(0, 20, 2)})
    srv = Server(budget_bytes=3000, slots=4, executor=ex, footprint=lambda r: r.n)
    ref[0] = srv
    reqs = make(20, [1000] * 20, np.zeros(20))
    srv.run(reqs, realtime=False)
    assert all(r.status == "ok" for r in reqs)
    assert srv.max_in_use <= 3000 and ex.max_in_use <= 3000
    assert all(r.footprint == (1500 if r.rid % 2 == 0 else 1000) for r in reqs)
    assert srv.in_use == 0 and srv.running == 0


def test_growth_waits_for_other_requests_then_runs():
    # two requests fill the budget; one needs 1000 more, which only the
    # other's completion frees
    ref = [None]
    ex = GrowingExecutor(ref, {0: 1000})
    srv = Server(budget_bytes=2500, slots=2, executor=ex, footprint=lambda r: r.n)
    ref[0] = srv
    reqs = make(2, [1000, 1200], np.zeros(2))
    srv.run(reqs, realtime=False)
    assert [r.status for r in reqs] == ["ok", "ok"]
    assert srv.max_in_use <= 2500
    assert reqs[0].t_finish >= reqs[1].t_finish


def test_growth_that_can_never_fit_fails_only_that_request():
    ref = [None]
    ex = GrowingExecutor(ref, {1: 5000})
    srv = Server(budget_bytes=3000, slots=2, executor=ex, footprint=lambda r: r.n)
    ref[0] = srv
    reqs = make(4, [1000] * 4, np.zeros(4))
    srv.run(reqs, realtime=False)
    assert [r.status for r in reqs] == ["ok", "failed", "ok", "ok"]
    assert "budget" in reqs[1].error
    assert srv.in_use == 0 and srv.max_in_use <= 3000
