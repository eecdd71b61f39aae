"""Serving form on the GPU: every result is the same alone and in the mix
(bitwise: the kernels are deterministic and requests share nothing), and
results match the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _requests(serve, keep):
    trace = W.request_trace(n_req=24, seed=7, rate=2000.0, n_lo=1e3, n_hi=3e4,
                            orders=(6, 8))
    return serve.trace_requests(trace, keep=keep)


def test_alone_equals_mix():
    need_gpu()
    from paper_1010_1482_amd import serve
    keep = set(range(24))
    say("serve: alone")
    alone = _requests(serve, keep)
    s1 = serve.Server(budget_bytes=8 << 30, slots=1, executor=serve.HipExecutor(1),
                      footprint=serve.hip_footprint)
    s1.run(alone, realtime=False)
    say("serve: mix")
    mix = _requests(serve, keep)
    s4 = serve.Server(budget_bytes=8 << 30, slots=4, executor=serve.HipExecutor(4),
                      footprint=serve.hip_footprint)
    s4.run(mix, realtime=True)
    assert all(r.status == "ok" for r in alone + mix), [r.error for r in alone + mix]
    overlap = sum(1 for a in mix for b in mix if a.rid < b.rid and
                  a.t_start < b.t_finish and b.t_start < a.t_finish)
    say(f"  overlapping request pairs in the mix: {overlap}")
    # continuous batching: requests really ran at the same time in the mix
    # (24 arrivals 0.5 ms apart on average, each longer than that)
    assert overlap > 0
    for a, b in zip(sorted(alone, key=lambda r: r.rid), sorted(mix, key=lambda r: r.rid)):
        for u, v in zip(a.output, b.output):
            assert np.array_equal(u, v), a.rid
    # and against the oracle on two of them
    for r in sorted(alone, key=lambda r: r.n)[:2]:
        x, y, z, m = r.make_inputs()
        ref = O.fmm(x, y, z, m, r.p, r.leaf_max)
        e = O.rel_l2(np.stack(r.output[1:]), np.stack(ref[1:]))
        say(f"  request {r.rid} n={r.n} p={r.p}: acc err vs oracle {e:.2e}")
        assert e < 1e-5


def test_budget_limits_concurrency():
    need_gpu()
    from paper_1010_1482_amd import serve
    reqs = _requests(serve, set())
    big = max(serve.hip_footprint(r) for r in reqs)
    srv = serve.Server(budget_bytes=big, slots=4, executor=serve.HipExecutor(4),
                       footprint=serve.hip_footprint)
    srv.run(reqs, realtime=False)
    assert all(r.status == "ok" for r in reqs)
    ev = sorted([(r.t_start, 1, r.footprint) for r in reqs] +
                [(r.t_finish, -1, r.footprint) for r in reqs])
    live = 0
    for _, d, f in ev:
        live += d * f
        assert live <= big
