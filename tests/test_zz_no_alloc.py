"""hfmm_direct_noalloc (the direct sum on the library's own device scratch
array, for callers that cannot allocate) against hfmm_direct (the same sum
on a caller arena) and the oracle, through the C ABI: two calls in a row,
the second smaller, so that the second runs on what the first left in the
array."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import assert_close, cancellation, host, need_gpu, say, to_dev


def _lib():
    from paper_1010_1482_amd import hfmm
    return hfmm, hfmm.library()


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _call(fn, dev, targets, prec, eps2, arena=None):
    hfmm, L = _lib()
    x, y, z, m = dev
    nt = x.numel() if targets is None else targets[0].numel()
    dt = hfmm.out_dtype(prec)
    out = [torch.full((nt,), float("nan"), dtype=dt, device="cuda") for _ in range(4)]
    tx, ty, tz = (None, None, None) if targets is None else targets
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    head = [_p(x), _p(y), _p(z), _p(m), x.numel(), _p(tx), _p(ty), _p(tz),
            0 if targets is None else nt, prec, float(eps2)]
    if fn == "direct":
        rc = L.hfmm_direct(*head, _p(arena), arena.numel(), *[_p(o) for o in out], s)
    else:
        rc = L.hfmm_direct_noalloc(*head, *[_p(o) for o in out], s)
    torch.cuda.synchronize()
    assert rc == hfmm.OK, (fn, rc)
    return host(out)


@pytest.mark.gpu
@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_noalloc_direct_matches_direct_twice(prec_name):
    need_gpu()
    hfmm, L = _lib()
    prec = hfmm.PRECISIONS[prec_name]
    tol = 1e-13 if prec_name == "fp64" else 1e-5
    # call 1: self-evaluation of 5000 points (mixed-sign masses); call 2:
    # 1200 sources at 700 distinct targets, softened
    x, y, z, _ = W.plummer(5000, 81)
    m = W.masses(5000, 82, "mixed")
    tx, ty, tz, _ = W.uniform(700, 83)
    cases = [(5000, None, 0.0), (1200, (tx, ty, tz), 1e-4)]
    for n, tg, eps2 in cases:
        say(f"noalloc direct {prec_name} n={n} targets={'self' if tg is None else len(tg[0])}")
        src = (x[:n], y[:n], z[:n], m[:n])
        dev = to_dev(*src)
        dtg = None if tg is None else to_dev(*tg)
        sz = C.c_size_t(0)
        assert L.hfmm_direct_bytes(n, 0 if tg is None else len(tg[0]), prec,
                                   C.byref(sz)) == hfmm.OK
        arena = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
        ref_dev = _call("direct", dev, dtg, prec, eps2, arena)
        got = _call("noalloc", dev, dtg, prec, eps2)
        # the same kernels on the same inputs: the same bits
        for a, b in zip(got, ref_dev):
            assert np.array_equal(a, b)
        if tg is None:
            ref = O.direct(*src, eps2=eps2)
            kap = cancellation(*src, *src[:3], ref)
        else:
            ref = O.direct_points(*src, *tg, eps2=eps2)
            kap = cancellation(*src, *tg, ref)
        assert_close(got, ref, tol, "vs oracle direct", kap)


def test_noalloc_rejects_jobs_beyond_the_scratch_array():
    # host-side check, before any device work: 2^21 FP64 points need
    # 64 MiB plus alignment, one more than the array holds
    hfmm, L = _lib()
    out = [None] * 4
    rc = L.hfmm_direct_noalloc(None, None, None, None, (64 << 20) // 32, None, None, None, 0,
                               hfmm.FP64, 0.0, *out, None)
    assert rc == hfmm.E_NOMEM
    rc = L.hfmm_direct_noalloc(None, None, None, None, 10, None, None, None, 0, 7, 0.0, *out,
                               None)
    assert rc == hfmm.E_UNSUPPORTED
