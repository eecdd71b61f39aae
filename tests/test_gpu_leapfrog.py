"""GPU time stepping (kick-drift-kick leapfrog around the force evaluation)
against the oracle leapfrog with the same field: direct sum (FP64), FMM
(FP64 and FP32), the Barnes-Hut treecode and the treecode over the FMM
lists, with a new tree every step and with the tree kept while the
particles stay near their leaves (the same trees built as the oracle's);
the closed-form circular orbit; and calls whose arena is too small, at the
first evaluation and in the middle of the run, leaving the state of the last
whole step."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import host, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_1010_1482_amd import hfmm
    hfmm.library()


def H():
    from paper_1010_1482_amd import hfmm
    return hfmm


def _state(n, seed):
    x, y, z, m = W.plummer(n, seed)
    rng = np.random.default_rng(seed + 1000)
    vx, vy, vz = (0.3 * rng.standard_normal(n) for _ in range(3))
    return x, y, z, vx, vy, vz, m


def _run_gpu(st, dt, steps, **kw):
    x, y, z, vx, vy, vz, m = to_dev(*st)
    f = H().leapfrog(x, y, z, vx, vy, vz, m, dt, steps, **kw)
    torch.cuda.synchronize()
    return host([x, y, z, vx, vy, vz]) + host(f)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", ["direct-fp64", "fmm-fp64", "fmm-fp32", "tl-fp64",
                                  "bh-fp64", "bh-fp32"])
def test_leapfrog_matches_oracle(case):
    meth, prec = case.split("-")
    n, dt, steps, p, leaf = 3000, 2e-3, 4, 10, 16
    say(f"leapfrog {meth} {prec} n={n} steps={steps}")
    st = _state(n, 71)
    if meth == "bh":  # centres of mass that move with unequal masses
        st = st[:6] + (W.masses(n, 171, "unequal"),)
    method = {"direct": "direct", "fmm": "fmm", "tl": "treecode_fmmlist",
              "bh": "treecode"}[meth]
    if meth == "bh":
        p = 4
    got = _run_gpu(st, dt, steps, p=p, method=method, precision=prec, leaf_max=leaf,
                   theta=0.5)
    if meth == "direct":
        field = None
    elif meth == "fmm":
        field = lambda x, y, z, m: O.fmm(x, y, z, m, p, leaf)
    elif meth == "bh":
        field = lambda x, y, z, m: O.treecode(x, y, z, m, p, 0.5, leaf, mode=0)
    else:
        field = lambda x, y, z, m: O.treecode(x, y, z, m, p, 0.5, leaf, mode=2)
    ref = O.leapfrog(*st, dt, steps, field=field)
    x0, v0 = st[:3], st[3:6]
    # displacements and velocity changes over the run, relative
    ex = _rel(np.stack(got[:3]) - np.stack(x0), np.stack(ref[:3]) - np.stack(x0))
    ev = _rel(np.stack(got[3:6]) - np.stack(v0), np.stack(ref[3:6]) - np.stack(v0))
    ea = _rel(np.stack(got[7:10]), np.stack(ref[7:10]))
    say(f"  vs oracle: dx {ex:.2e} dv {ev:.2e} a {ea:.2e}")
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert ex <= tol and ev <= tol and ea <= tol


def test_leapfrog_circular_binary_quarter_period():
    say("leapfrog circular binary, direct fp64")
    st = (np.array([0.5, -0.5]), np.zeros(2), np.zeros(2), np.zeros(2),
          np.array([0.5, -0.5]), np.zeros(2), np.array([0.5, 0.5]))
    k = 2000
    got = _run_gpu(st, 0.5 * np.pi / k, k, method="direct", precision="fp64")
    # a quarter turn: body 0 at (0, 1/2) moving at (-1/2, 0)
    assert np.allclose([got[0][0], got[1][0], got[3][0], got[4][0]], [0.0, 0.5, -0.5, 0.0],
                       atol=2e-6)
    # momentum stays zero
    assert abs(0.5 * got[3][0] + 0.5 * got[3][1]) < 1e-14


def test_leapfrog_small_arena_keeps_state_then_continues():
    say("leapfrog arena too small: state kept, then continued")
    st = _state(5000, 72)
    dev = to_dev(*st)
    x, y, z, vx, vy, vz, m = dev
    n = x.numel()
    out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4)]
    small = torch.empty(48 * n + (3 << 19), dtype=torch.uint8, device="cuda")
    done = C.c_int(-1)
    L = H()._lib()
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = L.hfmm_leapfrog(p(x), p(y), p(z), p(vx), p(vy), p(vz), p(m), n, 2e-3, 3, 16, 8, 0.5,
                         H().FMM, H().FP32, 0.0, -1.0, p(small), small.numel(),
                         *[p(o) for o in out], C.byref(done), None,
                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == H().E_NOMEM and done.value == 0
    assert L.hfmm_last_required_bytes() > small.numel()
    for a, b in zip(host(dev[:6]), st[:6]):
        assert np.array_equal(a, b)
    # the binding grows the arena and gives the same result as a fresh run
    f1 = host(H().leapfrog(x, y, z, vx, vy, vz, m, 2e-3, 3, p=8, method="fmm",
                           precision="fp32", leaf_max=16))
    got2 = _run_gpu(st, 2e-3, 3, p=8, method="fmm", precision="fp32", leaf_max=16)
    for a, b in zip(host(dev[:6]) + f1, got2):
        assert np.array_equal(a, b)


def _fast_state(n, seed):
    x, y, z, _ = W.plummer(n, seed)
    rng = np.random.default_rng(seed + 1000)
    vx, vy, vz = (rng.standard_normal(n) for _ in range(3))
    return x, y, z, vx, vy, vz, W.masses(n, seed + 1, "unequal")


@pytest.mark.parametrize("case", ["fmm-fp64", "fmm-fp32", "tl-fp64", "bh-fp64", "bh-fp32",
                                  "rot-fp64"])
def test_leapfrog_kept_tree_matches_oracle(case):
    # the tree is kept while every particle stays within 1/2 + 1/16 leaf
    # sides of its leaf's centre: the same steps keep it as in the oracle
    meth, prec = case.split("-")
    n, dt, steps, leaf, slack = 3000, 4e-3, 6, 16, 1.0 / 16.0
    p = 4 if meth == "bh" else 10
    say(f"leapfrog kept tree {meth} {prec} n={n} steps={steps}")
    st = _fast_state(n, 73)
    method = {"fmm": "fmm", "tl": "treecode_fmmlist", "bh": "treecode", "rot": "fmm_rot"}[meth]
    info = {}
    got = _run_gpu(st, dt, steps, p=p, method=method, precision=prec, leaf_max=leaf,
                   theta=0.5, slack=slack, info=info)
    if meth in ("fmm", "rot"):
        ev = lambda T, m: T.fmm(m, p)
    elif meth == "bh":
        ev = lambda T, m: T.treecode(m, p, 0.5, mode=0)
    else:
        ev = lambda T, m: T.treecode(m, p, 0.5, mode=2)
    ref = O.leapfrog_tree(*st, dt, steps, leaf, slack, ev)
    say(f"  builds: gpu {info['builds']} oracle {ref[-1]}")
    assert info["builds"] == ref[-1] and 1 < ref[-1] < steps + 1
    x0, v0 = st[:3], st[3:6]
    ex = _rel(np.stack(got[:3]) - np.stack(x0), np.stack(ref[:3]) - np.stack(x0))
    ev_ = _rel(np.stack(got[3:6]) - np.stack(v0), np.stack(ref[3:6]) - np.stack(v0))
    ea = _rel(np.stack(got[7:10]), np.stack(ref[7:10]))
    say(f"  vs oracle: dx {ex:.2e} dv {ev_:.2e} a {ea:.2e}")
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert ex <= tol and ev_ <= tol and ea <= tol


def test_leapfrog_kept_tree_equals_rebuilt_when_never_kept():
    # a slack that no step passes builds every step: the same bits as slack < 0
    st = _fast_state(2000, 74)
    a_info, b_info = {}, {}
    a = _run_gpu(st, 0.05, 3, p=8, method="fmm", precision="fp32", leaf_max=16, slack=0.0,
                 info=a_info)
    b = _run_gpu(st, 0.05, 3, p=8, method="fmm", precision="fp32", leaf_max=16, slack=-1.0,
                 info=b_info)
    assert a_info["builds"] == b_info["builds"] == 4
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def _collapsing_clusters(groups, per, seed, dt):
    """Groups of `per` particles 0.02 wide whose velocities bring each group
    to a point after two steps: the tree of the second step is far deeper."""
    rng = np.random.default_rng(seed)
    c = rng.random((3, groups)).repeat(per, axis=1)
    pos = c + 0.02 * rng.uniform(-1.0, 1.0, (3, groups * per))
    vel = (c - pos) / (2.0 * dt)
    m = np.full(groups * per, 1.0 / (groups * per))
    return (*pos, *vel, m)


def test_leapfrog_arena_runs_out_in_the_middle_of_the_run():
    say("leapfrog arena too small at step 2: back to step 1, then continued")
    dt, leaf, p, eps2 = 1e-3, 16, 6, 1e-6
    st = _collapsing_clusters(600, 17, 75, dt)
    n = len(st[0])
    kw = dict(p=p, method="fmm", precision="fp32", leaf_max=leaf, eps2=eps2, slack=-1.0)

    def need(pos):  # the most arena a tree of these positions takes
        t = H().Tree(*to_dev(*pos), leaf_max=leaf)
        try:
            t.upward(to_dev(st[6])[0], p, "fmm", "fp32")
            t.evaluate(eps2=eps2)
            torch.cuda.synchronize()
        except H().HfmmError as e:
            assert e.code == H().E_NOMEM
        return t.required_bytes()

    one = _run_gpu(st, dt, 1, **kw)
    two = _run_gpu(st, dt, 2, **kw)
    n0, n1, n2 = need(st[:3]), need(one[:3]), need(two[:3])
    say(f"  arena need by step: {n0} {n1} {n2}")
    assert n2 > 2 * max(n0, n1)
    state = (48 * n + 255) // 256 * 256
    L = H()._lib()
    ptr = lambda t: C.c_void_p(t.data_ptr())

    def run_c(steps, nbytes):  # the C entry point in such an arena, from the initial state
        ar = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dev = to_dev(*st)
        out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4)]
        done, builds = C.c_int(-1), C.c_int(-1)
        rc = L.hfmm_leapfrog(*[ptr(a) for a in dev], n, dt, steps, leaf, p, 0.5, H().FMM,
                             H().FP32, eps2, -1.0, ptr(ar), ar.numel(), *[ptr(o) for o in out],
                             C.byref(done), C.byref(builds),
                             C.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        say(f"  {steps} steps in {nbytes} bytes: rc {rc} done {done.value} "
            f"builds {builds.value}")
        return rc, done.value, builds.value, dev

    # the smallest arena (to 256 KiB) in which one step runs: the library
    # spreads the M2L over fewer partial results when the arena is tight, so
    # the peak of a roomy arena is not the least a step needs
    lo, hi = state, state + max(n0, n1) + (4 << 20)
    assert run_c(1, hi)[0] == H().OK
    while hi - lo > (256 << 10):
        mid = (lo + hi) // 2 // 256 * 256
        if run_c(1, mid)[0] == H().OK:
            hi = mid
        else:
            lo = mid
    nbytes = hi
    # one step fits this arena
    rc, done, builds, dev1 = run_c(1, nbytes)
    assert rc == H().OK and done == 1 and builds == 2
    # two do not: the tree of step 2 (or its expansions) no longer fits, and
    # the state goes back to that of step 1 (the same bits: an arena of the
    # same size gives the same evaluation)
    rc, done, builds, dev = run_c(2, nbytes)
    assert rc == H().E_NOMEM and done == 1 and builds in (2, 3)
    assert L.hfmm_last_required_bytes() > nbytes
    for a, b in zip(host(dev[:6]), host(dev1[:6])):
        assert np.array_equal(a, b)
    # the remaining step from there, in the binding's larger arena, follows
    # the uninterrupted two-step run to the FP32 field's rounding
    x, y, z, vx, vy, vz, m = dev
    f = H().leapfrog(x, y, z, vx, vy, vz, m, dt, 1, **kw)
    got = host(dev[:6]) + host(f)
    x0, v0 = np.stack(st[:3]), np.stack(st[3:6])
    assert _rel(np.stack(got[:3]) - x0, np.stack(two[:3]) - x0) <= 1e-6
    assert _rel(np.stack(got[3:6]) - v0, np.stack(two[3:6]) - v0) <= 1e-5
