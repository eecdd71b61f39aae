"""The C-ABI library loads and exports every symbol include/hfmm.h declares;
host-only entry points behave as documented (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfmm.h")
LIB = os.path.join(ROOT, "paper_1010_1482_amd", "libhfmm.so")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hfmm_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhfmm.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_lists_every_symbol():
    from paper_1010_1482_amd import hfmm
    assert sorted(hfmm.SYMBOLS) == declared_symbols()


def test_host_only_entry_points(lib):
    from paper_1010_1482_amd import hfmm
    b = hfmm.arena_bytes(1 << 20, 0, 64, 10, hfmm.FMM, hfmm.FP32)
    assert b > (1 << 20) * 100
    assert hfmm.arena_bytes(1000, 0, 64, 4, hfmm.TREECODE, hfmm.FP64) > 0
    with pytest.raises(hfmm.HfmmError) as e:
        hfmm.arena_bytes(1000, 0, 64, 17, hfmm.FMM, hfmm.FP32)
    assert e.value.code == hfmm.E_UNSUPPORTED
    with pytest.raises(hfmm.HfmmError) as e:
        hfmm.arena_bytes(1000, 0, 0, 4, hfmm.FMM, hfmm.FP32)
    assert e.value.code == hfmm.E_INVAL
    lib.hfmm_strerror.restype = C.c_char_p
    assert lib.hfmm_strerror(-2) == b"arena too small"
    out = C.c_void_p()
    L = hfmm._lib()
    # null arena / negative sizes are rejected before any device work
    assert L.hfmm_build_tree(None, None, None, -1, 64, None, 0, None,
                             C.byref(out)) == hfmm.E_INVAL
    assert L.hfmm_build_tree(None, None, None, 10, 64, C.c_void_p(1), 1 << 20, None,
                             C.byref(out)) == hfmm.E_INVAL  # null coordinates
    assert L.hfmm_get_stats(None, None) == hfmm.E_INVAL
    # null tree handles
    assert L.hfmm_evaluate(None, None, None, None, 0, 4, 0.5, hfmm.FMM, hfmm.FP32, 0.0,
                           None, None, None, None, None) == hfmm.E_INVAL
    flags = C.c_uint32(7)
    assert L.hfmm_status(None, None, C.byref(flags)) == hfmm.E_INVAL and flags.value == 0
    assert L.hfmm_export_targets(None, None, None) == hfmm.E_INVAL
    assert L.hfmm_export_target_lists(None, 0, None, None, None) == hfmm.E_INVAL
    L.hfmm_strerror.restype = C.c_char_p
    assert b"overflow" in L.hfmm_strerror(hfmm.E_OVERFLOW)


def test_new_methods_and_time_loop_host_checks(lib):
    from paper_1010_1482_amd import hfmm
    assert hfmm.arena_bytes(1 << 20, 0, 64, 3, hfmm.TREECODE_FMMLIST, hfmm.FP32) > 0
    with pytest.raises(hfmm.HfmmError) as e:
        hfmm.arena_bytes(1000, 0, 64, 4, 7, hfmm.FP32)
    assert e.value.code == hfmm.E_UNSUPPORTED
    L = hfmm._lib()
    done = C.c_int(-1)
    arena = C.c_void_p(1)  # never dereferenced: every call below fails its checks
    # negative n, negative steps, NaN dt, null arena: rejected before device work
    for n, steps, dt, ar in ((-1, 1, 1e-3, arena), (10, -1, 1e-3, arena),
                             (10, 1, float("nan"), arena), (10, 1, 1e-3, None)):
        rc = L.hfmm_leapfrog(*([None] * 7), n, dt, steps, 64, 4, 0.5, hfmm.FMM, hfmm.FP32,
                             0.0, 0.0625, ar, 1 << 30, *([None] * 4), C.byref(done), None, None)
        assert rc == hfmm.E_INVAL and done.value == 0
    # n > 0 with null state pointers
    rc = L.hfmm_leapfrog(*([None] * 7), 10, 1e-3, 1, 64, 4, 0.5, hfmm.FMM, hfmm.FP32, 0.0,
                         -1.0, arena, 1 << 30, *([None] * 4), C.byref(done), None, None)
    assert rc == hfmm.E_INVAL
    # NaN slack
    rc = L.hfmm_leapfrog(*([None] * 7), 10, 1e-3, 1, 64, 4, 0.5, hfmm.FMM, hfmm.FP32, 0.0,
                         float("nan"), arena, 1 << 30, *([None] * 4), C.byref(done), None, None)
    assert rc == hfmm.E_INVAL
    # refit: null handle or output, negative or non-finite slack
    kept = C.c_int(7)
    assert L.hfmm_refit(None, None, None, None, 0.1, None, C.byref(kept)) == hfmm.E_INVAL
    assert kept.value == 0
    # n = 0: nothing to do, every step counted
    builds = C.c_int(-1)
    rc = L.hfmm_leapfrog(*([None] * 7), 0, 1e-3, 3, 64, 4, 0.5, hfmm.FMM, hfmm.FP32, 0.0,
                         0.0625, arena, 1 << 30, *([None] * 4), C.byref(done), C.byref(builds),
                         None)
    assert rc == hfmm.OK and done.value == 3 and builds.value == 0


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
