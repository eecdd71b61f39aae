"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

The oracle (plain C) is built with gcc and both sanitizers and driven
through every entry point of hfmm_oracle.h on small seeded inputs
(oracle/sanitize_main.c): empty, single, tiny and adaptive trees, every list
kind, separate targets, the rotation and a kept tree.

The library's host code is built with the sanitizers on its host half only
(the device code for gfx950 as usual) and driven through every entry point
on the paths that end before device work, and on the no-device path
(tests/sanitize_host_main.cpp).  That build compiles every kernel again
(minutes), so it runs only with HFMM_SANITIZE_HOST=1."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _clean(out: str) -> bool:
    return "ERROR: AddressSanitizer" not in out and "runtime error" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
           os.path.join(ROOT, "oracle", "sanitize_main.c"),
           os.path.join(ROOT, "oracle", "hfmm_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    out = r.stdout + r.stderr
    assert r.returncode == 0 and _clean(out), out[-4000:]
    assert "sanitized oracle run complete" in out


@pytest.mark.skipif(os.environ.get("HFMM_SANITIZE_HOST") != "1",
                    reason="set HFMM_SANITIZE_HOST=1 (recompiles every kernel)")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    flags = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-std=c++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-I", os.path.join(ROOT, "include")]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1010_1482_amd", "csrc", "*.hip")))
    procs, objs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(["hipcc", *flags, "-c", src, "-o", obj],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        assert p.wait() == 0, p.stderr.read().decode()[-3000:]
    exe = str(tmp_path / "host_san")
    subprocess.run(["hipcc", *flags, "-x", "c++",
                    os.path.join(ROOT, "tests", "sanitize_host_main.cpp"), "-x", "none",
                    *objs, "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    out = r.stdout + r.stderr
    assert r.returncode == 0 and _clean(out), out[-4000:]
    assert "sanitized host run complete" in out
