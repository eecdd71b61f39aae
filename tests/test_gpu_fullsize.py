"""GPU results at the full sizes of the measured workloads, in the bench's
launch configuration, on sampled targets the FP64 oracle evaluates one by one:

* N = 2^20 uniform, p = 10, leaf <= 64: the FMM in FP32 and in every
  low-precision M2L form against the oracle FMM (the same approximation;
  differences are rounding), at 256 sampled targets;
* N = 2^22 Plummer, leaf <= 32: FMM p = 8, treecode p = 3, theta = 0.5, and
  the treecode over the FMM lists at p = 3, in FP32 and FP64, against the
  oracle FMM / treecode (group lists) / treecode (FMM lists);
* N = 2^22 uniform, p = 12: every M2L form against the oracle's exact direct
  sum, at the accuracy bar the metric is quoted at (1e-4 relative); BF16,
  which misses that bar, at its own rounding bar.

Each check bounds the normalised L2 error and the largest error at any one
target.
"""
import pytest
import torch

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import assert_close, host, need_gpu, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5   # FP32 against the FP64 evaluation of the same approximation
FP64_TOL = 1e-10  # FP64 against FP64 (summation order only)
METRIC_TOL = 1e-4  # relative L2 error bar of the metric (p >= 8, FP32 forms)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_1010_1482_amd import hfmm
    hfmm.library()


def H():
    from paper_1010_1482_amd import hfmm
    return hfmm


def _gpu_solve(x, y, z, m, **kw):
    out = host(H().solve(*to_dev(x, y, z, m), **kw))
    torch.cuda.synchronize()
    return out


@pytest.fixture(scope="module")
def uniform_1m():
    n = 1 << 20
    x, y, z, m = W.uniform(n, 2)
    tg = W.sample_targets(n, 256, 17)
    say(f"oracle fmm: uniform n={n} p=10 leaf=64 at {len(tg)} targets")
    return x, y, z, m, tg, O.fmm(x, y, z, m, 10, 64, targets=tg)


# rounding bars of the precision forms (relative rms of a product of two
# rounded operands, sqrt(2/3) u; BF16x3 ~3u^2; FP16x3 on the floor of its
# subnormal lo parts, 2^-15 (the derivation is beside the small-size tests))
_U = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}
FORM_TOL = {"fp32": FP32_TOL, "bf16": (2.0 / 3.0) ** 0.5 * _U["bf16"],
            "fp16": (2.0 / 3.0) ** 0.5 * _U["fp16"], "bf16x3": 3 * _U["bf16"] ** 2,
            "fp16x3": 2.0 ** -15}


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp16", "fp16x3"])
def test_uniform_1M_p10_forms_against_oracle_fmm(uniform_1m, prec):
    x, y, z, m, tg, ref = uniform_1m
    say(f"full size: uniform n={len(x)} p=10 leaf=64 {prec}")
    out = [o[tg] for o in _gpu_solve(x, y, z, m, p=10, method="fmm", precision=prec,
                                      leaf_max=64)]
    assert_close(out, ref, FORM_TOL[prec], "vs oracle fmm")


@pytest.fixture(scope="module")
def plummer_4m():
    n = 1 << 22
    x, y, z, m = W.plummer(n, 3)
    tg = W.sample_targets(n, 48, 11)
    return x, y, z, m, tg, {}


def _oracle(cache, key, fn):
    if key not in cache:
        cache[key] = fn()
    return cache[key]


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_plummer_4M_fmm_p8_against_oracle(plummer_4m, prec, tol):
    x, y, z, m, tg, cache = plummer_4m
    say(f"full size: plummer n={len(x)} fmm p=8 leaf=32 {prec}")
    ref = _oracle(cache, "fmm", lambda: O.fmm(x, y, z, m, 8, 32, targets=tg))
    out = [o[tg] for o in _gpu_solve(x, y, z, m, p=8, method="fmm", precision=prec,
                                      leaf_max=32)]
    assert_close(out, ref, tol, "vs oracle fmm")


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_plummer_4M_treecode_p3_against_oracle(plummer_4m, prec, tol):
    x, y, z, m, tg, cache = plummer_4m
    say(f"full size: plummer n={len(x)} treecode p=3 theta=0.5 leaf=32 {prec}")
    ref = _oracle(cache, "tc", lambda: O.treecode(x, y, z, m, 3, 0.5, 32, targets=tg, mode=0))
    out = [o[tg] for o in _gpu_solve(x, y, z, m, p=3, method="treecode", theta=0.5,
                                      precision=prec, leaf_max=32)]
    assert_close(out, ref, tol, "vs oracle treecode")


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_plummer_4M_fmmlist_treecode_p3_against_oracle(plummer_4m, prec, tol):
    x, y, z, m, tg, cache = plummer_4m
    say(f"full size: plummer n={len(x)} treecode over the FMM lists p=3 leaf=32 {prec}")
    ref = _oracle(cache, "tl", lambda: O.treecode(x, y, z, m, 3, 0.5, 32, targets=tg, mode=2))
    out = [o[tg] for o in _gpu_solve(x, y, z, m, p=3, method="treecode_fmmlist",
                                      precision=prec, leaf_max=32)]
    assert_close(out, ref, tol, "vs oracle treecode (FMM lists)")


def test_uniform_4M_p12_forms_against_direct():
    n = 1 << 22
    say(f"full size: uniform n={n} p=12 leaf=64, every M2L form vs direct")
    x, y, z, m = W.uniform(n, 2)
    tg = W.sample_targets(n, 64, 23)
    ref = O.direct(x, y, z, m, targets=tg)
    dev = to_dev(x, y, z, m)
    errs = {}
    for prec in ("fp32", "bf16x3", "fp16x3", "fp16", "bf16", "fp64"):
        out = [o.double().cpu().numpy()[tg]
               for o in H().solve(*dev, p=12, method="fmm", precision=prec, leaf_max=64)]
        errs[prec] = rel_err(out, ref)
        bar = METRIC_TOL if prec != "bf16" else FORM_TOL["bf16"]
        assert_close(out, ref, bar, f"{prec} vs direct")
    # BF16x3 keeps FP32's accuracy within a small factor (FP16x3 loses the
    # low parts of the smallest scaled entries to FP16's range; it is held
    # to the metric's bar above)
    assert errs["bf16x3"][1] <= 4 * errs["fp32"][1] + 1e-6
