"""The FMM with the rotation-based M2L (HFMM_FMM_ROT: rotate to the
translation axis, translate order by order, rotate back) against the
oracle: the local expansions of every cell, the FMM result in FP64 and FP32
over the orders 4..16, and separate targets.  The rotated translation is
exact, so the reference is the oracle's FMM with the literal Eq. 4 (the
oracle's own rotation-based M2L equals it to 1e-13, a pin of its own)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import assert_close, host, inputs, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_1010_1482_amd import hfmm
    hfmm.library()


def H():
    from paper_1010_1482_amd import hfmm
    return hfmm


def _paper_half(X, p):
    idx = [n * n + n + m for n in range(p) for m in range(n + 1)]
    return X[:, idx]


@pytest.mark.parametrize("dist,n,leaf,p", [("uniform", 8000, 32, 6), ("plummer", 6000, 16, 9),
                                           ("uniform", 4000, 32, 16)])
def test_rotation_m2l_local_expansions_match_oracle(dist, n, leaf, p):
    say(f"rotation M2L expansions {dist} n={n} p={p}")
    x, y, z, m = inputs(dist, n, 131, "mixed")
    T = O.Tree(x, y, z, leaf)
    Mo, Lo = T.fmm_expansions(m, p)
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
    t.upward(to_dev(m)[0], p, "fmm_rot", "fp64")
    t.evaluate()
    Lg = t.expansions(1).cpu().numpy()
    Lr = _paper_half(Lo, p)
    scale = np.max(np.abs(Lr), axis=1, keepdims=True) + 1e-300
    err = np.max(np.abs(Lg - Lr) / scale)
    say(f"  max relative L error {err:.2e}")
    assert err <= 1e-11


@pytest.mark.parametrize("p", [4, 8, 10, 12, 16])
def test_rotation_fmm_matches_oracle(p):
    say(f"fmm_rot p={p}")
    x, y, z, m = inputs("plummer", 6000, 132, "unequal")
    tg = W.sample_targets(6000, 512, 133)
    ref = O.fmm(x, y, z, m, p, 16, targets=tg)
    dev = to_dev(x, y, z, m)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        out = [o[tg] for o in host(H().solve(*dev, p=p, method="fmm_rot", precision=prec,
                                             leaf_max=16))]
        assert_close(out, ref, tol, f"{prec} vs oracle fmm")


def test_rotation_equals_dense_operator_fmm():
    say("fmm_rot == fmm (fp64)")
    x, y, z, m = inputs("uniform", 16384, 134, "unequal")
    dev = to_dev(x, y, z, m)
    a = host(H().solve(*dev, p=10, method="fmm", precision="fp64", leaf_max=64))
    b = host(H().solve(*dev, p=10, method="fmm_rot", precision="fp64", leaf_max=64))
    assert_close(b, a, 1e-12, "rotation vs dense operators")


def test_rotation_fmm_separate_targets():
    say("fmm_rot at separate targets")
    x, y, z, m = inputs("plummer", 5000, 135, "unequal")
    tx, ty, tz, _ = W.uniform(700, 136)
    tx, ty, tz = (4.0 * a - 2.0 for a in (tx, ty, tz))
    ref = O.fmm_points(x, y, z, m, 8, 16, tx, ty, tz)
    out = host(H().solve(*to_dev(x, y, z, m), p=8, method="fmm_rot", precision="fp64",
                         leaf_max=16, targets=to_dev(tx, ty, tz)))
    assert_close(out, ref, 1e-12, "vs oracle fmm at points")


def test_rotation_rejects_low_precision_forms():
    x, y, z, m = to_dev(*W.uniform(100, 137))
    with pytest.raises(H().HfmmError) as e:
        H().solve(x, y, z, m, p=6, method="fmm_rot", precision="bf16")
    assert e.value.code == H().E_UNSUPPORTED
