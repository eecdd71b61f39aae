"""A resident tree kept across a move of its sources (hfmm_refit) against
the oracle's kept tree: the keep-or-rebuild decision, then the FMM, both
treecodes and separate targets evaluated on the kept tree with the moved
positions, in FP64 and FP32; two moves in a row; and the handle left
unusable when a source moves too far or becomes non-finite."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import assert_close, cancellation, host, need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_1010_1482_amd import hfmm
    hfmm.library()


def H():
    from paper_1010_1482_amd import hfmm
    return hfmm


def _moved(x, y, z, T, frac, seed):
    hmin = T.centres()[3].min()
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, (3, len(x))) * frac * hmin
    return x + d[0], y + d[1], z + d[2]


def _ref(T, method, m, p, theta):
    if method in ("fmm", "fmm_rot"):
        return T.fmm(m, p)
    return T.treecode(m, p, theta, mode=0 if method == "treecode" else 2)


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
@pytest.mark.parametrize("method,p,leaf", [("fmm", 8, 16), ("fmm_rot", 10, 16),
                                           ("treecode", 4, 16), ("treecode_fmmlist", 6, 8)])
def test_kept_tree_matches_oracle(method, p, leaf, kind):
    say(f"refit {method} p={p} masses {kind}")
    x, y, z, _ = W.plummer(5000, 161)
    m = W.masses(5000, 162, kind)
    T = O.Tree(x, y, z, leaf)
    x1, y1, z1 = _moved(x, y, z, T, 0.05, 163)
    assert T.stays(x1, y1, z1, 1.0 / 16.0)
    T.move(x1, y1, z1)
    ref = _ref(T, method, m, p, 0.5)
    kap = (1.0, 1.0) if kind == "unequal" else cancellation(x1, y1, z1, m, x1, y1, z1, ref)
    md = to_dev(m)[0]
    precs = (("fp64", 1e-12),) if method == "fmm_rot" else (("fp64", 1e-12), ("fp32", 1e-5))
    for prec, tol in precs:
        t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
        t.upward(md, p, method, prec)
        t.evaluate()
        assert t.refit(*to_dev(x1, y1, z1), 1.0 / 16.0)
        t.upward(md, p, method, prec)
        out = host(t.evaluate(theta=0.5))
        assert t.status() == (H().OK, 0)
        assert_close(out, ref, tol, f"{prec} kept tree vs oracle", kap)


@pytest.mark.parametrize("method,p", [("fmm", 8), ("treecode", 4), ("treecode_fmmlist", 5)])
def test_two_moves_then_separate_targets(method, p):
    say(f"refit twice, then separate targets: {method}")
    x, y, z, _ = W.plummer(4000, 164)
    m = W.masses(4000, 165, "unequal")
    T = O.Tree(x, y, z, 16)
    x1, y1, z1 = _moved(x, y, z, T, 0.03, 166)
    x2, y2, z2 = _moved(x1, y1, z1, T, 0.03, 167)
    assert T.stays(x2, y2, z2, 1.0 / 16.0)
    T.move(x2, y2, z2)
    r = T.root()
    rng = np.random.default_rng(168)
    pts = r[:3, None] + 2 * r[3] * (rng.random((3, 700)) * 1.4 - 0.2)
    md = to_dev(m)[0]
    t = H().Tree(*to_dev(x, y, z), leaf_max=16, max_targets=700)
    t.upward(md, p, method, "fp64")
    assert t.refit(*to_dev(x1, y1, z1), 1.0 / 16.0)
    assert t.refit(*to_dev(x2, y2, z2), 1.0 / 16.0)
    t.upward(md, p, method, "fp64")
    assert_close(host(t.evaluate(theta=0.5)), _ref(T, method, m, p, 0.5), 1e-12,
                 "sources after two moves")
    if method == "fmm":
        ref = T.fmm_points(m, p, *pts)
    else:
        ref = T.treecode_points(m, p, 0.5, *pts, mode=0 if method == "treecode" else 2)
    out = host(t.evaluate(theta=0.5, targets=to_dev(*pts)))
    assert_close(out, ref, 1e-12, "separate targets on the kept tree")


def test_decision_matches_oracle_and_failed_refit_leaves_no_tree():
    say("refit decisions")
    x, y, z, _ = W.plummer(3000, 169)
    m = W.masses(3000, 170, "unequal")
    T = O.Tree(x, y, z, 16)
    md = to_dev(m)[0]
    for frac, slack in ((0.05, 1.0 / 16.0), (0.3, 1.0 / 16.0), (0.3, 0.5), (2.0, 0.5)):
        x1, y1, z1 = _moved(x, y, z, T, frac, 171)
        want = T.stays(x1, y1, z1, slack)
        t = H().Tree(*to_dev(x, y, z), leaf_max=16)
        t.upward(md, 6, "fmm", "fp32")
        t.evaluate()
        got = t.refit(*to_dev(x1, y1, z1), slack)
        say(f"  move {frac} slack {slack}: kept {got}")
        assert got == want
        if not got:
            with pytest.raises(H().HfmmError) as e:
                t.upward(md, 6, "fmm", "fp32")
            assert e.value.code == H().E_STATE
            with pytest.raises(H().HfmmError) as e:
                t.refit(*to_dev(x1, y1, z1), slack)
            assert e.value.code == H().E_STATE
        else:
            # evaluate before the new upward pass is refused
            with pytest.raises(H().HfmmError) as e:
                t.evaluate()
            assert e.value.code == H().E_STATE
    # a non-finite position never stays; a negative slack is refused
    t = H().Tree(*to_dev(x, y, z), leaf_max=16)
    bad = x.copy()
    bad[5] = np.nan
    assert not t.refit(*to_dev(bad, y, z), 0.5)
    t = H().Tree(*to_dev(x, y, z), leaf_max=16)
    with pytest.raises(H().HfmmError) as e:
        t.refit(*to_dev(x, y, z), -0.1)
    assert e.value.code == H().E_INVAL
    # at its own positions a tree is kept and gives the fresh tree's bits
    t.upward(md, 6, "fmm", "fp32")
    a = host(t.evaluate())
    assert t.refit(*to_dev(x, y, z), 1e-3)
    t.upward(md, 6, "fmm", "fp32")
    for u, v in zip(host(t.evaluate()), a):
        assert np.array_equal(u, v)
    torch.cuda.synchronize()
