"""Separate targets on the GPU, through the C ABI, against the oracle's
separate-target evaluation: every target binned into the resident source
tree (a leaf, an empty octant of a split cell, or outside the root cube).

Checked: the box of every target exactly; the near and far lists of every
box as sets; the FMM and both treecodes in FP64 and FP32; one tree
evaluated at several target sets and at its sources in turn; targets at the
source positions reproducing the self-evaluation; and the status word
(non-finite targets and masses)."""
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


def _sources(n, seed, kind="unequal"):
    x, y, z, _ = W.plummer(n, seed)
    return x, y, z, W.masses(n, seed + 1, kind)


def _targets(x, y, z, leaf, seed, n_in=900):
    """Targets inside leaves, in empty octants, and outside the root cube
    (partly adjacent to it, partly far)."""
    T = O.Tree(x, y, z, leaf)
    r = T.root()
    lo, side = r[:3], 2 * r[3]
    rng = np.random.default_rng(seed)
    pts = np.concatenate([lo[:, None] + side * rng.random((3, n_in)),
                          lo[:, None] + side * (rng.random((3, 60)) * 1.6 - 0.3),
                          lo[:, None] + side * (4.0 + rng.random((3, 12)))], axis=1)
    kinds = T.target_boxes(*pts)[:, 0]
    assert min(np.bincount(kinds, minlength=3)) >= 10, np.bincount(kinds, minlength=3)
    return T, pts[0], pts[1], pts[2]


def _kappa(x, y, z, m, tx, ty, tz, ref):
    return (1.0, 1.0) if np.all(m >= 0) else cancellation(x, y, z, m, tx, ty, tz, ref)


@pytest.mark.parametrize("method,p,leaf", [("fmm", 8, 16), ("treecode", 4, 16),
                                           ("treecode_fmmlist", 3, 16),
                                           ("treecode_fmmlist", 6, 8)])
def test_target_boxes_and_lists_match_oracle(method, p, leaf):
    say(f"target boxes and lists: {method} p={p} leaf={leaf}")
    x, y, z, m = _sources(4000, 111)
    T, tx, ty, tz = _targets(x, y, z, leaf, 112)
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf, max_targets=len(tx))
    t.upward(to_dev(m)[0], p, method, "fp64")
    t.evaluate(theta=0.5, targets=to_dev(tx, ty, tz))
    g = t.target_boxes().cpu().numpy()
    ob = T.target_boxes(tx, ty, tz)
    assert np.array_equal(g[:, :7], ob), "target boxes"
    (foff, fit), (noff, nit) = ((a.cpu().numpy() for a in t.target_list(w)) for w in range(2))
    c = T.cells()
    lists = [T.list(w) for w in range(4)]
    # (one target per box suffices: the lists are the box's)
    seen = set()
    for k in range(len(tx)):
        b = g[k, 7]
        if b in seen:
            continue
        seen.add(b)
        kind, host, leafc = ob[k, 0], ob[k, 5], ob[k, 6]
        pt = (tx[k], ty[k], tz[k])
        U, V, Wl, X = (list(T.box_list(pt, w)) for w in range(4))
        if method == "treecode":
            continue  # Barnes-Hut box lists: checked through the results below
        if method == "fmm":
            far, near = Wl + (V if kind else []), U + (X if kind else [])
        else:
            far, near = Wl + V, U + X
            a = c["parent"][leafc] if kind == 0 else host
            while a >= 0:
                off, it = lists[1]
                far += list(it[off[a]:off[a + 1]])
                off, it = lists[3]
                near += list(it[off[a]:off[a + 1]])
                a = c["parent"][a]
            if p == 3:  # the far kernel reads the V lists of the cells above itself
                far = Wl + (V if kind else [])
        assert sorted(nit[noff[b]:noff[b + 1]]) == sorted(near), (k, kind, "near")
        assert sorted(fit[foff[b]:foff[b + 1]]) == sorted(far), (k, kind, "far")
    say(f"  {len(seen)} boxes checked")


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
@pytest.mark.parametrize("method,p,leaf,theta", [("fmm", 8, 16, 0.5), ("fmm", 12, 32, 0.5),
                                                 ("treecode", 4, 16, 0.5),
                                                 ("treecode", 3, 8, 0.6),
                                                 ("treecode_fmmlist", 3, 16, 0.5),
                                                 ("treecode_fmmlist", 6, 8, 0.5)])
def test_separate_targets_match_oracle(method, p, leaf, theta, kind):
    say(f"separate targets: {method} p={p} leaf={leaf} masses {kind}")
    x, y, z, m = _sources(5000, 113, kind)
    T, tx, ty, tz = _targets(x, y, z, leaf, 114)
    if method == "fmm":
        ref = O.fmm_points(x, y, z, m, p, leaf, tx, ty, tz)
    else:
        ref = O.treecode_points(x, y, z, m, p, theta, leaf, tx, ty, tz,
                                mode=0 if method == "treecode" else 2)
    kap = _kappa(x, y, z, m, tx, ty, tz, ref)
    dev, dtg = to_dev(x, y, z, m), to_dev(tx, ty, tz)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        out = host(H().solve(*dev, p=p, method=method, precision=prec, leaf_max=leaf,
                             theta=theta, targets=dtg))
        assert_close(out, ref, tol, f"{prec} vs oracle", kap)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16"])
def test_separate_targets_precision_forms(prec):
    say(f"separate targets: fmm {prec}")
    x, y, z, m = _sources(6000, 115)
    T, tx, ty, tz = _targets(x, y, z, 16, 116)
    ref = O.fmm_points(x, y, z, m, 10, 16, tx, ty, tz)
    out = host(H().solve(*to_dev(x, y, z, m), p=10, method="fmm", precision=prec, leaf_max=16,
                         targets=to_dev(tx, ty, tz)))
    tol = {"bf16x3": 3 * 2.0 ** -16, "fp16": np.sqrt(2.0 / 3.0) * 2.0 ** -11}[prec]
    assert_close(out, ref, tol, "vs oracle")


def test_one_tree_many_target_sets():
    # the tree and its expansions stay resident: two target sets, then the
    # sources, then the first set again (the same bits)
    say("one tree, several evaluations")
    x, y, z, m = _sources(6000, 117)
    T, tx, ty, tz = _targets(x, y, z, 16, 118)
    ux, uy, uz, _ = W.uniform(700, 119)
    t = H().Tree(*to_dev(x, y, z), leaf_max=16, max_targets=len(tx))
    t.upward(to_dev(m)[0], 8, "fmm", "fp64")
    a1 = host(t.evaluate(targets=to_dev(tx, ty, tz)))
    assert_close(a1, O.fmm_points(x, y, z, m, 8, 16, tx, ty, tz), 1e-12, "set 1")
    b = host(t.evaluate(targets=to_dev(ux, uy, uz)))
    assert_close(b, O.fmm_points(x, y, z, m, 8, 16, ux, uy, uz), 1e-12, "set 2")
    s = host(t.evaluate())
    assert_close(s, O.fmm(x, y, z, m, 8, 16), 1e-12, "sources")
    a2 = host(t.evaluate(targets=to_dev(tx, ty, tz)))
    for u, v in zip(a1, a2):
        assert np.array_equal(u, v)
    assert t.status() == (H().OK, 0)


@pytest.mark.parametrize("method", ["fmm", "treecode", "treecode_fmmlist"])
def test_targets_at_the_sources_equal_self_evaluation(method):
    say(f"targets at the sources: {method}")
    x, y, z, m = _sources(4000, 120, "mixed")
    tg = W.sample_targets(4000, 900, 121)
    dev = to_dev(x, y, z, m)
    kw = dict(p=6, method=method, precision="fp64", leaf_max=16, theta=0.5)
    selfv = [o[tg] for o in host(H().solve(*dev, **kw))]
    sep = host(H().solve(*dev, targets=to_dev(x[tg], y[tg], z[tg]), **kw))
    kap = _kappa(x, y, z, m, x[tg], y[tg], z[tg], selfv)
    assert_close(sep, selfv, 1e-13, "separate vs self", kap)


def test_no_sources_and_no_targets():
    say("empty source or target sets")
    e = to_dev(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    tx, ty, tz, _ = W.uniform(10, 122)
    out = host(H().solve(*e, p=4, method="fmm", precision="fp64", targets=to_dev(tx, ty, tz)))
    assert all(np.all(o == 0.0) for o in out)
    x, y, z, m = _sources(500, 123)
    out = H().solve(*to_dev(x, y, z, m), p=4, method="fmm", precision="fp32",
                    targets=to_dev(np.zeros(0), np.zeros(0), np.zeros(0)))
    assert all(o.numel() == 0 for o in out)


def test_status_word_reports_bad_targets_and_masses():
    say("status word")
    x, y, z, m = _sources(3000, 124)
    tx, ty, tz, _ = W.uniform(50, 125)
    tx[7] = np.nan
    t = H().Tree(*to_dev(x, y, z), leaf_max=16, max_targets=50)
    t.upward(to_dev(m)[0], 4, "fmm", "fp32")
    assert t.status() == (H().OK, 0)
    t.evaluate(targets=to_dev(tx, ty, tz))
    assert t.status() == (H().E_DATA, H().ST_TGT_NONFINITE)
    # a clean evaluation clears the target bit
    tx[7] = 0.5
    t.evaluate(targets=to_dev(tx, ty, tz))
    assert t.status() == (H().OK, 0)
    bad = m.copy()
    bad[3] = np.inf
    t.upward(to_dev(bad)[0], 4, "fmm", "fp32")
    assert t.status() == (H().E_DATA, H().ST_MASS_NONFINITE)
    with pytest.raises(H().HfmmError) as e:
        H().solve(*to_dev(x, y, z, bad), p=4, method="fmm", precision="fp32")
    assert e.value.code == H().E_DATA
