"""GPU parity against the FP64 oracle: direct sum, tree and lists (exact),
expansions (stage by stage) and the FMM / treecode results.

Every end-to-end check bounds both the normalised L2 error over the targets
and the largest error at any one target.  Masses are equal, unequal
(positive, two decades) or mixed in sign; mixed-sign bars are the
equal-sign bars times the cancellation factor of the signed sums at the
targets (rounding errors scale with the sum of the magnitudes)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W
from tests.gpu_util import (assert_close, cancellation, host, inputs, need_gpu, rel_err,
                            say, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_1010_1482_amd import hfmm
    hfmm.library()


def H():
    from paper_1010_1482_amd import hfmm
    return hfmm


# ---------------------------------------------------------------- direct
@pytest.mark.parametrize("n,prec,tol", [(1000, "fp64", 1e-13), (3001, "fp32", 1e-5),
                                        (1, "fp64", 0.0)])
def test_direct_sum(n, prec, tol):
    say(f"direct n={n} {prec}")
    x, y, z, m = W.plummer(n, 31)
    ref = O.direct(x, y, z, m)
    out = host(H().direct(*to_dev(x, y, z, m), precision=prec))
    torch.cuda.synchronize()
    if n == 1:
        assert all(float(o[0]) == 0.0 for o in out)
        return
    assert_close(out, ref, max(tol, 1e-300), f"direct {prec}")


def test_direct_sum_distinct_targets_and_softening():
    say("direct targets + eps2")
    x, y, z, m = W.uniform(2000, 32)
    tx, ty, tz, _ = W.uniform(333, 33)
    ref = O.direct_points(x, y, z, m, tx, ty, tz, eps2=1e-4)
    out = host(H().direct(*to_dev(x, y, z, m), precision="fp64", eps2=1e-4,
                          targets=to_dev(tx, ty, tz)))
    assert_close(out, ref, 1e-13, "direct targets eps2")


# ---------------------------------------------------------------- tree
def _cells_oracle(T):
    c = T.cells()
    return np.stack([c["level"], c["ix"], c["iy"], c["iz"], c["first"], c["count"],
                     c["parent"], c["first_child"], c["nchild"]], 1)


@pytest.mark.parametrize("dist,n,leaf", [("uniform", 16384, 64), ("plummer", 20000, 16),
                                         ("plummer", 3000, 1), ("uniform", 70, 64)])
def test_tree_matches_oracle_exactly(dist, n, leaf):
    say(f"tree {dist} n={n} leaf={leaf}")
    x, y, z, m = W.make(dist, n, 41)
    T = O.Tree(x, y, z, leaf)
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
    st = t.stats()
    assert st["n_cells"] == T.ncells and st["depth"] == T.depth
    assert np.array_equal(np.array(st["root"]), T.root())
    gc = t.cells().cpu().numpy().astype(np.int64)
    oc = _cells_oracle(T).astype(np.int64)
    gc[:, 7] = np.where(gc[:, 8] == 0, -1, gc[:, 7])
    assert np.array_equal(gc, oc)
    # particles per leaf: the same sets (order inside a leaf is free)
    gp = t.perm().cpu().numpy()
    op = T.perm()
    for i in np.nonzero(oc[:, 8] == 0)[0]:
        a, k = oc[i, 4], oc[i, 5]
        assert np.array_equal(np.sort(gp[a:a + k]), np.sort(op[a:a + k]))


@pytest.mark.parametrize("dist,n,leaf", [("uniform", 16384, 64), ("plummer", 20000, 16),
                                         ("plummer", 2000, 2)])
def test_fmm_lists_match_oracle(dist, n, leaf):
    say(f"lists {dist} n={n} leaf={leaf}")
    x, y, z, m = W.make(dist, n, 42)
    T = O.Tree(x, y, z, leaf)
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
    t.upward(to_dev(m)[0], 4, H().FMM, H().FP64)
    for w in range(4):
        off, it = T.list(w)
        goff, git = (a.cpu().numpy() for a in t.fmm_list(w))
        assert len(git) == len(it), w
        for b in range(T.ncells):
            assert np.array_equal(np.sort(git[goff[b]:goff[b + 1]]),
                                  np.sort(it[off[b]:off[b + 1]])), (w, b)


# ---------------------------------------------------------------- expansions
def _paper_half(X, p):
    """oracle complex [nc, p*p] (all m) -> [nc, p(p+1)/2] (m >= 0)"""
    idx = [n * n + n + m for n in range(p) for m in range(n + 1)]
    return X[:, idx]


@pytest.mark.parametrize("dist,n,leaf,p,kind", [("uniform", 16384, 64, 6, "equal"),
                                                ("plummer", 6000, 16, 8, "equal"),
                                                ("plummer", 6000, 16, 8, "unequal"),
                                                ("uniform", 8000, 32, 7, "mixed")])
def test_fmm_expansions_fp64_match_oracle(dist, n, leaf, p, kind):
    say(f"expansions {dist} n={n} p={p} masses {kind}")
    x, y, z, m = inputs(dist, n, 43, kind)
    T = O.Tree(x, y, z, leaf)
    Mo, Lo = T.fmm_expansions(m, p)
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
    xd, yd, zd, md = to_dev(x, y, z, m)
    t.upward(md, p, H().FMM, H().FP64)
    Mg = t.expansions(0).cpu().numpy()
    Mr = _paper_half(Mo, p)
    assert np.max(np.abs(Mg - Mr)) <= 1e-12 * np.max(np.abs(Mr))
    t.evaluate()
    Lg = t.expansions(1).cpu().numpy()
    Lr = _paper_half(Lo, p)
    scale = np.max(np.abs(Lr), axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(Lg - Lr) / scale) <= 1e-11


# ---------------------------------------------------------------- end to end
def _kappa(x, y, z, m, tg, ref):
    if np.all(m >= 0):
        return (1.0, 1.0)
    return cancellation(x, y, z, m, x[tg], y[tg], z[tg], ref)


@pytest.mark.parametrize("dist,n,leaf,p,kind", [("uniform", 16384, 64, 6, "equal"),
                                                ("plummer", 8000, 16, 8, "equal"),
                                                ("plummer", 500, 2, 5, "equal"),
                                                ("uniform", 40, 64, 6, "equal"),
                                                ("plummer", 8000, 16, 8, "unequal"),
                                                ("plummer", 8000, 16, 8, "mixed"),
                                                ("uniform", 16384, 64, 6, "mixed")])
def test_fmm_fp64_matches_oracle(dist, n, leaf, p, kind):
    say(f"fmm fp64 {dist} n={n} leaf={leaf} p={p} masses {kind}")
    x, y, z, m = inputs(dist, n, 44, kind)
    ref = O.fmm(x, y, z, m, p, leaf)
    out = host(H().solve(*to_dev(x, y, z, m), p=p, method="fmm", precision="fp64",
                         leaf_max=leaf))
    kap = _kappa(x, y, z, m, np.arange(min(n, 512)), [r[:512] for r in ref])
    assert_close(out, ref, 1e-12, "vs oracle fmm", kap)


@pytest.mark.parametrize("dist,n,leaf,p,kind", [("uniform", 16384, 64, 6, "equal"),
                                                ("uniform", 16384, 64, 10, "equal"),
                                                ("plummer", 8000, 16, 8, "equal"),
                                                ("uniform", 20000, 64, 12, "equal"),
                                                ("plummer", 8000, 16, 8, "unequal"),
                                                ("uniform", 16384, 64, 10, "mixed")])
def test_fmm_fp32_matches_oracle(dist, n, leaf, p, kind):
    say(f"fmm fp32 {dist} n={n} leaf={leaf} p={p} masses {kind}")
    x, y, z, m = inputs(dist, n, 45, kind)
    tg = W.sample_targets(n, 512, 7)
    ref = O.fmm(x, y, z, m, p, leaf, targets=tg)
    out = host(H().solve(*to_dev(x, y, z, m), p=p, method="fmm", precision="fp32",
                         leaf_max=leaf))
    out = [o[tg] for o in out]
    assert_close(out, ref, 1e-5, "vs oracle fmm", _kappa(x, y, z, m, tg, ref))


# the orders where the M2L path changes: FP64 on the matrix cores up to
# p = 11 and on the vector units above; FP32 on the matrix cores up to
# p = 13, with the last output block of p^2 mod 16 in {1, 4, 9} rows on
# 4 x 4 products (p = 3: every row; p = 5, 11: three 4-row groups; p = 9:
# one row); the extremes p = 1 and p = HFMM_MAX_P
_ORDER_CASES = [("fp64", 1), ("fp64", 11), ("fp64", 12), ("fp64", 16),
                ("fp32", 1), ("fp32", 3), ("fp32", 5), ("fp32", 9), ("fp32", 11),
                ("fp32", 13), ("fp32", 14)]


@pytest.fixture(scope="module")
def order_inputs():
    x, y, z, m = W.make("uniform", 3000, 46)
    return x, y, z, m, W.sample_targets(3000, 64, 9)


@pytest.mark.parametrize("prec,p", _ORDER_CASES)
def test_fmm_order_boundaries(order_inputs, prec, p):
    x, y, z, m, tg = order_inputs
    say(f"fmm {prec} uniform n=3000 leaf=32 p={p}")
    ref = O.fmm(x, y, z, m, p, 32, targets=tg)
    out = [o[tg] for o in host(H().solve(*to_dev(x, y, z, m), p=p, method="fmm",
                                         precision=prec, leaf_max=32))]
    assert_close(out, ref, 1e-12 if prec == "fp64" else 1e-5, "vs oracle fmm")


# ---------------------------------------------------------------- treecode
@pytest.mark.parametrize("dist,n,leaf,p,theta,kind", [("plummer", 8000, 16, 3, 0.5, "equal"),
                                                      ("uniform", 6000, 32, 4, 0.4, "equal"),
                                                      ("plummer", 8000, 16, 3, 0.5, "unequal"),
                                                      ("plummer", 6000, 8, 5, 0.6, "unequal"),
                                                      ("uniform", 6000, 32, 3, 0.5, "mixed")])
def test_treecode_matches_oracle(dist, n, leaf, p, theta, kind):
    # Barnes-Hut about the centres of mass (weights |m|): the acceptance
    # distances, hence the lists, and the expansion centres all depend on them
    say(f"treecode {dist} n={n} p={p} theta={theta} masses {kind}")
    x, y, z, m = inputs(dist, n, 48, kind)
    T = O.Tree(x, y, z, leaf)
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
    md = to_dev(m)[0]
    t.upward(md, p, H().TREECODE, H().FP64)
    out = host(t.evaluate(theta=theta))
    # lists: identical except where l == theta d to rounding
    for w in range(2):
        off, it = T.bh_lists(m, theta, w)
        goff, git = (a.cpu().numpy() for a in t.bh_list(w))
        diff = 0
        for b in range(T.ncells):
            diff += len(set(git[goff[b]:goff[b + 1]]) ^ set(it[off[b]:off[b + 1]]))
        assert diff == 0, (w, diff)
    ref = O.treecode(x, y, z, m, p, theta, leaf)
    kap = _kappa(x, y, z, m, np.arange(512), [r[:512] for r in ref])
    assert_close(out, ref, 1e-12, "fp64 vs oracle treecode", kap)
    d = O.direct(x, y, z, m)
    t.upward(md, p, H().TREECODE, H().FP32)
    out32 = host(t.evaluate(theta=theta))
    assert_close(out32, ref, 1e-5, "fp32 vs oracle treecode", kap)
    assert rel_err(out, d)[1] < 5e-3 * kap[1]


@pytest.mark.parametrize("dist,n,leaf,p,kind", [("plummer", 8000, 8, 3, "equal"),
                                                ("uniform", 6000, 32, 6, "equal"),
                                                ("plummer", 5000, 4, 8, "equal"),
                                                ("plummer", 8000, 8, 3, "unequal"),
                                                ("uniform", 6000, 32, 6, "mixed")])
def test_fmmlist_treecode_matches_oracle(dist, n, leaf, p, kind):
    # the treecode of Sec. 4: M2P over V of the leaf and its ancestors and W
    # of the leaf, P2P over U of the leaf and X of the leaf and its ancestors
    say(f"treecode over the FMM lists {dist} n={n} leaf={leaf} p={p} masses {kind}")
    x, y, z, m = inputs(dist, n, 49, kind)
    T = O.Tree(x, y, z, leaf)
    c = T.cells()
    lists = [T.list(w) for w in range(4)]

    def items(w, b):
        off, it = lists[w]
        return list(it[off[b]:off[b + 1]])
    t = H().Tree(*to_dev(x, y, z), leaf_max=leaf)
    md = to_dev(m)[0]
    t.upward(md, p, H().TREECODE_FMMLIST, H().FP64)
    out = host(t.evaluate())
    (goff, git), (hoff, hit) = ((a.cpu().numpy() for a in t.bh_list(w)) for w in range(2))
    for b in range(T.ncells):
        far, near = [], []
        if c["nchild"][b] == 0:
            far, near = items(O.LIST_W, b), items(O.LIST_U, b)
            a = b
            while a >= 0:
                far += items(O.LIST_V, a)
                near += items(O.LIST_X, a)
                a = c["parent"][a]
        assert sorted(git[goff[b]:goff[b + 1]]) == sorted(far), b
        assert sorted(hit[hoff[b]:hoff[b + 1]]) == sorted(near), b
    ref = O.treecode(x, y, z, m, p, 0.5, leaf, mode=2)
    kap = _kappa(x, y, z, m, np.arange(512), [r[:512] for r in ref])
    assert_close(out, ref, 1e-12, "fp64 vs oracle", kap)
    t.upward(md, p, H().TREECODE_FMMLIST, H().FP32)
    assert_close(host(t.evaluate()), ref, 1e-5, "fp32 vs oracle", kap)
    # against the exact sum: the far field's truncation at this p
    d = O.direct(x, y, z, m)
    assert rel_err(out, d)[1] < {3: 5e-3, 6: 5e-4, 8: 1e-4}[p] * kap[1]


def test_empty_and_single():
    say("empty and single")
    x, y, z, m = to_dev(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    out = H().solve(x, y, z, m, p=4, method="fmm", precision="fp32")
    assert all(o.numel() == 0 for o in out)
    x, y, z, m = to_dev([0.5], [0.25], [0.125], [2.0])
    out = host(H().solve(x, y, z, m, p=4, method="fmm", precision="fp64"))
    assert all(o[0] == 0.0 for o in out)


def test_coincident_points():
    say("coincident points")
    x = np.zeros(300) + 0.5
    y = np.zeros(300) + 0.5
    z = np.zeros(300) + 0.5
    x[:3] = [0.0, 1.0, 0.25]
    m = np.full(300, 1.0 / 300)
    ref = O.fmm(x, y, z, m, 6, 8)
    out = host(H().solve(*to_dev(x, y, z, m), p=6, method="fmm", precision="fp64", leaf_max=8))
    for a, b in zip(out, ref):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("method,mode,p", [("treecode", 0, 3), ("treecode", 0, 5),
                                           ("treecode_fmmlist", 2, 3),
                                           ("treecode_fmmlist", 2, 5)])
def test_coincident_points_treecodes(method, mode, p):
    # 297 coincident points make one leaf at the deepest level, far above
    # leaf_max: the far kernels' loop over target chunks of a leaf
    say(f"coincident points {method} p={p}")
    x = np.zeros(300) + 0.5
    y = np.zeros(300) + 0.5
    z = np.zeros(300) + 0.5
    x[:3] = [0.0, 1.0, 0.25]
    m = np.full(300, 1.0 / 300)
    ref = O.treecode(x, y, z, m, p, 0.5, 8, mode=mode)
    out = host(H().solve(*to_dev(x, y, z, m), p=p, method=method, precision="fp64",
                         leaf_max=8, theta=0.5))
    # tolerances on the scale of phi and of the whole acceleration (a_z is
    # zero exactly: every point has z = 1/2)
    assert np.allclose(out[0], ref[0], rtol=1e-12, atol=1e-12 * np.abs(ref[0]).max())
    amax = max(np.abs(a).max() for a in ref[1:])
    for a, b in zip(out[1:], ref[1:]):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * amax)
    out32 = host(H().solve(*to_dev(x, y, z, m), p=p, method=method, precision="fp32",
                           leaf_max=8, theta=0.5))
    ephi, eacc = rel_err(out32, ref)
    assert ephi < 1e-5 and eacc < 1e-5


@pytest.mark.parametrize("method", ["treecode", "treecode_fmmlist"])
def test_empty_and_single_treecodes(method):
    say(f"empty and single {method}")
    x, y, z, m = to_dev(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0))
    out = H().solve(x, y, z, m, p=3, method=method, precision="fp32")
    assert all(o.numel() == 0 for o in out)
    x, y, z, m = to_dev([0.5], [0.25], [0.125], [2.0])
    out = host(H().solve(x, y, z, m, p=3, method=method, precision="fp64"))
    assert all(o[0] == 0.0 for o in out)


# ---------------------------------------------------------------- softening
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("method,mode", [("fmm", None), ("treecode", 0),
                                         ("treecode_fmmlist", 2)])
def test_softened_tree_evaluation(method, mode, prec, tol):
    # eps2 enters the near field (P2P) only, in the oracle as on the device
    say(f"softened {method} {prec}")
    x, y, z, m = inputs("plummer", 6000, 52, "unequal")
    eps2, p, leaf = 1e-3, 6, 16
    tg = W.sample_targets(6000, 512, 53)
    if mode is None:
        ref = O.fmm(x, y, z, m, p, leaf, targets=tg, eps2=eps2)
        hard = O.fmm(x, y, z, m, p, leaf, targets=tg)
    else:
        ref = O.treecode(x, y, z, m, p, 0.5, leaf, targets=tg, mode=mode, eps2=eps2)
        hard = O.treecode(x, y, z, m, p, 0.5, leaf, targets=tg, mode=mode)
    assert rel_err(hard, ref)[1] > 1e-3  # the softening matters at this eps2
    out = host(H().solve(*to_dev(x, y, z, m), p=p, method=method, precision=prec,
                         leaf_max=leaf, theta=0.5, eps2=eps2))
    assert_close([o[tg] for o in out], ref, tol, "vs oracle, softened")


# ---------------------------------------------------------------- precision form
# Bars from the arithmetic.  A product of two operands each rounded to a
# format of unit roundoff u carries a relative error of at most 2u; with
# rounding errors spread evenly over [-u, u] its rms is sqrt(2/3) u, and a
# sum of such products with independent errors and terms of one sign keeps
# that relative rms (mixed signs multiply it by the cancellation factor).
# The hi/lo split leaves the dropped lo*lo term and the two representation
# errors, ~3u^2.  BF16: u = 2^-8, FP16: u = 2^-11 (after the power-of-two
# range scaling).  FP16x3 sits on a floor below that: its lo parts are FP16
# subnormals (step 2^-24 of the largest scaled entry of a level or operator
# row), so each of the K ~ 189 p^2 terms of a coefficient carries an
# absolute error of up to 2^-25 of that scale; independent, they grow like
# sqrt(K) 2^-24 (1e-5 at p = 12), and three times that bounds the largest
# target error: 2^-15.
_U = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}
_TOL = {"bf16": np.sqrt(2.0 / 3.0) * _U["bf16"], "fp16": np.sqrt(2.0 / 3.0) * _U["fp16"],
        "bf16x3": 3 * _U["bf16"] ** 2, "fp16x3": 2.0 ** -15}


@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "fp16", "fp16x3"])
@pytest.mark.parametrize("dist,n,leaf,p,kind", [("uniform", 16384, 64, 8, "equal"),
                                                ("uniform", 20000, 64, 12, "equal"),
                                                ("plummer", 8000, 16, 8, "equal"),
                                                ("plummer", 8000, 16, 10, "unequal"),
                                                ("uniform", 16384, 64, 8, "mixed")])
def test_fmm_low_precision_m2l(prec, dist, n, leaf, p, kind):
    say(f"fmm {prec} {dist} n={n} leaf={leaf} p={p} masses {kind}")
    x, y, z, m = inputs(dist, n, 49, kind)
    tg = W.sample_targets(n, 512, 8)
    ref = O.fmm(x, y, z, m, p, leaf, targets=tg)
    out = host(H().solve(*to_dev(x, y, z, m), p=p, method="fmm", precision=prec,
                         leaf_max=leaf))
    out = [o[tg] for o in out]
    assert_close(out, ref, _TOL[prec], "vs oracle fmm", _kappa(x, y, z, m, tg, ref))


@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "fp16", "fp16x3"])
def test_fmm_low_precision_net_neutral_levels(prec):
    # every cell of every level net-neutral (each particle paired with an
    # opposite mass at a nearby point): the monopoles nearly vanish while the
    # dipoles carry the field; the operand scale comes from all coefficients
    say(f"fmm {prec} dipole pairs")
    x, y, z, _ = W.uniform(6000, 54)
    rng = np.random.default_rng(55)
    d = 1e-3 * rng.standard_normal((3, 6000))
    X, Y, Z = (np.concatenate([a, a + b]) for a, b in zip((x, y, z), d))
    mag = W.masses(6000, 56, "unequal")
    M = np.concatenate([mag, -mag])
    tg = W.sample_targets(12000, 512, 57)
    ref = O.fmm(X, Y, Z, M, 8, 32, targets=tg)
    out = [o[tg] for o in host(H().solve(*to_dev(X, Y, Z, M), p=8, method="fmm",
                                         precision=prec, leaf_max=32))]
    # the terms of the sums are the pairs' dipole fields: bar relative to the
    # sum of their magnitudes (|m d| / r^2 for phi, 2 |m d| / r^3 for a)
    tx, ty, tz = X[tg], Y[tg], Z[tg]
    r = np.sqrt((x[None, :] - tx[:, None]) ** 2 + (y[None, :] - ty[:, None]) ** 2 +
                (z[None, :] - tz[:, None]) ** 2)
    r = np.maximum(r, 1e-2)  # a target's own pair is summed directly, exactly
    md = mag * np.linalg.norm(d, axis=0)
    s_phi, s_acc = (md / r ** 2).sum(1), (2 * md / r ** 3).sum(1)
    kap = (max(1.0, np.linalg.norm(s_phi) / np.linalg.norm(ref[0])),
           max(1.0, np.linalg.norm(s_acc) / np.linalg.norm(np.stack(ref[1:]))))
    assert_close(out, ref, _TOL[prec], "vs oracle fmm", kap)
