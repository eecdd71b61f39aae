"""Pins of the oracle's FMM and treecode drivers: reduction to the direct sum,
convergence in p and theta, brute force on tiny inputs, exact invariances,
and the upward pass against a single P2M."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W


def _err(out, ref):
    return (O.rel_l2(out[0], ref[0]),
            O.rel_l2(np.stack(out[1:]), np.stack(ref[1:])))


def test_single_leaf_is_direct_sum():
    x, y, z, m = W.uniform(50, 1)
    f = O.fmm(x, y, z, m, p=6, leaf_max=64)
    d = O.direct(x, y, z, m)
    for a, b in zip(f, d):
        assert np.allclose(a, b, rtol=1e-14, atol=0)
    t = O.treecode(x, y, z, m, p=3, theta=0.5, leaf_max=64)
    for a, b in zip(t, d):
        assert np.allclose(a, b, rtol=1e-14, atol=0)


def test_fmm_error_falls_with_p():
    x, y, z, m = W.uniform(4096, 2)
    d = O.direct(x, y, z, m)
    errs = [_err(O.fmm(x, y, z, m, p=p, leaf_max=16), d)[1] for p in (2, 4, 6, 8)]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-4


@pytest.mark.parametrize("leaf", [1, 2, 4])
def test_tiny_deep_adaptive_trees_brute_force(leaf):
    x, y, z, m = W.plummer(200, 17)
    m = m * (0.5 + np.random.default_rng(1).random(200))
    d = O.direct(x, y, z, m)
    f = O.fmm(x, y, z, m, p=14, leaf_max=leaf)
    ephi, eacc = _err(f, d)
    assert ephi < 1e-6 and eacc < 1e-6


def test_plummer_adaptive_fmm_accuracy():
    x, y, z, m = W.plummer(3000, 3)
    d = O.direct(x, y, z, m)
    e6 = _err(O.fmm(x, y, z, m, p=6, leaf_max=16), d)
    e10 = _err(O.fmm(x, y, z, m, p=10, leaf_max=16), d)
    assert e10[1] < e6[1] and e10[1] < 1e-4


def test_power_of_two_scaling_is_bitwise():
    # positions x2 and masses x4: phi scales by exactly 2 and a by exactly 1
    x, y, z, m = W.plummer(2000, 4)
    f = O.fmm(x, y, z, m, p=8, leaf_max=16)
    g = O.fmm(2 * x, 2 * y, 2 * z, 4 * m, p=8, leaf_max=16)
    assert np.array_equal(g[0], 2 * f[0])
    for a, b in zip(f[1:], g[1:]):
        assert np.array_equal(a, b)


def test_input_order_invariance_is_bitwise():
    x, y, z, m = W.uniform(3000, 6)
    perm = np.random.default_rng(0).permutation(3000)
    f = O.fmm(x, y, z, m, p=6, leaf_max=32)
    g = O.fmm(x[perm], y[perm], z[perm], m[perm], p=6, leaf_max=32)
    for a, b in zip(f, g):
        assert np.array_equal(a[perm], b)


def test_mass_superposition():
    x, y, z, m = W.uniform(3000, 8)
    rng = np.random.default_rng(2)
    m1, m2 = rng.random(3000), rng.random(3000)
    f1 = O.fmm(x, y, z, m1, p=6, leaf_max=32)
    f2 = O.fmm(x, y, z, m2, p=6, leaf_max=32)
    f = O.fmm(x, y, z, m1 + m2, p=6, leaf_max=32)
    for a, b, c in zip(f, f1, f2):
        assert np.allclose(a, b + c, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_target_subset_matches_full_evaluation():
    x, y, z, m = W.plummer(4000, 12)
    t = W.sample_targets(4000, 37, 99)
    full = O.fmm(x, y, z, m, p=7, leaf_max=16)
    sub = O.fmm(x, y, z, m, p=7, leaf_max=16, targets=t)
    for a, b in zip(full, sub):
        assert np.array_equal(a[t], b)
    fullt = O.treecode(x, y, z, m, p=3, theta=0.5, leaf_max=16)
    subt = O.treecode(x, y, z, m, p=3, theta=0.5, leaf_max=16, targets=t)
    for a, b in zip(fullt, subt):
        assert np.array_equal(a[t], b)


def test_upward_pass_root_equals_single_p2m():
    x, y, z, m = W.plummer(1500, 14)
    T = O.Tree(x, y, z, 8)
    p = 8
    M, L = T.fmm_expansions(m, p)
    cx, cy, cz, _ = T.centres()
    ref = O.p2m(p, [cx[0], cy[0], cz[0]], x, y, z, m)
    assert np.max(np.abs(M[0] - ref)) < 1e-12 * np.max(np.abs(ref))
    # the root and level-1 cells receive no far field
    c = T.cells()
    assert np.all(L[c["level"] <= 1] == 0)


def test_treecode_converges_in_theta_and_p():
    x, y, z, m = W.plummer(3000, 15)
    d = O.direct(x, y, z, m)
    e = [_err(O.treecode(x, y, z, m, p=3, theta=th, leaf_max=16), d)[1]
         for th in (0.8, 0.5, 0.3)]
    assert e[0] > e[1] > e[2]
    ep = [_err(O.treecode(x, y, z, m, p=p, theta=0.5, leaf_max=16), d)[1]
          for p in (1, 3, 6)]
    assert ep[0] > ep[1] > ep[2]
    assert _err(O.treecode(x, y, z, m, p=3, theta=0.0, leaf_max=16), d)[1] < 1e-14


def test_treecode_per_particle_mode():
    x, y, z, m = W.plummer(2000, 16)
    d = O.direct(x, y, z, m)
    e = _err(O.treecode(x, y, z, m, p=4, theta=0.4, leaf_max=16, mode=1), d)[1]
    assert e < 1e-3


# ---- the treecode of Sec. 4 (mode 2: FMM lists, geometric centres) ----------

def _fmm_list_sets(T, leaf):
    """Far cells (V of the leaf and its ancestors, W of the leaf) and near
    leaves (U of the leaf, X of the leaf and its ancestors) of a target leaf,
    from the oracle's lists (pinned against their brute-force definitions)."""
    c = T.cells()
    lists = [T.list(w) for w in range(4)]

    def items(w, b):
        off, it = lists[w]
        return list(it[off[b]:off[b + 1]])
    far, near = items(O.LIST_W, leaf), items(O.LIST_U, leaf)
    a = leaf
    while a >= 0:
        far += items(O.LIST_V, a)
        near += items(O.LIST_X, a)
        a = c["parent"][a]
    return c, far, near


def test_fmm_list_treecode_single_leaf_is_direct_sum():
    x, y, z, m = W.uniform(50, 1)
    t = O.treecode(x, y, z, m, p=3, theta=0.5, leaf_max=64, mode=2)
    for a, b in zip(t, O.direct(x, y, z, m)):
        assert np.allclose(a, b, rtol=1e-14, atol=0)


@pytest.mark.parametrize("dist,n,leaf", [("uniform", 4000, 16), ("plummer", 3000, 8)])
def test_fmm_list_treecode_converges_to_direct_sum(dist, n, leaf):
    # the far field is a truncated multipole series whose terms fall as
    # (r/R)^n with r/R <= 0.76 for these lists: the error must fall
    # geometrically with p and reach the direct sum (a dropped, doubled or
    # mis-centred cell would leave an error floor)
    x, y, z, m = W.make(dist, n, 31)
    d = O.direct(x, y, z, m)
    e = [_err(O.treecode(x, y, z, m, p=p, theta=0.5, leaf_max=leaf, mode=2), d)
         for p in (2, 4, 8, 14)]
    assert all(b[1] < 0.4 * a[1] for a, b in zip(e, e[1:]))
    assert e[-1][0] < 1e-7 and e[-1][1] < 1e-6
    # theta is not used by this mode
    t1 = O.treecode(x, y, z, m, p=4, theta=0.3, leaf_max=leaf, mode=2)
    t2 = O.treecode(x, y, z, m, p=4, theta=0.9, leaf_max=leaf, mode=2)
    for a, b in zip(t1, t2):
        assert np.array_equal(a, b)


def test_fmm_list_treecode_near_field_is_exact():
    # with every particle outside the near set of one target leaf massless,
    # each far expansion is exactly zero and the result is the direct sum
    x, y, z, m = W.plummer(3000, 32)
    T = O.Tree(x, y, z, 8)
    perm = T.perm()
    c = T.cells()
    leaves = np.nonzero(c["nchild"] == 0)[0]
    rng = np.random.default_rng(5)
    checked = 0
    for leaf in rng.permutation(leaves)[:12]:
        _, far, near = _fmm_list_sets(T, leaf)
        mm = np.zeros_like(m)
        for b in near:
            idx = perm[c["first"][b]:c["first"][b] + c["count"][b]]
            mm[idx] = m[idx]
        tg = perm[c["first"][leaf]:c["first"][leaf] + c["count"][leaf]]
        got = O.treecode(x, y, z, mm, p=2, theta=0.5, leaf_max=8, targets=tg, mode=2)
        ref = O.direct(x, y, z, mm, targets=tg)
        for a, b in zip(got, ref):
            assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max())
        checked += len(far) > 0 and any(c["nchild"][b] == 0 and b != leaf for b in near)
    assert checked > 0


@pytest.mark.parametrize("p", [2, 4, 7])
def test_fmm_list_treecode_potential_within_truncation_bound(p):
    # Greengard-Rokhlin bound of a p-term multipole expansion of charges of
    # total |mass| A within radius r of the centre, at distance R > r:
    # |phi - phi_p| <= A / (R - r) * (r / R)^p.  Per target, the error
    # against the direct sum is at most the sum over its far cells.
    x, y, z, m = W.plummer(2500, 33)
    T = O.Tree(x, y, z, 8)
    perm = T.perm()
    c = T.cells()
    cx, cy, cz, _ = T.centres()
    pos = np.stack([x, y, z], 1)
    leaves = np.nonzero(c["nchild"] == 0)[0]
    rng = np.random.default_rng(6)
    for leaf in rng.permutation(leaves)[:10]:
        _, far, _ = _fmm_list_sets(T, leaf)
        tg = perm[c["first"][leaf]:c["first"][leaf] + c["count"][leaf]]
        got = O.treecode(x, y, z, m, p=p, theta=0.5, leaf_max=8, targets=tg, mode=2)[0]
        ref = O.direct(x, y, z, m, targets=tg)[0]
        bound = np.zeros(len(tg))
        for C in far:
            idx = perm[c["first"][C]:c["first"][C] + c["count"][C]]
            ctr = np.array([cx[C], cy[C], cz[C]])
            r = np.max(np.linalg.norm(pos[idx] - ctr, axis=1))
            R = np.linalg.norm(pos[tg] - ctr, axis=1)
            assert np.all(R > r)
            bound += np.sum(np.abs(m[idx])) / (R - r) * (r / R) ** p
        assert np.all(np.abs(got - ref) <= bound + 1e-13 * np.abs(ref))
