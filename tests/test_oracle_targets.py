"""Pins of the oracle's separate-target evaluation: targets binned into the
source tree (a leaf, an empty octant of a split cell, or outside the root).

A target box without sources is a leaf added to the tree.  Its lists are
therefore fixed by a second, independent construction: append one massless
particle at the target to the sources and build the tree again with the
oracle's colleague-based list builder (itself pinned against brute force).
The particle lands alone in a new leaf, which is exactly the box, and
nothing else in the tree changes.  The treecodes have no local expansions,
so their results at the target must equal those of the appended particle.
The FMM replaces the box's M2L/P2L/L2L by M2P/P2P at the target and must
converge to the direct sum."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W


def _geom(T, ids):
    c = T.cells()
    return sorted((int(c["level"][i]), int(c["ix"][i]), int(c["iy"][i]), int(c["iz"][i]))
                  for i in ids)


def _sources(n=3000, seed=91, kind="unequal"):
    x, y, z, _ = W.plummer(n, seed)
    return x, y, z, W.masses(n, seed + 1, kind)


def _targets_all_kinds(x, y, z, T, seed=92):
    """Targets inside leaves, in empty octants and outside the root cube."""
    rng = np.random.default_rng(seed)
    r = T.root()
    lo, side = r[:3], 2 * r[3]
    inside = lo[:, None] + side * rng.random((3, 600))
    near_out = lo[:, None] + side * (rng.random((3, 40)) * 1.6 - 0.3)  # partly outside
    far_out = lo[:, None] + side * (5.0 + rng.random((3, 8)))
    pts = np.concatenate([inside, near_out, far_out], axis=1)
    return pts[0], pts[1], pts[2]


def test_binning_of_the_three_kinds():
    x, y, z, m = _sources()
    T = O.Tree(x, y, z, 16)
    tx, ty, tz = _targets_all_kinds(x, y, z, T)
    b = T.target_boxes(tx, ty, tz)
    kinds = np.bincount(b[:, 0], minlength=3)
    assert kinds[0] > 100 and kinds[1] > 20 and kinds[2] > 8, kinds
    c = T.cells()
    r = T.root()
    for k in range(len(tx)):
        kind, lev, ix, iy, iz, host, leaf = b[k]
        h = 2 * r[3] / 2 ** lev
        box_lo = r[:3] + h * np.array([ix, iy, iz])
        pt = np.array([tx[k], ty[k], tz[k]])
        if kind == 2:
            assert host == -1 and leaf == -1 and lev == 0
            assert np.any(pt < r[:3]) or np.any(pt > r[:3] + 2 * r[3])
            continue
        # the box holds the point (up to the key's resolution at the faces)
        assert np.all(pt >= box_lo - 1e-9 * r[3]) and np.all(pt <= box_lo + h + 1e-9 * r[3])
        if kind == 0:
            assert host == leaf and c["nchild"][leaf] == 0 and c["level"][leaf] == lev
            assert (c["ix"][leaf], c["iy"][leaf], c["iz"][leaf]) == (ix, iy, iz)
        else:
            # a split cell whose child at the box's octant does not exist
            assert leaf == -1 and c["nchild"][host] > 0 and c["level"][host] == lev - 1
            assert (ix >> 1, iy >> 1, iz >> 1) == (c["ix"][host], c["iy"][host], c["iz"][host])
            kids = range(c["first_child"][host], c["first_child"][host] + c["nchild"][host])
            assert all((c["ix"][d], c["iy"][d], c["iz"][d]) != (ix, iy, iz) for d in kids)


def _in_bbox(x, y, z, pt):
    # the root cube is centred on the sources' bounding box: an appended point
    # leaves the tree's root as it is only inside that box
    return all(a.min() <= v <= a.max() for a, v in zip((x, y, z), pt))


def _appended_leaf(x, y, z, pt, leaf_max):
    X, Y, Z = (np.append(a, v) for a, v in zip((x, y, z), pt))
    A = O.Tree(X, Y, Z, leaf_max)
    s = int(np.nonzero(A.perm() == len(x))[0][0])
    c = A.cells()
    leaf = [i for i in range(A.ncells) if c["nchild"][i] == 0 and
            c["first"][i] <= s < c["first"][i] + c["count"][i]][0]
    return A, leaf


def test_box_lists_equal_the_lists_of_the_appended_leaf():
    x, y, z, m = _sources(2500, 93)
    leaf_max = 16
    T = O.Tree(x, y, z, leaf_max)
    tx, ty, tz = _targets_all_kinds(x, y, z, T, 94)
    b = T.target_boxes(tx, ty, tz)
    c = T.cells()
    checked = [0, 0]
    for k in range(len(tx)):
        kind, leaf = b[k, 0], b[k, 6]
        pt = (tx[k], ty[k], tz[k])
        if kind == 2 or (kind == 0 and c["count"][leaf] >= leaf_max) or not _in_bbox(x, y, z, pt):
            continue  # the appended particle would move the root or split the leaf
        if checked[kind] >= 25:
            continue
        A, al = _appended_leaf(x, y, z, pt, leaf_max)
        assert A.ncells == T.ncells + (1 if kind == 1 else 0)
        for w in range(4):
            off, it = A.list(w)
            want = _geom(A, [i for i in it[off[al]:off[al + 1]]])
            got = _geom(T, T.box_list(pt, w))
            if w == 0 and kind == 1:  # the appended leaf is in its own U list
                want = [g for g in want if g != (b[k, 1], *b[k, 2:5])]
            assert got == want, (k, kind, w)
        checked[kind] += 1
    assert checked[0] >= 10 and checked[1] >= 10, checked


def test_box_lists_cover_every_source_once():
    x, y, z, m = _sources(2000, 95)
    T = O.Tree(x, y, z, 8)
    tx, ty, tz = _targets_all_kinds(x, y, z, T, 96)
    b = T.target_boxes(tx, ty, tz)
    c = T.cells()
    lists = [T.list(w) for w in range(4)]
    for k in range(0, len(tx), 3):
        kind, host, leaf = b[k, 0], b[k, 5], b[k, 6]
        pt = (tx[k], ty[k], tz[k])
        cells = [list(T.box_list(pt, w)) for w in range(4)]
        cover = cells[0] + cells[1] + cells[2] + cells[3]
        a = c["parent"][leaf] if kind == 0 else host
        while a >= 0:  # V and X of the ancestors (carried by the host's L)
            for w in (1, 3):
                off, it = lists[w]
                cover += list(it[off[a]:off[a + 1]])
            a = c["parent"][a]
        hits = np.zeros(len(x), dtype=int)
        for ci in cover:
            hits[c["first"][ci]:c["first"][ci] + c["count"][ci]] += 1
        assert np.all(hits == 1), (k, kind, np.bincount(hits))


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
def test_targets_at_the_sources_equal_self_evaluation(kind):
    x, y, z, m = _sources(3000, 97, kind)
    tg = W.sample_targets(3000, 300, 98)
    tx, ty, tz = x[tg], y[tg], z[tg]
    pairs = [(O.fmm_points(x, y, z, m, 7, 16, tx, ty, tz),
              O.fmm(x, y, z, m, 7, 16, targets=tg))]
    for mode in (0, 2):
        pairs.append((O.treecode_points(x, y, z, m, 4, 0.5, 16, tx, ty, tz, mode=mode),
                      O.treecode(x, y, z, m, 4, 0.5, 16, targets=tg, mode=mode)))
    for got, ref in pairs:
        for a, r in zip(got, ref):
            assert np.allclose(a, r, rtol=1e-13, atol=1e-13 * np.abs(r).max())


@pytest.mark.parametrize("mode", [0, 2])
def test_treecodes_at_targets_equal_the_appended_massless_particle(mode):
    x, y, z, m = _sources(2500, 99)
    T = O.Tree(x, y, z, 16)
    tx, ty, tz = _targets_all_kinds(x, y, z, T, 100)
    b = T.target_boxes(tx, ty, tz)
    c = T.cells()
    pick = [k for k in range(len(tx)) if (b[k, 0] == 1 or
            (b[k, 0] == 0 and c["count"][b[k, 6]] < 16)) and
            _in_bbox(x, y, z, (tx[k], ty[k], tz[k]))][:40]
    assert sum(b[k, 0] == 1 for k in pick) >= 5
    got = O.treecode_points(x, y, z, m, 5, 0.6, 16, tx[pick], ty[pick], tz[pick], mode=mode)
    for j, k in enumerate(pick):
        X, Y, Z = (np.append(a, v) for a, v in zip((x, y, z), (tx[k], ty[k], tz[k])))
        ref = O.treecode(X, Y, Z, np.append(m, 0.0), 5, 0.6, 16, targets=[len(x)], mode=mode)
        for a, r in zip(got, ref):
            assert abs(a[j] - r[0]) <= 1e-13 * max(abs(r[0]), 1e-300) + 1e-15, (k, b[k, 0])


def test_fmm_at_targets_converges_to_the_direct_sum():
    x, y, z, m = _sources(4000, 101)
    T = O.Tree(x, y, z, 16)
    tx, ty, tz = _targets_all_kinds(x, y, z, T, 102)
    kinds = T.target_boxes(tx, ty, tz)[:, 0]
    d = O.direct_points(x, y, z, m, tx, ty, tz)
    for kd in (0, 1, 2):
        sel = kinds == kd
        errs = []
        for p in (3, 6, 10):
            f = O.fmm_points(x, y, z, m, p, 16, tx[sel], ty[sel], tz[sel])
            errs.append(O.rel_l2(np.stack([a for a in f[1:]]),
                                 np.stack([a[sel] for a in d[1:]])))
        assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], (kd, errs)
        # outside the root the W cells of a level-0 box are one level-1 cell
        # away: M2P at a separation ratio up to sqrt(3)/3 (0.58^10 = 4e-3 per
        # term); inside, the FMM's own accuracy at p = 10
        assert errs[2] < (1e-4 if kd < 2 else 5e-4), (kd, errs)


def test_root_leaf_targets_are_the_direct_sum():
    # every source in the root leaf: targets inside it and in the cubes
    # adjacent to it are summed directly; far cubes take the root's M2P
    x, y, z, _ = W.uniform(60, 103)
    m = W.masses(60, 104, "mixed")
    rng = np.random.default_rng(105)
    near = rng.random((3, 50)) * 2.6 - 0.8
    far = 4.0 + rng.random((3, 10))
    f = O.fmm_points(x, y, z, m, 12, 64, *near)
    d = O.direct_points(x, y, z, m, *near)
    for a, r in zip(f, d):
        assert np.allclose(a, r, rtol=1e-13, atol=1e-14 * np.abs(r).max())
    ff = O.fmm_points(x, y, z, m, 12, 64, *far)
    df = O.direct_points(x, y, z, m, *far)
    assert O.rel_l2(np.stack(ff[1:]), np.stack(df[1:])) < 1e-6
    for mode in (0, 2):
        t = O.treecode_points(x, y, z, m, 12, 0.5, 64, *near, mode=mode)
        for a, r in zip(t, d):
            assert np.allclose(a, r, rtol=1e-13, atol=1e-14 * np.abs(r).max())
