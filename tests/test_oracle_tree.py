"""Pins of the oracle's octree and interaction lists: Morton keys, the split
rule, closed-form list totals on full grids, the paper's structural constants
(27 P2P cells, 189 M2L cells, theta = 2/3), the adaptive lists against their
brute-force definitions, and exact once-only coverage of every pair."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_constants.json")))


def grid_points(n):
    """One point per cell of an n^3 grid of unit spacing."""
    i = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def test_keys_by_hand():
    # Root cube of the bounding box; the lower corner maps to key 0, the upper
    # corner to all 63 bits set; x bit above y bit above z bit.
    x = np.array([0.0, 1.0, 0.75, 0.0])
    y = np.array([0.0, 1.0, 0.0, 0.0])
    z = np.array([0.0, 1.0, 0.0, 0.5])
    T = O.Tree(x, y, z, 1)
    k = T.keys()
    assert k[0] == 0
    assert k[1] == (1 << 63) - 1
    # x = 0.75 -> q_x = 0b11 << 19: bits 3*20+2 and 3*19+2
    assert k[2] == (1 << 62) | (1 << 59)
    # z = 0.5 -> q_z = 1 << 20: bit 60
    assert k[3] == 1 << 60
    b = T.root()
    assert np.array_equal(b, [0.0, 0.0, 0.0, 0.5])


def test_sort_is_stable_and_cells_partition():
    x, y, z, _ = W.plummer(5000, 7)
    # duplicate some points so equal keys occur
    x[100:110] = x[0]
    y[100:110] = y[0]
    z[100:110] = z[0]
    T = O.Tree(x, y, z, 8)
    k = T.keys()
    perm = T.perm()
    ks = k[perm]
    assert np.all(ks[1:] >= ks[:-1])
    same = ks[1:] == ks[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])       # ties by index
    c = T.cells()
    nc = T.ncells
    assert c["first"][0] == 0 and c["count"][0] == 5000
    for i in range(nc):
        nch = c["nchild"][i]
        if nch == 0:
            assert c["count"][i] <= 8 or c["level"][i] == 21
            continue
        assert c["count"][i] > 8
        kids = range(c["first_child"][i], c["first_child"][i] + nch)
        assert c["first"][kids[0]] == c["first"][i]
        assert sum(c["count"][j] for j in kids) == c["count"][i]
        for a, b_ in zip(kids, list(kids)[1:]):
            assert c["first"][a] + c["count"][a] == c["first"][b_]
        for j in kids:
            assert c["parent"][j] == i and c["level"][j] == c["level"][i] + 1
    # each particle's key prefix matches its leaf's coordinates
    for i in range(nc):
        if c["nchild"][i]:
            continue
        lev = int(c["level"][i])
        for s in range(c["first"][i], c["first"][i] + c["count"][i]):
            pre = int(ks[s]) >> (3 * (21 - lev))
            q = [0, 0, 0]
            for t in range(lev):
                q[0] |= ((pre >> (3 * t + 2)) & 1) << t
                q[1] |= ((pre >> (3 * t + 1)) & 1) << t
                q[2] |= ((pre >> (3 * t)) & 1) << t
            assert q == [c["ix"][i], c["iy"][i], c["iz"][i]]


def test_uniform_tree_list_totals_closed_form():
    # Full 16^3 grid, one point per finest cell, leaf_max = 1: a uniform tree
    # of depth 4.  Per axis, (cell, neighbour) pairs on an n-grid number
    # 3n - 2 and pairs whose parents are neighbours 6n - 8, so
    #   |U| = (3n-2)^3 at the leaves and |V| = (6n-8)^3 - (3n-2)^3 per level.
    x, y, z = grid_points(16)
    T = O.Tree(x, y, z, 1)
    assert T.depth == 4
    c = T.cells()
    offU, _ = T.list(O.LIST_U)
    offV, _ = T.list(O.LIST_V)
    cntU = np.diff(offU)
    cntV = np.diff(offV)
    for lev in range(1, 5):
        n = 2 ** lev
        sel = c["level"] == lev
        assert cntV[sel].sum() == (6 * n - 8) ** 3 - (3 * n - 2) ** 3
    assert cntU[c["level"] == 4].sum() == (3 * 16 - 2) ** 3
    assert T.list(O.LIST_W)[1].size == 0 and T.list(O.LIST_X)[1].size == 0
    # the paper's maxima: 27 P2P cells (Sec. 5.1), 189 M2L cells (Sec. 5.2)
    assert cntU.max() == GOLD["max_p2p_cells"]["value"]
    assert cntV.max() == GOLD["max_m2l_cells"]["value"]


def test_316_offset_classes():
    x, y, z = grid_points(16)
    T = O.Tree(x, y, z, 1)
    c = T.cells()
    off, it = T.list(O.LIST_V)
    offs = set()
    for b in np.nonzero(c["level"] == 4)[0]:
        for s in it[off[b]:off[b + 1]]:
            offs.add((c["ix"][s] - c["ix"][b], c["iy"][s] - c["iy"][b],
                      c["iz"][s] - c["iz"][b]))
    assert len(offs) == 7 ** 3 - 3 ** 3
    assert all(max(map(abs, d)) in (2, 3) for d in offs)


def test_fmm_lists_equal_treecode_mac_two_thirds():
    # Sec. 4: the FMM neighbour list amounts to a MAC theta = 2/3.  Over every
    # target particle and every cell it takes through M2L (the V lists of its
    # leaf and of the leaf's ancestors), max l/d = 2/3 (reached only on the
    # target cell's boundary, so the sample max lies just below).
    x, y, z, _ = W.uniform(6000, 3)
    T = O.Tree(x, y, z, 16)
    c = T.cells()
    cx, cy, cz, side = T.centres()
    off, it = T.list(O.LIST_V)
    perm = T.perm()
    pos = np.stack([x[perm], y[perm], z[perm]], 1)
    worst = 0.0
    for leaf in np.nonzero(c["nchild"] == 0)[0]:
        pts = pos[c["first"][leaf]:c["first"][leaf] + c["count"][leaf]]
        a = leaf
        while a >= 0:
            for s in it[off[a]:off[a + 1]]:
                d = np.linalg.norm(pts - [cx[s], cy[s], cz[s]], axis=1)
                worst = max(worst, float(np.max(side[s] / d)))
            a = c["parent"][a]
    theta = GOLD["fmm_list_equivalent_mac"]["value"]
    assert worst <= theta * (1 + 1e-12)
    assert worst > 0.6


@pytest.mark.parametrize("dist,n,leaf", [("plummer", 3000, 8), ("plummer", 800, 2),
                                         ("uniform", 1500, 5)])
def test_lists_match_bruteforce_definitions(dist, n, leaf):
    x, y, z, _ = W.make(dist, n, 21)
    T = O.Tree(x, y, z, leaf)
    for w in range(4):
        off, it = T.list(w)
        offb, itb = T.list(w, bruteforce=True)
        assert np.array_equal(off, offb), w
        for b in range(T.ncells):
            assert sorted(it[off[b]:off[b + 1]]) == sorted(itb[offb[b]:offb[b + 1]]), (w, b)


def _coverage_fmm(T):
    """count[leaf B, particle j] of how many list entries bring j to B."""
    c = T.cells()
    nc, n = T.ncells, T.n
    lists = [T.list(w) for w in range(4)]
    cov = np.zeros((nc, n), dtype=np.int32)

    def add(b, cell):
        cov[b, c["first"][cell]:c["first"][cell] + c["count"][cell]] += 1

    for b in np.nonzero(c["nchild"] == 0)[0]:
        for w in (O.LIST_U, O.LIST_W):
            off, it = lists[w]
            for s in it[off[b]:off[b + 1]]:
                add(b, s)
        a = b
        while a >= 0:      # far field reaching B through its ancestors
            for w in (O.LIST_V, O.LIST_X):
                off, it = lists[w]
                for s in it[off[a]:off[a + 1]]:
                    add(b, s)
            a = c["parent"][a]
    return cov, c


@pytest.mark.parametrize("dist,n,leaf", [("plummer", 2000, 4), ("uniform", 2000, 16),
                                         ("plummer", 300, 1)])
def test_fmm_lists_cover_every_pair_exactly_once(dist, n, leaf):
    x, y, z, _ = W.make(dist, n, 5)
    T = O.Tree(x, y, z, leaf)
    cov, c = _coverage_fmm(T)
    leaves = np.nonzero(c["nchild"] == 0)[0]
    assert np.all(cov[leaves] == 1)


def test_adaptive_tree_has_w_and_x():
    x, y, z, _ = W.plummer(4000, 9)
    T = O.Tree(x, y, z, 4)
    assert T.list(O.LIST_W)[1].size > 0
    assert T.list(O.LIST_X)[1].size > 0


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8])
def test_bh_lists_cover_every_pair_exactly_once(theta):
    x, y, z, m = W.plummer(2500, 13)
    T = O.Tree(x, y, z, 8)
    c = T.cells()
    comx, comy, comz = T.com(m)
    cx, cy, cz, side = T.centres()
    offa, ita = T.bh_lists(m, theta, 0)
    offp, itp = T.bh_lists(m, theta, 1)
    root = T.root()
    for b in np.nonzero(c["nchild"] == 0)[0]:
        cov = np.zeros(T.n, dtype=np.int32)
        h = side[b]
        lo = root[:3] + h * np.array([c["ix"][b], c["iy"][b], c["iz"][b]])
        for s in ita[offa[b]:offa[b + 1]]:
            cov[c["first"][s]:c["first"][s] + c["count"][s]] += 1
            com = np.array([comx[s], comy[s], comz[s]])
            d = np.linalg.norm(np.maximum(0, np.maximum(lo - com, com - (lo + h))))
            assert side[s] < theta * d
        for s in itp[offp[b]:offp[b + 1]]:
            assert c["nchild"][s] == 0
            cov[c["first"][s]:c["first"][s] + c["count"][s]] += 1
        assert np.all(cov == 1)


def test_theta_zero_accepts_nothing():
    x, y, z, m = W.uniform(1000, 2)
    T = O.Tree(x, y, z, 16)
    assert T.bh_lists(m, 0.0, 0)[1].size == 0
