"""Pins of the oracle's tree kept across time steps: the particles take new
positions while the cells, their membership and order, the root and the
lists stay as built, and the rebuild rule (every particle within 1/2 + slack
leaf sides of its leaf's centre along each axis).

A kept tree must still give the field of the moved particles: with the
Barnes-Hut acceptance switched off (theta = 0) the treecode is the direct
sum, and the FMM converges to the direct sum at the new positions as p
grows, while the old positions are far off.  Any step left reading the
positions of the build (P2M, P2P, L2P, the W and X lists, the centres of
mass) fails one of these.  The rule is checked on a hand-built tree."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W


def _moved(x, y, z, T, frac, seed):
    """Positions displaced by up to frac of the smallest leaf side."""
    hmin = T.centres()[3].min()
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, (3, len(x))) * frac * hmin
    return x + d[0], y + d[1], z + d[2]


def _maxrel(a, ref):
    return max(float(np.max(np.abs(u - v)) / np.max(np.abs(v))) for u, v in zip(a, ref))


def test_stays_rule_on_a_hand_built_tree():
    # two particles at opposite corners of the unit cube, one per leaf: the
    # root is the unit cube, the leaves are its level-1 octants (side 1/2,
    # centres 1/4 and 3/4)
    x = np.array([0.0, 1.0])
    T = O.Tree(x, x.copy(), x.copy(), 1)
    assert np.allclose(T.root(), [0.0, 0.0, 0.0, 0.5])
    slack = 0.125
    lim = (0.5 + slack) * 0.5  # from the centre 1/4 of particle 0's leaf
    for dx, ok in ((0.25 + lim - 1e-9, True), (0.25 + lim + 1e-9, False),
                   (0.25 - lim + 1e-9, True), (0.25 - lim - 1e-9, False)):
        assert T.stays(np.array([dx, 1.0]), x.copy(), x.copy(), slack) is ok, dx
    # each axis counts, either particle counts, and non-finite never stays
    assert not T.stays(x.copy(), np.array([0.0, 0.75 - lim - 1e-9]), x.copy(), slack)
    assert T.stays(x.copy(), np.array([0.0, 0.75 - lim + 1e-9]), x.copy(), slack)
    assert not T.stays(x.copy(), x.copy(), np.array([np.nan, 1.0]), slack)
    # a slack of a whole leaf side keeps a particle a leaf away
    assert T.stays(np.array([0.7, 1.0]), x.copy(), x.copy(), 1.0)


def test_kept_tree_at_its_own_positions_is_the_fresh_tree():
    x, y, z, _ = W.plummer(1500, 141)
    m = W.masses(1500, 142, "mixed")
    T = O.Tree(x, y, z, 16)
    T.move(x, y, z)
    for a, b in zip(T.fmm(m, 8), O.fmm(x, y, z, m, 8, 16)):
        assert np.array_equal(a, b)
    for a, b in zip(T.treecode(m, 4, 0.5), O.treecode(x, y, z, m, 4, 0.5, 16)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
def test_kept_tree_treecode_at_theta_zero_is_the_direct_sum(kind):
    x, y, z, _ = W.plummer(2500, 143)
    m = W.masses(2500, 144, kind)
    T = O.Tree(x, y, z, 16)
    x1, y1, z1 = _moved(x, y, z, T, 0.5, 145)
    T.move(x1, y1, z1)
    ref = O.direct(x1, y1, z1, m)
    assert _maxrel(T.treecode(m, 4, 0.0), ref) <= 1e-12


def test_kept_tree_fmm_converges_to_the_moved_field():
    x, y, z, _ = W.plummer(2000, 146)
    m = W.masses(2000, 147, "unequal")
    T = O.Tree(x, y, z, 16)
    x1, y1, z1 = _moved(x, y, z, T, 0.06, 148)
    assert T.stays(x1, y1, z1, 1.0 / 16.0)
    T.move(x1, y1, z1)
    ref = O.direct(x1, y1, z1, m)
    old = O.direct(x, y, z, m)
    errs = []
    for p in (4, 8, 12):
        a = T.fmm(m, p)
        errs.append(max(O.rel_l2(u, v) for u, v in zip(a, ref)))
    # geometric convergence to the field at the new positions
    assert all(e1 < 0.2 * e0 for e0, e1 in zip(errs, errs[1:])), errs
    assert errs[-1] <= 1e-5, errs
    # the field at the old positions differs by far more
    assert max(O.rel_l2(u, v) for u, v in zip(old, ref)) > 1e3 * errs[-1]


def test_kept_tree_fmm_list_treecode_converges_to_the_moved_field():
    x, y, z, _ = W.plummer(3000, 149)
    m = W.masses(3000, 150, "unequal")
    T = O.Tree(x, y, z, 8)
    x1, y1, z1 = _moved(x, y, z, T, 0.06, 151)
    T.move(x1, y1, z1)
    ref = O.direct(x1, y1, z1, m)
    e = [max(O.rel_l2(u, v) for u, v in zip(T.treecode(m, p, 0.5, mode=2), ref))
         for p in (3, 8, 14)]
    assert e[1] < 0.1 * e[0] and e[2] < 0.1 * e[1] and e[2] <= 1e-6, e


def test_kept_tree_centres_of_mass_follow_the_particles():
    # about the kept tree's centre of mass the |m| dipole of each cell's
    # moved particles vanishes
    x, y, z, _ = W.plummer(2000, 152)
    m = W.masses(2000, 153, "mixed")
    T = O.Tree(x, y, z, 8)
    x1, y1, z1 = _moved(x, y, z, T, 0.5, 154)
    T.move(x1, y1, z1)
    com = T.com(m)
    c, perm, side = T.cells(), T.perm(), T.centres()[3]
    for i in range(T.ncells):
        idx = perm[c["first"][i]:c["first"][i] + c["count"][i]]
        a = np.abs(m[idx])
        M = O.p2m(2, (com[0][i], com[1][i], com[2][i]), x1[idx], y1[idx], z1[idx], a)
        assert np.abs(M[1:4]).max() <= 1e-13 * M[0].real * side[i], i


def _state(n, seed):
    x, y, z, _ = W.plummer(n, seed)
    rng = np.random.default_rng(seed + 1)
    v = 0.3 * rng.standard_normal((3, n))
    return (x, y, z, v[0], v[1], v[2], W.masses(n, seed + 2, "unequal"))


def test_leapfrog_tree_building_every_step_is_the_plain_leapfrog():
    st = _state(1000, 155)
    ev = lambda T, m: T.fmm(m, 8)
    a = O.leapfrog_tree(*st, 2e-3, 3, 16, -1.0, ev)
    b = O.leapfrog(*st, 2e-3, 3, field=lambda x, y, z, m: O.fmm(x, y, z, m, 8, 16))
    assert a[-1] == 4
    for u, v in zip(a[:-1], b):
        assert np.array_equal(u, v)


def test_leapfrog_tree_kept_tracks_the_direct_leapfrog():
    # (this run keeps its first tree throughout)
    st = _state(1000, 156)
    dt, steps = 2e-3, 4
    kept = O.leapfrog_tree(*st, dt, steps, 16, 1.0 / 16.0, lambda T, m: T.fmm(m, 10))
    assert kept[-1] == 1
    ref = O.leapfrog(*st, dt, steps)
    x0 = np.stack(st[:3])
    dx = np.stack(kept[:3]) - x0
    dref = np.stack(ref[:3]) - x0
    assert np.linalg.norm(dx - dref) <= 1e-6 * np.linalg.norm(dref)
    assert O.rel_l2(np.stack(kept[7:10]), np.stack(ref[7:10])) <= 3e-5


def test_leapfrog_tree_builds_fall_as_the_slack_grows():
    st = _state(1500, 157)
    ev = lambda T, m: T.fmm(m, 4)
    b = [O.leapfrog_tree(*st, 4e-3, 8, 16, s, ev)[-1] for s in (0.0, 1.0 / 16.0, 0.5, 1e9)]
    assert b[0] >= b[1] >= b[2] >= b[3] == 1
    assert b[0] > b[2]
