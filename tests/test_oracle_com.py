"""Pins of the oracle's centres of mass and of the Barnes-Hut treecode built
on them, with unequal and mixed-sign masses.

Sec. 4 measures the acceptance distance from a cell's centre of mass and the
treecode expands about it.  The centre is fixed by a property, not by its
formula: about the |m|-weighted centre the |m| dipole of the cell vanishes.
An unweighted centroid, signed weights or a wrong particle range each leave a
dipole and fail here; so does a treecode whose expansions are not centred
there (with positive masses a dipole-free expansion makes the p = 2 result
equal to the p = 1 result).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W


def _cells_and_members(T):
    c = T.cells()
    perm = T.perm()
    members = [perm[c["first"][i]:c["first"][i] + c["count"][i]] for i in range(T.ncells)]
    return c, members


def _dipole(M):
    """|M_1^m| for m = -1, 0, 1 of an oracle coefficient array (index n*n+n+m)."""
    return np.abs(M[1:4])


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
def test_com_makes_the_abs_mass_dipole_vanish(kind):
    x, y, z, _ = W.plummer(3000, 61)
    m = W.masses(3000, 62, kind)
    T = O.Tree(x, y, z, 8)
    cx, cy, cz = T.com(m)
    cen = T.centres()
    c, members = _cells_and_members(T)
    checked = 0
    for i in range(T.ncells):
        idx = members[i]
        if len(idx) < 2:
            continue
        a = np.abs(m[idx])
        com = (cx[i], cy[i], cz[i])
        M = O.p2m(2, com, x[idx], y[idx], z[idx], a)
        side = cen[3][i]
        # the dipole about the centre of mass is rounding only, relative to
        # the total |m| times the cell size
        assert _dipole(M).max() <= 1e-13 * M[0].real * side, i
        # about the geometric centre it is of the order of |m| h
        Mg = O.p2m(2, (cen[0][i], cen[1][i], cen[2][i]), x[idx], y[idx], z[idx], a)
        checked += _dipole(Mg).max() > 1e-6 * M[0].real * side
    assert checked > T.ncells // 4


def test_com_weights_are_abs_not_signed_masses():
    # with signed weights the centre would sit where the signed dipole
    # vanishes; the |m| centre leaves a signed dipole in most cells
    x, y, z, _ = W.uniform(2000, 63)
    m = W.masses(2000, 64, "mixed")
    T = O.Tree(x, y, z, 16)
    cx, cy, cz = T.com(m)
    c, members = _cells_and_members(T)
    signed_left = 0
    for i in range(T.ncells):
        idx = members[i]
        M = O.p2m(2, (cx[i], cy[i], cz[i]), x[idx], y[idx], z[idx], m[idx])
        signed_left += _dipole(M).max() > 1e-8 * np.abs(m[idx]).sum() * T.centres()[3][i]
    assert signed_left > T.ncells // 2


def test_com_of_a_massless_cell_is_its_geometric_centre():
    x, y, z, _ = W.uniform(4000, 65)
    m = W.masses(4000, 66, "unequal")
    m[x < 0.5] = 0.0
    T = O.Tree(x, y, z, 16)
    cx, cy, cz = T.com(m)
    cen = T.centres()
    c, members = _cells_and_members(T)
    massless = [i for i in range(T.ncells) if np.all(m[members[i]] == 0.0)]
    assert len(massless) > 20
    for i in massless:
        assert (cx[i], cy[i], cz[i]) == (cen[0][i], cen[1][i], cen[2][i])
    # a cell with mass somewhere is centred on it
    for i in range(T.ncells):
        if i not in massless:
            idx = members[i][m[members[i]] != 0.0]
            lo = np.array([x[idx].min(), y[idx].min(), z[idx].min()])
            hi = np.array([x[idx].max(), y[idx].max(), z[idx].max()])
            com = np.array([cx[i], cy[i], cz[i]])
            assert np.all(com >= lo - 1e-15) and np.all(com <= hi + 1e-15)


@pytest.mark.parametrize("mode", [0, 1])
def test_bh_treecode_is_dipole_free_about_the_com(mode):
    # positive unequal masses: the degree-1 terms of every accepted cell are
    # zero about its centre of mass, so p = 2 adds nothing to p = 1
    x, y, z, _ = W.plummer(3000, 67)
    m = W.masses(3000, 68, "unequal")
    tg = W.sample_targets(3000, 200, 69)
    t1 = O.treecode(x, y, z, m, 1, 0.6, 16, targets=tg, mode=mode)
    t2 = O.treecode(x, y, z, m, 2, 0.6, 16, targets=tg, mode=mode)
    d = O.direct(x, y, z, m, targets=tg)
    e1 = O.rel_l2(np.stack(t1[1:]), np.stack(d[1:]))
    assert e1 > 1e-4  # the far field is really used
    for a, b in zip(t1, t2):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    # the geometric-centre expansions of mode 2 do carry a dipole
    g1 = O.treecode(x, y, z, m, 1, 0.6, 16, targets=tg, mode=2)
    g2 = O.treecode(x, y, z, m, 2, 0.6, 16, targets=tg, mode=2)
    assert O.rel_l2(np.stack(g1[1:]), np.stack(g2[1:])) > 1e-4


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
@pytest.mark.parametrize("mode", [0, 1])
def test_bh_treecode_theta_zero_is_the_direct_sum(kind, mode):
    x, y, z, _ = W.plummer(1500, 70)
    m = W.masses(1500, 71, kind)
    t = O.treecode(x, y, z, m, 3, 0.0, 8, mode=mode)
    d = O.direct(x, y, z, m)
    for a, b in zip(t, d):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max())


@pytest.mark.parametrize("kind", ["unequal", "mixed"])
def test_bh_treecode_converges_with_unequal_masses(kind):
    x, y, z, _ = W.plummer(4000, 72)
    m = W.masses(4000, 73, kind)
    tg = W.sample_targets(4000, 256, 74)
    d = O.direct(x, y, z, m, targets=tg)
    errs = []
    for theta, p in ((0.8, 3), (0.5, 3), (0.5, 6), (0.3, 8)):
        t = O.treecode(x, y, z, m, p, theta, 16, targets=tg, mode=0)
        errs.append(O.rel_l2(np.stack(t[1:]), np.stack(d[1:])))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-5, errs
