"""Pins of the oracle's expansion operators: exact cases, exactness of the
translations, convergence in p, and gradients against finite differences."""
import numpy as np
import pytest

from oracle import oracle as O

RNG = np.random.default_rng(42)


def _cluster(c, n, half, rng):
    pts = np.asarray(c) + (rng.random((n, 3)) - 0.5) * 2 * half
    return pts[:, 0], pts[:, 1], pts[:, 2], rng.random(n) + 0.1


def _exact(pts, m, x):
    d = np.stack(pts, 1) - np.asarray(x)
    r = np.linalg.norm(d, axis=1)
    return np.concatenate([[np.sum(m / r)], (m / r ** 3) @ d])


def test_centred_mass_multipole_is_exact():
    c = np.array([0.3, -0.2, 0.5])
    M = O.p2m(8, c, [c[0]], [c[1]], [c[2]], [2.0])
    assert M[0] == 2.0 and np.all(M[1:] == 0)
    x = np.array([1.7, 0.4, -1.0])
    out = O.m2p(8, c, M, x)
    ref = _exact(([c[0]], [c[1]], [c[2]]), np.array([2.0]), x)
    assert np.allclose(out, ref, rtol=1e-15, atol=0)


def test_p2m_m2p_converges_geometrically():
    c = np.zeros(3)
    x, y, z, m = _cluster(c, 20, 0.25, RNG)
    tgt = np.array([1.3, 0.9, -0.8])
    ref = _exact((x, y, z), m, tgt)
    errs = [np.abs(O.m2p(p, c, O.p2m(p, c, x, y, z, m), tgt)[0] - ref[0]) / ref[0]
            for p in (2, 4, 6, 8, 10, 12)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-9


def test_p2l_l2p_converges():
    c = np.zeros(3)
    x, y, z, m = _cluster([2.0, -1.5, 1.0], 15, 0.3, RNG)
    tgt = np.array([0.2, 0.1, -0.15])
    ref = _exact((x, y, z), m, tgt)
    errs = [np.abs(O.l2p(p, c, O.p2l(p, c, x, y, z, m), tgt)[0] - ref[0]) / ref[0]
            for p in (2, 5, 8, 11, 14)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-9


@pytest.mark.parametrize("p", [4, 10, 13])
def test_m2m_is_exact(p):
    # M2M(P2M about the child centre) == P2M about the parent centre, for all
    # degrees < p: degree j only draws on degrees <= j.
    cc = np.array([0.25, -0.25, 0.25])
    cp = np.zeros(3)
    x, y, z, m = _cluster(cc, 12, 0.25, RNG)
    Mc = O.p2m(p, cc, x, y, z, m)
    ref = O.p2m(p, cp, x, y, z, m)
    got = O.m2m(p, cc, cp, Mc)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [4, 10, 13])
def test_l2l_is_exact(p):
    # A local expansion truncated at degree p-1 is a harmonic polynomial that
    # L2L re-expands exactly about the child centre.
    cp = np.zeros(3)
    cc = np.array([-0.125, 0.125, 0.125])
    x, y, z, m = _cluster([3.0, 2.0, -2.5], 10, 0.5, RNG)
    Lp = O.p2l(p, cp, x, y, z, m)
    Lc = O.l2l(p, cp, cc, Lp)
    for _ in range(4):
        pt = cc + (RNG.random(3) - 0.5) * 0.25
        a = O.l2p(p, cp, Lp, pt)
        b = O.l2p(p, cc, Lc, pt)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(a).max())


@pytest.mark.parametrize("off", [(3.0, 1.0, -2.0), (0.0, 0.0, 2.0), (2.0, 2.0, 2.0)])
def test_m2l_of_centred_mass_equals_p2l(off):
    # Reading of the direction in Eq. 4: (rho, alpha, beta) of c_tgt - c_src.
    # A unit mass at the source centre must give its P2L expansion exactly.
    cs = np.zeros(3)
    ct = np.asarray(off)
    p = 10
    M = O.p2m(p, cs, [0.0], [0.0], [0.0], [1.0])
    L = O.m2l(p, cs, ct, M)
    ref = O.p2l(p, ct, [0.0], [0.0], [0.0], [1.0])
    assert np.max(np.abs(L - ref)) <= 1e-15 * np.max(np.abs(ref)) + 1e-18


def test_m2l_reversed_direction_is_wrong():
    # The opposite direction is a plausible slip; it must fail the same check.
    cs = np.zeros(3)
    ct = np.array([3.0, 1.0, -2.0])
    M = O.p2m(8, cs, [0.0], [0.0], [0.0], [1.0])
    L_bad = O.m2l(8, ct, cs, M)   # vector c_src - c_tgt instead
    ref = O.p2l(8, ct, [0.0], [0.0], [0.0], [1.0])
    assert np.max(np.abs(L_bad - ref)) > 1e-3 * np.max(np.abs(ref))


def test_m2l_l2p_converges_to_exact():
    cs = np.zeros(3)
    ct = np.array([2.0, 0.0, 1.0])
    x, y, z, m = _cluster(cs, 10, 0.5, RNG)
    tgt = ct + np.array([0.2, -0.3, 0.1])
    ref = _exact((x, y, z), m, tgt)
    errs = []
    for p in (3, 6, 9, 12):
        L = O.m2l(p, cs, ct, O.p2m(p, cs, x, y, z, m))
        out = O.l2p(p, ct, L, tgt)
        errs.append(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6


def _fd_grad(f, x, h=1e-5):
    g = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[a] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("pt", [(0.11, -0.07, 0.05), (0.0, 0.0, 0.13),
                                (0.0, 0.0, -0.09), (0.0, 0.0, 0.0)])
def test_l2p_gradient_matches_finite_differences(pt):
    # includes points on the z axis and the expansion centre itself
    c = np.zeros(3)
    x, y, z, m = _cluster([2.0, -1.0, 1.5], 8, 0.3, RNG)
    L = O.p2l(9, c, x, y, z, m)
    pt = np.asarray(pt, float)
    g = _fd_grad(lambda q: O.l2p(9, c, L, q)[0], pt)
    out = O.l2p(9, c, L, pt)
    assert np.max(np.abs(out[1:] - g)) < 1e-8 * np.abs(g).max()


@pytest.mark.parametrize("pt", [(1.2, -0.7, 0.5), (0.0, 0.0, 1.3), (0.0, 0.0, -1.1)])
def test_m2p_gradient_matches_finite_differences(pt):
    c = np.zeros(3)
    x, y, z, m = _cluster(c, 8, 0.2, RNG)
    M = O.p2m(9, c, x, y, z, m)
    pt = np.asarray(pt, float)
    g = _fd_grad(lambda q: O.m2p(9, c, M, q)[0], pt)
    out = O.m2p(9, c, M, pt)
    assert np.max(np.abs(out[1:] - g)) < 1e-8 * np.abs(g).max()


def test_expansion_gradient_converges_to_direct_force():
    c = np.zeros(3)
    x, y, z, m = _cluster(c, 10, 0.25, RNG)
    tgt = np.array([1.5, -1.0, 0.7])
    ref = _exact((x, y, z), m, tgt)
    out = O.m2p(14, c, O.p2m(14, c, x, y, z, m), tgt)
    assert np.linalg.norm(out[1:] - ref[1:]) < 1e-9 * np.linalg.norm(ref[1:])
