"""Pins of the oracle's direct sum (Eq. 1 with the Sec. 5.1 sign)."""
import numpy as np

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W


def test_single_point_mass():
    # one source of mass M at the origin, probes of mass 0
    x = np.array([0.0, 1.0, 0.0, -2.0])
    y = np.array([0.0, 0.0, 3.0, 1.0])
    z = np.array([0.0, 0.0, 4.0, 2.0])
    m = np.array([2.5, 0.0, 0.0, 0.0])
    phi, ax, ay, az = O.direct(x, y, z, m, targets=[1, 2, 3])
    for k, i in enumerate([1, 2, 3]):
        r = np.sqrt(x[i] ** 2 + y[i] ** 2 + z[i] ** 2)
        assert abs(phi[k] - 2.5 / r) < 1e-15
        # attraction towards the source: a = -M r_hat / r^2
        assert abs(ax[k] + 2.5 * x[i] / r ** 3) < 1e-15
        assert abs(ay[k] + 2.5 * y[i] / r ** 3) < 1e-15
        assert abs(az[k] + 2.5 * z[i] / r ** 3) < 1e-15


def test_self_pair_and_coincident_points_skipped():
    x = np.array([0.0, 0.0, 1.0])
    y = np.zeros(3)
    z = np.zeros(3)
    m = np.array([1.0, 1.0, 1.0])
    phi, ax, _, _ = O.direct(x, y, z, m)
    assert phi[0] == 1.0 and ax[0] == 1.0        # only the particle at x = 1
    assert phi[2] == 2.0 and ax[2] == -2.0


def test_softening():
    x = np.array([0.0, 3.0])
    y = np.array([0.0, 4.0])
    z = np.zeros(2)
    m = np.array([1.0, 0.0])
    phi, ax, ay, _ = O.direct(x, y, z, m, targets=[1], eps2=11.0)
    assert abs(phi[0] - 1 / 6.0) < 1e-16
    assert abs(ax[0] + 3 / 216.0) < 1e-16 and abs(ay[0] + 4 / 216.0) < 1e-16


def test_momentum_conservation():
    # sum_i m_i a_i = 0 by pairwise antisymmetry
    x, y, z, m = W.plummer(3000, 11)
    m = m * (1 + np.random.default_rng(3).random(3000))
    _, ax, ay, az = O.direct(x, y, z, m)
    scale = np.sum(np.abs(m * ax)) + np.sum(np.abs(m * ay)) + np.sum(np.abs(m * az))
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) < 1e-13 * scale


def test_matches_independent_numpy_sum():
    x, y, z, m = W.uniform(700, 5)
    phi, ax, ay, az = O.direct(x, y, z, m)
    pos = np.stack([x, y, z], 1)
    d = pos[None, :, :] - pos[:, None, :]
    r2 = np.sum(d * d, -1)
    np.fill_diagonal(r2, np.inf)
    rinv = 1 / np.sqrt(r2)
    ref_phi = rinv @ m
    ref_a = np.einsum("ij,ijk->ik", m[None, :] * rinv ** 3, d)
    assert O.rel_l2(phi, ref_phi) < 1e-14
    assert O.rel_l2(np.stack([ax, ay, az], 1), ref_a) < 1e-14


def _fibonacci_sphere(n, R):
    k = np.arange(n) + 0.5
    cz = 1 - 2 * k / n
    ph = np.pi * (1 + 5 ** 0.5) * k
    s = np.sqrt(1 - cz * cz)
    return R * s * np.cos(ph), R * s * np.sin(ph), R * cz


def test_uniform_shell_closed_form():
    # Shell theorem: phi = M / max(r, R), and a = 0 inside. A quasi-uniform
    # Fibonacci point set approximates the shell; probes carry zero mass.
    n, R, M = 40000, 1.0, 3.0
    sx, sy, sz = _fibonacci_sphere(n, R)
    probes = np.array([[0.0, 0.0, 0.0], [0.2, -0.1, 0.3], [2.0, 1.0, -1.5],
                       [0.0, 0.0, 5.0]])
    phi, ax, ay, az = O.direct_points(sx, sy, sz, np.full(n, M / n),
                                      probes[:, 0], probes[:, 1], probes[:, 2])
    for k, q in enumerate(probes):
        r = np.linalg.norm(q)
        assert abs(phi[k] - M / max(r, R)) < 1e-4 * M
        if r < R:
            assert np.sqrt(ax[k] ** 2 + ay[k] ** 2 + az[k] ** 2) < 1e-4 * M
        else:
            a_ref = -M * q / r ** 3
            assert np.linalg.norm([ax[k], ay[k], az[k]] - a_ref) < 1e-4 * M


def test_points_and_indices_agree():
    x, y, z, m = W.uniform(500, 9)
    t = np.array([3, 77, 499])
    a = O.direct(x, y, z, m, targets=t)
    b = O.direct_points(x, y, z, m, x[t], y[t], z[t])
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
