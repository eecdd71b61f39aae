"""Pins of the oracle's time stepping (kick-drift-kick leapfrog over the
direct-sum field): a closed-form circular orbit with second-order
convergence in dt, exact time reversibility and momentum conservation."""
import numpy as np

from oracle import oracle as O
from paper_1010_1482_amd import workloads as W


def _binary():
    # two masses 1/2 at separation 1 on a circular orbit about their centre
    # of mass: relative angular velocity sqrt(G (m1 + m2) / r^3) = 1, each
    # body at radius 1/2 moving at speed 1/2
    x = np.array([0.5, -0.5]); y = np.zeros(2); z = np.zeros(2)
    vx = np.zeros(2); vy = np.array([0.5, -0.5]); vz = np.zeros(2)
    return x, y, z, vx, vy, vz, np.array([0.5, 0.5])


def test_circular_binary_returns_after_one_period_second_order():
    errs = []
    for k in (200, 400, 800):
        x, y, z, vx, vy, vz, m = _binary()
        out = O.leapfrog(x, y, z, vx, vy, vz, m, 2 * np.pi / k, k)
        # closed form after one period: the initial state
        errs.append(max(np.max(np.abs(out[0] - x)), np.max(np.abs(out[1] - y)),
                        np.max(np.abs(out[4] - vy))))
    assert errs[0] < 2e-3
    # second order: halving dt divides the error by about 4
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5


def test_circular_binary_quarter_period_closed_form():
    x, y, z, vx, vy, vz, m = _binary()
    k = 2000
    out = O.leapfrog(x, y, z, vx, vy, vz, m, 0.5 * np.pi / k, k)
    # after a quarter turn body 0 sits at (0, 1/2) moving at (-1/2, 0)
    assert np.allclose([out[0][0], out[1][0], out[3][0], out[4][0]], [0.0, 0.5, -0.5, 0.0],
                       atol=2e-6)


def test_time_reversible():
    x, y, z, m = W.plummer(300, 61)
    rng = np.random.default_rng(3)
    vx, vy, vz = (0.3 * rng.standard_normal(300) for _ in range(3))
    dt, k = 1e-3, 20
    f = O.leapfrog(x, y, z, vx, vy, vz, m, dt, k)
    b = O.leapfrog(f[0], f[1], f[2], -f[3], -f[4], -f[5], m, dt, k)
    scale = np.max(np.abs(x))
    for a, c in zip(b[:3], (x, y, z)):
        assert np.max(np.abs(a - c)) < 1e-11 * scale
    for a, c in zip(b[3:6], (vx, vy, vz)):
        assert np.max(np.abs(-a - c)) < 1e-9


def test_momentum_conserved():
    x, y, z, m = W.plummer(400, 62)
    m = m * (0.5 + np.random.default_rng(4).random(400))
    vx = vy = vz = np.zeros(400)
    out = O.leapfrog(x, y, z, vx, vy, vz, m, 1e-3, 10)
    for v in out[3:6]:
        assert abs(np.sum(m * v)) < 1e-14 * np.sum(m * np.abs(v))


def test_energy_error_bounded_and_second_order():
    # a symplectic second-order integrator: on a softened cluster the energy
    # error stays small over the run and falls by 4 when dt halves
    x, y, z, m = W.plummer(64, 81)
    rng = np.random.default_rng(9)
    v = [0.3 * rng.standard_normal(64) for _ in range(3)]
    eps2 = 0.01

    def field(x, y, z, m):
        return O.direct(x, y, z, m, eps2=eps2)

    def energy(st):
        phi = O.direct(st[0], st[1], st[2], m, eps2=eps2)[0]
        return 0.5 * np.sum(m * (st[3] ** 2 + st[4] ** 2 + st[5] ** 2)) - 0.5 * np.sum(m * phi)
    worst = []
    for dt, k in ((1e-2, 100), (5e-3, 200), (2.5e-3, 400)):
        st = [x, y, z, *v]
        e0 = energy(st)
        w = 0.0
        for _ in range(10):
            st = list(O.leapfrog(*st, m, dt, k // 10, field=field)[:6])
            w = max(w, abs(energy(st) - e0) / abs(e0))
        worst.append(w)
    assert worst[0] < 1e-4
    for a, b in zip(worst, worst[1:]):
        assert 3.5 < a / b < 4.5
