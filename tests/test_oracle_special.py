"""Pins of the oracle's special functions (Eqs. 5-9 and the identity of
Sec. 5.2) against library routines and classical identities."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, lpmv

from oracle import oracle as O


@pytest.mark.parametrize("x", [-0.97, -0.3, 0.0, 0.41, 0.999])
def test_legendre_matches_scipy(x):
    # scipy's lpmv carries the Condon-Shortley phase, as Eq. 8 does.
    nmax = 16
    P = O.legendre(nmax, x)
    for n in range(nmax + 1):
        for m in range(n + 1):
            ref = lpmv(m, n, x)
            assert abs(P[n, m] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, m)


def test_legendre_double_factorial_reading():
    # Eq. 8 read with (2m-1)!!: at x = 0, P_m^m = (-1)^m (2m-1)!!.
    P = O.legendre(6, 0.0)
    dfact = [1, 1, 3, 15, 105, 945, 10395]
    for m in range(7):
        assert P[m, m] == (-1) ** m * dfact[m]


def test_anm_values():
    # Eq. 5 by hand: A_n^m = 1/sqrt((n-m)!(n+m)!)
    assert O.anm(0, 0) == 1.0
    assert O.anm(1, 0) == 1.0
    assert abs(O.anm(1, 1) - 1 / math.sqrt(2)) < 1e-16
    assert abs(O.anm(2, 1) - 1 / math.sqrt(6)) < 1e-16
    assert abs(O.anm(3, -2) - 1 / math.sqrt(120)) < 1e-16


def test_ynm_sum_rule_is_legendre_of_angle():
    # Classical addition theorem for Legendre polynomials: for unit vectors
    # a, b at angle gamma, sum_m Y_n^{-m}(a) Y_n^m(b) = P_n(cos gamma).
    rng = np.random.default_rng(0)
    for _ in range(5):
        a1, b1, a2, b2 = rng.random(4) * np.array([np.pi, 2 * np.pi] * 2)
        Ya = O.ynm(12, a1, b1)
        Yb = O.ynm(12, a2, b2)
        u = np.array([np.sin(a1) * np.cos(b1), np.sin(a1) * np.sin(b1), np.cos(a1)])
        v = np.array([np.sin(a2) * np.cos(b2), np.sin(a2) * np.sin(b2), np.cos(a2)])
        cg = float(u @ v)
        for n in range(13):
            s = sum(Ya[n * n + n - m] * Yb[n * n + n + m] for m in range(-n, n + 1))
            assert abs(s.imag) < 1e-12
            assert abs(s.real - eval_legendre(n, cg)) < 1e-12, n


def test_scaled_harmonic_identity():
    # Identity of Sec. 5.2: Y_n^m / (rho^{n+1} A_n^m) = (n-m)! P_n^m e^{im beta}
    # / rho^{n+1}, checked with scipy's Legendre function on the right.
    al, be, rho = 1.1, -2.3, 1.7
    Y = O.ynm(10, al, be)
    for n in range(11):
        for m in range(n + 1):
            lhs = Y[n * n + n + m] / (rho ** (n + 1) * O.anm(n, m))
            rhs = (math.factorial(n - m) * lpmv(m, n, math.cos(al)) *
                   np.exp(1j * m * be) / rho ** (n + 1))
            assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs)), (n, m)


def test_multipole_addition_theorem():
    # 1/|x - y| = sum rho^n / r^{n+1} Y_n^{-m}(y) Y_n^m(x)  (the factorisation
    # behind Eq. 2) converges geometrically in rho/r.
    y = np.array([0.1, -0.2, 0.15])
    x = np.array([0.9, 0.7, -1.1])
    rho = np.linalg.norm(y)
    r = np.linalg.norm(x)
    ay, by = math.acos(y[2] / rho), math.atan2(y[1], y[0])
    ax, bx = math.acos(x[2] / r), math.atan2(x[1], x[0])
    Yy = O.ynm(30, ay, by)
    Yx = O.ynm(30, ax, bx)
    s = 0
    for n in range(31):
        for m in range(-n, n + 1):
            s += rho ** n / r ** (n + 1) * Yy[n * n + n - m] * Yx[n * n + n + m]
    assert abs(s - 1 / np.linalg.norm(x - y)) < 1e-15
