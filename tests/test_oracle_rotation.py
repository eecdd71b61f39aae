"""Pins of the oracle's rotation-based M2L (the O(p^3) translation Sec. 6
lists): rotate the multipole expansion to the translation axis, translate
along it, rotate the local expansion back.

The rotation of a degree-n expansion is fixed by what it must do to the
field (the rotated coefficients give the same potential at the rotated
point) and by the group it represents (identity, inverse, composition,
unitarity).  The whole translation is exact, so it must equal the literal
Eq. 4 M2L to rounding for any direction; and along the z axis Eq. 4 couples
each order m only to itself, which is what makes the rotated form O(p^3)."""
import numpy as np
import pytest

from oracle import oracle as O


def _real_field(p, rng):
    """Random coefficients of a real field: X_n^-m = conj(X_n^m)."""
    X = rng.standard_normal(p * p) + 1j * rng.standard_normal(p * p)
    for n in range(p):
        X[n * n + n] = X[n * n + n].real
        for m in range(1, n + 1):
            X[n * n + n - m] = np.conj(X[n * n + n + m])
    return X


def _rot(axis, angle):
    a = np.asarray(axis, dtype=float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


_DIRS = [(1.7, -2.1, 2.6), (0, 0, 3.0), (0, 0, -2.5), (1e-9, 0, 2.0), (2.0, 0, 0),
         (0, -3.0, 0), (-2.0, -2.0, -1.0), (3.0, 3.0, 3.0)]


@pytest.mark.parametrize("p", [1, 2, 5, 10, 16])
@pytest.mark.parametrize("d", _DIRS)
def test_rotation_m2l_equals_eq4(p, d):
    rng = np.random.default_rng(p)
    M = _real_field(p, rng)
    cs = np.array([0.3, -0.1, 0.2])
    ct = cs + np.array(d)
    a = O.m2l(p, cs, ct, M)
    b = O.m2l_rot(p, cs, ct, M)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_eq4_along_z_couples_each_order_to_itself():
    p = 8
    for k in range(-(p - 1), p):
        M = np.zeros(p * p, dtype=complex)
        for n in range(abs(k), p):
            M[n * n + n + k] = 1.0 + 0.5j * n
        L = O.m2l(p, (0, 0, 0), (0, 0, 2.5), M)
        for j in range(p):
            for m in range(-j, j + 1):
                if m != k:
                    assert abs(L[j * j + j + m]) < 1e-16 * np.max(np.abs(L))


@pytest.mark.parametrize("p", [3, 9, 14])
def test_rotation_group_properties(p):
    rng = np.random.default_rng(10 + p)
    X = _real_field(p, rng)
    Q1, Q2 = _rot((1, 2, -1), 0.7), _rot((-2, 0.5, 1), 2.1)
    # identity; a rotation and its inverse; composition: rotating by Q1 then
    # by Q2 gives u -> f(Q1 Q2 u)
    assert np.allclose(O.rotate(p, np.eye(3), X), X, rtol=0, atol=1e-14 * np.abs(X).max())
    back = O.rotate(p, Q1.T, O.rotate(p, Q1, X))
    assert np.allclose(back, X, rtol=0, atol=1e-13 * np.abs(X).max())
    two = O.rotate(p, Q2, O.rotate(p, Q1, X))
    one = O.rotate(p, Q1 @ Q2, X)
    assert np.allclose(two, one, rtol=0, atol=1e-13 * np.abs(X).max())
    # unitary per degree (the harmonics share the norm 4 pi / (2n + 1))
    Y = O.rotate(p, Q1, X)
    for n in range(p):
        s = slice(n * n, (n + 1) * (n + 1))
        assert abs(np.sum(np.abs(Y[s]) ** 2) - np.sum(np.abs(X[s]) ** 2)) < \
            1e-13 * np.sum(np.abs(X[s]) ** 2)


@pytest.mark.parametrize("p", [4, 11])
def test_rotated_multipole_gives_the_same_field(p):
    # the field of the rotated coefficients at Q^T x equals the original at x:
    # f'(u) = f(Q u) for the multipole's angular parts, radial parts unchanged
    rng = np.random.default_rng(20 + p)
    M = _real_field(p, rng)
    Q = _rot((0.3, -1.0, 0.4), 1.3)
    Mq = O.rotate(p, Q, M)
    for _ in range(5):
        x = rng.standard_normal(3) * 3
        a = O.m2p(p, (0, 0, 0), M, Q @ x)
        b = O.m2p(p, (0, 0, 0), Mq, x)
        assert abs(a[0] - b[0]) < 1e-12 * abs(a[0]) + 1e-14
        # the gradient rotates as a vector
        assert np.allclose(Q.T @ a[1:], b[1:], rtol=1e-11, atol=1e-13)
