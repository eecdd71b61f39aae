"""Python access to the FP64 CPU oracle (``hfmm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow FP64 reference the
HIP library is checked against; only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  Nothing in the
product package imports it.

Coefficient arrays are complex128 of length p*p, index n*n + n + m for
degrees n < p and orders m = -n..n (Eqs. 2-4 of the paper).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hfmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_u64p = C.POINTER(C.c_uint64)


def build() -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LIB)
        L.oracle_anm.restype = C.c_double
        L.oracle_anm.argtypes = [C.c_int, C.c_int]
        L.oracle_tree_build.restype = C.c_void_p
        L.oracle_tree_build.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int]
        L.oracle_tree_move.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.oracle_tree_stays.restype = C.c_int
        L.oracle_tree_stays.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double]
        L.oracle_tree_free.argtypes = [C.c_void_p]
        L.oracle_tree_ncells.restype = C.c_int64
        L.oracle_tree_ncells.argtypes = [C.c_void_p]
        L.oracle_tree_depth.restype = C.c_int
        L.oracle_tree_depth.argtypes = [C.c_void_p]
        L.oracle_list_size.restype = C.c_int64
        L.oracle_list_size.argtypes = [C.c_void_p, C.c_int]
        L.oracle_list_size_bruteforce.restype = C.c_int64
        L.oracle_list_size_bruteforce.argtypes = [C.c_void_p, C.c_int]
        L.oracle_bh_lists.restype = C.c_int64
        L.oracle_num_threads.restype = C.c_int
        L.oracle_box_list.restype = C.c_int64
        L.oracle_box_list.argtypes = [C.c_void_p, _dp, C.c_int, _i32p]
        L.oracle_target_boxes.argtypes = [C.c_void_p, C.c_int64, _dp, _dp, _dp, _i64p]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(C.c_int(n))


def fmm_phase_seconds():
    """(upward, downward, evaluation) wall seconds of the last oracle FMM."""
    out = np.zeros(3)
    lib().oracle_fmm_phase_seconds(_d(out))
    return tuple(float(v) for v in out)


def num_threads() -> int:
    return lib().oracle_num_threads()


# ---- special functions -------------------------------------------------

def legendre(nmax: int, x: float) -> np.ndarray:
    P = np.zeros((nmax + 1) * (nmax + 1))
    lib().oracle_legendre(C.c_int(nmax), C.c_double(x), _d(P))
    return P.reshape(nmax + 1, nmax + 1)


def ynm(nmax: int, alpha: float, beta: float) -> np.ndarray:
    Y = np.zeros((nmax + 1) ** 2, dtype=np.complex128)
    lib().oracle_ynm(C.c_int(nmax), C.c_double(alpha), C.c_double(beta),
                     Y.ctypes.data_as(_dp))
    return Y


def anm(n: int, m: int) -> float:
    return lib().oracle_anm(n, m)


# ---- single operators --------------------------------------------------

def _c3(c):
    return (C.c_double * 3)(*[float(v) for v in c])


def p2m(p, c, x, y, z, m):
    x, y, z, m = map(_f64, (x, y, z, m))
    M = np.zeros(p * p, dtype=np.complex128)
    lib().oracle_p2m(C.c_int(p), _c3(c), C.c_int64(len(x)), _d(x), _d(y),
                     _d(z), _d(m), M.ctypes.data_as(_dp))
    return M


def p2l(p, c, x, y, z, m):
    x, y, z, m = map(_f64, (x, y, z, m))
    L = np.zeros(p * p, dtype=np.complex128)
    lib().oracle_p2l(C.c_int(p), _c3(c), C.c_int64(len(x)), _d(x), _d(y),
                     _d(z), _d(m), L.ctypes.data_as(_dp))
    return L


def _translate(fn, p, a, b, Cin):
    Cin = np.ascontiguousarray(Cin, dtype=np.complex128)
    out = np.zeros(p * p, dtype=np.complex128)
    fn(C.c_int(p), _c3(a), _c3(b), Cin.ctypes.data_as(_dp),
       out.ctypes.data_as(_dp))
    return out


def m2m(p, c_child, c_parent, M):
    return _translate(lib().oracle_m2m, p, c_child, c_parent, M)


def m2l(p, c_src, c_tgt, M):
    return _translate(lib().oracle_m2l, p, c_src, c_tgt, M)


def m2l_rot(p, c_src, c_tgt, M):
    """M2L by rotation to the translation axis, coaxial translation and
    rotation back (Sec. 6)."""
    return _translate(lib().oracle_m2l_rot, p, c_src, c_tgt, M)


def rotate(p, Q, C_in):
    """Coefficients of the field u -> f(Q u) (Q: 3x3 rotation)."""
    Qc = (C.c_double * 9)(*[float(v) for v in np.asarray(Q, dtype=np.float64).ravel()])
    C_in = np.ascontiguousarray(C_in, dtype=np.complex128)
    out = np.zeros(p * p, dtype=np.complex128)
    lib().oracle_rotate(C.c_int(p), Qc, C_in.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def l2l(p, c_parent, c_child, L):
    return _translate(lib().oracle_l2l, p, c_parent, c_child, L)


def _evaluate(fn, p, c, Cin, x):
    Cin = np.ascontiguousarray(Cin, dtype=np.complex128)
    out = np.zeros(4)
    fn(C.c_int(p), _c3(c), Cin.ctypes.data_as(_dp), _c3(x), _d(out))
    return out


def l2p(p, c, L, x):
    """[phi, ax, ay, az] of a local expansion at point x."""
    return _evaluate(lib().oracle_l2p, p, c, L, x)


def m2p(p, c, M, x):
    """[phi, ax, ay, az] of a multipole expansion at point x."""
    return _evaluate(lib().oracle_m2p, p, c, M, x)


# ---- direct sum ----------------------------------------------------------

def direct(x, y, z, m, targets=None, eps2=0.0):
    """phi, ax, ay, az at source indices `targets` (all when None)."""
    x, y, z, m = map(_f64, (x, y, z, m))
    n = len(x)
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = len(targets), targets.ctypes.data_as(_i64p)
    out = [np.zeros(nt) for _ in range(4)]
    lib().oracle_direct(C.c_int64(n), _d(x), _d(y), _d(z), _d(m),
                        C.c_int64(nt), tp, C.c_double(eps2),
                        *[_d(o) for o in out])
    return tuple(out)


def direct_points(x, y, z, m, tx, ty, tz, eps2=0.0):
    x, y, z, m, tx, ty, tz = map(_f64, (x, y, z, m, tx, ty, tz))
    nt = len(tx)
    out = [np.zeros(nt) for _ in range(4)]
    lib().oracle_direct_points(C.c_int64(len(x)), _d(x), _d(y), _d(z), _d(m),
                               C.c_int64(nt), _d(tx), _d(ty), _d(tz),
                               C.c_double(eps2), *[_d(o) for o in out])
    return tuple(out)


# ---- tree ---------------------------------------------------------------

LIST_U, LIST_V, LIST_W, LIST_X = 0, 1, 2, 3


class Tree:
    """Oracle octree over caller-order positions (Morton keys, split rule
    count > leaf_max, level < 21)."""

    def __init__(self, x, y, z, leaf_max):
        self._keep = [_f64(x), _f64(y), _f64(z)]
        self.n = len(self._keep[0])
        self.h = lib().oracle_tree_build(C.c_int64(self.n),
                                         *[_d(a) for a in self._keep],
                                         C.c_int(leaf_max))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oracle_tree_free(C.c_void_p(h))
            self.h = None

    @property
    def ncells(self):
        return lib().oracle_tree_ncells(C.c_void_p(self.h))

    @property
    def depth(self):
        return lib().oracle_tree_depth(C.c_void_p(self.h))

    def root(self):
        r = np.zeros(4)
        lib().oracle_tree_root(C.c_void_p(self.h), _d(r))
        return r

    def keys(self):
        k = np.zeros(self.n, dtype=np.uint64)
        lib().oracle_tree_keys(C.c_void_p(self.h), k.ctypes.data_as(_u64p))
        return k

    def perm(self):
        p = np.zeros(self.n, dtype=np.int64)
        lib().oracle_tree_perm(C.c_void_p(self.h), p.ctypes.data_as(_i64p))
        return p

    def cells(self):
        nc = self.ncells
        i32 = {k: np.zeros(nc, dtype=np.int32) for k in
               ("level", "ix", "iy", "iz", "parent", "first_child", "nchild")}
        i64 = {k: np.zeros(nc, dtype=np.int64) for k in ("first", "count")}
        lib().oracle_tree_cells(
            C.c_void_p(self.h),
            *[i32[k].ctypes.data_as(_i32p) for k in ("level", "ix", "iy", "iz")],
            *[i64[k].ctypes.data_as(_i64p) for k in ("first", "count")],
            *[i32[k].ctypes.data_as(_i32p) for k in ("parent", "first_child",
                                                      "nchild")])
        i32.update(i64)
        return i32

    def centres(self):
        nc = self.ncells
        out = [np.zeros(nc) for _ in range(4)]
        lib().oracle_tree_centres(C.c_void_p(self.h), *[_d(o) for o in out])
        return tuple(out)

    def com(self, m):
        m = _f64(m)
        nc = self.ncells
        out = [np.zeros(nc) for _ in range(3)]
        lib().oracle_tree_com(C.c_void_p(self.h), _d(m), *[_d(o) for o in out])
        return tuple(out)

    def list(self, which, bruteforce=False):
        """CSR (off[ncells+1], items) of list U/V/W/X."""
        h = C.c_void_p(self.h)
        if bruteforce:
            tot = lib().oracle_list_size_bruteforce(h, which)
        else:
            tot = lib().oracle_list_size(h, which)
        off = np.zeros(self.ncells + 1, dtype=np.int64)
        items = np.zeros(max(tot, 1), dtype=np.int32)
        fn = lib().oracle_list_get_bruteforce if bruteforce else \
            lib().oracle_list_get
        fn(h, C.c_int(which), off.ctypes.data_as(_i64p),
           items.ctypes.data_as(_i32p))
        return off, items[:tot]

    def bh_lists(self, m, theta, which):
        """Barnes-Hut group lists: which 0 = accepted (M2P), 1 = P2P."""
        m = _f64(m)
        h = C.c_void_p(self.h)
        tot = lib().oracle_bh_lists(h, _d(m), C.c_double(theta),
                                    C.c_int(which), None, None)
        off = np.zeros(self.ncells + 1, dtype=np.int64)
        items = np.zeros(max(tot, 1), dtype=np.int32)
        lib().oracle_bh_lists(h, _d(m), C.c_double(theta), C.c_int(which),
                              off.ctypes.data_as(_i64p),
                              items.ctypes.data_as(_i32p))
        return off, items[:tot]

    def target_boxes(self, tx, ty, tz):
        """Per target point: (kind, level, ix, iy, iz, host, leaf) of the box
        it is binned into (kind 0 leaf, 1 empty octant, 2 outside the root)."""
        tx, ty, tz = map(_f64, (tx, ty, tz))
        out = np.zeros((len(tx), 7), dtype=np.int64)
        lib().oracle_target_boxes(C.c_void_p(self.h), C.c_int64(len(tx)), _d(tx), _d(ty),
                                  _d(tz), out.ctypes.data_as(_i64p))
        return out

    def box_list(self, point, which):
        """List U/V/W/X (0..3) of the box of one target point (cell ids)."""
        pt = (C.c_double * 3)(*[float(v) for v in point])
        h = C.c_void_p(self.h)
        n = lib().oracle_box_list(h, pt, C.c_int(which), None)
        items = np.zeros(max(n, 1), dtype=np.int32)
        lib().oracle_box_list(h, pt, C.c_int(which), items.ctypes.data_as(_i32p))
        return items[:n]

    def move(self, x, y, z):
        """New positions (caller order) for the same cells, membership,
        order, root and lists (a tree kept across a time step)."""
        self._keep = [_f64(x), _f64(y), _f64(z)]
        lib().oracle_tree_move(C.c_void_p(self.h), *[_d(a) for a in self._keep])

    def stays(self, x, y, z, slack):
        """Every particle at x, y, z within (1/2 + slack) leaf sides of the
        centre of its leaf, along each axis."""
        x, y, z = map(_f64, (x, y, z))
        return bool(lib().oracle_tree_stays(C.c_void_p(self.h), _d(x), _d(y), _d(z),
                                            C.c_double(slack)))

    def fmm(self, m, p, targets=None, eps2=0.0):
        """The FMM on this tree (phi, ax, ay, az) at caller indices."""
        m = _f64(m)
        nt, tg = _targets(targets, self.n)
        out = [np.zeros(nt) for _ in range(4)]
        lib().oracle_fmm_tree(C.c_void_p(self.h), _d(m), C.c_int(p), C.c_double(eps2),
                              C.c_int64(nt), None if tg is None else tg.ctypes.data_as(_i64p),
                              *[_d(o) for o in out])
        return tuple(out)

    def treecode(self, m, p, theta, mode=0, targets=None, eps2=0.0):
        """The treecode (modes as `treecode`) on this tree."""
        m = _f64(m)
        nt, tg = _targets(targets, self.n)
        out = [np.zeros(nt) for _ in range(4)]
        lib().oracle_treecode_tree(C.c_void_p(self.h), _d(m), C.c_int(p), C.c_double(theta),
                                   C.c_int(mode), C.c_double(eps2), C.c_int64(nt),
                                   None if tg is None else tg.ctypes.data_as(_i64p),
                                   *[_d(o) for o in out])
        return tuple(out)

    def fmm_points(self, m, p, tx, ty, tz, eps2=0.0):
        """The FMM on this tree at separate target points."""
        m, tx, ty, tz = map(_f64, (m, tx, ty, tz))
        out = [np.zeros(len(tx)) for _ in range(4)]
        lib().oracle_fmm_points_tree(C.c_void_p(self.h), _d(m), C.c_int(p), C.c_double(eps2),
                                     C.c_int64(len(tx)), _d(tx), _d(ty), _d(tz),
                                     *[_d(o) for o in out])
        return tuple(out)

    def treecode_points(self, m, p, theta, tx, ty, tz, mode=0, eps2=0.0):
        """The treecode (mode 0 or 2) on this tree at separate target points."""
        if mode not in (0, 2):
            raise ValueError("mode 0 or 2")
        m, tx, ty, tz = map(_f64, (m, tx, ty, tz))
        out = [np.zeros(len(tx)) for _ in range(4)]
        lib().oracle_treecode_points_tree(C.c_void_p(self.h), _d(m), C.c_int(p),
                                          C.c_double(theta), C.c_int(mode), C.c_double(eps2),
                                          C.c_int64(len(tx)), _d(tx), _d(ty), _d(tz),
                                          *[_d(o) for o in out])
        return tuple(out)

    def fmm_expansions(self, m, p):
        m = _f64(m)
        nc = self.ncells
        M = np.zeros(nc * p * p, dtype=np.complex128)
        L = np.zeros(nc * p * p, dtype=np.complex128)
        lib().oracle_fmm_expansions(C.c_void_p(self.h), _d(m), C.c_int(p),
                                    M.ctypes.data_as(_dp),
                                    L.ctypes.data_as(_dp))
        return M.reshape(nc, p * p), L.reshape(nc, p * p)


# ---- drivers --------------------------------------------------------------

def _targets(targets, n):
    if targets is None:
        return n, None
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    return len(targets), targets


def fmm(x, y, z, m, p, leaf_max, targets=None, eps2=0.0):
    """Oracle FMM (phi, ax, ay, az) at caller indices `targets`."""
    x, y, z, m = map(_f64, (x, y, z, m))
    nt, tg = _targets(targets, len(x))
    out = [np.zeros(nt) for _ in range(4)]
    lib().oracle_fmm(C.c_int64(len(x)), _d(x), _d(y), _d(z), _d(m),
                     C.c_int(leaf_max), C.c_int(p), C.c_double(eps2),
                     C.c_int64(nt),
                     None if tg is None else tg.ctypes.data_as(_i64p),
                     *[_d(o) for o in out])
    return tuple(out)


def treecode(x, y, z, m, p, theta, leaf_max, targets=None, mode=0, eps2=0.0):
    """Oracle treecode.  Barnes-Hut acceptance l < theta d about centres of
    mass: mode 0 per target leaf, 1 per particle.  Mode 2: the treecode of
    Sec. 4 over the FMM lists (M2P from the V lists of the leaf and its
    ancestors and the leaf's W list, P2P over U and the X lists, expansions
    about geometric centres; theta unused)."""
    x, y, z, m = map(_f64, (x, y, z, m))
    nt, tg = _targets(targets, len(x))
    out = [np.zeros(nt) for _ in range(4)]
    lib().oracle_treecode(C.c_int64(len(x)), _d(x), _d(y), _d(z), _d(m),
                          C.c_int(leaf_max), C.c_int(p), C.c_double(theta),
                          C.c_int(mode), C.c_double(eps2), C.c_int64(nt),
                          None if tg is None else tg.ctypes.data_as(_i64p),
                          *[_d(o) for o in out])
    return tuple(out)


def fmm_points(x, y, z, m, p, leaf_max, tx, ty, tz, eps2=0.0):
    """Oracle FMM at separate target points binned into the source tree."""
    x, y, z, m, tx, ty, tz = map(_f64, (x, y, z, m, tx, ty, tz))
    out = [np.zeros(len(tx)) for _ in range(4)]
    lib().oracle_fmm_points(C.c_int64(len(x)), _d(x), _d(y), _d(z), _d(m),
                            C.c_int(leaf_max), C.c_int(p), C.c_double(eps2),
                            C.c_int64(len(tx)), _d(tx), _d(ty), _d(tz),
                            *[_d(o) for o in out])
    return tuple(out)


def treecode_points(x, y, z, m, p, theta, leaf_max, tx, ty, tz, mode=0, eps2=0.0):
    """Oracle treecode (mode 0 Barnes-Hut group lists, mode 2 the FMM lists)
    at separate target points binned into the source tree."""
    if mode not in (0, 2):
        raise ValueError("mode 0 or 2")
    x, y, z, m, tx, ty, tz = map(_f64, (x, y, z, m, tx, ty, tz))
    out = [np.zeros(len(tx)) for _ in range(4)]
    lib().oracle_treecode_points(C.c_int64(len(x)), _d(x), _d(y), _d(z), _d(m),
                                 C.c_int(leaf_max), C.c_int(p), C.c_double(theta),
                                 C.c_int(mode), C.c_double(eps2), C.c_int64(len(tx)),
                                 _d(tx), _d(ty), _d(tz), *[_d(o) for o in out])
    return tuple(out)


def rel_l2(a, ref):
    """Normalised L2 error sqrt(sum |a-ref|^2) / sqrt(sum |ref|^2)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((a - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))


# ---- time stepping ----------------------------------------------------------

def leapfrog(x, y, z, vx, vy, vz, m, dt, steps, field=None):
    """Kick-drift-kick leapfrog over `steps` steps of length dt (the paper
    leaves the integrator of its N-body simulation unnamed; this is the
    standard second-order symplectic one).  The acceleration of each particle
    is the field of all the others, a_i = sum_j m_j (x_j - x_i) / r^3
    (`field(x, y, z, m)` -> (phi, ax, ay, az); the oracle direct sum when
    None).  Per step: v += a dt/2; x += v dt; a = field(x); v += a dt/2.
    Returns (x, y, z, vx, vy, vz, phi, ax, ay, az) after the last step, the
    field being that of the final positions."""
    if field is None:
        field = direct
    pos = [np.array(a, dtype=np.float64) for a in (x, y, z)]
    vel = [np.array(a, dtype=np.float64) for a in (vx, vy, vz)]
    m = _f64(m)
    phi, *acc = field(*pos, m)
    for _ in range(steps):
        for v, a in zip(vel, acc):
            v += 0.5 * dt * a
        for q, v in zip(pos, vel):
            q += dt * v
        phi, *acc = field(*pos, m)
        for v, a in zip(vel, acc):
            v += 0.5 * dt * a
    return (*pos, *vel, phi, *acc)


def leapfrog_tree(x, y, z, vx, vy, vz, m, dt, steps, leaf_max, slack, evaluate):
    """Kick-drift-kick leapfrog (as `leapfrog`) whose field comes from an
    octree kept across steps.  After each drift the tree takes the new
    positions (Tree.move) when every particle lies within (1/2 + slack) leaf
    sides of its leaf's centre along each axis (Tree.stays), and a new tree
    is built otherwise; slack < 0 builds one every step.
    evaluate(tree, m) -> (phi, ax, ay, az) in caller order.  Returns the
    state and field as `leapfrog` does, then the number of trees built."""
    pos = [np.array(a, dtype=np.float64) for a in (x, y, z)]
    vel = [np.array(a, dtype=np.float64) for a in (vx, vy, vz)]
    m = _f64(m)
    tree = Tree(*pos, leaf_max)
    builds = 1
    phi, *acc = evaluate(tree, m)
    for _ in range(steps):
        for v, a in zip(vel, acc):
            v += 0.5 * dt * a
        for q, v in zip(pos, vel):
            q += dt * v
        if slack >= 0 and tree.stays(*pos, slack):
            tree.move(*pos)
        else:
            tree = Tree(*pos, leaf_max)
            builds += 1
        phi, *acc = evaluate(tree, m)
        for v, a in zip(vel, acc):
            v += 0.5 * dt * a
    return (*pos, *vel, phi, *acc, builds)
