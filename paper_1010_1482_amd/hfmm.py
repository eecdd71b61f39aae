"""Python binding of the hfmm C ABI (include/hfmm.h).

Argument marshalling only: every step of the computation runs in the HIP
library libhfmm.so.  PyTorch provides device memory and the stream.  There is
no fallback: importing this module on a machine without the built library,
or calling it without a HIP device, raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfmm.so")

DIRECT, TREECODE, FMM, TREECODE_FMMLIST, FMM_ROT = 0, 1, 2, 3, 4
FP64, FP32, M2L_BF16, M2L_BF16X3, M2L_FP16, M2L_FP16X3 = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": M2L_BF16, "bf16x3": M2L_BF16X3,
              "fp16": M2L_FP16, "fp16x3": M2L_FP16X3}
METHODS = {"direct": DIRECT, "treecode": TREECODE, "fmm": FMM,
           "treecode_fmmlist": TREECODE_FMMLIST, "fmm_rot": FMM_ROT}
OK, E_INVAL, E_NOMEM, E_UNSUPPORTED, E_HIP, E_STATE, E_DATA, E_OVERFLOW = \
    0, -1, -2, -3, -4, -5, -6, -7
ST_SRC_NONFINITE, ST_TGT_NONFINITE, ST_MASS_NONFINITE, ST_OVERFLOW = 1, 2, 4, 8
MAX_P = 16

# exported symbols, in the order include/hfmm.h declares them
SYMBOLS = ("hfmm_arena_bytes", "hfmm_build_tree", "hfmm_upward", "hfmm_evaluate",
           "hfmm_solve", "hfmm_refit", "hfmm_status", "hfmm_direct_bytes", "hfmm_direct", "hfmm_direct_noalloc",
           "hfmm_leapfrog",
           "hfmm_tree_release",
           "hfmm_required_bytes", "hfmm_last_required_bytes", "hfmm_get_stats",
           "hfmm_strerror", "hfmm_export_perm", "hfmm_export_targets",
           "hfmm_export_target_lists", "hfmm_export_cells", "hfmm_export_list",
           "hfmm_export_bh_list", "hfmm_export_expansions", "hfmm_set_timing")


class HfmmError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib().hfmm_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class Stats(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_cells", C.c_int64),
                ("n_leaves", C.c_int64), ("depth", C.c_int32), ("sort_bits", C.c_int32),
                ("root", C.c_double * 4), ("list_u", C.c_int64), ("list_v", C.c_int64),
                ("list_w", C.c_int64), ("list_x", C.c_int64), ("list_m2p", C.c_int64),
                ("list_p2p", C.c_int64), ("p2p_pairs", C.c_int64), ("m2l_pairs", C.c_int64),
                ("arena_used", C.c_size_t), ("phase_ms", C.c_double * 10),
                ("n_targets", C.c_int64), ("n_target_boxes", C.c_int64),
                ("target_near", C.c_int64), ("target_far", C.c_int64)]

    PHASES = ("build", "lists", "upward", "m2l_ops", "m2l", "downward", "far", "p2p",
              "targets", "m2l_prep")

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["root"] = list(self.root)
        d["phase_ms"] = {k: v for k, v in zip(self.PHASES, self.phase_ms) if v >= 0}
        return d


_LIB = None
_vp = C.c_void_p


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_1010_1482_amd/build.py")
        L = C.CDLL(LIB_PATH)
        i64, i32, d, sz = C.c_int64, C.c_int, C.c_double, C.c_size_t
        L.hfmm_arena_bytes.argtypes = [i64, i64, i32, i32, i32, i32, C.POINTER(sz)]
        L.hfmm_build_tree.argtypes = [_vp, _vp, _vp, i64, i32, _vp, sz, _vp, C.POINTER(_vp)]
        L.hfmm_upward.argtypes = [_vp, _vp, i32, i32, i32, _vp]
        L.hfmm_evaluate.argtypes = [_vp, _vp, _vp, _vp, i64, i32, d, i32, i32, d, _vp, _vp, _vp,
                                    _vp, _vp]
        L.hfmm_status.argtypes = [_vp, _vp, C.POINTER(C.c_uint32)]
        L.hfmm_solve.argtypes = [_vp, _vp, _vp, _vp, i64, _vp, _vp, _vp, i64, i32, i32, d,
                                 i32, i32, d, _vp, sz, _vp, _vp, _vp, _vp, _vp]
        L.hfmm_direct_bytes.argtypes = [i64, i64, i32, C.POINTER(sz)]
        L.hfmm_direct.argtypes = [_vp, _vp, _vp, _vp, i64, _vp, _vp, _vp, i64, i32, d, _vp,
                                  sz, _vp, _vp, _vp, _vp, _vp]
        L.hfmm_direct_noalloc.argtypes = [_vp, _vp, _vp, _vp, i64, _vp, _vp, _vp, i64, i32, d,
                                          _vp, _vp, _vp, _vp, _vp]
        L.hfmm_leapfrog.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, i64, d, i32, i32, i32,
                                    d, i32, i32, d, d, _vp, sz, _vp, _vp, _vp, _vp,
                                    C.POINTER(i32), C.POINTER(i32), _vp]
        L.hfmm_refit.argtypes = [_vp, _vp, _vp, _vp, d, _vp, C.POINTER(i32)]
        L.hfmm_tree_release.argtypes = [_vp]
        L.hfmm_tree_release.restype = None
        L.hfmm_required_bytes.argtypes = [_vp]
        L.hfmm_required_bytes.restype = sz
        L.hfmm_last_required_bytes.argtypes = []
        L.hfmm_last_required_bytes.restype = sz
        L.hfmm_get_stats.argtypes = [_vp, C.POINTER(Stats)]
        L.hfmm_strerror.argtypes = [i32]
        L.hfmm_strerror.restype = C.c_char_p
        L.hfmm_export_perm.argtypes = [_vp, _vp, _vp]
        L.hfmm_export_targets.argtypes = [_vp, _vp, _vp]
        L.hfmm_export_target_lists.argtypes = [_vp, i32, _vp, _vp, _vp]
        L.hfmm_export_cells.argtypes = [_vp, _vp, _vp]
        L.hfmm_export_list.argtypes = [_vp, i32, _vp, _vp, _vp]
        L.hfmm_export_bh_list.argtypes = [_vp, i32, _vp, _vp, _vp]
        L.hfmm_export_expansions.argtypes = [_vp, i32, _vp, _vp]
        L.hfmm_set_timing.argtypes = [i32]
        L.hfmm_set_timing.restype = None
        _LIB = L
    return _LIB


def set_timing(on: bool):
    """Per-phase device timers for trees built afterwards."""
    _lib().hfmm_set_timing(1 if on else 0)


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


def _check(rc: int, what: str):
    if rc != OK:
        raise HfmmError(rc, what)


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _dev(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t


def _prec(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def _meth(method):
    return METHODS[method] if isinstance(method, str) else int(method)


def arena_bytes(n_src, n_tgt=0, leaf_max=64, p=10, method=FMM, precision=FP32):
    out = C.c_size_t(0)
    _check(_lib().hfmm_arena_bytes(n_src, n_tgt, leaf_max, p, _meth(method), _prec(precision),
                                   C.byref(out)), "hfmm_arena_bytes")
    return out.value


def out_dtype(precision):
    return torch.float64 if _prec(precision) == FP64 else torch.float32


def _targets(targets):
    """Device target coordinates and their count.  An empty target set never
    reaches the library: torch gives an empty tensor a null data pointer,
    and a null tx selects self-evaluation there."""
    if targets is None:
        return None, None, None, 0
    tx, ty, tz = (_dev(t, "target") for t in targets)
    if not (tx.numel() == ty.numel() == tz.numel()):
        raise ValueError("target coordinate arrays differ in length")
    return tx, ty, tz, tx.numel()


def _empty_out(dt, device, out):
    return out if out is not None else tuple(torch.empty(0, dtype=dt, device=device)
                                             for _ in range(4))


class Tree:
    """A device-resident octree over the sources, living in one caller-owned
    arena tensor, evaluated at the sources or at separate target sets of up
    to `max_targets` points."""

    def __init__(self, x, y, z, leaf_max=64, arena=None, stream=None, arena_bytes_hint=None,
                 max_targets=0):
        self.ns = x.numel()
        self.leaf_max = leaf_max
        for nm, t in (("x", x), ("y", y), ("z", z)):
            _dev(t, nm)
        self._keep = (x, y, z)
        nbytes = arena_bytes_hint or arena_bytes(self.ns, max_targets, leaf_max, 12, FMM, FP32)
        self.h = None
        for _ in range(6):
            self.arena = arena if arena is not None else torch.empty(
                nbytes, dtype=torch.uint8, device=x.device)
            h = _vp()
            rc = _lib().hfmm_build_tree(_ptr(x), _ptr(y), _ptr(z), self.ns, leaf_max,
                                        _ptr(self.arena), self.arena.numel(), _stream(stream),
                                        C.byref(h))
            if rc == E_NOMEM and arena is None:
                need = _lib().hfmm_last_required_bytes()
                nbytes = max(int(need * 1.25), nbytes * 2)
                continue
            _check(rc, "hfmm_build_tree")
            self.h = h
            break
        if self.h is None:
            raise HfmmError(E_NOMEM, "hfmm_build_tree")
        self.p = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _LIB is not None:
            _LIB.hfmm_tree_release(h)
            self.h = None

    def upward(self, m, p, method=FMM, precision=FP32, stream=None):
        _dev(m, "m")
        self._m = m
        rc = _lib().hfmm_upward(self.h, _ptr(m), p, _meth(method), _prec(precision),
                                _stream(stream))
        _check(rc, "hfmm_upward")
        self.p, self.method, self.precision = p, _meth(method), _prec(precision)

    def evaluate(self, theta=0.5, eps2=0.0, targets=None, out=None, stream=None):
        """phi, ax, ay, az at the sources (targets=None) or at targets=(tx, ty, tz)."""
        dt = out_dtype(self.precision)
        dev = self._keep[0].device
        tx, ty, tz, nt = _targets(targets)
        if targets is None:
            nt = self.ns
        elif nt == 0:
            return _empty_out(dt, dev, out)
        if out is None:
            out = tuple(torch.empty(nt, dtype=dt, device=dev) for _ in range(4))
        self._tkeep = (tx, ty, tz)
        rc = _lib().hfmm_evaluate(self.h, _ptr(tx), _ptr(ty), _ptr(tz),
                                  0 if targets is None else nt, self.p, float(theta),
                                  self.method, self.precision, float(eps2),
                                  *[_ptr(o) for o in out], _stream(stream))
        _check(rc, "hfmm_evaluate")
        return out

    def refit(self, x, y, z, slack, stream=None):
        """Move the sources to x, y, z keeping the tree when every one stays
        within (1/2 + slack) leaf sides of its leaf's centre on each axis
        (True; upward must run again before evaluate), else False (the tree
        is unusable: build a new one)."""
        for nm, t in (("x", x), ("y", y), ("z", z)):
            _dev(t, nm)
        kept = C.c_int(0)
        _check(_lib().hfmm_refit(self.h, _ptr(x), _ptr(y), _ptr(z), float(slack),
                                 _stream(stream), C.byref(kept)), "hfmm_refit")
        self._keep = (x, y, z)
        return bool(kept.value)

    def status(self, stream=None):
        """(code, flags) of the device status word after the enqueued work."""
        f = C.c_uint32(0)
        rc = _lib().hfmm_status(self.h, _stream(stream), C.byref(f))
        return rc, f.value

    def stats(self):
        s = Stats()
        _check(_lib().hfmm_get_stats(self.h, C.byref(s)), "hfmm_get_stats")
        return s.as_dict()

    def required_bytes(self):
        return _lib().hfmm_required_bytes(self.h)

    # ---- inspection ----
    def perm(self, stream=None):
        n = self.stats()["n_particles"]
        out = torch.empty(n, dtype=torch.int32, device=self.arena.device)
        _check(_lib().hfmm_export_perm(self.h, _ptr(out), _stream(stream)), "export_perm")
        return out

    def target_boxes(self, stream=None):
        """Per target of the last evaluation (caller order): kind, level, ix,
        iy, iz, host, leaf, box index."""
        n = self.stats()["n_targets"]
        out = torch.empty((n, 8), dtype=torch.int32, device=self.arena.device)
        _check(_lib().hfmm_export_targets(self.h, _ptr(out), _stream(stream)),
               "export_targets")
        return out

    def target_list(self, which, stream=None):
        """CSR by box of the last separate-target evaluation: which 0 far
        (M2P), 1 near (P2P)."""
        st = self.stats()
        nn = [st["target_far"], st["target_near"]][which]
        off = torch.empty(st["n_target_boxes"] + 1, dtype=torch.int32, device=self.arena.device)
        items = torch.empty(max(nn, 1), dtype=torch.int32, device=self.arena.device)
        _check(_lib().hfmm_export_target_lists(self.h, which, _ptr(off), _ptr(items),
                                               _stream(stream)), "export_target_lists")
        return off, items[:nn]

    def cells(self, stream=None):
        nc = self.stats()["n_cells"]
        out = torch.empty((nc, 9), dtype=torch.int32, device=self.arena.device)
        _check(_lib().hfmm_export_cells(self.h, _ptr(out), _stream(stream)), "export_cells")
        return out

    def fmm_list(self, which, stream=None):
        st = self.stats()
        nn = [st["list_u"], st["list_v"], st["list_w"], st["list_x"]][which]
        off = torch.empty(st["n_cells"] + 1, dtype=torch.int32, device=self.arena.device)
        items = torch.empty(max(nn, 1), dtype=torch.int32, device=self.arena.device)
        _check(_lib().hfmm_export_list(self.h, which, _ptr(off), _ptr(items), _stream(stream)),
               "export_list")
        return off, items[:nn]

    def bh_list(self, which, stream=None, offsets_only=False):
        st = self.stats()
        nn = [st["list_m2p"], st["list_p2p"]][which]
        off = torch.empty(st["n_cells"] + 1, dtype=torch.int32, device=self.arena.device)
        if offsets_only:
            _check(_lib().hfmm_export_bh_list(self.h, which, _ptr(off), None, _stream(stream)),
                   "export_bh_list")
            return off
        items = torch.empty(max(nn, 1), dtype=torch.int32, device=self.arena.device)
        _check(_lib().hfmm_export_bh_list(self.h, which, _ptr(off), _ptr(items),
                                          _stream(stream)), "export_bh_list")
        return off, items[:nn]

    def expansions(self, which, stream=None):
        """which 0 = M, 1 = L in the paper's normalisation, complex [ncells, p(p+1)/2]
        for n < p, m = 0..n."""
        nc = self.stats()["n_cells"]
        p = self.p
        out = torch.empty((nc, p * (p + 1) // 2, 2), dtype=torch.float64,
                          device=self.arena.device)
        _check(_lib().hfmm_export_expansions(self.h, which, _ptr(out), _stream(stream)),
               "export_expansions")
        return torch.view_as_complex(out)


def solve(x, y, z, m, p=10, method=FMM, precision=FP32, leaf_max=64, theta=0.5, eps2=0.0,
          targets=None, arena=None, out=None, stream=None):
    """phi, ax, ay, az at the sources (targets=None) or at targets=(tx, ty, tz)."""
    method, precision = _meth(method), _prec(precision)
    for nm, t in (("x", x), ("y", y), ("z", z), ("m", m)):
        _dev(t, nm)
    ns = x.numel()
    tx, ty, tz, nt = _targets(targets)
    dt = out_dtype(precision)
    if targets is None:
        nt = ns
    elif nt == 0:
        return _empty_out(dt, x.device, out)
    if out is None:
        out = tuple(torch.empty(nt, dtype=dt, device=x.device) for _ in range(4))
    nbytes = arena.numel() if arena is not None else arena_bytes(
        ns, 0 if targets is None else nt, leaf_max, p, method, precision)
    for _ in range(6):
        ar = arena if arena is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                         device=x.device)
        rc = _lib().hfmm_solve(_ptr(x), _ptr(y), _ptr(z), _ptr(m), ns, _ptr(tx), _ptr(ty),
                               _ptr(tz), 0 if targets is None else nt, leaf_max, p,
                               float(theta), method, precision, float(eps2), _ptr(ar),
                               ar.numel(), *[_ptr(o) for o in out], _stream(stream))
        if rc == E_NOMEM and arena is None:
            need = _lib().hfmm_last_required_bytes()
            nbytes = max(int(need * 1.25), nbytes * 2)
            continue
        _check(rc, "hfmm_solve")
        return out
    raise HfmmError(E_NOMEM, "hfmm_solve")


def leapfrog(x, y, z, vx, vy, vz, m, dt, steps, p=10, method=FMM, precision=FP32,
             leaf_max=64, theta=0.5, eps2=0.0, slack=-1.0, out=None, info=None, stream=None):
    """`steps` kick-drift-kick steps of length dt on the device, positions and
    velocities (contiguous float64 CUDA tensors) updated in place; returns
    the field (phi, ax, ay, az) at the final positions.  slack < 0 builds a
    tree per evaluation; slack >= 0 keeps it while the particles stay within
    (1/2 + slack) leaf sides of their leaves' centres (Tree.refit).  When
    the arena turns out too small the library stops at a whole step and the
    call continues from there with a larger one.  `info` (a dict) receives
    the trees built ("builds") and the calls made ("calls")."""
    method, precision = _meth(method), _prec(precision)
    for nm, t in (("x", x), ("y", y), ("z", z), ("vx", vx), ("vy", vy), ("vz", vz),
                  ("m", m)):
        _dev(t, nm)
    n = x.numel()
    dt_ = out_dtype(precision)
    if out is None:
        out = tuple(torch.empty(n, dtype=dt_, device=x.device) for _ in range(4))
    if method == DIRECT:
        sz = C.c_size_t(0)
        _check(_lib().hfmm_direct_bytes(n, 0, precision, C.byref(sz)), "hfmm_direct_bytes")
        nbytes = sz.value
    else:
        nbytes = arena_bytes(n, 0, leaf_max, p, method, precision)
    nbytes += 48 * n + (2 << 20)
    left = int(steps)
    builds = 0
    for calls in range(1, 9):
        ar = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        done, nb = C.c_int(0), C.c_int(0)
        rc = _lib().hfmm_leapfrog(_ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz),
                                  _ptr(m), n, float(dt), left, leaf_max, p, float(theta),
                                  method, precision, float(eps2), float(slack), _ptr(ar),
                                  ar.numel(), *[_ptr(o) for o in out], C.byref(done),
                                  C.byref(nb), _stream(stream))
        builds += nb.value
        if info is not None:
            info.update(builds=builds, calls=calls)
        if rc == E_NOMEM:
            left -= done.value
            nbytes = max(int(_lib().hfmm_last_required_bytes() * 1.25), nbytes * 2)
            continue
        _check(rc, "hfmm_leapfrog")
        return out
    raise HfmmError(E_NOMEM, "hfmm_leapfrog")


def direct(x, y, z, m, precision=FP32, eps2=0.0, targets=None, out=None, stream=None):
    """Direct sum of Eq. 1 on the device."""
    precision = _prec(precision)
    ns = x.numel()
    tx = ty = tz = None
    nt = ns
    if targets is not None:
        tx, ty, tz, nt = _targets(targets)
        if nt == 0:
            return _empty_out(out_dtype(precision), x.device, out)
    sz = C.c_size_t(0)
    _check(_lib().hfmm_direct_bytes(ns, 0 if targets is None else nt, precision, C.byref(sz)),
           "hfmm_direct_bytes")
    ar = torch.empty(sz.value, dtype=torch.uint8, device=x.device)
    dt = out_dtype(precision)
    if out is None:
        out = tuple(torch.empty(nt, dtype=dt, device=x.device) for _ in range(4))
    _check(_lib().hfmm_direct(_ptr(x), _ptr(y), _ptr(z), _ptr(m), ns, _ptr(tx), _ptr(ty),
                              _ptr(tz), 0 if targets is None else nt, precision, float(eps2),
                              _ptr(ar), ar.numel(), *[_ptr(o) for o in out], _stream(stream)),
           "hfmm_direct")
    return out
