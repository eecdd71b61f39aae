"""Helpers for the GPU parity tests (inputs on the device, oracle on the host)."""
import sys

import numpy as np
import pytest
import torch

from paper_1010_1482_amd import workloads as W


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def host(ts):
    return [t.double().cpu().numpy() for t in ts]


def inputs(dist, n, seed, kind="equal"):
    """Positions of workload `dist` and masses of `kind` (equal, unequal,
    mixed), both seeded."""
    x, y, z, m = W.make(dist, n, seed)
    if kind != "equal":
        m = W.masses(n, seed + 500, kind)
    return x, y, z, m


def rel_err(out, ref):
    """Normalised L2 errors (phi, acceleration) over the targets."""
    a = np.stack([np.asarray(o, dtype=np.float64) for o in out[1:]])
    r = np.stack([np.asarray(o, dtype=np.float64) for o in ref[1:]])
    ephi = np.linalg.norm(np.asarray(out[0]) - ref[0]) / np.linalg.norm(ref[0])
    eacc = np.linalg.norm(a - r) / np.linalg.norm(r)
    return float(ephi), float(eacc)


def elem_err(out, ref):
    """Largest error at any one target, relative to the largest reference
    value: max_i |phi_i - ref_i| / max_i |ref_i|, and the same for the
    acceleration vectors.  An error confined to a few targets, which the L2
    norm over many targets dilutes, shows here."""
    a = np.stack([np.asarray(o, dtype=np.float64) for o in out[1:]])
    r = np.stack([np.asarray(o, dtype=np.float64) for o in ref[1:]])
    ephi = np.max(np.abs(np.asarray(out[0]) - ref[0])) / np.max(np.abs(ref[0]))
    eacc = np.max(np.linalg.norm(a - r, axis=0)) / np.max(np.linalg.norm(r, axis=0))
    return float(ephi), float(eacc)


def cancellation(x, y, z, m, tx, ty, tz, ref):
    """How much the signed sums cancel at the targets: ||sum |m|/r|| / ||phi||
    and ||sum |m|/r^2|| / ||a||.  Rounding errors scale with the sum of the
    magnitudes of the terms, so a relative error bar of a mixed-sign case is
    the equal-sign bar times this factor (1 for positive masses)."""
    am = np.abs(m)
    s_phi = np.zeros(len(tx))
    s_acc = np.zeros(len(tx))
    for k0 in range(0, len(tx), 64):
        dx = x[None, :] - tx[k0:k0 + 64, None]
        dy = y[None, :] - ty[k0:k0 + 64, None]
        dz = z[None, :] - tz[k0:k0 + 64, None]
        r2 = dx * dx + dy * dy + dz * dz
        ok = r2 > 0
        inv = np.where(ok, 1.0 / np.sqrt(np.where(ok, r2, 1.0)), 0.0)
        s_phi[k0:k0 + 64] = inv @ am
        s_acc[k0:k0 + 64] = (inv * inv) @ am
    a = np.stack([np.asarray(o, dtype=np.float64) for o in ref[1:]])
    k_phi = np.linalg.norm(s_phi) / np.linalg.norm(ref[0])
    k_acc = np.linalg.norm(s_acc) / np.linalg.norm(a)
    return max(1.0, float(k_phi)), max(1.0, float(k_acc))


def assert_close(out, ref, tol, what="", kappa=(1.0, 1.0)):
    """Normalised L2 and per-target errors both within tol (times the
    cancellation factor kappa for phi and acceleration)."""
    l2 = rel_err(out, ref)
    el = elem_err(out, ref)
    say(f"  {what}: L2 phi {l2[0]:.2e} acc {l2[1]:.2e}; per target phi {el[0]:.2e} "
        f"acc {el[1]:.2e} (tol {tol:.1e}, kappa {kappa[0]:.1f} {kappa[1]:.1f})")
    assert np.all(np.isfinite(np.stack(out))), what
    assert l2[0] <= tol * kappa[0] and l2[1] <= tol * kappa[1], (what, l2)
    assert el[0] <= tol * kappa[0] and el[1] <= tol * kappa[1], (what, el)
    return l2, el
