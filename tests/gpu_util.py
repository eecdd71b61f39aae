"""Helpers for the GPU parity tests (inputs on the device, oracle on the host)."""
import sys

import numpy as np
import pytest
import torch


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


def rel_err(out, ref):
    a = np.stack([np.asarray(o, dtype=np.float64) for o in out[1:]])
    r = np.stack([np.asarray(o, dtype=np.float64) for o in ref[1:]])
    ephi = np.linalg.norm(np.asarray(out[0]) - ref[0]) / np.linalg.norm(ref[0])
    eacc = np.linalg.norm(a - r) / np.linalg.norm(r)
    return float(ephi), float(eacc)
