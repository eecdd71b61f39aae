"""Seeded synthetic inputs for the N-body workloads.

This module holds input generation only: no arithmetic of the treecode or
FMM.  Both the HIP path and the FP64 oracle are fed from it.  The paper
measures on synthetic particle sets (no public dataset), so these recipes
stand in for its workloads:

* uniform: positions ~ U[0,1)^3, masses 1/N;
* plummer: Plummer sphere of scale radius a, radii r = a / sqrt(U^(-2/3) - 1)
  with U ~ (0,1], resampled while r > r_max, isotropic directions, masses 1/N.
"""
from __future__ import annotations

import numpy as np


def uniform(n: int, seed: int):
    """N points uniform in the unit cube, masses 1/N (FP64 SoA)."""
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n))
    m = np.full(n, 1.0 / max(n, 1))
    return pos[0].copy(), pos[1].copy(), pos[2].copy(), m


def plummer(n: int, seed: int, a: float = 1.0, r_max: float = 20.0):
    """Plummer sphere (scale radius a, truncated at r_max), masses 1/N."""
    rng = np.random.default_rng(seed)
    r = np.empty(n)
    filled = 0
    while filled < n:
        k = n - filled
        u = 1.0 - rng.random(k)                      # (0, 1]
        rr = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        rr = rr[np.isfinite(rr) & (rr <= r_max)]
        take = min(len(rr), k)
        r[filled:filled + take] = rr[:take]
        filled += take
    cz = 2.0 * rng.random(n) - 1.0
    ph = 2.0 * np.pi * rng.random(n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    m = np.full(n, 1.0 / max(n, 1))
    return r * sz * np.cos(ph), r * sz * np.sin(ph), r * cz, m


def masses(n: int, seed: int, kind: str = "unequal") -> np.ndarray:
    """Per-particle masses of total |m| = 1.

    * "equal": 1/N each;
    * "unequal": positive, log-uniform over two decades (ratio up to 100);
    * "mixed": the same magnitudes with seeded random signs (about half
      negative), as for charges; the sum of the signed masses is near zero.
    """
    if kind == "equal":
        return np.full(n, 1.0 / max(n, 1))
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-1.0, 1.0, n)
    mag /= max(mag.sum(), 1e-300)
    if kind == "unequal":
        return mag
    if kind == "mixed":
        return np.where(rng.random(n) < 0.5, -mag, mag)
    raise ValueError(f"unknown mass kind {kind!r}")


def sample_targets(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices in [0, n), sorted."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def make(dist: str, n: int, seed: int):
    if dist == "uniform":
        return uniform(n, seed)
    if dist == "plummer":
        return plummer(n, seed)
    raise ValueError(f"unknown distribution {dist!r}")


def request_trace(n_req: int = 2000, seed: int = 5, rate: float = 200.0,
                  n_lo: float = 1e3, n_hi: float = 1e6, orders=(6, 8, 10)):
    """Serving trace: N log-uniform in [n_lo, n_hi], half uniform / half
    Plummer (seeded permutation), order p uniform over `orders`, Poisson
    arrivals at `rate` per second; request i draws its data with seed
    1e6 + i."""
    rng = np.random.default_rng(seed)
    ns = np.rint(10.0 ** rng.uniform(np.log10(n_lo), np.log10(n_hi),
                                     n_req)).astype(np.int64)
    dist = np.array(["uniform"] * (n_req // 2) +
                    ["plummer"] * (n_req - n_req // 2))
    dist = dist[rng.permutation(n_req)]
    ps = rng.choice(np.asarray(orders), size=n_req)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    return [dict(i=i, n=int(ns[i]), dist=str(dist[i]), p=int(ps[i]),
                 t_arrive=float(arrivals[i]), seed=int(1_000_000 + i))
            for i in range(n_req)]
