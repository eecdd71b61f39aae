#!/usr/bin/env python3
"""Throughput of the FMM hot path on one MI355X.

Workload: N = 1,048,576 particles uniform in the unit cube, masses 1/N,
p = 10 expansion terms, leaves of at most 64 particles, FP32 far and near
field (M2M/L2L in FP64).  One step = the whole path from device-resident
FP64 inputs to device-resident outputs: tree build (bounding cube, keys,
sort, cells), FMM lists, P2M, M2M, M2L, L2L, L2P, P2P and the scatter back
to the caller's order.  The value is N / (time per step).

Printed as one JSON line; see the keys below.  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp32_TFs": 157.3,   # FP32 vector (dual-issue/packed) and FP32 matrix
    "fp64_TFs": 78.6,
    "bf16_TFs": 2500.0,
    "fp16_TFs": 2500.0,
}
P2P_FLOPS = 21  # per pair: the paper's 19 (Sec. 5.1) plus the potential
# Issue ceiling of the FP32 P2P loop (the AMD assembly of this build): per
# pair 14 VALU operations (3 sub, 5 fma, 4 mul, 1 max, 1 add), one v_rsq_f32
# at a quarter of the rate, and a quarter of an instruction of loop
# overhead: 18.25 issue slots of a 16-lane SIMD, 4 SIMDs per CU, 256 CUs,
# 2.4 GHz
P2P_SLOTS = 14 + 4 + 0.25
P2P_CEILING = 256 * 4 * 16 * 2.4e9 / P2P_SLOTS


def p2p_pairs(tree) -> int:
    """sum over leaves of (targets in leaf) x (sources in its U list)."""
    cells = tree.cells().cpu().numpy()
    off, items = (a.cpu().numpy() for a in tree.fmm_list(0))
    cnt = cells[:, 5].astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(cnt[items])])
    src = cs[off[1:]] - cs[off[:-1]]
    leaf = cells[:, 8] == 0
    return int(np.sum(cnt[leaf] * src[leaf]))


# FP32 flops one M2P evaluation executes (FMA = 2), by expansion order p,
# counted from the instruction mix of the treecode far-field kernel's inner
# loop: irregular solid harmonics to degree p by recurrence, the potential
# and the three gradient contractions, the scaled offset and rsqrt; at p = 3
# the Cartesian quadrupole form (monopole, dipole and traceless quadrupole
# with their analytic gradient)
M2P_FLOPS = {1: 48, 2: 106, 3: 80, 4: 334, 5: 499, 6: 698, 7: 931, 8: 1198}


def treecode_work(tree):
    """(M2P evaluations, P2P pairs) of the Barnes-Hut group lists: per leaf,
    (its particles) x (accepted cells), and (its particles) x (particles of
    the leaves in its near list)."""
    cells = tree.cells().cpu().numpy()
    cnt = cells[:, 5].astype(np.int64)
    leaf = cells[:, 8] == 0
    aoff = tree.bh_list(0, offsets_only=True).cpu().numpy()
    boff, bitems = (a.cpu().numpy() for a in tree.bh_list(1))
    alen = (aoff[1:] - aoff[:-1]).astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(cnt[bitems])])
    src = cs[boff[1:]] - cs[boff[:-1]]
    return int(np.sum(cnt[leaf] * alen[leaf])), int(np.sum(cnt[leaf] * src[leaf]))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(x, y, z, m, p: int, leaf: int, dist: str, ntarget: int = 1024,
                 ntarget_1core: int = 16):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload, on all host threads and on one: the whole tree and upward pass
    for all N particles, the downward pass for the cells the sampled target
    particles need (their leaves and ancestors), and their far and near
    field; and the direct sum at the same targets.  The whole-problem time
    is estimated from the measured phases: tree + upward + the downward
    scaled by (all V pairs / V pairs of the needed cells) + the per-target
    evaluation times N; `value` = N / that time."""
    from oracle import oracle as O
    from paper_1010_1482_amd import workloads as W
    n = len(x)
    threads = O.num_threads()
    tg = W.sample_targets(n, ntarget, 7)
    t0 = time.perf_counter()
    T = O.Tree(x, y, z, leaf)
    t_tree = time.perf_counter() - t0
    # V pairs of the cells the targets need, against all V pairs
    c = T.cells()
    voff, _ = T.list(1)
    vlen = voff[1:] - voff[:-1]
    inv = np.empty(n, dtype=np.int64)
    inv[T.perm()] = np.arange(n)
    leaf_of = np.empty(n, dtype=np.int64)
    for ci in np.nonzero(c["nchild"] == 0)[0]:
        leaf_of[c["first"][ci]:c["first"][ci] + c["count"][ci]] = ci
    need = set()
    for s_ in inv[tg]:
        ci = int(leaf_of[s_])
        while ci >= 0 and ci not in need:
            need.add(ci)
            ci = int(c["parent"][ci])
    v_need = int(vlen[list(need)].sum())
    v_all = int(vlen.sum())

    def fmm_leg(k):
        t0 = time.perf_counter()
        T.fmm(m, p, targets=tg[:k])
        wall = time.perf_counter() - t0
        up, down, ev = O.fmm_phase_seconds()
        return wall, up, down, ev

    def direct_leg(k):
        t0 = time.perf_counter()
        O.direct(x, y, z, m, targets=tg[:k])
        return time.perf_counter() - t0

    wall, up, down, ev = fmm_leg(ntarget)
    td = direct_leg(ntarget)
    full = t_tree + up + down * v_all / max(v_need, 1) + ev / ntarget * n
    # one core: fewer targets (the downward of their cells only)
    O.set_num_threads(1)
    try:
        need1 = set()
        for s_ in inv[tg[:ntarget_1core]]:
            ci = int(leaf_of[s_])
            while ci >= 0 and ci not in need1:
                need1.add(ci)
                ci = int(c["parent"][ci])
        v_need1 = int(vlen[list(need1)].sum())
        t0 = time.perf_counter()
        T1 = O.Tree(x, y, z, leaf)
        t_tree1 = time.perf_counter() - t0
        del T1
        wall1, up1, down1, ev1 = fmm_leg(ntarget_1core)
        td1 = direct_leg(ntarget_1core)
    finally:
        O.set_num_threads(threads)
    full1 = t_tree1 + up1 + down1 * v_all / max(v_need1, 1) + ev1 / ntarget_1core * n
    return {"value": n / full, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": (f"oracle FMM (FP64, Eq. 4 M2L as complex sums) on the same N={n} "
                       f"{dist} particles, p={p}, leaf<={leaf}: tree and upward pass for all "
                       f"N, downward for the cells {ntarget} seeded targets need "
                       f"({v_need} of {v_all} V pairs), their far and near field; "
                       f"value = N / (tree + upward + downward x {v_all}/{v_need} + "
                       f"evaluation per target x N), an estimate from measured phases"),
            "fmm_all_threads": {"targets": ntarget, "wall_s": wall, "tree_s": t_tree,
                                "upward_s": up, "downward_s": down, "evaluation_s": ev,
                                "full_n_estimate_s": full},
            "fmm_one_core": {"targets": ntarget_1core, "wall_s": wall1, "tree_s": t_tree1,
                             "upward_s": up1, "downward_s": down1, "evaluation_s": ev1,
                             "full_n_estimate_s": full1, "particles_per_s": n / full1},
            "direct_all_threads": {"targets": ntarget, "s": td,
                                   "pairs_per_s": ntarget * n / td,
                                   "full_n_estimate_s": td * n / ntarget},
            "direct_one_core": {"targets": ntarget_1core, "s": td1,
                                "pairs_per_s": ntarget_1core * n / td1,
                                "full_n_estimate_s": td1 * n / ntarget_1core}}


def serving_bench(n_req: int, slots: int, budget_gb: float, plain: bool):
    """The serving form: the seeded request trace (N log-uniform in
    [1e3, 1e6], half uniform / half Plummer, p in {6, 8, 10}, Poisson arrivals
    at 200 req/s), served with continuous batching on `slots` streams under an
    HBM budget, and (plain=True) one request at a time for comparison.
    Inputs are generated on the host before the clock starts."""
    from paper_1010_1482_amd import serve
    from paper_1010_1482_amd import workloads as W
    trace = W.request_trace(n_req=n_req, seed=5)
    data = {e["i"]: W.make(e["dist"], e["n"], e["seed"]) for e in trace}

    def reqs():
        rs = serve.trace_requests(trace)
        for r in rs:
            r.make_inputs = (lambda i=r.rid: data[i])
        return rs

    # warm up code objects and the allocator on a few requests
    warm = serve.Server(int(budget_gb * 2 ** 30), slots, serve.HipExecutor(slots),
                        serve.hip_footprint)
    warm.run(reqs()[:2 * slots], realtime=False)
    out = {}
    modes = [("batched", slots)] + ([("one_at_a_time", 1)] if plain else [])
    for name, k in modes:
        srv = serve.Server(int(budget_gb * 2 ** 30), k, serve.HipExecutor(k),
                           serve.hip_footprint)
        t0 = time.perf_counter()
        done = srv.run(reqs(), realtime=True)
        out[name] = serve.summarize(done, time.perf_counter() - t0)
        out[name]["slots"] = k
    off = sum(e["n"] for e in trace) / trace[-1]["t_arrive"]
    out["offered_particles_per_s"] = off
    out["trace"] = (f"{n_req} requests, N log-uniform [1e3, 1e6], half uniform / half "
                    f"Plummer, p in {{6, 8, 10}}, Poisson 200 req/s, FP32 FMM, leaf<=64, "
                    f"HBM budget {budget_gb} GiB")
    return out


def source_digest(path: str) -> str:
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic(kernel: str, config: str):
    """HBM bytes per launch of `kernel` on `config` from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a
    plain copy), or None when the kernel's source changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config}_counters.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-json:"):
                rec = json.loads(line.split(":", 1)[1])
                if rec.get("source_sha") != source_digest(rec["source"]):
                    return None
                return rec
    return None


def copy_probe(mib: int = 1024) -> int:
    """A plain device copy of known size, for calibrating the FETCH_SIZE and
    WRITE_SIZE counters (rocprofv3 --pmc ... -- python3 bench.py --copy-probe)."""
    import torch
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}), flush=True)
    return 0


def measure(args, prec_name, x, y, z, m, dev, steps, warmup, accuracy, p=None, leaf=None,
            method=None, theta=None, ref=None, host_copies=True):
    """Time `steps` whole steps (after `warmup`) of one configuration
    (p, leaf, method and theta default to the command line's); `ref` is a
    precomputed (targets, FP64 direct sum there) for the accuracy check."""
    import torch
    from paper_1010_1482_amd import hfmm
    from paper_1010_1482_amd import workloads as W
    n = len(x)
    p = args.p if p is None else p
    leaf = args.leaf if leaf is None else leaf
    theta = args.theta if theta is None else theta
    prec = hfmm.PRECISIONS[prec_name]
    meth = hfmm.METHODS[args.method if method is None else method]
    xd, yd, zd, md = (torch.from_numpy(a).to(dev) for a in (x, y, z, m))
    dt = hfmm.out_dtype(prec)
    out = tuple(torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    hold = {"arena": torch.empty(hfmm.arena_bytes(n, 0, leaf, p, meth, prec),
                                 dtype=torch.uint8, device=dev)}
    hfmm.set_timing(True)

    def step(sizing=False):
        try:
            t = hfmm.Tree(xd, yd, zd, leaf_max=leaf, arena=hold["arena"])
        except hfmm.HfmmError as e:
            if sizing and e.code == hfmm.E_NOMEM:
                return hfmm._lib().hfmm_last_required_bytes()
            raise
        try:
            t.upward(md, p, meth, prec)
            t.evaluate(theta=theta, out=out)
        except hfmm.HfmmError as e:
            if sizing and e.code == hfmm.E_NOMEM:
                return t.required_bytes()
            raise
        return t

    # sizing pass, outside the clock: the arena estimate can fall short for
    # clustered data (long treecode lists); grow it to what the call needed
    for _ in range(4):
        need = step(sizing=True)
        if not isinstance(need, int):
            break
        hold["arena"] = None
        torch.cuda.synchronize()
        hold["arena"] = torch.empty(int(need * 1.25) + (64 << 20), dtype=torch.uint8,
                                    device=dev)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, phases = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        tr = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        phases.append(tr.stats()["phase_ms"])
    t1 = time.perf_counter()
    ms = (t1 - t0) / steps * 1e3
    res = {"ms_per_step": ms, "value": n / (ms * 1e-3),
           "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                          "p99": float(np.percentile(lat, 99) * 1e3)},
           "phase_ms": {k: float(np.mean([d[k] for d in phases])) for k in phases[-1]},
           "stats": tr.stats(), "tree": tr}
    if host_copies:
        # the same step with the inputs copied in from pinned host memory and
        # the outputs copied back (reported beside `value`, never as it)
        hx = [torch.from_numpy(a).pin_memory() for a in (x, y, z, m)]
        ho = [torch.empty(n, dtype=dt, pin_memory=True) for _ in range(4)]
        nh = max(1, min(steps, 3))
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        for _ in range(nh):
            for d, h in zip((xd, yd, zd, md), hx):
                d.copy_(h, non_blocking=True)
            step()
            for h, d in zip(ho, out):
                h.copy_(d, non_blocking=True)
            torch.cuda.synchronize()
        hms = (time.perf_counter() - h0) / nh * 1e3
        res["with_host_copies"] = {"ms_per_step": hms, "particles_per_s": n / (hms * 1e-3),
                                   "note": "FP64 inputs host->device and outputs "
                                           "device->host (pinned) inside each step"}
    if accuracy:
        from oracle import oracle as O
        if ref is None:
            tg = W.sample_targets(n, args.accuracy_targets, 100 + args.seed)
            ref = (tg, O.direct(x, y, z, m, targets=tg))
        tg, ref = ref
        got = [o.double().cpu().numpy()[tg] for o in out]
        res["accuracy"] = {
            "targets": len(tg), "reference": "FP64 oracle direct sum over all N",
            "rel_l2_phi": O.rel_l2(got[0], ref[0]),
            "rel_l2_acc": O.rel_l2(np.stack(got[1:]), np.stack(ref[1:]))}
    return res


def p2p_line(pairs, ms, peak):
    """P2P throughput against the FP32 vector peak (21 flops per pair) and
    against the issue ceiling of its instruction mix."""
    if not pairs or not ms:
        return None
    rate = pairs / (ms * 1e-3)
    tf = rate * P2P_FLOPS / 1e12
    return {"pairs": pairs, "ms": ms, "pairs_per_s": rate, "tflops": tf,
            "frac_of_vector_peak": tf / peak, "instruction_mix_ceiling_pairs_per_s": P2P_CEILING,
            "frac_of_instruction_mix_ceiling": rate / P2P_CEILING,
            "note": "21 flops per pair (the paper's 19 plus the potential); ceiling: 14 VALU "
                    "+ 1 quarter-rate v_rsq_f32 + 0.25 overhead = 18.25 issue slots per pair"}


def clustered_and_4m_forms(args, dev):
    """The two 4M workloads measured beside the headline one (3 timed steps
    after one warm-up each, accuracy against the FP64 oracle direct sum at
    the same number of seeded targets):
    N = 4,194,304 Plummer (scale radius 1, truncated at 20), equal masses,
    leaf <= 32: FMM p = 8, Barnes-Hut treecode theta = 0.5 with quadrupole
    moments (p = 3), both in FP32 and FP64, and the treecode over the FMM
    lists (p = 3, FP32);
    N = 4,194,304 uniform, p = 12, leaf <= 64: the FMM with the M2L in FP32
    and in each low-precision form."""
    from oracle import oracle as O
    from paper_1010_1482_amd import workloads as W
    n = 1 << 22
    keep = ("build", "lists", "upward", "m2l", "downward", "far", "p2p", "bh")
    out = {}

    def run(x, y, z, m, ref, prec, **kw):
        r = measure(args, prec, x, y, z, m, dev, 3, 1, True, ref=ref, host_copies=False,
                    **kw)
        return {"value": r["value"], "ms_per_step": r["ms_per_step"],
                "rel_l2_acc": r["accuracy"]["rel_l2_acc"],
                "rel_l2_phi": r["accuracy"]["rel_l2_phi"],
                "phase_ms": {k: v for k, v in r["phase_ms"].items() if k in keep and v}}

    x, y, z, m = W.plummer(n, 3)
    tg = W.sample_targets(n, args.accuracy_targets, 103)
    ref = (tg, O.direct(x, y, z, m, targets=tg))
    res = {}
    for name, meth, p in (("fmm_p8", "fmm", 8), ("treecode_theta0.5_p3", "treecode", 3)):
        for prec in ("fp32", "fp64"):
            res[f"{name}_{prec}"] = run(x, y, z, m, ref, prec, p=p, leaf=32, method=meth,
                                        theta=0.5)
    res["treecode_fmmlist_p3_fp32"] = run(x, y, z, m, ref, "fp32", p=3, leaf=32,
                                          method="treecode_fmmlist")
    out["plummer_4M_leaf32"] = {
        "workload": "N=4194304 Plummer sphere (a=1, r<=20), masses 1/N, leaf<=32",
        "results": res}
    del x, y, z, m
    x, y, z, m = W.uniform(n, 4)
    tg = W.sample_targets(n, args.accuracy_targets, 104)
    ref = (tg, O.direct(x, y, z, m, targets=tg))
    res = {}
    for prec in ("fp32", "bf16x3", "fp16x3", "bf16", "fp16"):
        res[prec] = run(x, y, z, m, ref, prec, p=12, leaf=64, method="fmm")
    out["uniform_4M_p12"] = {
        "workload": "FMM N=4194304 uniform unit cube, masses 1/N, p=12, leaf<=64, M2L "
                    "forms (P2P FP32, M2M/L2L FP64)",
        "results": res}
    return out


def leapfrog_rate(args, x, y, z, m, dev):
    """Time steps of the N-body loop (kick-drift-kick leapfrog, one force
    evaluation per step) at the same configuration, from rest, once with a
    new tree every step and once with the tree kept while every particle
    stays within 1/2 + 1/16 leaf sides of its leaf's centre: per-step time =
    (time of K steps - time of 0 steps) / K, the 0-step call being the
    initial evaluation both make.  The near field is softened
    (eps^2 = 1e-6) and dt = 1e-4: unsoftened close pairs of a random cube
    would be flung out in the first steps and blow up the root cell."""
    import torch
    from paper_1010_1482_amd import hfmm
    k = args.leapfrog_steps
    xd, yd, zd, md = (torch.from_numpy(a).to(dev) for a in (x, y, z, m))
    v = [torch.zeros_like(xd) for _ in range(3)]
    dt, eps2 = 1e-4, 1e-6
    res = {"steps": k, "dt": dt, "eps2": eps2}
    for name, slack in (("new_tree", -1.0), ("kept_tree", 1.0 / 16.0)):
        kw = dict(p=args.p, method=args.method, precision=args.precision, leaf_max=args.leaf,
                  theta=args.theta, eps2=eps2, slack=slack)
        hfmm.leapfrog(xd.clone(), yd.clone(), zd.clone(), *[a.clone() for a in v], md, dt, 1,
                      **kw)  # warm-up
        times, info = {}, {}
        for steps in (0, k):
            pos = [a.clone() for a in (xd, yd, zd)]
            vel = [a.clone() for a in v]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hfmm.leapfrog(*pos, *vel, md, dt, steps, info=info, **kw)
            torch.cuda.synchronize()
            times[steps] = time.perf_counter() - t0
        ms = (times[k] - times[0]) / k * 1e3
        res[name] = {"slack": slack, "ms_per_step": ms, "trees_built": info.get("builds"),
                     "particle_steps_per_s": len(x) / (ms * 1e-3)}
    res["note"] = ("kick-drift-kick leapfrog from rest; new_tree builds a tree per step, "
                   "kept_tree refits the first one while the particles stay within "
                   "1/2 + slack leaf sides of their leaves' centres")
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--dist", default="uniform")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--accuracy-targets", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--method", default="fmm", choices=["fmm", "treecode", "treecode_fmmlist"])
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--leapfrog-steps", type=int, default=5,
                    help="time this many steps of the N-body loop (0 skips it)")
    ap.add_argument("--forms", default="bf16x3,fp16x3,bf16,fp16",
                    help="M2L precision forms measured beside the headline one "
                         "('' for none)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving trace (0 skips the serving form)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--no-serve-plain", action="store_true",
                    help="skip serving the trace one request at a time")
    ap.add_argument("--no-4m", action="store_true",
                    help="skip the 4M Plummer and 4M p=12 workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain copy of known size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        return 2
    if args.copy_probe:
        return copy_probe()

    import torch
    from paper_1010_1482_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    n, p, leaf = args.n, args.p, args.leaf
    x, y, z, m = W.make(args.dist, n, args.seed)
    r = measure(args, args.precision, x, y, z, m, dev, args.steps, args.warmup,
                not args.no_accuracy)
    tr, stats, ph = r["tree"], r["stats"], r["phase_ms"]
    workload = (f"FMM N={n} {args.dist} unit cube, masses 1/N, p={p}, leaf<={leaf}, "
                f"{args.precision}") if args.method == "fmm" else (
                f"treecode N={n} {args.dist}, p={p}, theta={args.theta}, leaf<={leaf}, "
                f"{args.precision}") if args.method == "treecode" else (
                f"treecode over the FMM lists N={n} {args.dist}, p={p}, leaf<={leaf}, "
                f"{args.precision}")

    # Roofline of the dominant kernel: algorithmic work per launch over the
    # kernel's own device time (HIP events on its stream, averaged over the
    # timed steps).  M2L: 2 p^4 flops per V pair (the real p^2 x p^2
    # operator), on the matrix cores of its operand type.  P2P: 21 flops per
    # pair (the paper's count plus the potential) on the FP32 vector units.
    alu_peak = PEAK["fp64_TFs"] if args.precision == "fp64" else PEAK["fp32_TFs"]
    m2p_evals = 0
    if args.method == "fmm":
        pairs = p2p_pairs(tr)
    else:
        m2p_evals, pairs = treecode_work(tr)
    m2l_pairs = stats["m2l_pairs"]
    m2l_peak = {"fp32": PEAK["fp32_TFs"], "fp64": PEAK["fp64_TFs"]}.get(
        args.precision, PEAK["bf16_TFs"])
    cand = {
        "m2l": (ph.get("m2l", 0.0), 2.0 * p ** 4 * m2l_pairs, "mfma", m2l_peak),
        "p2p": (ph.get("p2p", 0.0), P2P_FLOPS * pairs, "alu", alu_peak),
    }
    if args.method != "fmm" and p in M2P_FLOPS:
        cand["far"] = (ph.get("far", 0.0), M2P_FLOPS[p] * m2p_evals, "alu", alu_peak)
    dom = max(cand, key=lambda k: cand[k][0])
    dms, dwork, dbound, dpeak = cand[dom]
    ach = dwork / (dms * 1e-3) / 1e12
    m2l_kernel = "k_m2l_valu" if p > (11 if args.precision == "fp64" else 13) else "k_m2l_mma"
    far_kernel = "k_treecode_far3" if p == 3 else "k_treecode_far"
    kname = {"m2l": m2l_kernel, "p2p": "k_p2p", "far": far_kernel}[dom]
    cfg = f"{args.dist}_{n >> 20}M_p{p}_{args.precision}" if n >= 1 << 20 else \
        f"{args.dist}_{n}_p{p}_{args.precision}"
    rec = recorded_traffic(kname, cfg)
    roof = {"bound": dbound, "achieved": ach, "peak": dpeak, "unit": "TFLOP/s",
            "frac": ach / dpeak, "traffic": rec["bytes_per_launch"] if rec else None,
            "kernel": kname, "work_per_launch": dwork, "launch_ms": dms}
    if rec:
        roof["traffic_note"] = rec["note"]

    res = {
        "metric": "particles/s, FMM N=1M at rel err<=1e-4 vs FP64; p50/p99 request latency",
        "value": r["value"], "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision != "fp64" else "f64", "data": "synthetic",
        "config": {"workload": workload, "n": n, "p": p, "leaf_max": leaf,
                   "dist": args.dist, "precision": args.precision, "method": args.method},
        "latency_ms": r["latency_ms"],
        "with_host_copies": r["with_host_copies"],
        "direct_equivalent_pairs_per_s": float(n) * float(n) / (r["ms_per_step"] * 1e-3),
        "phase_ms": ph,
        "tree": {"cells": stats["n_cells"], "leaves": stats["n_leaves"],
                 "depth": stats["depth"], "list_u": stats["list_u"],
                 "list_v": stats["list_v"], "list_m2p": stats["list_m2p"],
                 "list_p2p": stats["list_p2p"], "p2p_pairs": pairs,
                 "m2p_evaluations": m2p_evals},
        "p2p_interactions_per_s": pairs / (ph.get("p2p", 1.0) * 1e-3) if pairs else None,
        "p2p": p2p_line(pairs, ph.get("p2p"), alu_peak),
        "m2l_pairs_per_s": m2l_pairs / (ph.get("m2l", 1.0) * 1e-3) if m2l_pairs else None,
        "m2p_evaluations_per_s": (m2p_evals / (ph.get("far", 1.0) * 1e-3)
                                  if m2p_evals else None),
        "roofline": roof,
    }
    if "accuracy" in r:
        res["accuracy"] = r["accuracy"]
    if args.leapfrog_steps > 0:
        res["leapfrog"] = leapfrog_rate(args, x, y, z, m, dev)
    forms = [f for f in args.forms.split(",") if f and f != args.precision]
    if forms and args.method == "fmm":
        res["precision_forms"] = {}
        for f in forms:
            rf = measure(args, f, x, y, z, m, dev, args.steps, args.warmup,
                         not args.no_accuracy)
            res["precision_forms"][f] = {
                "value": rf["value"], "ms_per_step": rf["ms_per_step"],
                "m2l_ms": rf["phase_ms"].get("m2l"),
                "rel_l2_acc": rf.get("accuracy", {}).get("rel_l2_acc"),
                "rel_l2_phi": rf.get("accuracy", {}).get("rel_l2_phi")}
    if args.serve_requests > 0:
        res["serving"] = serving_bench(args.serve_requests, args.serve_slots,
                                       args.serve_budget_gb, not args.no_serve_plain)
    if not args.no_4m:
        res["workloads_4M"] = clustered_and_4m_forms(args, dev)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(x, y, z, m, p, leaf, args.dist)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
