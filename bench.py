#!/usr/bin/env python3
"""Throughput of the MLMC finite-element hot path on one MI355X.

Workload: the single-level batched solve of 1024 samples on the 64^3 Q1 mesh
(M = 64 KL modes, correlation length 0.3, sigma^2 = 1, f = 1, homogeneous
Dirichlet data, QoI = mean of u over [1/4, 3/4]^3), each sample solved by
GMG-preconditioned CG to true relative residual 1e-8.  One step = one pass of
the whole path over one batch: Philox draw of xi, MFMA KLE field, multigrid
hierarchy, batched solve, QoI and level statistics.  Every step draws fresh
samples (sample indices advance by the batch size).

Prints one JSON line:  value = sample-DOFs solved per second (interior
unknowns (n-1)^3 summed over the solves of the timed steps / wall time).
Also reported: the fp64 path on the same workload, the roofline of the
dominant kernel (algorithmic bytes / event-timed duration on the library's
stream), and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s

# HBM bytes per launch of each kernel class, from two rocprofv3 counter runs
# of this bench command (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, the factors
# read off a 1 GiB copy kernel in the same runs), averaged over the launches of
# the event-timed pass like the roofline's achieved rate (same samples and
# tuning, so the same launch mix).  They stand
# for the kernels only while the device sources (the .hip launchers and the
# headers they include) and this tuning are unchanged; the per-kernel table and
# the commands are in the committed counter summary.
TRAFFIC = {
    "profile": "profiles/batched-64cube-1024_hbm_traffic.txt",
    "tuning": {"zvar_fp32": 2, "zvar_fp64": 2, "vsmall_fp32": 16, "vsmall_fp64": 8, "cheb_degree": 1, "max_batch": 256, "graph_batch": 1, "fuse": 447, "lanes": 4},
    "sha256_16": {"common.hpp": "84103274fa2b6280", "grid.hpp": "b240c0e6cdf9fd1c", "kernels.hpp": "037887b66ba1ce4b", "krylov.hip": "cdf3168b8678bec1", "stencil.hip": "e58c30d0c1b92bf7"},
    "bytes_per_launch": {
        "PCG_APPLY (f32)": 1654327456,
        "CHEB_PROLONG (f32)": 522266031,
        "RESIDUAL_RESTRICT (f32)": 395964223,
        "PCG_UPDATE (f32)": 792139355,
        "TRUE_RESIDUAL (f64)": 2168757237,
    },
}


# the tuning choices a class's launch mix depends on, with the bits that matter
# (None: the whole value); the coarse V-cycle and the smoothing degree set the
# iteration (and so launch) counts, the LDS-engine bit of zvar selects the
# apply's engine, the DIRECTION and REFINE fusion bits its form.  Fusion bit 128 (the
# whole solve of 4^3 / 8^3 meshes) never acts on the 64^3 workload.
FUSE_64 = 127
TRAFFIC_TUNING_KEYS = {
    "PCG_UPDATE (f32)": {"max_batch": None, "vsmall_fp32": None, "cheb_degree": None, "fuse": FUSE_64},
    "PCG_APPLY (f32)": {"max_batch": None, "vsmall_fp32": None, "cheb_degree": None, "zvar_fp32": 2, "fuse": 32 | 4},
    "TRUE_RESIDUAL (f64)": {"max_batch": None, "vsmall_fp32": None, "cheb_degree": None, "zvar_fp64": 2,
                            "fuse": FUSE_64},
}


def measured_traffic(kernel: str, tuning: dict):
    """Counter-measured HBM bytes per launch of `kernel`, or None when the
    kernel sources or the tuning differ from those the counters were taken on."""
    import hashlib
    by = TRAFFIC["bytes_per_launch"].get(kernel)
    if by is None:
        return None
    keys = TRAFFIC_TUNING_KEYS.get(kernel, {k: (FUSE_64 if k == "fuse" else None) for k in TRAFFIC["tuning"]})
    for k, mask in keys.items():
        a, b = tuning.get(k), TRAFFIC["tuning"][k]
        if (a != b) if mask is None else (a is None or (a & mask) != (b & mask)):
            return None
    src = os.path.join(ROOT, "paper_2111_11788_amd", "csrc")
    for name, want in TRAFFIC["sha256_16"].items():
        with open(os.path.join(src, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != want:
                return None
    return by
METRIC = "MLMC sample-DOFs solved/s at rel.res 1e-8"


def _cpu_worker(args):
    seed_first, wl_name = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import mlmc as omlmc
    import workloads
    wl = {w.name: w for w in workloads.ALL}[wl_name]
    t = time.perf_counter()
    y, qf, qc, it = omlmc.sample_level(wl, 0, seed_first, 1)
    return time.perf_counter() - t, float(qf[0]), int(it[0])


def cpu_baseline(wl, samples: int):
    """The oracle (assembled CSR + Jacobi-PCG, fp64) on `samples` samples of
    the workload, one single-threaded process per core."""
    import multiprocessing as mp
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(samples, avail, 16))
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(i, wl.name) for i in range(samples)])
    wall = time.perf_counter() - t0
    dofs = (wl.n0 - 1) ** 3
    return {"value": samples * dofs / wall, "unit": "sample-DOFs/s", "cores": cores, "kind": "oracle",
            "qoi": [r[1] for r in res],
            "sample": f"{samples} samples of the 64^3 workload (level 0, indices 0..{samples - 1}), "
                      f"assembled CSR + Jacobi-PCG to rel.res 1e-8, {cores} processes x 1 thread",
            "wall_s": round(wall, 3), "mean_sample_s": round(sum(r[0] for r in res) / samples, 3),
            "cpu": platform.processor() or platform.machine(), "cpu_count": os.cpu_count(), "affinity": avail}


def copy_probe(mib: int):
    """A plain copy kernel of known size (reads and writes `mib` MiB once):
    the yardstick that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def run_gpu(wl, precision: int, steps: int, warmup: int, batch: int, profile: bool, autotune: bool = False,
            tuning: dict | None = None, probe_mib: int = 0, validate: bool = False):
    import numpy as np
    import torch
    import paper_2111_11788_amd as mm

    ctx = mm.Context(wl, precision=precision, max_batch=batch)
    dofs = (wl.n0 - 1) ** 3
    tuning_in = tuning
    if tuning:
        ctx.set_tuning(**{k: v for k, v in tuning.items() if k != "seconds"})
        tuning = ctx.tuning()
    else:
        tuning = ctx.autotune(0, batch) if autotune else ctx.tuning()
    if probe_mib:
        copy_probe(probe_mib)
    check = None
    if validate:
        # untimed pass over sample indices 0 .. batch-1 with the same tuning:
        # the QoIs the oracle values (stored goldens, the CPU baseline's) are
        # compared with
        _, qf0, _, it0 = ctx.sample_level(0, 0, batch)
        check = {"qf": [float(x) for x in qf0], "iters_max": int(it0.max())}
    first = batch if validate else 0
    for _ in range(warmup):
        ctx.sample_level(0, first, batch)
        first += batch
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for _ in range(steps):
        y, qf, qc, it = ctx.sample_level(0, first, batch)
        its.append(it)
        first += batch
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"value": steps * batch * dofs / wall, "ms_per_step": 1e3 * wall / steps,
           "iters_mean": float(np.mean(its)), "iters_max": int(np.max(its)), "tuning": tuning, "check": check}
    if profile:
        ctx.set_profiling(True)
        ctx.sample_level(0, first, batch)
        rows = []
        for name in mm.KERNELS:
            for p in (0, 1):
                n, ms, by = ctx.kernel_time(name, p)
                if n:
                    rows.append((ms, name, "f64" if p == 0 else "f32", n, by))
        ctx.set_profiling(False)
        rows.sort(reverse=True)
        ms, name, dt, n, by = rows[0]
        avg_ms = ms / n
        achieved = by / n / (avg_ms * 1e-3) / 1e9
        label = f"{name} ({dt})"
        traffic = measured_traffic(label, tuning)
        out["roofline"] = {"bound": "hbm", "kernel": label, "achieved": round(achieved, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": traffic, "launches": n, "avg_launch_us": round(1e3 * avg_ms, 2),
                           "bytes_per_launch": by / n,
                           "traffic_over_algorithmic": None if traffic is None else round(traffic / (by / n), 4),
                           "traffic_source": TRAFFIC["profile"] if traffic is not None else None}
        out["kernels"] = [{"kernel": f"{r[1]} ({r[2]})", "ms": round(r[0], 3), "launches": r[3],
                           "GBps": round(r[4] / (r[0] * 1e-3) / 1e9, 1) if r[0] > 0 else None} for r in rows[:12]]
    ctx.close()
    return out


def qoi_vs_oracle(check, golden: str, cpu=None):
    """Relative QoI error of the GPU's samples 0 .. batch-1 against the stored
    oracle values (Jacobi-PCG to 1e-12) and the CPU baseline's own solves (to
    the bench tolerance 1e-8)."""
    if not check:
        return None
    out = {}
    gp = os.path.join(ROOT, "tests", "golden", golden)
    if os.path.exists(gp):
        gold = json.load(open(gp))
        rel = [abs(check["qf"][g["index"]] - g["q"]) / abs(g["q"]) for g in gold["samples"]
               if g["index"] < len(check["qf"])]
        out["stored_oracle"] = {"samples": [g["index"] for g in gold["samples"]], "oracle_rtol": gold["rtol"],
                                "max_rel": max(rel) if rel else None, "source": f"tests/golden/{golden}"}
    if cpu and cpu.get("qoi"):
        rel = [abs(check["qf"][i] - q) / abs(q) for i, q in enumerate(cpu["qoi"])]
        out["cpu_baseline_oracle"] = {"samples": f"0..{len(rel) - 1}", "oracle_rtol": 1e-8, "max_rel": max(rel)}
    return out


# the 256^3 leg's tuning: the autotuner's pick on that workload with 16
# samples per call: four concurrent batches of 4, Chebyshev degree 1, two
# captured PCG iterations per convergence check, the prolongation fusion off
# (the pre-smoothing and residual-update bits, set, act only with it, so the
# kernels are those of the earlier pick, which ran the 16 samples as one
# batch): about 93 against 98 ms per 16 samples
C5_TUNING = {"zvar_fp32": 2, "zvar_fp64": 2, "vsmall_fp32": 16, "vsmall_fp64": 8, "cheb_degree": 1, "max_batch": 4,
             "graph_batch": 2, "fuse": 510, "field": 0, "lanes": 4}


# the fp64 leg's tuning: the autotuner's pick for the same workload in fp64
# (Chebyshev degree 1, four concurrent batches of 256, eager launches): about
# 74 against 90 ms per step at the library's defaults (degree 2, one batch)
FP64_TUNING = {"zvar_fp32": 6, "zvar_fp64": 2, "vsmall_fp32": 16, "vsmall_fp64": 8, "cheb_degree": 1,
               "max_batch": 256, "graph_batch": 0, "fuse": 443, "field": 0, "lanes": 4}


def run_c5_leg(steps: int = 3, B: int = 16, tuning=None):
    """The largest single-GPU workload (256^3, sigma^2 = 2, correlation length
    0.1, M = 512), B samples per call with the given tuning (None: the
    library's defaults): sample-DOFs/s, ms per call, iterations, the dominant
    kernel's HBM roofline and the QoI error against the stored oracle values
    of samples 0 and 1."""
    import numpy as np
    import torch
    import paper_2111_11788_amd as mm
    import workloads
    wl = workloads.C5
    ctx = mm.Context(wl, max_batch=B)
    tuning_in = tuning
    if tuning:
        ctx.set_tuning(**{k: v for k, v in tuning.items() if k != "seconds"})
    _, qf0, _, it0 = ctx.sample_level(0, 0, B)      # untimed: carving, graphs, the QoI check
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for k in range(steps):
        _, _, _, it = ctx.sample_level(0, B * (k + 1), B)
        its.append(it)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ctx.set_profiling(True)
    ctx.sample_level(0, B * (steps + 1), B)
    rows = []
    for name in mm.KERNELS:
        for p in (0, 1):
            n, ms, by = ctx.kernel_time(name, p)
            if n:
                rows.append((ms, name, "f64" if p == 0 else "f32", n, by))
    ctx.set_profiling(False)
    tuning = ctx.tuning()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    rows.sort(reverse=True)
    ms, name, dt, n, by = rows[0]
    achieved = by / n / (ms / n * 1e-3) / 1e9
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "c5_stress_qoi.json")))
    err = [{"sample": g["index"], "rel_err": abs(float(qf0[g["index"]]) - g["q"]) / abs(g["q"])}
           for g in gold["samples"]]
    dofs = (wl.n0 - 1) ** 3
    return {"workload": wl.name, "mesh": "256^3", "samples_per_batch": B, "dofs_per_sample": dofs,
            "value": B * dofs / wall, "unit": "sample-DOFs/s", "ms_per_batch": 1e3 * wall,
            "iterations": {"mean": float(np.mean(its)), "max": int(np.max(its))},
            "roofline": {"bound": "hbm", "kernel": f"{name} ({dt})", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "launches": n, "avg_launch_us": round(1e3 * ms / n, 2), "bytes_per_launch": by / n},
            "kernels": [{"kernel": f"{r[1]} ({r[2]})", "ms": round(r[0], 3), "launches": r[3],
                         "GBps": round(r[4] / (r[0] * 1e-3) / 1e9, 1) if r[0] > 0 else None} for r in rows[:8]],
            "qoi_vs_oracle": {"samples": err, "oracle_rtol": gold["rtol"], "max_rel": max(e["rel_err"] for e in err),
                              "source": "tests/golden/c5_stress_qoi.json"},
            "tuning": tuning, "tuning_source": "pinned autotuner pick" if tuning_in else "library defaults",
            "steps": steps}


def _round_tuning(ctx, args):
    """--lanes and --no-pack of the sampling rounds."""
    import paper_2111_11788_amd as mm
    if args.lanes:
        ctx.set_tuning(lanes=args.lanes)
    if args.no_pack:
        ctx.set_tuning(fuse=ctx.tuning()["fuse"] & ~mm.FUSE_PACK)


def run_c3(args):
    """Time-to-eps of the 5-level MLMC workload (pilot + optimal allocation)."""
    import numpy as np
    import torch
    import paper_2111_11788_amd as mm
    import workloads
    wl = workloads.C3

    def one(eps, seed=None):
        ctx = mm.Context(wl, max_batch=1024, arena_bytes=40 << 30, cheb_degree=args.cheb_degree,
                         **({} if seed is None else {"seed": seed}))
        _round_tuning(ctx, args)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nl, est = ctx.estimate(eps, n_pilot=32, cost_model=0, max_rounds=3)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.close()
        dofs = sum(int(nl[l]) * ((wl.n(l) - 1) ** 3 + ((wl.n(l) // 2 - 1) ** 3 if l else 0))
                   for l in range(wl.levels))
        return {"eps": eps, "seconds": wall, "n_per_level": [int(x) for x in nl], "qtilde": est["qtilde"],
                "var_qtilde": est["var_qtilde"], "eps2_over_2": eps ** 2 / 2,
                "var_per_level": [l["var"] for l in est["levels"]],
                "cost_per_sample_s": [l["cost"] for l in est["levels"]], "sample_dofs": dofs,
                "sample_dofs_per_s": dofs / wall, "lanes": est["lanes"], "active_ratio": est["active_ratio"]}

    # process set-up outside the timed runs: one untimed run on another seed
    # loads the kernels' code objects (the HIP runtime loads them at first
    # launch) and the host thread pool
    if not args.no_warm:
        one(wl.eps, seed=wl.seed + 1)
    absolute = one(wl.eps)
    # the relative reading of the same target: eps = 1e-3 |Qtilde|, Qtilde from the absolute run
    relative = one(wl.eps * abs(absolute["qtilde"]))

    def adaptive(eps, l0):
        """Adaptive MLMC from levels 0..l0: L grows by eq. mlmc_num_levels (the
        configured meshes cap it), N_l by eq. mlmc_num_samples."""
        ctx = mm.Context(wl, max_batch=1024, arena_bytes=40 << 30, cheb_degree=args.cheb_degree)
        _round_tuning(ctx, args)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nl, info, est = ctx.estimate_adaptive(eps, l0=l0, n_pilot=32, cost_model=0, max_rounds=10)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.close()
        L = info["L"]
        dofs = sum(int(nl[l]) * ((wl.n(l) - 1) ** 3 + ((wl.n(l) // 2 - 1) ** 3 if l else 0)) for l in range(L + 1))
        return {"eps": eps, "l0": l0, "seconds": wall, "L": L, "meshes_used": [wl.n(l) for l in range(L + 1)],
                "n_per_level": [int(nl[l]) for l in range(L + 1)], "qtilde": est["qtilde"],
                "var_qtilde": est["var_qtilde"], "bias": info["bias"], "err": info["err"], "alpha": info["alpha"],
                "beta": info["beta"], "rounds": info["rounds"], "sample_dofs_per_s": dofs / wall,
                "lanes": est["lanes"], "active_ratio": est["active_ratio"]}

    adapt = adaptive(wl.eps * abs(absolute["qtilde"]), 1)
    return {"metric": "time-to-eps", "value": absolute["seconds"], "unit": "s", "higher_is_better": False,
            "config": {"workload": wl.name, "meshes": [wl.n(l) for l in range(wl.levels)], "eps": wl.eps,
                       "n_pilot": 32, "n_modes": wl.n_modes, "corr_len": wl.corr_len, "precision": "mixed",
                       "cost_model": "measured GPU seconds per sample",
                       "untimed_warm_up": None if args.no_warm else "one run on seed + 1 (code objects, threads)"},
            "absolute": absolute, "relative": relative, "adaptive_relative": adapt, "dtype": "f32+f64",
            "data": "synthetic"}


def run_c4(args):
    """Serving: Poisson arrivals over levels 16^3..256^3 weighted 16^(4-l).

    Saturation is the closed-loop completion rate with `clients` requests kept
    outstanding (each completion is replaced at once by a fresh draw from the
    level law), measured after a warm-up second.  Each open-loop run then
    offers Poisson arrivals at a fraction of it; latency is completion time
    minus scheduled arrival time (the submission lag of this driver plus the
    library's submit-to-completion time), nearest-rank percentiles."""
    import numpy as np
    import torch
    import paper_2111_11788_amd as mm
    import workloads
    wl = workloads.C4
    weights = np.array([16.0 ** (wl.levels - 1 - l) for l in range(wl.levels)])
    weights /= weights.sum()
    slots = [int(x) for x in args.slots.split(",")] if args.slots else [2048, 1024, 128, 8, 2]
    # the bf16 KLE against the fp64 KLE on the same samples (64 per mesh 16^3..64^3)
    kle_check = None
    if wl.precision == 2:
        kle_check = []
        for l in range(3):
            qs = []
            for prec in (1, 2):
                c = mm.Context(wl, precision=prec, max_batch=64)
                _, qf, _, _ = c.sample_level(l, 0, 64)
                qs.append(np.asarray(qf))
                c.close()
                del c
            rel = np.abs(qs[1] - qs[0]) / np.abs(qs[0])
            kle_check.append({"mesh": wl.n(l), "samples": 64, "qoi_rel_dev_max": float(rel.max()),
                              "qoi_rel_dev_mean": float(rel.mean())})
        torch.cuda.empty_cache()
    ctx = mm.Context(wl, arena_bytes=int(args.arena_gb * 2**30), cheb_degree=args.cheb_degree)
    ctx.serve_start(slots)
    rng = np.random.default_rng(4)
    dofs = np.array([(wl.n(l) - 1) ** 3 + ((wl.n(l) // 2 - 1) ** 3 if l else 0) for l in range(wl.levels)],
                    dtype=np.float64)
    next_id = np.zeros(wl.levels, dtype=np.uint64)

    def draw(k):
        lv = rng.choice(wl.levels, size=k, p=weights).astype(np.int32)
        ids = np.empty(k, dtype=np.uint64)
        for l in range(wl.levels):
            m = lv == l
            c = int(m.sum())
            ids[m] = next_id[l] + np.arange(c, dtype=np.uint64)
            next_id[l] += np.uint64(c)
        return lv, ids

    def active_ratio(a, b):
        """A = a / (p t_w) of eq. active_ratio between two serve_stats
        snapshots: slot-seconds in use weighted by each slot's share of the HBM
        budget, over the budget held by all slots times the wall time."""
        num = sum((b["slot_busy_s"][m] - a["slot_busy_s"][m]) * b["slot_bytes"][m] for m in range(16))
        den = sum(b["slots"][m] * b["slot_bytes"][m] for m in range(16)) * (b["uptime_s"] - a["uptime_s"])
        return num / den if den > 0 else None

    def pct(x, q):
        """nearest-rank percentile"""
        xs = np.sort(x)
        return float(xs[max(0, int(np.ceil(q / 100.0 * len(xs))) - 1)])

    # warm-up
    lv, ids = draw(2000)
    ctx.wait(ctx.submit_batch(lv, ids), timeout=600)

    # closed-loop saturation
    clients = args.clients if args.clients else 2 * sum(slots)
    lv, ids = draw(clients)
    ctx.submit_batch(lv, ids)
    outstanding = clients
    t0 = time.perf_counter()
    warm_end, end = t0 + 1.0, t0 + 1.0 + args.sat_seconds
    snap0 = None
    n_done = 0
    dofs_done = 0.0
    while True:
        r = ctx.drain_array(timeout=0.005)
        now = time.perf_counter()
        outstanding -= len(r)
        if now >= warm_end and snap0 is None:
            snap0 = ctx.serve_stats()
        if now >= warm_end and now < end:
            n_done += len(r)
            dofs_done += float(dofs[r["level"]].sum())
        if now >= end:
            break
        if len(r):
            lv, ids = draw(len(r))
            ctx.submit_batch(lv, ids)
            outstanding += len(r)
    snap1 = ctx.serve_stats()
    while outstanding > 0:
        outstanding -= len(ctx.drain_array(timeout=0.05))
    sat_rate = n_done / args.sat_seconds
    sat_dofs = dofs_done / args.sat_seconds
    out = {"metric": "serving p50/p99 latency and sample-DOFs/s", "unit": "s",
           "config": {"workload": wl.name, "meshes": [wl.n(l) for l in range(wl.levels)], "slots": slots,
                      "level_weights": weights.tolist(), "n_modes": wl.n_modes,
                      "kle": "bf16 MFMA, fp32 accumulate" if wl.precision == 2 else "fp64 MFMA",
                      "precision": "mixed"},
           "kle_bf16_vs_fp64": kle_check,
           "saturation": {"requests_per_s": sat_rate, "sample_dofs_per_s": sat_dofs, "clients": clients,
                          "seconds": args.sat_seconds, "kind": "closed loop",
                          "active_ratio": active_ratio(snap0, snap1) if snap0 else None,
                          "lends": snap1["lends"], "reclaims": snap1["reclaims"]},
           "rates": []}
    for frac in (0.5, 0.8, 0.95):
        rate = frac * sat_rate
        n = int(args.serve_seconds * rate)
        lv, ids = draw(n)
        arrive = np.cumsum(rng.exponential(1.0 / rate, size=n))
        tickets = np.zeros(n, dtype=np.uint64)
        lag = np.zeros(n)
        got = []
        s0 = ctx.serve_stats()
        t0 = time.perf_counter()
        i = 0
        while i < n:
            # submit every request whose arrival time has passed, drain finished ones
            now = time.perf_counter() - t0
            j = int(np.searchsorted(arrive, now, side="right"))
            if j > i:
                tickets[i:j] = ctx.submit_batch(lv[i:j], ids[i:j])
                lag[i:j] = (time.perf_counter() - t0) - arrive[i:j]
                i = j
            r = ctx.drain_array(timeout=0.0)
            if len(r):
                got.append(r)
        done = sum(len(g) for g in got)
        while done < n:
            r = ctx.drain_array(timeout=0.05)
            if len(r):
                got.append(r)
                done += len(r)
            if time.perf_counter() - t0 > args.serve_seconds + 600:
                raise TimeoutError("serving run did not finish")
        wall = time.perf_counter() - t0
        s1 = ctx.serve_stats()
        a_ratio = active_ratio(s0, s1)
        res = np.concatenate(got)
        order = np.argsort(tickets)
        pos = order[np.searchsorted(tickets[order], res["ticket"])]
        lat = np.empty(n)
        lat[pos] = res["latency_s"] + lag[pos]
        per = {}
        for l in range(wl.levels):
            m = lv == l
            if m.sum():
                per[str(l)] = {"n": int(m.sum()), "p50_ms": 1e3 * pct(lat[m], 50), "p99_ms": 1e3 * pct(lat[m], 99)}
        out["rates"].append({"fraction_of_saturation": frac, "offered_requests_per_s": rate, "requests": n,
                             "p50_ms": 1e3 * pct(lat, 50), "p99_ms": 1e3 * pct(lat, 99),
                             "max_submit_lag_ms": 1e3 * float(lag.max()),
                             "sample_dofs_per_s": float(dofs[lv].sum()) / wall, "per_level": per,
                             "active_ratio": a_ratio, "lends": s1["lends"] - s0["lends"],
                             "reclaims": s1["reclaims"] - s0["reclaims"],
                             "all_ok": bool((res["status"] == 0).all())})
    ctx.serve_stop()
    return out


def run_c5(args):
    """256^3 stress: batches of 4, 8, 16; iterations, GB/s, QoI vs the oracle on 2 samples."""
    import numpy as np
    import torch
    import paper_2111_11788_amd as mm
    import workloads
    wl = workloads.C5
    gold = None
    gp = os.path.join(ROOT, "tests", "golden", "c5_stress_qoi.json")
    if os.path.exists(gp):
        gold = json.load(open(gp))
    out = {"metric": "MLMC sample-DOFs solved/s at rel.res 1e-8", "unit": "sample-DOFs/s",
           "config": {"workload": wl.name, "mesh": "256^3", "sigma2": wl.sigma2, "corr_len": wl.corr_len,
                      "n_modes": wl.n_modes, "precision": "mixed"}, "batches": []}
    for B in (4, 8, 16):
        ctx = mm.Context(wl, max_batch=B, cheb_degree=args.cheb_degree)
        tuned = ctx.autotune(0, B) if args.autotune else None
        if tuned is None and args.c5_tuning:
            ctx.set_tuning(**{k: v for k, v in json.loads(args.c5_tuning).items() if k != "seconds"})
            tuned = ctx.tuning()
        y, qf, qc, it = ctx.sample_level(0, 0, B)       # warm-up (carve, graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y, qf, qc, it = ctx.sample_level(0, 0, B)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.set_profiling(True)
        ctx.sample_level(0, 0, B)
        rows = []
        for name in mm.KERNELS:
            for p in (0, 1):
                n, ms, by = ctx.kernel_time(name, p)
                if n:
                    rows.append((ms, name, p, n, by))
        ctx.set_profiling(False)
        rows.sort(reverse=True)
        ms, name, p, n, by = rows[0]
        rec = {"batch": B, "ms": 1e3 * wall, "sample_dofs_per_s": B * 255 ** 3 / wall,
               "iters": [int(x) for x in it], "dominant": f"{name} ({'f32' if p else 'f64'})", "tuning": tuned,
               "dominant_GBps": by / (ms * 1e-3) / 1e9}
        if gold:
            rec["qoi_vs_oracle"] = [{"sample": g["index"], "gpu": float(qf[g["index"]]), "oracle": g["q"],
                                     "rel_err": abs(float(qf[g["index"]]) - g["q"]) / abs(g["q"])}
                                    for g in gold["samples"]]
        out["batches"].append(rec)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    return out


def run_pause(args):
    """Pause-model scheduler stress (Sec. 5.1 benchmark): active ratio A(p) of
    eq. active_ratio for short / medium / long models, three spreads and
    batch sampling, on P = 2048 workgroup slots with task widths 1, 8, 64 (the
    8 / 64 / 512-core partitions scaled by 1/8) and N_l = C (1024, 64, 4)."""
    import workloads
    import paper_2111_11788_amd as mm
    C = args.pause_c
    counts = [C * 1024, C * 64, C * 4]
    widths = [1, 8, 64]
    P = 2048
    ctx = mm.Context(workloads.C1, arena_bytes=64 << 20)
    out = {"metric": "pause-model active ratio A(p)", "unit": "fraction", "higher_is_better": True,
           "config": {"workload": "pause model", "capacity_slots": P, "widths": widths, "counts": counts,
                      "law": "U(mu - sqrt(3) sigma, mu + sqrt(3) sigma)"}, "runs": []}
    ctx.pause_model([8], [1], 10.0, 0.0, P)            # warm-up: module load, first launches
    runs = [("short", 10.0, 0.2, 1), ("medium", 1000.0, 0.2, 1), ("long", 100000.0, 0.2, 1),
            ("medium", 1000.0, 0.5 / 3 ** 0.5, 1), ("medium", 1000.0, 0.01, 1),
            ("short", 10.0, 0.2, 8), ("medium", 1000.0, 0.2, 8)]
    for name, mu, rel_sigma, batch in runs:
        r, ticks, done = ctx.pause_model(counts, widths, mu, rel_sigma * mu, P, batch)
        ideal_wall = r["active_slot_s"] / (P * r["ideal_ratio"]) if r["ideal_ratio"] > 0 else 0.0
        out["runs"].append({"model": name, "mu_us": mu, "sigma_over_mu": rel_sigma, "batch": batch,
                            "tasks": r["tasks"], "steps": r["steps"], "wall_s": r["wall_s"],
                            "ideal_wall_s": ideal_wall, "A": r["ratio"], "A_ideal": r["ideal_ratio"],
                            "overhead_us_per_step": 1e6 * (r["wall_s"] - ideal_wall) / max(1, r["steps"]),
                            "measured_over_scheduled": r["measured_slot_s"] / r["active_slot_s"]})
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--precision", choices=["mixed", "fp64", "bf16kle"], default="mixed",
                    help="mixed: fp32 multigrid in fp64 refinement; fp64; bf16kle: mixed with the KLE on bf16 MFMA")
    ap.add_argument("--mode", choices=["c2", "c3", "c4", "c5", "pause"], default="c2",
                    help="c2: the throughput line (default); c3: time-to-eps; c4: serving; c5: 256^3 stress; "
                    "pause: pause-model scheduler stress")
    ap.add_argument("--pause-c", type=int, default=4, help="pause: sample multiplier C of N_l = C N*_l")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune before timing (default: the pinned tuning the HBM counters were taken with, "
                    "itself the autotuner's pick on this workload)")
    ap.add_argument("--tuning", default="", help="JSON tuning to apply instead of autotuning "
                    "(e.g. the 'tuning' object of an earlier line)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain copy of this many MiB first (counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the fp64 comparison run")
    ap.add_argument("--no-c5", action="store_true", help="skip the 256^3 leg of the default line")
    ap.add_argument("--c5-tuning", default="", help="JSON tuning of the 256^3 leg ('{}': library defaults); "
                    "with --mode c5, the tuning of its three batch sizes (default there: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=16)
    ap.add_argument("--slots", default="", help="c4: slots per mesh, comma separated")
    ap.add_argument("--arena-gb", type=float, default=40.0)
    ap.add_argument("--clients", type=int, default=0, help="c4: outstanding requests of the closed loop "
                    "(0: twice the slots)")
    ap.add_argument("--sat-seconds", type=float, default=3.0, help="c4: measured closed-loop seconds")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-warm", action="store_true", help="c3: no untimed run before the timed ones")
    ap.add_argument("--no-pack", action="store_true",
                    help="c3: solves of two levels on one mesh in separate tasks")
    ap.add_argument("--lanes", type=int, default=0,
                    help="c3: concurrent lanes of the sampling rounds (0: the library default)")
    ap.add_argument("--cheb-degree", type=int, default=0,
                    help="c3/c4/c5: Chebyshev smoothing degree (0: the library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); samples are independent, "
              "so a multi-GPU run is N copies of this one on disjoint sample ranges", file=sys.stderr)
        sys.exit(2)
    if args.mode != "c2":
        fn = {"c3": run_c3, "c4": run_c4, "c5": run_c5, "pause": run_pause}[args.mode]
        print(json.dumps(fn(args)))
        return

    import workloads
    wl = workloads.C2
    prec = {"mixed": 1, "fp64": 0, "bf16kle": 2}[args.precision]
    pinned = FP64_TUNING if prec == 0 else TRAFFIC["tuning"]
    tuning = json.loads(args.tuning) if args.tuning else (None if args.autotune else dict(pinned))
    main_run = run_gpu(wl, prec, args.steps, args.warmup, args.batch, profile=True,
                       autotune=args.autotune and tuning is None, tuning=tuning,
                       probe_mib=args.copy_probe_mib, validate=True)
    fp64 = None
    if prec == 1 and not args.no_fp64:
        fp64 = run_gpu(wl, 0, max(1, args.steps // 2), 1, args.batch, profile=False, tuning=FP64_TUNING,
                       validate=True)
    c5 = None if args.no_c5 else run_c5_leg(tuning=json.loads(args.c5_tuning) if args.c5_tuning else C5_TUNING)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_samples)
    check = qoi_vs_oracle(main_run.get("check"), "c2_batched_qoi.json", cpu)

    line = {
        "metric": METRIC, "value": main_run["value"], "unit": "sample-DOFs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {1: "f32+f64", 0: "f64", 2: "bf16+f32+f64"}[prec], "data": "synthetic",
        "config": {"workload": wl.name, "mesh": f"{wl.n0}^3 Q1 hexahedra", "samples_per_step": args.batch,
                   "dofs_per_sample": (wl.n0 - 1) ** 3, "n_modes": wl.n_modes, "corr_len": wl.corr_len,
                   "sigma2": wl.sigma2, "qoi": "subcube [1/4,3/4]^3 average", "rtol": wl.rtol,
                   "solver": "GMG-PCG (Chebyshev-Jacobi smoothing, V-cycle to 2^3)",
                   "precision": {1: "fp32 GMG-PCG inside fp64 refinement", 0: "fp64",
                                 2: "fp32 GMG-PCG inside fp64 refinement, KLE on bf16 MFMA"}[prec]},
        "iterations": {"mean": main_run["iters_mean"], "max": main_run["iters_max"]},
        "tuning": main_run["tuning"],
        "roofline": main_run.get("roofline"),
        "kernels": main_run.get("kernels"),
        "qoi_vs_oracle": check,
        "fp64_path": None if fp64 is None else {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                                                "iters_mean": fp64["iters_mean"], "tuning": fp64["tuning"],
                                                "qoi_vs_oracle": qoi_vs_oracle(fp64.get("check"),
                                                                               "c2_batched_qoi.json", cpu)},
        "largest_single_gpu_config": c5,
        "cpu_baseline": None if cpu is None else {k: v for k, v in cpu.items() if k != "qoi"},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
