#!/usr/bin/env python3
"""Benchmark of the flip Monte Carlo hot path on one MI355X.

Default workload: 1000 rigid A/B/C triangles at T = 0.75 (the lowest
equilibrated temperature of the paper), density 1.2, seeded lattice start,
checkerboard sweeps with FP32 energy differences and an FP64 re-sum every 100
sweeps; a step is 100 sweeps (one re-sum window) including the cell builds,
the re-sum, E/M samples, the g(r) frame and C_2 samples.  The same run in
plain FP64 is timed beside it, then the first 200 jobs of the serving stream
give the p50/p99 request latency ("serving"), the 8000-molecule system ("c2"),
the 256-replica batch ("c3") and the paper's flexible triangles, one system
and 256 replicas ("flexible"), each report their own roofline, and the
CPU oracle runs on a bounded sample on one core and on all cores
("cpu_baseline").  Prints one JSON line.

Other workloads (--workload): c2, c3, c4 (the serving loop at any job count and
memory budget), tau (relaxation times of flip MC against local MC from
equilibrated states, with the four-point susceptibilities and the Pearson
coefficient), flex (the flexible engine alone, one system of each body and
replicas of the triangles), flex_tau (the same relaxation comparison on the
paper's own flexible triangles) and copy (the HBM calibration of the counter
summaries).
"""
from __future__ import annotations

import argparse
import hashlib
import math
import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "attempted molecule-moves/s on 1 MI355X (+ p50/p99 request latency) vs plain FP64"
FLOP_PER_PAIR_TERM = 25  # 3 sub, 3 mul + 2 fma for r^2, cut-off test, rcp, 3 mul, fma, mul, add, ...
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
SWEEPS_PER_STEP = 100


def progress(msg):
    """A line on stderr when a stage of a long workload ends."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


RIGID_SOURCES = ("kernels.hip", "engine.h", "wave.h")
FLEX_SOURCES = ("flex_sweep.h", "engine.h", "wave.h")


def kernel_source_hash(files=RIGID_SOURCES):
    """Hash of kernel sources with comments and blank lines left out (a change
    of wording does not change the kernel the counters were taken on)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2506_21290_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_counters(name):
    """The committed rocprofv3 counter summary of a kernel (HBM bytes per
    launch, VALU busy fraction), or {} when it is missing or was taken on
    another version of the kernel's sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash(tuple(t.get("sources", RIGID_SOURCES))):
        return {}
    return t


def measured_traffic(name):
    return measured_counters(name).get("bytes_per_launch")


def run_system(flipmc, torch, precision, steps, warmup, M=1000, T=0.75, k=0, nc=0, seed=1):
    p = flipmc.mc_params_default(
        n_molecules=M, temperature=T, precision=precision, colours_per_axis=k, cells_per_side=nc,
        seed=seed, resum_interval=100, obs_interval=10, gofr_interval=100, obs_start=0,
        max_samples=8192)
    _, k, nc = flipmc.mc_geometry(p)
    s = flipmc.System(p)
    for _ in range(warmup):
        s.sweep(SWEEPS_PER_STEP)
    torch.cuda.synchronize()
    o0 = s.observables()
    s.timing_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        s.sweep(SWEEPS_PER_STEP)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    tm = s.timing_read()
    o1 = s.observables()
    e, em, drift = s.energy()
    # drift of every re-sum window since the lattice start: the first window
    # holds the lattice transient (E/M of order 10^5), reported on its own
    _, dw = s.samples()
    s.close()
    moves = steps * SWEEPS_PER_STEP * M
    att = [int(o1["attempts"][i] - o0["attempts"][i]) for i in range(3)]
    acc = [int(o1["accepts"][i] - o0["accepts"][i]) for i in range(3)]
    return {
        "ms": ms,
        "moves": moves,
        "moves_per_s": moves / (ms / 1e3),
        "sweep_kernel_ms": tm["sweep_ms"],
        "sweep_launches": tm["sweep_launches"],
        "event_kernel_ms": tm["event_ms"],
        "pair_terms": int(o1["pair_terms"] - o0["pair_terms"]),
        "pair_tests": int(o1["pair_tests"] - o0["pair_tests"]),
        "exits": int(o1["exits"] - o0["exits"]),
        "near_overflows": int(o1["near_overflows"] - o0["near_overflows"]),
        "accept_rate": {kind: (acc[i] / att[i] if att[i] else None)
                        for i, kind in enumerate(["translate", "rotate", "flip"])},
        "energy_per_molecule": em,
        "max_abs_drift_per_window": o1["max_abs_drift"],
        "drift_first_window": float(dw[0]) if len(dw) else None,
        "max_abs_drift_after_first_window": float(np.max(np.abs(dw[1:]))) if len(dw) > 1 else None,
        "last_drift": drift,
        "sweeps_done": int(o1["sweep"]),
        "k": k,
        "n_c": nc,
    }


LIQUID = os.path.join(ROOT, "tests", "golden", "liquid_1000_T0.75_sweep500.npz")


def host_cpu():
    """(logical CPUs visible to this process, model name of the host CPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def _oracle_replica(seconds, seed_offset=0):
    """Sweeps of the oracle on the 1000-molecule workload from its liquid
    state at sweep 500 (the warm-up the GPU leg also runs), for `seconds`;
    returns (attempted moves, elapsed s).  One replica per process."""
    import numpy as np
    from oracle import oracle

    f = np.load(LIQUID)
    s = oracle.System(oracle.Params(n_molecules=1000, temperature=0.75, colours_per_axis=2,
                                    cells_per_side=4, seed=1 + seed_offset), lattice=False)
    s.set_state(f["com"], f["quat"], f["types"], int(f["sweep"]))
    n = 0
    t0 = time.perf_counter()
    while True:
        s.sweep_checkerboard(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return n * 1000, dt


def cpu_baseline(seconds, max_procs=16):
    """The serial FP64 oracle on the host: one replica on one core, then one
    replica process per core (up to max_procs) at once."""
    import multiprocessing as mp
    from oracle import oracle

    oracle.build()
    moves, dt = _oracle_replica(seconds)
    one = moves / dt
    ncpu, model = host_cpu()
    procs = max(1, min(ncpu, max_procs))
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.starmap(_oracle_replica, [(seconds, r + 1) for r in range(procs)])
    allc = sum(m / t for m, t in res)
    return {
        "value": one,
        "unit": "molecule-moves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{moves} attempted moves ({moves // 1000} checkerboard sweeps) of the 1000-molecule "
                  f"T=0.75 system from its liquid state at sweep 500 (the GPU leg's warm-up), "
                  f"serial FP64 oracle, {dt:.1f} s",
        "all_cores": {"value": allc, "processes": procs, "cores": procs,
                      "sample": f"{procs} oracle replicas (seeds 2-{procs + 1}), one process each, "
                                f"{seconds:.0f} s each"},
        "nproc": ncpu,
        "cpu_model": model,
    }


def bench_c1(args, flipmc, torch):
    f32 = run_system(flipmc, torch, flipmc.MC_FP32_DE, args.steps, args.warmup)
    f64 = run_system(flipmc, torch, flipmc.MC_FP64, args.steps, args.warmup)
    launches = max(1, f32["sweep_launches"])
    flops = f32["pair_terms"] * FLOP_PER_PAIR_TERM
    kern_s = f32["sweep_kernel_ms"] / 1e3
    achieved = flops / kern_s / 1e12
    traffic = measured_traffic("k_sweeps_c1")
    out = {
        "metric": METRIC,
        "value": f32["moves_per_s"],
        "unit": "molecule-moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "1000 rigid A/B/C triangles (sites 0.9/1.0/1.1, WCA), density 1.2, T=0.75, "
                        f"seeded lattice start, checkerboard k={f32['k']} n_c={f32['n_c']}, FP32 dE + "
                        "FP64 re-sum every 100 sweeps; step = 100 sweeps",
            "molecules": 1000,
            "sweeps_per_step": SWEEPS_PER_STEP,
            "temperature": 0.75,
            "precision": "FP32 dE, FP64 state/accept/re-sum",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_TFLOPS["f32"],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS["f32"],
            "traffic": traffic,
            "kernel": "k_sweeps<float, resident>",
            "cus_used": 1,
            "valu_busy_on_its_cu": measured_counters("k_sweeps_c1").get("valu_busy_on_its_cu"),
            "avg_launch_ms": f32["sweep_kernel_ms"] / launches,
            "flops_per_launch": flops / launches,
            "flop_per_pair_term": FLOP_PER_PAIR_TERM,
        },
        "fp64": {
            "value": f64["moves_per_s"],
            "ms_per_step": f64["ms"] / args.steps,
            "accept_rate": f64["accept_rate"],
            "max_abs_drift_per_window": f64["max_abs_drift_per_window"],
            "drift_first_window": f64["drift_first_window"],
            "max_abs_drift_after_first_window": f64["max_abs_drift_after_first_window"],
            "energy_per_molecule": f64["energy_per_molecule"],
        },
        "fp32_over_fp64": f32["moves_per_s"] / f64["moves_per_s"],
        "pair_interactions_per_s": f32["pair_terms"] / (f32["ms"] / 1e3),
        "candidate_pair_tests_per_s": f32["pair_tests"] / (f32["ms"] / 1e3),
        "accept_rate": f32["accept_rate"],
        "exits_per_move": f32["exits"] / f32["moves"],
        "near_overflows": f32["near_overflows"],
        "energy_per_molecule": f32["energy_per_molecule"],
        "max_abs_drift_per_window": f32["max_abs_drift_per_window"],
        "drift_first_window": f32["drift_first_window"],
        "max_abs_drift_after_first_window": f32["max_abs_drift_after_first_window"],
        "sweeps_done": f32["sweeps_done"],
    }
    if args.serving_jobs > 0:
        # the request latency of the metric: the serving stream, first jobs
        sv = bench_c4(args, flipmc, torch, n_jobs=args.serving_jobs, check_alone=0)
        out["serving"] = {k: sv[k] for k in ("workload", "completed", "p50_latency_s", "p99_latency_s",
                                              "moves_per_s", "wall_s", "peak_concurrent_jobs")}
    if not args.no_sub:
        # the 8000-molecule system and the 256-replica batch, each with the
        # roofline of its own dominant kernel, and the flexible molecules
        out["c2"] = bench_c2(args, flipmc, torch)
        out["c3"] = bench_c3(args, flipmc, torch)
        out["flexible"] = bench_flex(args, flipmc, torch, sweeps=200, bodies=("triangles",), replicas=256)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        out["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
        out["gpu_over_cpu_all_cores"] = out["value"] / out["cpu_baseline"]["all_cores"]["value"]
    return out


def bench_c2(args, flipmc, torch):
    """8000 molecules at T = 1.1 (mid-range), FP32 dE + FP64 re-sum every 100
    sweeps, 100 warm-up + 1000 timed sweeps; decomposition from the engine's
    table."""
    M, T = 8000, 1.1
    p = flipmc.mc_params_default(n_molecules=M, temperature=T, precision=flipmc.MC_FP32_DE,
                                 seed=1, resum_interval=100, obs_interval=10, gofr_interval=0)
    L, k, nc = flipmc.mc_geometry(p)
    resident, lds = flipmc.mc_placement(p)
    s = flipmc.System(p)
    s.sweep(100)
    torch.cuda.synchronize()
    o0 = s.observables()
    s.timing_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    n_sweeps = 1000
    s.sweep(n_sweeps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    tm = s.timing_read()
    o1 = s.observables()
    terms = int(o1["pair_terms"] - o0["pair_terms"])
    overflows = int(o1["near_overflows"] - o0["near_overflows"])
    kern_s = tm["sweep_ms"] / 1e3
    launches = max(1, tm["sweep_launches"])
    s.close()
    # HBM bytes of one 100-sweep launch from the committed counter summary
    # (null when it was taken on other kernel sources)
    traffic = measured_traffic("k_spread_c2")
    _, wg = flipmc.mc_engine(p)
    achieved = terms * FLOP_PER_PAIR_TERM / kern_s / 1e12
    return {
        "workload": "c2: 8000 molecules, T=1.1, FP32 dE + FP64 re-sum every 100 sweeps, 1000 timed sweeps",
        "k": k, "n_c": nc, "resident_in_lds": resident,
        "moves_per_s": M * n_sweeps / (ms / 1e3),
        "pair_interactions_per_s": terms / (ms / 1e3),
        "candidate_pair_tests_per_s": int(o1["pair_tests"] - o0["pair_tests"]) / (ms / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f32"],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f32"],
                     "traffic": traffic, "kernel": "k_spread<float>",
                     "cus_used": wg,
                     "valu_busy_on_its_cus": measured_counters("k_spread_c2").get("valu_busy_on_its_cus"),
                     "hbm_gb_per_s": (traffic * n_sweeps / 100 / kern_s / 1e9) if traffic else None,
                     "avg_launch_ms": tm["sweep_ms"] / launches,
                     "flops_per_launch": terms * FLOP_PER_PAIR_TERM / launches},
        "near_overflows": overflows,
        "ms": ms,
    }


def bench_tau(args, flipmc, torch):
    """Relaxation of flip MC against local MC (the protocol of Sec. III.B-C on
    the rigid molecules): R replicas of the 1000-molecule system, each from its
    own lattice start, are equilibrated by flip MC (p_flip = 0.2) for E sweeps;
    each equilibrated state then starts two runs, one of flip MC and one of
    local MC (p_flip = 0: translations and rotations only, in the same ratio),
    which sample F_s(7.4, t), F_s^cm(5.1, t) and C_2(t) at t in {1, 2, 5} x 10^j
    sweeps from a common origin.  The library forms the ensemble means, chi_4
    (Eq. 10), chi_4^self (Eq. 11), rho (Eq. 13) and the 1/e times (Sec. III.C)
    from the runs' observables (mc_dynamics).  Every stage runs in one batch."""
    M, T, R = 1000, args.tau_temperature, args.tau_replicas
    E, S = args.tau_equilibration, args.tau_sweeps
    b = flipmc.Batch(2 * R, flipmc.MC_FP32_DE)

    def params(seed, pf):
        return flipmc.mc_params_default(n_molecules=M, temperature=T, precision=flipmc.MC_FP32_DE, seed=seed,
                                        p_flip=pf, p_translate=(1.0 - pf) / 2, resum_interval=1000,
                                        obs_interval=0, gofr_interval=0)

    def run_all(systems, n):
        for s in systems:
            b.add(s, n)
        done = 0
        while done < len(systems):
            b.run(0)
            done += len(b.poll())

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flip = [flipmc.System(params(r + 1, 0.2), stream=b.stream) for r in range(R)]
    run_all(flip, E)
    progress(f"tau: {R} replicas equilibrated ({E} sweeps)")
    local = []
    for r, s in enumerate(flip):
        st = s.get_state()
        local.append(flipmc.System(params(R + r + 1, 0.0), com=st["com"], quat=st["quat"], types=st["types"],
                                   stream=b.stream))
    for s in flip + local:
        s.reset_observables()
    run_all(flip + local, S)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"tau: {2 * R} production runs done ({S} sweeps)")
    out = {"workload": f"tau: {R} replicas of {M} molecules, T={T}, FP32 dE; {E} sweeps of flip-MC "
                       f"equilibration, then {S} sweeps each of flip MC and of local MC from the same states",
           "wall_s": wall,
           "moves_per_s": M * (R * E + 2 * R * S) / wall}
    for kind, ss in (("flip", flip), ("local", local)):
        d = flipmc.mc_dynamics([s.obs_struct() for s in ss], M)
        res = {"t": [int(x) for x in d["t"]]}
        for key in ("fs", "fs_cm", "c2"):
            ratio = d["chi4_" + key] / np.maximum(d["chi4s_" + key], 1e-300)
            res[key] = {"mean": d[key].tolist(), "tau": d["tau_" + key],
                        "chi4_over_self_peak": float(np.max(ratio))}
        res["pearson_peak"] = float(np.max(d["rho"]))
        out[kind] = res
        for s in ss:
            s.close()
    b.close()
    out["equilibration_over_tau"] = {key: (E / out["flip"][key]["tau"] if out["flip"][key]["tau"] else None)
                                     for key in ("fs", "fs_cm", "c2")}
    out["speedup"] = {key: (out["local"][key]["tau"] / out["flip"][key]["tau"]
                            if out["local"][key]["tau"] and out["flip"][key]["tau"] else None)
                      for key in ("fs", "fs_cm", "c2")}
    return out


def bench_flex(args, flipmc, torch, sweeps=None, bodies=("triangles", "squares", "tetrahedra"), replicas=None):
    """The paper's own flexible molecules (FENE-bonded A/B/C triangles, Sec.
    II.A) and the squares and tetrahedra of Sec. VII on the flexible engine,
    FP64: attempted atom moves per second after a warm-up from the lattice
    start, with the roofline of the sweep kernel (pair terms x 25 FLOP over
    its launch time, against the FP64 vector peak)."""
    out = {}
    n_sweeps = sweeps or args.flex_sweeps
    replicas = args.flex_replicas if replicas is None else replicas
    counters = measured_counters("k_fx_sweeps_flex")
    for name, g, M, T, rho in (("triangles", flipmc.MC_TRIANGLE, 1000, 0.75, 1.2),
                               ("squares", flipmc.MC_SQUARE, 1000, 1.0, 1.2),
                               ("tetrahedra", flipmc.MC_TETRAHEDRON, 1000, 1.0, 1.2)):
        if name not in bodies:
            continue
        p = flipmc.mcf_params_default(g, n_molecules=M, temperature=T, density=rho, seed=1,
                                      resum_interval=100, gofr_interval=0)
        _, k, nc = flipmc.mcf_geometry(p)
        s = flipmc.FlexSystem(p)
        s.sweep(args.flex_warmup)
        torch.cuda.synchronize()
        o0 = s.observables()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        s.sweep(n_sweeps)
        z.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(z)
        o1 = s.observables()
        e, em, drift = s.energy()
        s.close()
        N = flipmc.SITES[g] * M
        att = o1["attempts"] - o0["attempts"]
        acc = o1["accepts"] - o0["accepts"]
        terms = int(o1["pair_terms"] - o0["pair_terms"])
        achieved = terms * FLOP_PER_PAIR_TERM / (ms / 1e3) / 1e12
        out[name] = {
            "workload": f"{M} flexible {name} ({N} atoms), density {rho}, T={T}, k={k} n_c={nc}, FP64, "
                        f"{args.flex_warmup} warm-up + {n_sweeps} timed sweeps of N attempts",
            "atom_moves_per_s": N * n_sweeps / (ms / 1e3),
            "molecule_equivalent_moves_per_s": M * n_sweeps / (ms / 1e3),
            "accept_rate": {"translate": float(acc[0] / max(1, att[0])), "flip": float(acc[2] / max(1, att[2]))},
            "energy_per_molecule": em,
            "pair_interactions_per_s": terms / (ms / 1e3),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                         "frac": achieved / PEAK_TFLOPS["f64"], "kernel": "k_fx_sweeps", "cus_used": 1,
                         # counters of the 1000 triangles' launches (null for
                         # the other bodies or other kernel sources)
                         "traffic": counters.get("bytes_per_launch") if name == "triangles" else None,
                         "valu_busy_on_its_cu": counters.get("valu_busy_on_its_cu") if name == "triangles" else None},
            "ms": ms,
        }
        progress(f"flex: {name} done")
    if replicas:
        out["replicas"] = bench_flex_replicas(args, flipmc, torch, replicas, n_sweeps)
    return out


def bench_flex_replicas(args, flipmc, torch, R, n_sweeps):
    """R replicas of the 1000 flexible triangles (seeds 1..R) advanced
    together by mcf_sweep_many, one workgroup each: the device-wide rate of
    the flexible engine when the paper's replica averages fill it."""
    M, T, rho = 1000, 0.75, 1.2
    ps = [flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=M, temperature=T, density=rho, seed=r + 1,
                                    resum_interval=100, gofr_interval=0) for r in range(R)]
    systems = [flipmc.FlexSystem(p) for p in ps]
    flipmc.flex_sweep_many(systems, args.flex_warmup)
    torch.cuda.synchronize()
    o0 = [s.observables() for s in systems]
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    flipmc.flex_sweep_many(systems, n_sweeps)
    z.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(z)
    o1 = [s.observables() for s in systems]
    terms = sum(int(b["pair_terms"] - x["pair_terms"]) for x, b in zip(o0, o1))
    for s in systems:
        s.close()
    N = 3 * M
    achieved = terms * FLOP_PER_PAIR_TERM / (ms / 1e3) / 1e12
    # counters of the 256-replica launch (null for another replica count or
    # other kernel sources)
    counted = measured_counters("k_fx_sweeps_flex").get("replicas", {}) if R == 256 else {}
    progress("flex: replicas done")
    return {
        "workload": f"{R} replicas of {M} flexible triangles ({N} atoms each), density {rho}, T={T}, FP64, "
                    f"{args.flex_warmup} warm-up + {n_sweeps} timed sweeps, one launch per event interval",
        "atom_moves_per_s": R * N * n_sweeps / (ms / 1e3),
        "pair_interactions_per_s": terms / (ms / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["f64"], "kernel": "k_fx_sweeps", "cus_used": min(R, 256),
                     "traffic": counted.get("bytes_per_launch"),
                     "valu_busy_on_its_cus": counted.get("valu_busy_on_its_cus")},
        "ms": ms,
    }


def bench_flex_tau(args, flipmc, torch):
    """Relaxation of flip MC against local MC on the paper's own flexible
    triangles (the protocol of Sec. III.B-C): R replicas of 1000 molecules,
    each from its own lattice start, are equilibrated by flip MC (p_flip = 0.2)
    for E sweeps, all replicas advanced together (mcf_sweep_many); each
    equilibrated state then starts one run of flip MC and one of local MC
    (p_flip = 0: atom translations only), which sample F_s(7.4, t) over the
    atoms, F_s^cm(5.1, t) and C_2(t) at t in {1, 2, 5} x 10^j sweeps from a
    common origin.  The library forms the ensemble means, chi_4, chi_4^self,
    rho and the 1/e times (mcf_dynamics)."""
    M, T, R = 1000, args.flex_tau_temperature, args.flex_tau_replicas
    E, S = args.flex_tau_equilibration, args.flex_tau_sweeps
    step = 2000

    def params(seed, pf):
        return flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=M, temperature=T, seed=seed, p_flip=pf,
                                         resum_interval=1000, obs_interval=0, gofr_interval=0)

    def advance(systems, n, what):
        done = 0
        while done < n:
            k = min(step, n - done)
            flipmc.flex_sweep_many(systems, k)
            torch.cuda.synchronize()
            done += k
            progress(f"flex tau: {what} {done} of {n} sweeps")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flip = [flipmc.FlexSystem(params(r + 1, 0.2)) for r in range(R)]
    advance(flip, E, f"{R} replicas equilibrating")
    local = []
    for r, s in enumerate(flip):
        st = s.get_state()
        local.append(flipmc.FlexSystem(params(R + r + 1, 0.0), pos=st["pos"], types=st["types"]))
    for s in flip + local:
        s.reset_observables()
    advance(flip + local, S, f"{2 * R} production runs")
    wall = time.perf_counter() - t0
    N = 3 * M
    out = {"workload": f"flex tau: {R} replicas of {M} flexible triangles ({N} atoms), T={T}, FP64; {E} sweeps "
                       f"of flip-MC equilibration, then {S} sweeps each of flip MC and of local MC from the same "
                       f"states",
           "wall_s": wall,
           "atom_moves_per_s": N * (R * E + 2 * R * S) / wall}
    for kind, ss in (("flip", flip), ("local", local)):
        d = flipmc.mc_dynamics([s.obs_struct() for s in ss], M, atoms_per_molecule=3)
        res = {"t": [int(x) for x in d["t"]]}
        for key in ("fs", "fs_cm", "c2"):
            ratio = d["chi4_" + key] / np.maximum(d["chi4s_" + key], 1e-300)
            res[key] = {"mean": d[key].tolist(), "tau": d["tau_" + key],
                        "chi4_over_self_peak": float(np.max(ratio))}
        res["pearson_peak"] = float(np.max(d["rho"]))
        out[kind] = res
        for s in ss:
            s.close()
    out["equilibration_over_tau"] = {key: (E / out["flip"][key]["tau"] if out["flip"][key]["tau"] else None)
                                     for key in ("fs", "fs_cm", "c2")}
    out["speedup"] = {key: (out["local"][key]["tau"] / out["flip"][key]["tau"]
                            if out["local"][key]["tau"] and out["flip"][key]["tau"] else None)
                      for key in ("fs", "fs_cm", "c2")}
    return out


def bench_c3(args, flipmc, torch):
    """256 independent replicas, M in {216, 512, 1000, 1728}, T over the
    paper's range, FP32 dE, 1000 sweeps each, all advanced by one batch."""
    from paper_2506_21290_amd import workloads

    jobs = workloads.replica_set(256, sweeps=1000, seed=1)
    b = flipmc.Batch(256, flipmc.MC_FP32_DE)
    systems = []
    for j in jobs:
        p = flipmc.mc_params_default(n_molecules=j.n_molecules, temperature=j.temperature,
                                     precision=flipmc.MC_FP32_DE, seed=j.seed,
                                     resum_interval=100, obs_interval=10, gofr_interval=0)
        s = flipmc.System(p, stream=b.stream)
        b.add(s, j.sweeps)
        systems.append(s)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    done = 0
    launches = 0
    while done < len(jobs):
        launches += b.run(0) > 0
        done += len(b.poll())
    stop.record(b.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    moves = sum(j.n_molecules * j.sweeps for j in jobs)
    obs = [s.observables() for s in systems]
    terms = sum(int(o["pair_terms"]) for o in obs)
    overflows = sum(int(o["near_overflows"]) for o in obs)
    achieved = terms * FLOP_PER_PAIR_TERM / (ms / 1e3) / 1e12
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    for s in systems:
        s.close()
    b.close()
    # the same kind of replica alone, plain FP64: a stratified sample of 8
    by_size = {}
    for j in jobs:
        by_size.setdefault(j.n_molecules, []).append(j)
    sample = [by_size[m][i] for m in sorted(by_size) for i in range(min(2, len(by_size[m])))]
    t_seq = 0.0
    m_seq = 0
    for j in sample:
        p = flipmc.mc_params_default(n_molecules=j.n_molecules, temperature=j.temperature,
                                     precision=flipmc.MC_FP64, seed=j.seed, resum_interval=100,
                                     obs_interval=10, gofr_interval=0)
        s = flipmc.System(p)
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        s.sweep(j.sweeps)
        z.record()
        torch.cuda.synchronize()
        t_seq += a.elapsed_time(z) / 1e3
        m_seq += j.n_molecules * j.sweeps
        s.close()
    return {
        "workload": "c3: 256 replicas, M in {216,512,1000,1728}, T in [0.75,3], FP32 dE, 1000 sweeps each",
        "moves_per_s": moves / (ms / 1e3),
        "ms": ms,
        "moves": moves,
        "launches": launches,
        "pair_interactions_per_s": terms / (ms / 1e3),
        "near_overflows": overflows,
        # the batch's run is one launch of the one-workgroup sweep kernel (all
        # 256 replicas, re-sums and C_2 samples inside it): its time is the
        # timed region, measured with events on the batch's stream
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f32"],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f32"],
                     "traffic": measured_traffic("k_sweeps_c3"),
                     "kernel": "k_sweeps<float, resident, inline events>",
                     "cus_used": min(ncu, len(jobs)),
                     "valu_busy": measured_counters("k_sweeps_c3").get("valu_busy"),
                     "avg_launch_ms": ms / max(1, launches),
                     "flops_per_launch": terms * FLOP_PER_PAIR_TERM / max(1, launches)},
        "fp64_one_by_one_moves_per_s": m_seq / t_seq,
        "fp64_sample": f"{len(sample)} replicas (2 per size) run alone in FP64",
    }


def bench_c4(args, flipmc, torch, n_jobs=None, check_alone=None):
    """Poisson stream of sampling jobs served with continuous batching."""
    from paper_2506_21290_amd import serve, workloads

    jobs = workloads.serving_stream(n_jobs=n_jobs or args.jobs, rate=200.0, seed=1, m_max=args.m_max,
                                    s_max=args.s_max)
    cap = None
    if args.policy == "sjf":
        cap = args.max_active or torch.cuda.get_device_properties(0).multi_processor_count
    srv = serve.Server(memory_budget=args.budget, backend=serve.GpuBackend(flipmc.MC_FP32_DE),
                       quantum_moves=args.quantum, policy=args.policy, max_active=cap)
    t0 = time.perf_counter()
    mark = [0]

    def on_done(n):
        if n >= mark[0] + 100 or n == len(jobs):
            mark[0] = n
            progress(f"c4: {n} of {len(jobs)} jobs done, {time.perf_counter() - t0:.1f} s")

    res = srv.serve(jobs, time_limit=args.time_limit, on_done=on_done)
    wall = time.perf_counter() - t0
    lat = np.array([r.latency for r in res])
    moves = sum(r.moves for r in res)
    # the same result alone and in the mix: sampled jobs re-run alone, bitwise
    same = checked = 0
    n_check = args.check_alone if check_alone is None else check_alone
    if n_check:
        by_index = {r.job.index: r for r in res}
        pick = sorted(by_index)[:: max(1, len(by_index) // n_check)][:n_check]
        be = srv.backend
        for i in pick:
            j = by_index[i].job
            s = flipmc.System(serve.job_params(j, flipmc.MC_FP32_DE))
            s.sweep(j.sweeps)
            alone = be.result(j, s)
            s.close()
            mixed = by_index[i]
            checked += 1
            same += (alone["energy_per_molecule"] == mixed.energy_per_molecule and
                     np.array_equal(alone["gofr"], mixed.gofr) and np.array_equal(alone["c2"], mixed.c2))
        progress(f"c4: {same} of {checked} sampled jobs identical alone and in the mix")
    offered = sum(j.n_molecules * j.sweeps for j in jobs) / (jobs[-1].arrival - jobs[0].arrival)
    return {
        "workload": f"c4: {len(jobs)} Poisson jobs at 200/s, M=n^3 log-uniform in [125,{args.m_max}], "
                    f"T in [0.75,3], sweeps log-uniform in [100,{args.s_max}], FP32 dE, memory budget "
                    f"{args.budget / 2**20:g} MiB, admission "
                    + ("in arrival order" if cap is None else f"shortest job first, at most {cap} jobs at once"),
        "completed": len(res),
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "moves_per_s": moves / wall,
        "offered_moves_per_s": offered,
        "wall_s": wall,
        "peak_concurrent_jobs": srv.peak_active,
        "peak_bytes": srv.peak_bytes,
        "budget_bytes": args.budget,
        "launches": srv.launches,
        "alone_vs_mix": {"checked": checked, "bitwise_identical": same},
    }


def bench_copy(args, flipmc, torch):
    """A plain device-to-device copy of a known size: the reference for
    scaling rocprofv3's FETCH_SIZE / WRITE_SIZE counters to HBM bytes."""
    n = 256 << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").random_(0, 255)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    reps = 5
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        dst.copy_(src)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    return {"workload": "copy: 256 MiB device-to-device, 5 repetitions",
            "bytes_read_per_copy": n, "bytes_written_per_copy": n,
            "ms_per_copy": ms, "gb_per_s": 2 * n / (ms / 1e3) / 1e9}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c1",
                    choices=["c1", "c2", "c3", "c4", "tau", "flex", "flex_tau", "copy"])
    ap.add_argument("--tau-temperature", type=float, default=2.2)
    ap.add_argument("--tau-replicas", type=int, default=16)
    ap.add_argument("--tau-equilibration", type=int, default=40000)
    ap.add_argument("--flex-warmup", type=int, default=200)
    ap.add_argument("--flex-sweeps", type=int, default=1000)
    ap.add_argument("--flex-replicas", type=int, default=256,
                    help="flex: replicas of the 1000 flexible triangles advanced together (0: none)")
    ap.add_argument("--tau-sweeps", type=int, default=50000)
    ap.add_argument("--flex-tau-temperature", type=float, default=2.0)
    ap.add_argument("--flex-tau-replicas", type=int, default=16)
    ap.add_argument("--flex-tau-equilibration", type=int, default=20000)
    ap.add_argument("--flex-tau-sweeps", type=int, default=20000)
    ap.add_argument("--jobs", type=int, default=200)
    ap.add_argument("--serving-jobs", type=int, default=200,
                    help="jobs of the serving stream run after the c1 line's own work (0: none)")
    ap.add_argument("--m-max", type=int, default=27000)
    ap.add_argument("--s-max", type=int, default=10000)
    ap.add_argument("--budget", type=int, default=4 << 30)
    ap.add_argument("--quantum", type=int, default=100_000)
    ap.add_argument("--policy", choices=["fifo", "sjf"], default="fifo",
                    help="serving admission: arrival order, or shortest job first")
    ap.add_argument("--max-active", type=int, default=0,
                    help="jobs admitted at once under sjf (0 = the device's compute units)")
    ap.add_argument("--time-limit", type=float, default=None)
    ap.add_argument("--check-alone", type=int, default=20,
                    help="c4: sampled jobs re-run alone and compared with their result in the mix")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-sub", action="store_true", help="leave out the c2 and c3 sub-objects")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": f"--gpus {args.gpus}: this engine runs on one GPU; "
                                   "it has no multi-GPU mode"}))
        sys.exit(2)
    import torch

    from paper_2506_21290_amd import flipmc

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.workload == "c1":
        out = bench_c1(args, flipmc, torch)
    else:
        out = {"c2": bench_c2, "c3": bench_c3, "c4": bench_c4, "tau": bench_tau, "flex": bench_flex,
               "flex_tau": bench_flex_tau, "copy": bench_copy}[args.workload](args, flipmc, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
