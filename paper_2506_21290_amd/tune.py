"""Autotuner of the checkerboard decomposition and of the molecules per
workgroup.

For a system size M and a precision, every valid (k, n_c) is a correct
sampler with its own trajectory; they differ in speed (colour phases, cells per
wave, neighbour-list length).  For each (k, n_c) the number of workgroups a
sweep runs on (one, or the multi-workgroup engine on a wave per cell of a
colour, or on fewer workgroups with several cells per wave) changes only the
speed: every count gives bitwise the same chain.  The tuner times each
candidate (k, n_c, workgroups) and records the fastest in ``tuned.json`` next
to this file.  ``choose`` reads the table (falling back to the engine's own
model when a size is missing), so a job's decomposition is a fixed function of
(M, precision) and can be reproduced by the oracle.

Run on the GPU:  python -m paper_2506_21290_amd.tune --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import flipmc

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned.json")
PREC_NAME = {flipmc.MC_FP64: "fp64", flipmc.MC_FP32_DE: "fp32"}
_table = None


def candidates(M, precision, per_k=4):
    """Valid (k, n_c) for an M-molecule box at the default density: the
    `per_k` finest grids of each k (coarser grids only lengthen the chains of
    trials inside a cell).  When some of them keep the state in one
    workgroup's LDS, only those: such a system then runs on one workgroup,
    the most efficient use of a compute unit when many jobs share the device
    (a finer grid beyond the LDS would be faster alone on many workgroups)."""
    out = []
    for k in (2, 3):
        ok = []
        for nc in range(k, 41, k):
            p = flipmc.mc_params_default(n_molecules=M, precision=precision,
                                         colours_per_axis=k, cells_per_side=nc)
            try:
                flipmc.mc_geometry(p)
            except flipmc.McError:
                continue
            ok.append((k, nc))
        out += ok[-per_k:]
    resident = []
    for k, nc in out:
        p = flipmc.mc_params_default(n_molecules=M, precision=precision, colours_per_axis=k,
                                     cells_per_side=nc)
        if flipmc.mc_placement(p)[0]:
            resident.append((k, nc))
    return resident or out


def workgroup_counts(M, precision, k, nc):
    """Workgroup counts worth timing for one decomposition: the most its cells
    allow (a wave per cell of a colour), half and a quarter of that, and one
    workgroup when the state fits its LDS."""
    p = flipmc.mc_params_default(n_molecules=M, precision=precision, colours_per_axis=k, cells_per_side=nc,
                                 workgroups=1 << 20)
    _, most = flipmc.mc_engine(p)
    counts = {w for w in (most, most // 2, most // 4) if w >= 2}
    p.workgroups = 1
    if flipmc.mc_placement(p)[0] or not counts:
        counts.add(1)
    return sorted(counts)


def table():
    global _table
    if _table is None:
        _table = {}
        if os.path.exists(TABLE):
            with open(TABLE) as f:
                _table = json.load(f)
    return _table


def choose(M, precision):
    """(k, n_c, workgroups) for M molecules: the tuned entry, else (0, 0, 0) =
    the engine's model."""
    entry = table().get(PREC_NAME[precision], {}).get(str(M))
    if entry:
        return int(entry["k"]), int(entry["n_c"]), int(entry.get("tuned_workgroups", 0))
    return 0, 0, 0


def time_candidate(M, precision, k, nc, sweeps, T=1.0, workgroups=0):
    import torch

    p = flipmc.mc_params_default(n_molecules=M, temperature=T, precision=precision,
                                 colours_per_axis=k, cells_per_side=nc, resum_interval=0,
                                 obs_interval=0, gofr_interval=0, workgroups=workgroups)
    s = flipmc.System(p)
    s.sweep(max(5, sweeps // 5))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(sweeps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / sweeps


def tune(sizes, precisions, budget_moves=600_000):
    result = {}
    for prec in precisions:
        name = PREC_NAME[prec]
        result[name] = {}
        for M in sizes:
            sweeps = max(10, min(200, budget_moves // M))
            timed = []
            for k, nc in candidates(M, prec):
                for wg in workgroup_counts(M, prec, k, nc):
                    dt = time_candidate(M, prec, k, nc, sweeps, workgroups=wg)
                    timed.append((dt, k, nc, wg))
                    print(f"{name} M={M} k={k} n_c={nc} workgroups={wg}: {dt * 1e6:.1f} us/sweep", flush=True)
            dt, k, nc, wg = min(timed)
            p = flipmc.mc_params_default(n_molecules=M, precision=prec, colours_per_axis=k,
                                         cells_per_side=nc, workgroups=wg)
            engine, used = flipmc.mc_engine(p)
            result[name][str(M)] = {"k": k, "n_c": nc, "tuned_workgroups": wg, "us_per_sweep": dt * 1e6,
                                    "moves_per_s": M / dt, "engine": engine, "workgroups": used,
                                    "molecules_per_workgroup": M / used}
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default=",".join(str(n ** 3) for n in range(4, 31)))
    ap.add_argument("--precisions", default="fp32")
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    sizes = [int(x) for x in args.sizes.split(",")]
    precs = [{"fp32": flipmc.MC_FP32_DE, "fp64": flipmc.MC_FP64}[x] for x in args.precisions.split(",")]
    res = tune(sizes, precs)
    old = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
    for name, entries in res.items():
        old.setdefault(name, {}).update(entries)
    with open(args.out, "w") as f:
        json.dump(old, f, indent=1, sort_keys=True)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
