"""Write the liquid-state fixture from the oracle alone.

The 1000-molecule system of the default workload (density 1.2, T = 0.75, the
lowest equilibrated temperature of Sec. III.B; checkerboard k = 2, n_c = 4,
seed 1) is advanced by the serial FP64 oracle for 500 sweeps from its seeded
lattice start, the warm-up after which the benchmark starts timing, and its
state is stored.  Tests load it to check the engine trial by trial in the
dense-liquid regime (and, tiled 2 x 2 x 2, at 8000 molecules).  Nothing here
runs the GPU engine.

    python tests/golden/make_liquid_state.py   (about two minutes)
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402

OUT = os.path.join(HERE, "liquid_1000_T0.75_sweep500.npz")
M, T, K, NC, SEED, SWEEPS = 1000, 0.75, 2, 4, 1, 500


def main():
    oracle.build()
    s = oracle.System(oracle.Params(n_molecules=M, temperature=T, colours_per_axis=K,
                                    cells_per_side=NC, seed=SEED))
    s.sweep_checkerboard(SWEEPS)
    st = s.get_state()
    np.savez_compressed(OUT, com=st["com"], quat=st["quat"], types=st["types"],
                        sweep=np.uint64(st["sweep"]), e_acc=np.float64(st["e_acc"]),
                        energy=np.float64(s.energy()),
                        recipe=np.array(f"oracle, M={M} T={T} k={K} n_c={NC} seed={SEED}, "
                                        f"{SWEEPS} checkerboard sweeps from the lattice start"))
    print(OUT, "E/M =", s.energy() / M)


if __name__ == "__main__":
    main()
