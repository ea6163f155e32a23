"""Parity in the dense liquid, at full size, inside batches, and statistics.

The liquid starts come from a fixture written by the oracle alone
(tests/golden/make_liquid_state.py: the 1000-molecule system at T = 0.75,
500 sweeps from its lattice start); the 8000-molecule start tiles it 2 x 2 x 2.
Trial-by-trial bars as in test_gpu_parity: proposals identical, dE within
1e-12 S (FP64) or 1e-5 S (FP32), decisions identical outside the near-tie
band (then the engine is re-seeded from the oracle's state).
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle  # noqa: E402
from paper_2506_21290_amd import flipmc  # noqa: E402

from test_gpu_parity import compare_sweep, gparams, oparams  # noqa: E402

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "liquid_1000_T0.75_sweep500.npz")


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def liquid(tile=1):
    """The oracle-made liquid state, optionally tiled tile^3 times (the box
    side of tile^3 * 1000 molecules is tile times that of 1000)."""
    f = np.load(FIXTURE)
    com, quat, types, sweep = f["com"], f["quat"], f["types"], int(f["sweep"])
    if tile > 1:
        L1 = oracle.box_length(1000)
        L = oracle.box_length(1000 * tile ** 3)
        shifts = np.array([(i, j, k) for k in range(tile) for j in range(tile) for i in range(tile)])
        com = np.concatenate([com + L1 * s for s in shifts])
        com = np.mod(com, L)
        quat = np.tile(quat, (tile ** 3, 1))
        types = np.tile(types, (tile ** 3, 1))
    return com, quat, types, sweep


def parity_from(gp, op, start, n_sweeps, fp32):
    """Both sides from the same start, n sweeps compared trial by trial."""
    com, quat, types, sweep = start
    g = flipmc.System(gp)
    g.set_state(com, quat, types, sweep)
    o = oracle.System(op, lattice=False)
    o.set_state(com, quat, types, sweep)
    resyncs = trials = 0
    for _ in range(n_sweeps):
        g.decision_log(1)
        g.sweep(1)
        lg = g.read_log()
        lo = o.sweep_checkerboard(1, log=True)
        trials += int((lo["exited"] == 0).sum())
        if compare_sweep(lg, lo, fp32):
            st = o.get_state()
            g.set_state(st["com"], st["quat"], st["types"], st["sweep"], st["e_acc"])
            resyncs += 1
        elif not fp32:
            sg, so = g.get_state(), o.get_state()
            assert np.array_equal(sg["com"], so["com"])
            assert np.array_equal(sg["types"], so["types"])
            assert np.max(np.abs(sg["quat"] - so["quat"])) < 1e-13
    return g, o, trials, resyncs


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("flags,engine", [(0, flipmc.MC_ENGINE_LDS),
                                          (flipmc.MC_FLAG_HBM_STATE, flipmc.MC_ENGINE_SPREAD)])
def test_liquid_1000_molecules_every_trial(fp32, flags, engine):
    # the timed configuration (k = 2, n_c = 4, T = 0.75) in its timed regime
    print(f"liquid 1000 fp32={fp32} engine={engine}", flush=True)
    gp = gparams(1000, 0.75, 2, 4, fp32=fp32, flags=flags)
    assert flipmc.mc_engine(gp)[0] == engine
    g, o, trials, resyncs = parity_from(gp, oparams(1000, 0.75, 2, 4), liquid(), 3, fp32)
    assert trials > 2500 and resyncs <= 3


def test_liquid_8000_molecules_every_trial():
    # 8000 molecules at T = 1.1 with the engine's own decomposition (the
    # multi-workgroup engine), FP32 dE, from the tiled liquid
    print("liquid 8000 fp32", flush=True)
    gp = flipmc.mc_params_default(n_molecules=8000, temperature=1.1, seed=1,
                                  precision=flipmc.MC_FP32_DE)
    _, k, nc = flipmc.mc_geometry(gp)
    assert flipmc.mc_engine(gp)[0] == flipmc.MC_ENGINE_SPREAD
    g, o, trials, resyncs = parity_from(gp, oparams(8000, 1.1, k, nc), liquid(2), 2, True)
    assert trials > 12000 and resyncs <= 3


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("flags", [0, flipmc.MC_FLAG_HBM_STATE | flipmc.MC_FLAG_SINGLE_WORKGROUP])
def test_near_list_overflow_path(fp32, flags):
    # k = 2, n_c = 2 (cells of side 6.79): every molecule of the box lies
    # within reach of every cell, far beyond the near list's 192 entries, so
    # every cell takes the overflow path (all stencil molecules evaluated)
    print(f"overflow fp32={fp32} flags={flags}", flush=True)
    gp = gparams(1000, 0.75, 2, 2, fp32=fp32, flags=flags, resum_interval=0, gofr_interval=0)
    g, o, trials, resyncs = parity_from(gp, oparams(1000, 0.75, 2, 2), liquid(), 2, fp32)
    assert trials > 1500 and resyncs <= 3
    assert g.observables()["near_overflows"] == 8 * 2  # 8 cells per sweep, 2 sweeps


def test_overflow_counter_is_zero_without_overflow():
    gp = gparams(216, 1.0, 3, 6, fp32=True, seed=5)
    g = flipmc.System(gp)
    g.sweep(5)
    assert g.observables()["near_overflows"] == 0


@pytest.mark.parametrize("fp32", [False, True])
def test_batched_systems_match_the_oracle(fp32):
    # systems advanced inside a batch (several per launch, slices of a few
    # sweeps) against the oracle run alone: every trial, and in FP64 the final
    # states bitwise.  The decision log is enabled before the systems join.
    n = 8
    cases = [(216, 1.0, 3, 6, 3), (343, 2.0, 3, 6, 4), (512, 0.8, 2, 4, 5)]
    b = flipmc.Batch(4, flipmc.MC_FP32_DE if fp32 else flipmc.MC_FP64)
    systems = []
    for M, T, k, nc, seed in cases:
        s = flipmc.System(gparams(M, T, k, nc, fp32=fp32, seed=seed), stream=b.stream)
        s.decision_log(n)
        b.add(s, n)
        systems.append(s)
    done = 0
    while done < len(cases):
        b.run(20_000)  # slices of about 20 sweeps of a 1000-molecule system
        done += len(b.poll())
    for s, (M, T, k, nc, seed) in zip(systems, cases):
        lg = s.read_log()
        o = oracle.System(oparams(M, T, k, nc, seed=seed))
        for sw in range(n):
            lo = o.sweep_checkerboard(1, log=True)
            if compare_sweep(lg[sw * M:(sw + 1) * M], lo, fp32):
                break  # a near tie: the chains part from here
        else:
            sg, so = s.get_state(), o.get_state()
            assert sg["sweep"] == so["sweep"] == n
            if not fp32:
                assert np.array_equal(sg["com"], so["com"])
                assert np.array_equal(sg["types"], so["types"])
                assert np.max(np.abs(sg["quat"] - so["quat"])) < 1e-13


def test_replica_batch_launch_sampled_against_the_oracle():
    # the 256-replica set in the launch the bench times (one batch, FP32 dE,
    # every replica on its workgroup, re-sums and C_2 samples inside the
    # sweep kernel), a few sweeps: 8 replicas sampled 2 per size, trial by
    # trial against the oracle run alone on the same seeds and decomposition
    from paper_2506_21290_amd import workloads

    n = 3
    jobs = workloads.replica_set(256, sweeps=n, seed=1)
    by_size = {}
    for j in jobs:
        by_size.setdefault(j.n_molecules, []).append(j)
    sample = [j for m in sorted(by_size) for j in by_size[m][:2]]
    print(f"replica batch: {len(jobs)} replicas, sampled {[j.index for j in sample]}", flush=True)
    b = flipmc.Batch(256, flipmc.MC_FP32_DE)
    systems = {}
    for j in jobs:
        p = flipmc.mc_params_default(n_molecules=j.n_molecules, temperature=j.temperature,
                                     precision=flipmc.MC_FP32_DE, seed=j.seed, resum_interval=100,
                                     obs_interval=10, gofr_interval=0)
        s = flipmc.System(p, stream=b.stream)
        if j in sample:
            s.decision_log(n)
        b.add(s, j.sweeps)
        systems[j.index] = (s, p)
    launches = done = 0
    while done < len(jobs):
        launches += b.run(0) > 0
        done += len(b.poll())
    assert launches == 1
    compared = 0
    for j in sample:
        s, p = systems[j.index]
        _, k, nc = flipmc.mc_geometry(p)
        lg = s.read_log()
        o = oracle.System(oparams(j.n_molecules, j.temperature, k, nc, seed=j.seed))
        M = j.n_molecules
        for sw in range(n):
            lo = o.sweep_checkerboard(1, log=True)
            compared += 1
            if compare_sweep(lg[sw * M:(sw + 1) * M], lo, True):
                break  # a near tie: the chains part from here
    assert compared >= 2 * len(sample)
    for s, _ in systems.values():
        s.close()
    b.close()
