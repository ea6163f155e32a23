"""Seeded synthetic workloads: which systems to simulate, not how.

Nothing here computes any part of the method; the functions only draw job
parameters (sizes, temperatures, sweep counts, arrival times) from numpy's
seeded generator, so the engine, the oracle and the benchmarks can share
them.  Temperatures span the paper's flip-MC range T = 0.75 ... 3 (Sec. III.B);
the molecule counts are perfect cubes so every job can start from the seeded
simple-cubic lattice.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

T_LOW, T_HIGH = 0.75, 3.0
REPLICA_SIZES = (216, 512, 1000, 1728)


@dataclass
class Job:
    index: int
    n_molecules: int
    temperature: float
    sweeps: int
    seed: int
    arrival: float = 0.0


def replica_set(n=256, sweeps=1000, seed=1):
    """Uneven replicas: M uniform over 216 / 512 / 1000 / 1728 molecules,
    T uniform over the paper's range, seed r + 1."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(REPLICA_SIZES, size=n)
    temps = rng.uniform(T_LOW, T_HIGH, size=n)
    return [Job(r, int(sizes[r]), float(temps[r]), int(sweeps), r + 1) for r in range(n)]


def serving_stream(n_jobs=2000, rate=200.0, seed=1, m_min=125, m_max=27000, s_min=100,
                   s_max=10000):
    """Poisson arrivals (mean `rate` per second) of sampling jobs with M = n^3
    log-uniform over [m_min, m_max], T uniform over the paper's range and the
    sweep count log-uniform over [s_min, s_max]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrival = np.cumsum(gaps) - gaps[0]
    logm = rng.uniform(np.log(m_min), np.log(m_max), size=n_jobs)
    n = np.clip(np.rint(np.exp(logm) ** (1.0 / 3.0)), round(m_min ** (1 / 3)), round(m_max ** (1 / 3)))
    temps = rng.uniform(T_LOW, T_HIGH, size=n_jobs)
    sweeps = np.rint(np.exp(rng.uniform(np.log(s_min), np.log(s_max), size=n_jobs)))
    return [Job(j, int(n[j]) ** 3, float(temps[j]), int(sweeps[j]), j + 1, float(arrival[j]))
            for j in range(n_jobs)]
