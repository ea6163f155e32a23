"""Continuous-batching sampling server on one GPU.

Requests are sampling jobs (M molecules at temperature T for S sweeps).  Their
configurations stay resident in HBM for the job's life; a job is admitted as
soon as a slot and enough of the memory budget are free, and every launch
advances all admitted jobs by a time slice (``quantum_moves`` attempted moves
per job), so jobs that arrive while others run join the next launch and their
work overlaps on the device.  Systems whose working set fits one workgroup's
LDS go to one batch, larger ones to a second batch on a second stream, so the
two kinds of launch run side by side.

Each finished job returns E/M (mean over the second half of its sweeps), g(r)
(frames over the second half) and C_2(t) (Sec. III, Eq. 3 and Eq. 7).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import flipmc


@dataclass
class Result:
    job: object
    latency: float        # done - arrival (s)
    wait: float           # admitted - arrival (s)
    energy_per_molecule: float
    gofr_r: np.ndarray
    gofr: np.ndarray
    c2_t: np.ndarray
    c2: np.ndarray
    moves: int
    accept: dict = field(default_factory=dict)


def job_params(job, precision):
    S = job.sweeps
    gofr_every = max(10, (S // 2) // 5 // 10 * 10)
    return flipmc.mc_params_default(
        n_molecules=job.n_molecules, temperature=job.temperature, precision=precision,
        seed=job.seed, resum_interval=100, obs_interval=10, gofr_interval=gofr_every,
        obs_start=S // 2, max_samples=max(16, S // 10 + 2))


def gofr_normalised(obs, n_sites, box):
    """Eq. (3): counts / (frames N rho 4 pi r^2 dr) with the exact shell volume."""
    nb = len(obs["gofr_all"])
    dr = obs["gofr_dr"]
    r = np.arange(nb + 1) * dr
    shell = 4.0 * math.pi / 3.0 * (r[1:] ** 3 - r[:-1] ** 3)
    rho = n_sites / box ** 3
    frames = max(1, obs["n_gofr_frames"])
    g = obs["gofr_all"] / (frames * n_sites * rho * shell)
    return 0.5 * (r[1:] + r[:-1]), g


class Server:
    def __init__(self, memory_budget, precision=flipmc.MC_FP32_DE, max_slots=1024,
                 quantum_moves=400_000):
        import torch

        self.torch = torch
        self.precision = precision
        self.budget = int(memory_budget)
        self.used = 0
        self.quantum = int(quantum_moves)
        self.streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        self.admit_stream = torch.cuda.Stream()
        self.batches = [flipmc.Batch(max_slots, precision, stream=s) for s in self.streams]
        self.max_slots = max_slots
        self.active = {}  # (batch, slot) -> (job, system, bytes, t_admit)
        self.peak_active = 0
        self.peak_bytes = 0
        self.launches = 0

    def _admit(self, job, now):
        p = job_params(job, self.precision)
        need = flipmc.mc_required_bytes(p)
        if need > self.budget:
            raise ValueError(f"job {job.index} needs {need} bytes, above the whole budget")
        if self.used + need > self.budget:
            return False
        resident, _ = flipmc.mc_placement(p)
        bi = 0 if resident else 1
        b = self.batches[bi]
        if len(b.members) >= self.max_slots:
            return False
        with self.torch.cuda.stream(self.admit_stream):
            s = flipmc.System(p, stream=self.admit_stream)
        slot = b.add(s, job.sweeps)
        self.active[(bi, slot)] = (job, s, need, now)
        self.used += need
        self.peak_active = max(self.peak_active, len(self.active))
        self.peak_bytes = max(self.peak_bytes, self.used)
        return True

    def _harvest(self, bi, slot, system, t0):
        job, s, need, t_admit = self.active.pop((bi, slot))
        obs = s.observables()
        now = time.perf_counter() - t0
        box = flipmc.mc_geometry(s.params)[0]
        r, g = gofr_normalised(obs, 3 * job.n_molecules, box)
        n_e = max(1, obs["n_energy_samples"])
        att, acc = obs["attempts"], obs["accepts"]
        res = Result(
            job=job, latency=now - job.arrival, wait=t_admit - job.arrival,
            energy_per_molecule=obs["energy_sum"] / n_e, gofr_r=r, gofr=g,
            c2_t=obs["c2_sweep"], c2=obs["c2"], moves=job.n_molecules * job.sweeps,
            accept={k: float(acc[i]) / max(1, int(att[i]))
                    for i, k in enumerate(["translate", "rotate", "flip"])},
        )
        self.used -= need
        del s
        return res

    def cancel(self, bi, slot):
        """Drop a running job: its slot and budget are free for the next admission."""
        job, s, need, _ = self.active.pop((bi, slot))
        self.batches[bi].cancel(slot)
        self.used -= need
        return job

    def serve(self, jobs, time_limit=None):
        """Run the arrival stream to completion; returns the results in
        completion order."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        queue = collections.deque()
        results = []
        i = 0
        t0 = time.perf_counter()
        while i < len(jobs) or queue or self.active:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while i < len(jobs) and jobs[i].arrival <= now:
                queue.append(jobs[i])
                i += 1
            while queue and self._admit(queue[0], now):
                queue.popleft()
            if not self.active:
                if i < len(jobs):
                    time.sleep(max(0.0, jobs[i].arrival - (time.perf_counter() - t0)))
                continue
            for b in self.batches:
                if b.members:
                    b.run(self.quantum)
                    self.launches += 1
            for bi, b in enumerate(self.batches):
                if b.members:
                    for slot, system in b.poll():
                        results.append(self._harvest(bi, slot, system, t0))
        return results
