"""Continuous-batching sampling server on one GPU.

Requests are sampling jobs (M molecules at temperature T for S sweeps).  Their
configurations stay resident in HBM for the job's life; a job is admitted as
soon as a slot and enough of the memory budget are free (in arrival order, or
the shortest queued job first with a cap on the jobs admitted), and every run
advances all admitted jobs by one time slice, so jobs that arrive while others
run join the next run and their work overlaps on the device.  Every job gets
one workgroup per run (systems whose working set fits one workgroup's LDS keep
it there); the workgroups left over go to the large jobs with the most work
left, which then run on the multi-workgroup engine in a cooperative launch
beside the others.

The time slice is given in attempted moves of a 1000-molecule job; the batch
turns it into a time and gives every job the sweeps it runs in that time on
its engine (a cost model against size, calibrated on the batch's own timed
launches), so the launches of a run take about the same time.

Each finished job returns E/M (mean over the second half of its sweeps), g(r)
(frames over the second half) and C_2(t) (Sec. III, Eq. 3 and Eq. 7).

The device work goes through a backend object (``GpuBackend`` by default); the
admission, budget and slot accounting is plain Python and can be exercised with
any object that offers the same few methods.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import flipmc, tune


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
    """Engine parameters of a job: the tuned decomposition and workgroup count
    for its size (the latter caps what a batch gives the job), FP64
    re-sum every 100 sweeps, E/M every 10 sweeps and about five g(r) frames over
    the second half of the run."""
    S = job.sweeps
    gofr_every = max(10, (S // 2) // 5 // 10 * 10)
    k, nc, wg = tune.choose(job.n_molecules, precision)
    return flipmc.mc_params_default(
        n_molecules=job.n_molecules, temperature=job.temperature, precision=precision,
        seed=job.seed, colours_per_axis=k, cells_per_side=nc, workgroups=wg, resum_interval=100,
        obs_interval=10, gofr_interval=gofr_every, obs_start=S // 2,
        max_samples=max(16, S // 10 + 2))


class GpuBackend:
    """Jobs as flipmc systems in one batch: every run gives each job one
    workgroup and the spare workgroups of the device to the large jobs with the
    most work left (multi-workgroup engine); the engines make the same
    decisions, so a job's result does not depend on how it was run."""

    def __init__(self, precision=flipmc.MC_FP32_DE, max_slots=1024, max_workgroups=0):
        import torch

        self.torch = torch
        self.precision = precision
        self.streams = [torch.cuda.Stream()]
        self.admit_stream = torch.cuda.Stream()
        self.batches = [flipmc.Batch(max_slots, precision, stream=s) for s in self.streams]
        for b in self.batches:
            b.set_workgroups(max_workgroups)
        self.max_slots = max_slots

    def size(self, job):
        """(bytes of device memory, batch index)"""
        p = job_params(job, self.precision)
        return flipmc.mc_required_bytes(p), 0

    def free_slots(self, bi):
        return self.max_slots - len(self.batches[bi].members)

    def start(self, job, bi):
        with self.torch.cuda.stream(self.admit_stream):
            s = flipmc.System(job_params(job, self.precision), stream=self.admit_stream)
        return self.batches[bi].add(s, job.sweeps), s

    def launch(self, quantum_moves):
        n = 0
        for b in self.batches:
            if b.members:
                b.run(quantum_moves)
                n += 1
        return n

    def harvest(self):
        """[(batch index, slot, system)] of finished jobs."""
        out = []
        for bi, b in enumerate(self.batches):
            if b.members:
                out += [(bi, slot, s) for slot, s in b.poll()]
        return out

    def cancel(self, bi, slot):
        self.batches[bi].cancel(slot)

    def result(self, job, s):
        obs = s.observables()
        g = obs["gofr_norm_all"]  # Eq. (3), normalised by the library
        r = (np.arange(len(g)) + 0.5) * obs["gofr_dr"]
        n_e = max(1, obs["n_energy_samples"])
        att, acc = obs["attempts"], obs["accepts"]
        return dict(energy_per_molecule=obs["energy_sum"] / n_e, gofr_r=r, gofr=g,
                    c2_t=obs["c2_sweep"], c2=obs["c2"],
                    accept={k: float(acc[i]) / max(1, int(att[i]))
                            for i, k in enumerate(["translate", "rotate", "flip"])})


class Server:
    """Admission policies: "fifo" admits jobs in arrival order as soon as the
    budget and a slot allow; "sjf" admits the queued job with the least work
    (molecules x sweeps) first, and at most max_active jobs at once, so that
    short jobs do not share the device with every long one (the smallest mean
    and median latency for known job sizes; the longest jobs finish last)."""

    def __init__(self, memory_budget, backend=None, quantum_moves=100_000, policy="fifo",
                 max_active=None):
        if policy not in ("fifo", "sjf"):
            raise ValueError(f"unknown admission policy {policy!r}")
        self.backend = backend if backend is not None else GpuBackend()
        self.budget = int(memory_budget)
        self.used = 0
        self.quantum = int(quantum_moves)
        self.policy = policy
        self.max_active = max_active
        self.active = {}  # (batch, slot) -> (job, handle, bytes, t_admit)
        self.peak_active = 0
        self.peak_bytes = 0
        self.launches = 0

    def try_admit(self, job, now):
        need, bi = self.backend.size(job)
        if need > self.budget:
            raise ValueError(f"job {job.index} needs {need} bytes, above the whole budget")
        if self.used + need > self.budget or self.backend.free_slots(bi) <= 0:
            return False
        slot, handle = self.backend.start(job, bi)
        self.active[(bi, slot)] = (job, handle, need, now)
        self.used += need
        self.peak_active = max(self.peak_active, len(self.active))
        self.peak_bytes = max(self.peak_bytes, self.used)
        return True

    def finish(self, bi, slot, now):
        job, handle, need, t_admit = self.active.pop((bi, slot))
        self.used -= need
        r = self.backend.result(job, handle)
        return Result(job=job, latency=now - job.arrival, wait=t_admit - job.arrival,
                      moves=job.n_molecules * job.sweeps, **r)

    def cancel(self, bi, slot):
        """Drop a running job: its slot and budget are free for the next admission."""
        job, handle, need, _ = self.active.pop((bi, slot))
        self.backend.cancel(bi, slot)
        self.used -= need
        return job

    def serve(self, jobs, time_limit=None, clock=None, on_done=None):
        """Run an arrival stream to completion; returns results in completion
        order.  `clock` (seconds since start) defaults to the wall clock;
        `on_done(n)` is called with the number of finished jobs after each
        harvest that finished some."""
        t0 = time.perf_counter()
        clock = clock or (lambda: time.perf_counter() - t0)
        jobs = sorted(jobs, key=lambda j: j.arrival)
        queue = collections.deque()
        results = []
        i = 0
        while i < len(jobs) or queue or self.active:
            now = clock()
            if time_limit is not None and now > time_limit:
                break
            arrived = False
            while i < len(jobs) and jobs[i].arrival <= now:
                queue.append(jobs[i])
                i += 1
                arrived = True
            if self.policy == "sjf" and arrived:
                queue = collections.deque(sorted(queue, key=lambda j: (j.n_molecules * j.sweeps, j.arrival)))
            while queue and (self.max_active is None or len(self.active) < self.max_active) and \
                    self.try_admit(queue[0], now):
                queue.popleft()
            if not self.active:
                if i < len(jobs):
                    time.sleep(max(0.0, min(0.05, jobs[i].arrival - clock())))
                continue
            n = self.backend.launch(self.quantum)
            self.launches += n
            done = self.backend.harvest()
            for bi, slot, _ in done:
                results.append(self.finish(bi, slot, clock()))
            if done and on_done is not None:
                on_done(len(results))
            if n == 0 and not done:
                time.sleep(2e-4)  # only slices in flight: wait a little

        return results
