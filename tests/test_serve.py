"""Host-side logic of batching and serving, with a stand-in backend (no GPU):
admission against the memory budget, FIFO order, cancellation freeing slots
and budget, completion of every job; and the seeded workload generators."""
import math

import numpy as np
import pytest

from paper_2506_21290_amd import serve, workloads


class FakeBackend:
    """Each job needs 3 * M bytes and finishes after ceil(M * S / quantum) launches."""

    def __init__(self, slots=4):
        self.slots = slots
        self.running = {}  # (bi, slot) -> remaining launches
        self.next_slot = [0, 0]
        self.launched = 0

    def size(self, job):
        return 3 * job.n_molecules, 0 if job.n_molecules <= 1000 else 1

    def free_slots(self, bi):
        return self.slots - sum(1 for (b, _) in self.running if b == bi)

    def start(self, job, bi):
        slot = self.next_slot[bi]
        self.next_slot[bi] += 1
        self.running[(bi, slot)] = math.ceil(job.n_molecules * job.sweeps / self.quantum)
        return slot, job

    def launch(self, quantum):
        self.quantum = quantum
        for key in self.running:
            self.running[key] -= 1
        self.launched += 1
        return 1

    def harvest(self):
        done = [k for k, v in self.running.items() if v <= 0]
        for k in done:
            del self.running[k]
        return [(b, s, None) for (b, s) in done]

    def cancel(self, bi, slot):
        del self.running[(bi, slot)]

    def result(self, job, handle):
        return dict(energy_per_molecule=0.0, gofr_r=np.zeros(1), gofr=np.zeros(1),
                    c2_t=np.zeros(0), c2=np.zeros(0))


def make_jobs(n, seed=0):
    rng = np.random.default_rng(seed)
    return [workloads.Job(i, int(rng.choice([125, 512, 1000, 1728])), 1.0,
                          int(rng.integers(100, 1000)), i + 1, 0.0) for i in range(n)]


def test_every_job_completes_within_budget():
    fb = FakeBackend(slots=3)
    fb.quantum = 50_000
    budget = 3 * (1728 + 1000 + 512)
    srv = serve.Server(budget, backend=fb, quantum_moves=50_000)
    jobs = make_jobs(40)
    res = srv.serve(jobs, clock=lambda: 0.0)
    assert sorted(r.job.index for r in res) == list(range(40))
    assert srv.peak_bytes <= budget and srv.used == 0
    assert srv.peak_active <= 6  # two batches of 3 slots


def test_admission_is_fifo_and_budget_bound():
    fb = FakeBackend(slots=100)
    fb.quantum = 1
    srv = serve.Server(3 * 1000 * 2, backend=fb, quantum_moves=1)
    jobs = [workloads.Job(i, 1000, 1.0, 100, i + 1, 0.0) for i in range(5)]
    assert srv.try_admit(jobs[0], 0.0) and srv.try_admit(jobs[1], 0.0)
    assert not srv.try_admit(jobs[2], 0.0)  # budget full
    assert srv.used == 6000
    big = workloads.Job(9, 10**6, 1.0, 100, 1, 0.0)
    with pytest.raises(ValueError):
        srv.try_admit(big, 0.0)


def test_cancel_frees_slot_and_budget():
    fb = FakeBackend(slots=1)
    fb.quantum = 1
    srv = serve.Server(10**9, backend=fb, quantum_moves=1)
    a, b = (workloads.Job(i, 512, 1.0, 100, i + 1, 0.0) for i in range(2))
    assert srv.try_admit(a, 0.0)
    assert not srv.try_admit(b, 0.0)  # no slot
    assert srv.cancel(0, 0) is a
    assert srv.used == 0 and not srv.active
    assert srv.try_admit(b, 0.0)


def test_serving_stream_statistics():
    jobs = workloads.serving_stream(n_jobs=4000, rate=200.0, seed=1)
    arr = np.array([j.arrival for j in jobs])
    gaps = np.diff(arr)
    assert arr[0] == 0.0 and np.all(gaps >= 0)
    assert gaps.mean() == pytest.approx(1 / 200, rel=0.05)
    n = np.array([round(j.n_molecules ** (1 / 3)) for j in jobs])
    assert n.min() >= 5 and n.max() <= 30
    assert all(j.n_molecules == k ** 3 for j, k in zip(jobs, n))
    s = np.array([j.sweeps for j in jobs])
    assert s.min() >= 100 and s.max() <= 10000
    # log-uniform sweeps: the median sits near the geometric mean 1000
    assert 700 < np.median(s) < 1400
    t = np.array([j.temperature for j in jobs])
    assert t.min() >= 0.75 and t.max() <= 3.0


def test_replica_set():
    jobs = workloads.replica_set(256, sweeps=1000, seed=1)
    assert len(jobs) == 256 and {j.n_molecules for j in jobs} == set(workloads.REPLICA_SIZES)
    assert [j.seed for j in jobs] == list(range(1, 257))
    assert all(0.75 <= j.temperature <= 3.0 for j in jobs)


def test_shortest_job_first_admits_the_least_work_and_respects_the_cap():
    fb = FakeBackend(slots=100)
    fb.quantum = 1000
    srv = serve.Server(10**9, backend=fb, quantum_moves=1000, policy="sjf", max_active=2)
    # all arrive together: work 125 * 900, 1728 * 100, 512 * 100, 1000 * 1000
    jobs = [workloads.Job(0, 125, 1.0, 900, 1, 0.0), workloads.Job(1, 1728, 1.0, 100, 2, 0.0),
            workloads.Job(2, 512, 1.0, 100, 3, 0.0), workloads.Job(3, 1000, 1.0, 1000, 4, 0.0)]
    admitted = []
    orig = fb.start

    def start(job, bi):
        admitted.append(job.index)
        assert len(fb.running) < 2  # never more than max_active at once
        return orig(job, bi)

    fb.start = start
    res = srv.serve(jobs, clock=lambda: 0.0)
    assert sorted(r.job.index for r in res) == [0, 1, 2, 3]
    assert admitted[:2] == [2, 0]  # 51 200 and 112 500 moves before 172 800 and 10^6
    assert srv.peak_active <= 2 and srv.used == 0


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        serve.Server(1, backend=FakeBackend(), policy="lifo")
