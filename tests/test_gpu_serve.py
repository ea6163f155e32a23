"""Serving on the GPU: every job's result is the same alone and in the mix.

A short Poisson stream is served with continuous batching under a small
memory budget (so admissions wait for completions); a sample of the jobs is
then run alone, one system per launch sequence, and the results must agree
bitwise: the chain of a job depends only on its seed, never on which other
jobs shared its launches."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_21290_amd import flipmc, serve, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("policy,cap", [("fifo", None), ("sjf", 4)])
def test_results_same_alone_and_in_the_mix(policy, cap):
    jobs = workloads.serving_stream(n_jobs=14, rate=200.0, seed=3, m_min=125, m_max=1728,
                                    s_min=60, s_max=300)
    # two jobs too large for one workgroup's LDS: the multi-workgroup engine
    t_last = jobs[-1].arrival
    jobs += [workloads.Job(14, 2197, 1.3, 40, 77, t_last), workloads.Job(15, 2744, 2.0, 30, 78, t_last)]
    prec = flipmc.MC_FP32_DE
    sizes = [flipmc.mc_required_bytes(serve.job_params(j, prec)) for j in jobs]
    budget = 3 * max(sizes)  # a few jobs at a time: later arrivals must wait
    srv = serve.Server(budget, backend=serve.GpuBackend(prec, max_slots=8), quantum_moves=20_000,
                       policy=policy, max_active=cap)
    res = srv.serve(jobs)
    assert sorted(r.job.index for r in res) == list(range(len(jobs)))
    assert srv.peak_bytes <= budget and srv.used == 0
    if cap:
        assert srv.peak_active <= cap
    assert srv.launches > len(jobs)  # time-sliced, not one launch per job
    assert any(r.wait > 0 for r in res)
    be = srv.backend
    for j in jobs[14:]:
        engine, _ = flipmc.mc_engine(serve.job_params(j, prec))
        assert engine == flipmc.MC_ENGINE_SPREAD
    by_index = {r.job.index: r for r in res}
    for j in jobs[::3] + jobs[14:]:
        s = flipmc.System(serve.job_params(j, prec))
        s.sweep(j.sweeps)
        alone = be.result(j, s)
        mixed = by_index[j.index]
        assert alone["energy_per_molecule"] == mixed.energy_per_molecule
        assert np.array_equal(alone["gofr"], mixed.gofr)
        assert np.array_equal(alone["c2"], mixed.c2) and np.array_equal(alone["c2_t"], mixed.c2_t)


def test_cancel_then_readmit_on_device():
    prec = flipmc.MC_FP32_DE
    jobs = [workloads.Job(i, 216, 1.5, 5000, i + 1, 0.0) for i in range(2)]
    srv = serve.Server(10 ** 9, backend=serve.GpuBackend(prec, max_slots=1), quantum_moves=10_000)
    assert srv.try_admit(jobs[0], 0.0)
    assert not srv.try_admit(jobs[1], 0.0)  # the only slot is busy
    srv.backend.launch(srv.quantum)
    srv.backend.harvest()
    assert srv.cancel(0, 0).index == 0
    assert srv.used == 0
    assert srv.try_admit(jobs[1], 0.0)
