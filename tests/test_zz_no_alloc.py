"""The allocation-free entry point mcf_init_system_noalloc against
mcf_init_system: the same kernels on the static scratch must give bitwise the
same attempts, decisions, states, energies and observables.  Two calls in a
row, the second with a smaller input; each system is closed before the
next, as they share the device's scratch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_21290_amd import flipmc  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(params, no_alloc, n):
    s = flipmc.FlexSystem(params, no_alloc=no_alloc)
    s.decision_log(n)
    s.sweep(n)
    out = {"log": s.read_log(), "state": s.get_state(), "energy": s.energy(), "obs": s.observables()}
    s.close()
    return out


@pytest.mark.parametrize("case", ["first", "second_smaller"])
def test_noalloc_equals_the_allocating_entry_point(case):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if case == "first":
        p = flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=1000, temperature=0.75, seed=4,
                                      resum_interval=5, gofr_interval=5)
    else:
        p = flipmc.mcf_params_default(flipmc.MC_TETRAHEDRON, n_molecules=125, temperature=2.0, seed=6,
                                      resum_interval=5, gofr_interval=5)
    print(f"no-alloc {case}: geometry {p.geometry}, {p.n_molecules} molecules", flush=True)
    n = 8
    a = _run(p, False, n)
    b = _run(p, True, n)
    la, lb = a["log"], b["log"]
    assert len(la) == len(lb) == n * flipmc.SITES[p.geometry] * p.n_molecules
    for f in la.dtype.names:
        assert np.array_equal(la[f], lb[f], equal_nan=True), f
    assert int(la["accepted"].sum()) > 0
    assert np.array_equal(a["state"]["pos"], b["state"]["pos"])
    assert np.array_equal(a["state"]["types"], b["state"]["types"])
    assert a["state"]["sweep"] == b["state"]["sweep"] == n
    assert a["energy"] == b["energy"]
    for key in ("gofr_all", "gofr_inter", "c2", "fs", "fs_cm", "attempts", "accepts"):
        assert np.array_equal(a["obs"][key], b["obs"][key]), key
    assert a["obs"]["e_acc"] == b["obs"]["e_acc"]
