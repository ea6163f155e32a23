"""Parity of the flexible-molecule engine (the paper's own FENE-bonded
molecule, Sec. II.A, and the squares and tetrahedra of Sec. VII) with the
serial FP64 oracle of oracle/flex_oracle.c, attempt by attempt through the C
ABI.  Bars: proposals (move, flip rotation, cell exits) identical; dE and S
within 1e-12 S, infinite on the same attempts (a bond at its limit);
decisions identical outside |dE + T ln u| < 1e-12 S + 1e-9; positions bitwise
and types equal while no decision differed; observables within 1e-12."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import flex  # noqa: E402
from oracle import oracle as rig  # noqa: E402
from paper_2506_21290_amd import flipmc  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "triangle": (flipmc.MC_TRIANGLE, 125, 2.0, 3, 3, 1.2),
    "square": (flipmc.MC_SQUARE, 125, 2.0, 3, 3, 0.3),
    "tetrahedron": (flipmc.MC_TETRAHEDRON, 125, 2.0, 3, 3, 1.2),
    "triangle_1000": (flipmc.MC_TRIANGLE, 1000, 0.75, 3, 6, 1.2),
    # same-colour cells closer than the worst-case reach 2 D + r_c: one cell
    # at a time (the gap is below the reach of any square) ...
    "square_serial": (flipmc.MC_SQUARE, 125, 1.0, 2, 4, 0.3),
    # ... and side by side while the squares stay small enough (the bench's
    # 1000 squares, 8 cells per colour instead of 1)
    "square_1000": (flipmc.MC_SQUARE, 1000, 1.0, 4, 8, 1.2),
}


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gp(g, M, T, k, nc, rho, seed=1, **kw):
    return flipmc.mcf_params_default(g, n_molecules=M, temperature=T, colours_per_axis=k, cells_per_side=nc,
                                     density=rho, seed=seed, **kw)


def op(g, M, T, k, nc, rho, seed=1, **kw):
    return flex.Params(n_molecules=M, temperature=T, geometry=g, colours_per_axis=k, cells_per_side=nc,
                       density=rho, seed=seed, **kw)


def compare(lg, lo):
    """One sweep's records, both indexed by atom; True when a near-tie
    decision differed."""
    assert np.array_equal(lg["molecule"], np.arange(len(lg)))
    assert np.array_equal(lg["sweep"], lo["sweep"])
    assert np.array_equal(lg["move"], lo["move"])
    assert np.array_equal(lg["exited"], lo["exited"])
    assert np.array_equal(lg["axis"], lo["kind"])
    np.testing.assert_allclose(lg["t_log_u"], lo["t_log_u"], rtol=1e-14, atol=1e-300)
    ok = lo["exited"] == 0
    inf_o = np.isinf(lo["delta_e"])
    assert np.array_equal(np.isinf(lg["delta_e"]), inf_o)
    fin = ok & ~inf_o
    tol = 1e-12 * lo["scale"][fin] + 1e-300
    assert np.all(np.abs(lg["delta_e"][fin] - lo["delta_e"][fin]) <= tol)
    assert np.all(np.abs(lg["scale"][fin] - lo["scale"][fin]) <= tol)
    assert not np.any(lg["accepted"][inf_o])
    band = np.abs(lo["delta_e"] + lo["t_log_u"]) < 1e-12 * lo["scale"] + 1e-9
    differ = lg["accepted"] != lo["accepted"]
    assert not np.any(differ & ~band)
    if fin.any():
        assert np.mean(lg["pair_terms"][fin] != lo["pair_terms"][fin]) < 1e-3
    return bool(np.any(differ))


def run(case, n_sweeps, seed=1):
    g, M, T, k, nc, rho = CASES[case]
    print(f"flex {case} M={M} sweeps={n_sweeps}", flush=True)
    p = gp(g, M, T, k, nc, rho, seed=seed)
    assert flipmc.mcf_geometry(p)[1:] == (k, nc)
    s = flipmc.FlexSystem(p)
    o = flex.System(op(g, M, T, k, nc, rho, seed=seed))
    # the engine's own lattice start equals the oracle's up to the last bits of
    # sin, cos and sqrt; the chains are then compared from the oracle's start
    st, so = s.get_state(), o.get_state()
    assert np.array_equal(st["types"], so["types"])
    assert np.max(np.abs(st["pos"] - so["pos"])) < 1e-12
    assert s.energy()[0] == pytest.approx(o.energy(), rel=1e-9)
    s.set_state(so["pos"], so["types"], 0)
    assert s.energy()[0] == pytest.approx(o.energy(), rel=1e-12)
    resyncs = 0
    for _ in range(n_sweeps):
        s.decision_log(1)
        s.sweep(1)
        lg = s.read_log()
        lo = o.sweep_checkerboard(1, log=True)
        if compare(lg, lo):
            x = o.get_state()
            s.set_state(x["pos"], x["types"], x["sweep"], x["e_acc"])
            resyncs += 1
            continue
        st, so = s.get_state(), o.get_state()
        assert st["sweep"] == so["sweep"]
        assert np.array_equal(st["pos"], so["pos"])
        assert np.array_equal(st["types"], so["types"])
    return s, o, resyncs


@pytest.mark.parametrize("case", ["triangle", "square", "tetrahedron"])
def test_every_attempt_matches_the_oracle(case):
    s, o, resyncs = run(case, 12)
    assert resyncs == 0
    e, _, drift = s.energy()
    assert e == pytest.approx(o.energy(), rel=1e-10)
    # E_0 + the accepted dE, against the fresh FP64 re-sum
    assert abs(drift) <= 1e-9 * abs(e)
    c = s.observables()
    oc = o.counters()
    assert list(c["attempts"]) == list(oc["attempts"]) and list(c["accepts"]) == list(oc["accepts"])
    assert c["exits"] == oc["exits"]


@pytest.mark.parametrize("case", ["square_serial", "square_1000"])
def test_cells_closer_than_the_reach_match_the_oracle(case):
    # the oracle attempts the cells of a colour in ascending index; the engine
    # runs them one at a time or, when this sweep's bodies cannot reach across
    # the gap, side by side: every attempt identical either way
    s, o, resyncs = run(case, 4 if case == "square_serial" else 2)
    assert resyncs == 0


def test_side_by_side_cells_equal_one_at_a_time():
    # MC_FLAG_SERIAL_CELLS forces one cell at a time: bitwise the same chain
    g, M, T, k, nc, rho = CASES["square_1000"]
    print("flex serial vs side by side", flush=True)
    a = flipmc.FlexSystem(gp(g, M, T, k, nc, rho, seed=5))
    b = flipmc.FlexSystem(gp(g, M, T, k, nc, rho, seed=5, flags=flipmc.MC_FLAG_SERIAL_CELLS))
    a.sweep(10)
    b.sweep(10)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["pos"], sb["pos"]) and np.array_equal(sa["types"], sb["types"])
    assert sa["e_acc"] == sb["e_acc"]


def test_full_size_1000_triangles():
    # the paper's system size (M = 1000, N = 3000 atoms) at T = 0.75
    s, o, resyncs = run("triangle_1000", 3)
    assert resyncs <= 1


@pytest.mark.parametrize("g,T", [(flipmc.MC_TRIANGLE, 0.75), (flipmc.MC_SQUARE, 1.0),
                                 (flipmc.MC_TETRAHEDRON, 1.0)], ids=["triangle", "square", "tetrahedron"])
def test_timed_regime_in_the_bench_decomposition(g, T):
    # the flexible bench's systems (1000 molecules, density 1.2, the
    # decomposition mcf_geometry picks) after the default line's 200 warm-up
    # sweeps on the device: that state into the oracle, then 2 sweeps attempt
    # by attempt
    print(f"flex timed regime geometry={g}", flush=True)
    p = flipmc.mcf_params_default(g, n_molecules=1000, temperature=T, density=1.2, seed=1)
    _, k, nc = flipmc.mcf_geometry(p)
    s = flipmc.FlexSystem(p)
    s.sweep(200)
    st = s.get_state()
    assert st["sweep"] == 200
    o = flex.System(op(g, 1000, T, k, nc, 1.2, seed=1))
    o.set_state(st["pos"], st["types"], st["sweep"], st["e_acc"])
    assert s.energy()[0] == pytest.approx(o.energy(), rel=1e-12)
    resyncs = 0
    for _ in range(2):
        s.decision_log(1)
        s.sweep(1)
        lg = s.read_log()
        lo = o.sweep_checkerboard(1, log=True)
        if compare(lg, lo):  # a near-tie decision differed: go on from the oracle's state
            x = o.get_state()
            s.set_state(x["pos"], x["types"], x["sweep"], x["e_acc"])
            resyncs += 1
            continue
        a, b = s.get_state(), o.get_state()
        assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["types"], b["types"])
    assert resyncs <= 1


def test_fene_wall_on_the_device():
    # a stretched triangle (bond 0-1 at 1.5 with types B, C): flips that put
    # A on that bond reach the bond's limit; the engine gives dE = inf on the
    # same attempts as the oracle and never accepts them
    print("flex fene wall", flush=True)
    kw = dict(p_flip=0.5)
    p = gp(flipmc.MC_TRIANGLE, 1, 1e6, 2, 2, 0.001, seed=5, **kw)
    o = flex.System(op(flipmc.MC_TRIANGLE, 1, 1e6, 2, 2, 0.001, seed=5, **kw), lattice=False)
    L = o.box
    pos = np.array([[L / 2, L / 2, L / 2], [L / 2 + 1.5, L / 2, L / 2], [L / 2 + 0.75, L / 2 + 0.9, L / 2]])
    types = np.array([1, 2, 0], dtype=np.uint8)
    s = flipmc.FlexSystem(p, pos=pos, types=types)
    o.set_state(pos, types, 0)
    walls = 0
    for _ in range(60):
        s.decision_log(1)
        s.sweep(1)
        lg = s.read_log()
        lo = o.sweep_checkerboard(1, log=True)
        assert not compare(lg, lo)
        walls += int(np.isinf(lg["delta_e"]).sum())
    assert walls > 0


def test_observables_match_the_oracle():
    # g(r) counts of every ordered atom pair (Eq. 3), C_2 (Eq. 7), F_s and
    # F_s^cm (Eqs. 5-6) at the sample sweeps, on the 125-triangle system
    g, M, T, k, nc, rho = CASES["triangle"]
    p = gp(g, M, T, k, nc, rho, seed=3, gofr_interval=5, obs_interval=5, resum_interval=10)
    o = flex.System(op(g, M, T, k, nc, rho, seed=3))
    so = o.get_state()
    s = flipmc.FlexSystem(p, pos=so["pos"], types=so["types"])
    n = 20
    s.sweep(n)
    obs = s.observables()
    nb = len(obs["gofr_all"])
    ca = np.zeros(nb, dtype=np.uint64)
    ci = np.zeros(nb, dtype=np.uint64)
    u0, kref = o.orientation_ref()
    a0, c0 = o.unwrapped()
    want, terms = {}, {}
    for t in range(1, n + 1):
        o.sweep_checkerboard(1)
        if t % 5 == 0:
            o.gofr_accumulate(ca, ci, dr=p.gofr_dr)
        if t in (1, 2, 5, 10, 20):
            a, c = o.unwrapped()
            want[t] = (float(np.mean(o.c2_terms(u0, kref))),
                       rig.fs_isotropic(a - a0, p.fs_q), rig.fs_isotropic(c - c0, p.fs_q_cm))
            # per-particle contributions (Sec. V.A): sin(q d)/(q d) of each
            # atom and centre, C_2 of each molecule
            fs_i = np.sinc(p.fs_q * np.linalg.norm(a - a0, axis=1) / np.pi)
            fcm_i = np.sinc(p.fs_q_cm * np.linalg.norm(c - c0, axis=1) / np.pi)
            terms[t] = (o.c2_terms(u0, kref), fcm_i, fs_i)
    assert obs["n_gofr_frames"] == 4
    assert np.abs(obs["gofr_all"].astype(np.int64) - ca.astype(np.int64)).sum() <= 4
    assert np.abs(obs["gofr_inter"].astype(np.int64) - ci.astype(np.int64)).sum() <= 4
    assert [int(t) for t in obs["c2_sweep"]] == [1, 2, 5, 10, 20]
    for j, t in enumerate([1, 2, 5, 10, 20]):
        assert obs["c2"][j] == pytest.approx(want[t][0], abs=1e-12)
        assert obs["fs"][j] == pytest.approx(want[t][1], abs=1e-12)
        assert obs["fs_cm"][j] == pytest.approx(want[t][2], abs=1e-12)
        c2_i, fcm_i, fs_i = terms[t]
        assert obs["c2_sq"][j] == pytest.approx(np.mean(c2_i ** 2), abs=1e-12)
        assert obs["fs_cm_sq"][j] == pytest.approx(np.mean(fcm_i ** 2), abs=1e-12)
        assert obs["c2_fs_cm"][j] == pytest.approx(np.mean(c2_i * fcm_i), abs=1e-12)
        assert obs["fs_sq"][j] == pytest.approx(np.mean(fs_i ** 2), abs=1e-12)
    g_norm = rig.gofr_normalise(obs["gofr_all"], 4, 3 * M, o.box, p.gofr_dr)
    np.testing.assert_allclose(obs["gofr_norm_all"], g_norm, rtol=1e-12)


def test_state_roundtrip_and_bad_types():
    g, M, T, k, nc, rho = CASES["tetrahedron"]
    s = flipmc.FlexSystem(gp(g, M, T, k, nc, rho))
    s.sweep(3)
    st = s.get_state()
    s2 = flipmc.FlexSystem(gp(g, M, T, k, nc, rho), pos=st["pos"], types=st["types"])
    assert np.array_equal(s2.get_state()["pos"], st["pos"])
    assert s2.energy()[0] == pytest.approx(s.energy()[0], rel=1e-12)
    bad = st["types"].copy()
    bad[0] = bad[1]
    with pytest.raises(flipmc.McError) as e:
        s2.set_state(st["pos"], bad, 0)
    assert e.value.code == flipmc.MC_EINVAL


@pytest.mark.parametrize("case", ["triangle", "square", "tetrahedron", "triangle_1000"])
def test_lds_and_buffer_state_agree(case):
    # the sweep kernel with positions, types and cell lists in LDS and the same
    # kernel on the arrays in the system's buffer give bitwise equal chains
    g, M, T, k, nc, rho = CASES[case]
    print(f"flex lds-vs-buffer {case}", flush=True)
    kw = dict(gofr_interval=5, obs_interval=5, resum_interval=10, max_samples=64)
    pr = gp(g, M, T, k, nc, rho, seed=7, **kw)
    ph = gp(g, M, T, k, nc, rho, seed=7, flags=flipmc.MC_FLAG_HBM_STATE, **kw)
    assert flipmc.mcf_placement(pr)[0] and not flipmc.mcf_placement(ph)[0]
    a, b = flipmc.FlexSystem(pr), flipmc.FlexSystem(ph)
    for n in (1, 7, 22):
        a.sweep(n)
        b.sweep(n)
        sa, sb = a.get_state(), b.get_state()
        assert sa["sweep"] == sb["sweep"]
        assert np.array_equal(sa["pos"], sb["pos"]) and np.array_equal(sa["types"], sb["types"])
    oa, ob = a.observables(), b.observables()
    for key in ("attempts", "accepts", "gofr_all", "gofr_inter", "c2", "fs", "fs_cm"):
        assert np.array_equal(np.asarray(oa[key]), np.asarray(ob[key])), key
    assert oa["exits"] == ob["exits"] and oa["e_acc"] == ob["e_acc"]
    assert a.energy() == b.energy()


def test_sweep_many_equals_each_system_alone():
    # one launch of four systems of different geometry, size and placement
    # (the 1000-triangle system keeps its state in the buffer) against each
    # system advanced alone: bitwise the same states and observables
    print("flex sweep_many", flush=True)
    kw = dict(gofr_interval=5, obs_interval=5, resum_interval=10, max_samples=64)
    specs = [("triangle", 1, 0), ("tetrahedron", 2, 0), ("square", 3, 0),
             ("triangle_1000", 4, flipmc.MC_FLAG_HBM_STATE)]
    many = [flipmc.FlexSystem(gp(*CASES[c], seed=sd, flags=fl, **kw)) for c, sd, fl in specs]
    alone = [flipmc.FlexSystem(gp(*CASES[c], seed=sd, flags=fl, **kw)) for c, sd, fl in specs]
    for n in (1, 7, 22):
        flipmc.flex_sweep_many(many, n)
        for s in alone:
            s.sweep(n)
    for a, b in zip(many, alone):
        sa, sb = a.get_state(), b.get_state()
        assert sa["sweep"] == sb["sweep"] == 30
        assert np.array_equal(sa["pos"], sb["pos"]) and np.array_equal(sa["types"], sb["types"])
        oa, ob = a.observables(), b.observables()
        for key in ("attempts", "accepts", "gofr_all", "c2", "fs", "fs_cm"):
            assert np.array_equal(np.asarray(oa[key]), np.asarray(ob[key])), key
        assert oa["e_acc"] == ob["e_acc"]
    with pytest.raises(flipmc.McError) as e:
        flipmc.flex_sweep_many([many[0], many[1], many[0]], 1)
    assert e.value.code == flipmc.MC_EINVAL
    assert many[0].get_state()["sweep"] == 30  # nothing was enqueued


def test_replica_launch_sampled_against_the_oracle():
    # the bench's replica launch: 256 systems of 1000 flexible triangles
    # (T = 0.75, seeds 1 .. 256) advanced together by mcf_sweep_many, two
    # sweeps; replicas 1 and 256 attempt by attempt against the oracle (both
    # from the oracle's lattice start)
    print("flex replica launch", flush=True)
    R, n, N = 256, 2, 3000
    ps = [flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=1000, temperature=0.75, density=1.2,
                                    seed=r + 1, gofr_interval=0) for r in range(R)]
    runs = [flipmc.FlexSystem(p) for p in ps]
    oracles = {}
    for r in (0, R - 1):
        _, k, nc = flipmc.mcf_geometry(ps[r])
        o = flex.System(op(flipmc.MC_TRIANGLE, 1000, 0.75, k, nc, 1.2, seed=r + 1))
        so = o.get_state()
        runs[r].set_state(so["pos"], so["types"], 0)
        runs[r].decision_log(n)
        oracles[r] = o
    flipmc.flex_sweep_many(runs, n)
    for r, o in oracles.items():
        lg = runs[r].read_log()
        tie = False
        for sw in range(n):
            lo = o.sweep_checkerboard(1, log=True)
            if compare(lg[sw * N:(sw + 1) * N], lo):
                tie = True
                break
        if not tie:
            a, b = runs[r].get_state(), o.get_state()
            assert a["sweep"] == b["sweep"] == n
            assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["types"], b["types"])
    for s in runs:
        s.close()
