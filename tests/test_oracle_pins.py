"""Pins for the serial FP64 oracle.

Each test checks the oracle against something other than itself: published
known-answer vectors, a third-party implementation, closed forms, a library
routine, an independent numpy brute force, exact enumeration or a
statistical law.  The aim is that a plausible slip anywhere in the oracle
(a dropped term, a wrong sign, a swapped index or operand) fails one of them.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ----

def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    # Random123 known-answer vectors (SC'11 reference implementation).
    for ctr, key, out in _kat():
        assert list(oracle_mod.philox(ctr, key)) == out
        assert list(brute.philox4x32_10(ctr, key)) == out


def test_philox_matches_rocrand(oracle_mod, tmp_path):
    # A third-party implementation (rocRAND's header) on 2000 counters.
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "probe"
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand_probe.cpp")
    subprocess.check_call([hipcc, "-O1", src, "-o", str(exe)], cwd=str(tmp_path))
    rng = np.random.default_rng(7)
    words = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    words[:5, 1:4] = 0xFFFFFFFF
    text = "\n".join(" ".join(str(int(x)) for x in row) for row in words) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in l.split()] for l in out.stdout.strip().splitlines()])
    for row, r in zip(words[:300], ref[:300]):
        assert list(oracle_mod.philox(row[:4], row[4:])) == list(r)
    got = brute.philox4x32_10(words[:, :4], words[:, 4:])
    assert np.array_equal(got.astype(np.int64), ref)


def test_uniform_conversions(oracle_mod):
    # (w + 1/2) 2^-32 is open at both ends; the 53-bit forms hit the ends
    # exactly where their definitions say.
    assert oracle_mod.u32(0) == 2.0**-33
    assert oracle_mod.u32(0xFFFFFFFF) == 1.0 - 2.0**-33
    assert oracle_mod.u53(0, 0) == 2.0**-53
    assert oracle_mod.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    assert oracle_mod.u53_left(0, 0) == 0.0
    assert oracle_mod.u53_left(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert oracle_mod.u53(0x800, 0) == 2 * 2.0**-53  # the 11 low bits are dropped


# ---------------------------------------------------------------- model ----

@pytest.mark.parametrize("sig", [0.9, 0.95, 1.0, 1.05, 1.1])
def test_wca_closed_forms(oracle_mod, sig):
    # Eq. (1): u(sigma) = eps; u = 0 at and beyond 2^(1/6) sigma; u >= 0;
    # the shifted potential equals (2 (s/r)^6 - 1)^2 below the cut-off.
    assert oracle_mod.wca(sig * sig, sig) == pytest.approx(1.0, abs=1e-15)
    rc = 2.0 ** (1.0 / 6.0) * sig
    assert oracle_mod.wca(rc * rc * (1 + 1e-15), sig) == 0.0
    assert oracle_mod.wca((1.3 * sig) ** 2, sig) == 0.0
    for x in [0.5, 0.8, 0.95, 1.05, 1.12]:
        r = x * sig
        u = oracle_mod.wca(r * r, sig)
        alt = (2.0 * x**-6 - 1.0) ** 2
        assert u == pytest.approx(alt, rel=1e-12, abs=1e-12)
        assert u >= 0.0
    # continuity at the cut-off: u -> 0 from below
    r = rc * (1 - 1e-9)
    assert 0.0 <= oracle_mod.wca(r * r, sig) < 1e-12


def test_fene_is_kremer_grest(oracle_mod):
    # Eq. (2) is the Kremer-Grest bond with K = 30, R0 = 1.5 sigma:
    # -(K R0^2 / 2) ln(1 - (r/R0)^2) with K R0^2 / 2 = 33.75 at sigma = 1.
    for sig in [0.95, 1.0, 1.05]:
        K, R0 = 30.0 / sig**2, 1.5 * sig
        for r in [0.5, 0.9, 1.2, 1.4]:
            kg = -0.5 * K * R0 * R0 * math.log1p(-((r * sig / R0) ** 2))
            assert oracle_mod.fene(r * sig, sig) == pytest.approx(kg, rel=1e-13)
    assert oracle_mod.fene(0.0, 1.0) == 0.0


def test_bond_length_is_minimum_of_wca_plus_fene(oracle_mod):
    # b* minimises U(x) = U_WCA + U_FENE of a sigma_ij = 1 bond: check with an
    # independent minimiser (scipy) and with the sign of U on both sides.
    from scipy.optimize import minimize_scalar

    b = oracle_mod.bond_length_star()

    def U(x):
        return oracle_mod.wca(x * x, 1.0) + oracle_mod.fene(x, 1.0)

    res = minimize_scalar(U, bounds=(0.9, 1.1), method="bounded", options={"xatol": 1e-12})
    assert b == pytest.approx(res.x, abs=2e-7)
    for h in [1e-4, 1e-5, 1e-6]:
        assert U(b) < U(b + h) and U(b) < U(b - h)
        # the central difference of the slope vanishes to O(h^2) (U''' h^2 / 6
        # with U''' of order 1e4), far below U'' * 3e-9 ~ 5e-6 that an error of
        # 3e-9 in b* would leave
        assert abs((U(b + h) - U(b - h)) / (2 * h)) < 1e4 * h * h + 1e-7


def test_box_body_frame_and_rotation(oracle_mod):
    from scipy.spatial.transform import Rotation

    # rho = N / V with N = 3 M sites (Sec. II.A)
    for M in [64, 1000, 8000]:
        L = oracle_mod.box_length(M, 1.2)
        assert L**3 == pytest.approx(3 * M / 1.2, rel=1e-14)
    b = oracle_mod.bond_length_star()
    body = oracle_mod.body_frame()
    assert np.allclose(body.sum(0), 0.0, atol=1e-16)
    for i in range(3):
        for j in range(i + 1, 3):
            assert np.linalg.norm(body[i] - body[j]) == pytest.approx(b, rel=1e-15)
    assert np.allclose(body, brute.triangle(b), atol=1e-15)
    # W = max cut-off + twice the circumradius
    W = oracle_mod.stencil_reach()
    assert W == pytest.approx(2 ** (1 / 6) * 1.1 + 2 * b / math.sqrt(3), rel=1e-15)
    rng = np.random.default_rng(3)
    for _ in range(50):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = oracle_mod.rotation_matrix(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.allclose(R, ref, atol=1e-14)


def test_lattice_start(oracle_mod):
    # Simple-cubic lattice at the paper's density, uniform random orientations.
    p = oracle_mod.Params(n_molecules=1000, temperature=0.75, colours_per_axis=3, cells_per_side=9)
    s = oracle_mod.System(p)
    st = s.get_state()
    n, L = 10, s.box
    a = L / n
    m = np.arange(1000)
    expect = np.stack([(m % n + 0.5) * a, ((m // n) % n + 0.5) * a, (m // (n * n) + 0.5) * a], 1)
    assert np.array_equal(st["com"], expect)
    q = st["quat"]
    assert np.allclose((q * q).sum(1), 1.0, atol=1e-15)
    # the exact map from the tag-2 Philox draws, rebuilt by the numpy code
    assert np.allclose(q, brute.lattice_quaternions(1000, 1), rtol=0, atol=1e-15)
    # Haar measure: each quaternion component has E[q_i^2] = 1/4, and a rotated
    # axis is uniform on the sphere (mean 0, second moment 1/3).
    assert np.allclose((q * q).mean(0), 0.25, atol=0.03)
    ez = brute.quat_to_matrix(q)[:, :, 2]
    assert np.all(np.abs(ez.mean(0)) < 0.1)
    assert np.allclose((ez * ez).mean(0), 1 / 3, atol=0.04)
    assert np.array_equal(st["types"], np.tile([0, 1, 2], (1000, 1)))
    # the lattice start is the seeded state of the paper's density, not relaxed
    assert s.energy() / 1000 > 1e3


def test_intramolecular_energy_constant(oracle_mod):
    p = oracle_mod.Params(n_molecules=27, temperature=3.0, colours_per_axis=3, cells_per_side=3)
    s = oracle_mod.System(p)
    b = oracle_mod.bond_length_star()
    per = 3 * (oracle_mod.wca(b * b, 1.0) + oracle_mod.fene(b, 1.0))
    # the three bonds have sigma_ij 0.95, 1.0, 1.05, so only the sum is checked
    e0 = s.energy_intra()
    s.sweep_checkerboard(5)
    assert s.energy_intra() == pytest.approx(e0, rel=1e-12)
    assert e0 / 27 == pytest.approx(62.918, abs=1e-3)
    assert per > 0


# --------------------------------------------------------------- energies ----

@pytest.mark.parametrize("M,seed", [(27, 1), (64, 5), (125, 9)])
def test_energy_matches_numpy_brute_force(oracle_mod, M, seed):
    nc = {27: 3, 64: 3, 125: 3}[M]
    p = oracle_mod.Params(n_molecules=M, temperature=3.0, seed=seed, colours_per_axis=3,
                          cells_per_side=nc)
    s = oracle_mod.System(p)
    st = s.get_state()
    b = oracle_mod.bond_length_star()
    e_np = brute.energy(st["com"], st["quat"], st["types"], s.box, b)
    assert s.energy() == pytest.approx(e_np, rel=1e-12)
    # after some moves too (liquid-like state with flipped types)
    s.sweep_checkerboard(20)
    st = s.get_state()
    e_np = brute.energy(st["com"], st["quat"], st["types"], s.box, b)
    assert s.energy() == pytest.approx(e_np, rel=1e-12)
    assert np.allclose(s.sites(), brute.sites(st["com"], st["quat"], b), atol=1e-13)


def _replay(oracle_mod, p, n_sweeps, schedule="checkerboard"):
    """Replay the oracle's log trial by trial with the numpy implementation."""
    s = oracle_mod.System(p)
    b = oracle_mod.bond_length_star()
    rp = brute.Replayer(p, s.box, b)
    st = s.get_state()
    com, quat, types = st["com"].copy(), st["quat"].copy(), st["types"].copy()
    e = rp.energy(com, quat, types)
    checked = 0
    for sw in range(n_sweeps):
        if schedule == "checkerboard":
            log = s.sweep_checkerboard(1, log=True)
        else:
            log = s.sweep_random(1, log=True)
        for rec in log[np.argsort(log["seq"], kind="stable")]:
            m = int(rec["molecule"])
            if schedule == "random":
                g = rp.draw(int(rec["slot"]), sw, 4)
                assert m == min(int(p.n_molecules * brute.uniform53_left(g[0], g[1])), p.n_molecules - 1)
            move, new, u_acc, moved = rp.propose(com, quat, types, m, int(rec["slot"]), sw,
                                                 schedule == "checkerboard")
            assert rec["move"] == move
            assert rec["t_log_u"] == pytest.approx(p.temperature * math.log(u_acc), rel=1e-14)
            if new is None:
                assert rec["exited"] == 1 and rec["accepted"] == 0
                continue
            assert rec["exited"] == 0
            e_new = rp.energy(*new)
            de = e_new - e
            # the interacting site-pair terms the trial evaluated: moved sites
            # against all other sites, before and after the move
            assert rec["pair_terms"] == rp.pairs(com, quat, types, m, moved) + rp.pairs(*new, m, moved)
            scale = abs(rec["scale"]) + abs(e) * 1e-3
            assert abs(rec["delta_e"] - de) <= 1e-10 * scale + 1e-10, (sw, m, move)
            accept = de <= 0 or p.temperature * math.log(u_acc) < -de
            if abs(de + p.temperature * math.log(u_acc)) > 1e-7 * scale:
                assert bool(rec["accepted"]) == accept
            if rec["accepted"]:
                com, quat, types = new
                e = e_new
            checked += 1
        st = s.get_state()
        assert np.array_equal(st["types"], types)
        assert np.allclose(st["com"], com, atol=1e-12)
        assert np.allclose(st["quat"], quat, atol=1e-12)
        assert st["e_acc"] == pytest.approx(e, rel=1e-9, abs=1e-9)
    return checked


def test_replay_checkerboard_trial_by_trial(oracle_mod):
    # T1: every trial's proposal, dE, cell exit and Metropolis decision agree
    # with the numpy re-implementation replayed from the definitions.
    p = oracle_mod.Params(n_molecules=27, temperature=3.0, seed=11, colours_per_axis=3,
                          cells_per_side=3)
    assert _replay(oracle_mod, p, 12) > 200


def test_replay_checkerboard_k2(oracle_mod):
    p = oracle_mod.Params(n_molecules=64, temperature=3.0, seed=1, colours_per_axis=2,
                          cells_per_side=2)
    assert _replay(oracle_mod, p, 3) > 150


def test_replay_random_schedule(oracle_mod):
    p = oracle_mod.Params(n_molecules=27, temperature=2.0, seed=4, colours_per_axis=3,
                          cells_per_side=3)
    assert _replay(oracle_mod, p, 8, schedule="random") > 150


def test_energy_invariant_accumulated_equals_resum(oracle_mod):
    # T2: E_0 + sum of accepted dE equals the re-summed energy.
    p = oracle_mod.Params(n_molecules=64, temperature=3.0, seed=1)
    s = oracle_mod.System(p)
    tot = abs(s.energy())
    for _ in range(10):
        log = s.sweep_checkerboard(20, log=True)
        tot += np.abs(log["delta_e"][log["accepted"] == 1]).sum()
        e_acc = s.get_state()["e_acc"]
        assert abs(e_acc - s.energy()) <= 1e-9 * (tot + abs(s.energy()))


def test_cell_order_does_not_matter(oracle_mod):
    # T7: cells of one colour do not interact, so the order they are visited
    # in leaves the state bitwise unchanged.
    p = oracle_mod.Params(n_molecules=216, temperature=1.0, seed=3, colours_per_axis=3,
                          cells_per_side=6)
    states = []
    for order_seed in [0, 123, 987654321]:
        s = oracle_mod.System(p)
        s.sweep_checkerboard(6, cell_order_seed=order_seed)
        states.append(s.get_state())
    for st in states[1:]:
        assert np.array_equal(st["com"], states[0]["com"])
        assert np.array_equal(st["quat"], states[0]["quat"])
        assert np.array_equal(st["types"], states[0]["types"])


def test_flip_is_a_half_turn(oracle_mod):
    # Swapping the types of sites a+1 and a+2 at fixed positions equals a
    # rotation by pi about the median through site a (equilateral triangle).
    body = oracle_mod.body_frame()
    for a in range(3):
        n = body[a] / np.linalg.norm(body[a])
        R = 2 * np.outer(n, n) - np.eye(3)  # rotation by pi about n
        rotated = body @ R.T
        s1, s2 = (a + 1) % 3, (a + 2) % 3
        assert np.allclose(rotated[a], body[a], atol=1e-15)
        assert np.allclose(rotated[s1], body[s2], atol=1e-15)
        assert np.allclose(rotated[s2], body[s1], atol=1e-15)


def test_flip_leaves_positions_and_orientation(oracle_mod):
    # Flip-only chain: positions never change and C_2 stays 1 (Sec. III.B).
    p = oracle_mod.Params(n_molecules=64, temperature=3.0, p_flip=1.0, p_translate=0.0)
    s = oracle_mod.System(p)
    st0 = s.get_state()
    u0, k = s.orientation_ref()
    log = s.sweep_checkerboard(5, log=True)
    st = s.get_state()
    assert np.all(log["move"] == 2)
    assert log["accepted"].sum() > 0
    assert np.array_equal(st["com"], st0["com"]) and np.array_equal(st["quat"], st0["quat"])
    assert not np.array_equal(st["types"], st0["types"])
    assert s.c2(u0, k) == pytest.approx(1.0, abs=1e-14)


# -------------------------------------------------- exact detailed balance ----

def _two_molecules(oracle_mod, T, seed, p_flip=1.0):
    p = oracle_mod.Params(n_molecules=2, temperature=T, density=0.05, seed=seed, p_flip=p_flip,
                          p_translate=0.0, colours_per_axis=2, cells_per_side=2)
    return p


PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def test_flip_chain_samples_boltzmann_exactly(oracle_mod):
    # T4: two molecules at fixed positions, flips only: 36 type states.  The
    # energies come from the numpy brute force; independent chains of the
    # oracle must visit the states with Boltzmann frequencies.
    from scipy.stats import chisquare

    T = 1.5
    p = _two_molecules(oracle_mod, T, 1)
    s = oracle_mod.System(p, lattice=False)
    b = oracle_mod.bond_length_star()
    states = [(a, c) for a in PERMS for c in PERMS]
    rng = np.random.default_rng(0)
    # pick a close pair of molecules whose 36 type states span a few kT
    for _ in range(200):
        com = np.array([[1.0, 1.0, 1.0], [1.0 + rng.uniform(1.0, 1.6), 1.2, 1.1]])
        quat = rng.normal(size=(2, 4))
        quat /= np.linalg.norm(quat, axis=1, keepdims=True)
        E = np.array([brute.energy(com, quat, np.array([a, c], dtype=np.uint8), s.box, b)
                      for a, c in states])
        if T < np.ptp(E) < 6 * T:
            break
    else:
        pytest.fail("no suitable configuration found")
    for i, (a, c) in enumerate(states):
        s.set_state(com, quat, np.array([a, c], dtype=np.uint8), 0)
        assert s.energy() == pytest.approx(E[i], rel=1e-12)
    pi = np.exp(-(E - E.min()) / T)
    pi /= pi.sum()
    # detailed balance of the single-molecule flip kernel built from these E:
    # pi_x min(1, e^{-dE/T}) is symmetric in (x, y)
    idx = {st: i for i, st in enumerate(states)}
    for (a, c), i in idx.items():
        for ax in range(3):
            a2 = list(a)
            s1, s2 = (ax + 1) % 3, (ax + 2) % 3
            a2[s1], a2[s2] = a2[s2], a2[s1]
            j = idx[(tuple(a2), c)]
            f = pi[i] * min(1.0, math.exp(-(E[j] - E[i]) / T))
            r = pi[j] * min(1.0, math.exp(-(E[i] - E[j]) / T))
            assert f == pytest.approx(r, rel=1e-12)
    # independent chains from a fixed start, 40 sweeps each
    n_chains = 6000
    counts = np.zeros(36)
    start = np.array([PERMS[0], PERMS[0]], dtype=np.uint8)
    for c in range(n_chains):
        p = _two_molecules(oracle_mod, T, 1000 + c)
        ch = oracle_mod.System(p, lattice=False)
        ch.set_state(com, quat, start, 0)
        ch.sweep_checkerboard(40)
        ty = ch.get_state()["types"]
        counts[idx[(tuple(ty[0]), tuple(ty[1]))]] += 1
    exp = pi * n_chains
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    stat, pval = chisquare(obs, ex * obs.sum() / ex.sum())
    assert pval > 1e-4, (stat, pval)


# ------------------------------------------------------------ special cases ----

def test_isolated_molecule_accepts_everything(oracle_mod):
    # T8: one molecule: dE is identically zero, every non-exit move is accepted.
    p = oracle_mod.Params(n_molecules=1, temperature=0.5, density=0.001, colours_per_axis=2,
                          cells_per_side=2)
    s = oracle_mod.System(p)
    log = s.sweep_checkerboard(500, log=True)
    ok = log["exited"] == 0
    assert np.all(log["delta_e"][ok] == 0.0) and np.all(log["accepted"][ok] == 1)
    assert log["exited"].sum() < 500 and set(np.unique(log["move"])) == {0, 1, 2}


def test_ideal_gas_limit(oracle_mod):
    # T8: at T = 1e12 almost every non-exit move is accepted and the
    # inter-molecular g(r) is 1 (Eq. 3 normalisation).
    p = oracle_mod.Params(n_molecules=216, temperature=1e12, colours_per_axis=3, cells_per_side=6,
                          seed=2)
    s = oracle_mod.System(p)
    s.sweep_checkerboard(60)
    log = s.sweep_checkerboard(5, log=True)
    ok = log["exited"] == 0
    assert log["accepted"][ok].mean() > 0.98
    nb, rmax = oracle_mod.gofr_bins(s.box, 0.05)
    ca = np.zeros(nb, dtype=np.uint64)
    ci = np.zeros(nb, dtype=np.uint64)
    frames = 40
    for _ in range(frames):
        s.sweep_checkerboard(5)
        s.gofr_accumulate(ca, ci, dr=0.05)
    g = oracle_mod.gofr_normalise(ci, frames, 3 * 216, s.box, 0.05)
    r = np.arange(nb + 1) * 0.05
    sel = r[:-1] >= 1.0
    assert abs(g[sel].mean() - 1.0) < 0.03
    # intramolecular pairs: 6 ordered pairs per molecule per frame at r = b*
    b = oracle_mod.bond_length_star()
    intra = (ca - ci).astype(np.int64)
    assert intra[int(b / 0.05)] == 6 * 216 * frames
    assert intra.sum() == 6 * 216 * frames


def test_c2_closed_forms(oracle_mod):
    # Eq. (7), l = 2: C_2 = 1 at the reference; a common rotation by theta
    # about an axis normal to every u gives P_2(cos theta).
    p = oracle_mod.Params(n_molecules=27, temperature=3.0, colours_per_axis=3, cells_per_side=3)
    s = oracle_mod.System(p)
    u0, k = s.orientation_ref()
    assert np.all(k == 1)
    assert s.c2(u0, k) == pytest.approx(1.0, abs=1e-14)
    st = s.get_state()
    M = 27
    # all molecules aligned with the body frame: site 1 direction is b_1 / R
    q_id = np.tile([1.0, 0, 0, 0], (M, 1))
    s.set_state(st["com"], q_id, st["types"], 0)
    u0, k = s.orientation_ref()
    theta = 0.7
    q_rot = np.tile([math.cos(theta / 2), 0, 0, math.sin(theta / 2)], (M, 1))  # about z
    s.set_state(st["com"], q_rot, st["types"], 0)
    assert s.c2(u0, k) == pytest.approx(0.5 * (3 * math.cos(theta) ** 2 - 1), abs=1e-14)


# --------------------------------------------------------------- statistics ----

@pytest.mark.slow
def test_flip_and_local_moves_sample_the_same_energy(oracle_mod):
    # Sec. II.C: flip MC and MC without flips give the same energy
    # distribution.  Batch means over independent seeds at T = 3.
    def run(p_flip, seed):
        p = oracle_mod.Params(n_molecules=64, temperature=3.0, seed=seed, p_flip=p_flip,
                              p_translate=0.4 if p_flip > 0 else 0.5)
        s = oracle_mod.System(p)
        s.sweep_checkerboard(300)
        e = []
        for _ in range(30):
            s.sweep_checkerboard(10)
            e.append(s.get_state()["e_acc"] / 64)
        return np.mean(e)

    a = np.array([run(0.2, 100 + i) for i in range(10)])
    b = np.array([run(0.0, 200 + i) for i in range(10)])
    se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
    assert abs(a.mean() - b.mean()) < 3.5 * se + 1e-3


@pytest.mark.slow
def test_checkerboard_and_random_schedules_agree(oracle_mod):
    # Both schedules sample the same Boltzmann distribution at T = 3.
    def run(kind, seed):
        p = oracle_mod.Params(n_molecules=64, temperature=3.0, seed=seed)
        s = oracle_mod.System(p)
        f = s.sweep_checkerboard if kind == "cb" else s.sweep_random
        f(300)
        e = []
        for _ in range(30):
            f(10)
            e.append(s.get_state()["e_acc"] / 64)
        return np.mean(e)

    a = np.array([run("cb", 300 + i) for i in range(10)])
    b = np.array([run("rs", 400 + i) for i in range(10)])
    se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
    assert abs(a.mean() - b.mean()) < 3.5 * se + 1e-3


def test_invalid_parameters_are_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.System(oracle_mod.Params(n_molecules=64, temperature=3.0, colours_per_axis=2,
                                            cells_per_side=3))
    with pytest.raises(ValueError):  # (k-1) w below the interaction reach
        oracle_mod.System(oracle_mod.Params(n_molecules=1000, temperature=3.0,
                                            colours_per_axis=2, cells_per_side=6))
    with pytest.raises(ValueError):  # not a cube: no lattice start
        oracle_mod.System(oracle_mod.Params(n_molecules=100, temperature=3.0,
                                            colours_per_axis=2, cells_per_side=2))


def test_gofr_normalisation_of_a_uniform_histogram(oracle_mod):
    # counts equal to frames * N * rho * shell volume give g = 1 (Eq. 3);
    # no frames give zeros
    box, n_sites, frames, dr, nb = 10.0, 300, 4, 0.05, 100
    r = np.arange(nb + 1) * dr
    shell = 4 * np.pi / 3 * (r[1:] ** 3 - r[:-1] ** 3)
    counts = frames * n_sites * (n_sites / box ** 3) * shell
    assert np.allclose(oracle_mod.gofr_normalise(counts, frames, n_sites, box, dr), 1.0, rtol=1e-14)
    assert not oracle_mod.gofr_normalise(counts, 0, n_sites, box, dr).any()
