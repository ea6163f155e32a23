"""Pins of the flexible-molecule oracle (the paper's own model, Sec. II.A:
FENE bonds, Eq. 2, and WCA, Eq. 1, between all atoms; and the squares and
tetrahedra of its outlook, Sec. VII) against what the mathematics fixes:
closed forms, the independent numpy brute force replayed trial by trial,
exact Boltzmann sampling of flip-only chains, the hard wall of the FENE bond.
"""
import math

import numpy as np
import pytest

from oracle import brute_flex as bf
from oracle import flex

# (geometry, molecules, k, n_c, density): the square's ring of bonds lets two
# atoms of one molecule sit up to two bonds apart, so its colours need cells
# of width >= (2 * 2 * 1.6 + 1.23) / (k - 1): a dilute box keeps it small
GEOMS = [(flex.TRIANGLE, 125, 3, 3, 1.2), (flex.SQUARE, 125, 3, 3, 0.3),
         (flex.TETRAHEDRON, 125, 3, 3, 1.2)]


def _sigma(g):
    return (0.9, 1.0, 1.1) if g == flex.TRIANGLE else flex.SIGMA4


def test_tables_match_the_geometry():
    # bonds = edges of the ideal body; flips = the permutations 180 degree
    # rotations about its two-fold axes induce (derived numerically in
    # brute_flex); the oracle must use the same (checked through a flip-only
    # replay below) and the counts it reports
    L = flex.lib()
    assert [L.fx_sites(g) for g in range(3)] == [3, 4, 4]
    assert [L.fx_flip_kinds(g) for g in range(3)] == [len(bf.flips(g)) for g in range(3)]
    assert len(bf.bonds(flex.TRIANGLE)) == 3 and len(bf.bonds(flex.SQUARE)) == 4
    assert len(bf.bonds(flex.TETRAHEDRON)) == 6
    for g in range(3):
        for perm in bf.flips(g):
            assert sorted(perm) == list(range(len(perm)))
            assert all(perm[perm[s]] == s for s in range(len(perm)))  # an involution


@pytest.mark.parametrize("g,M,k,nc,rho", GEOMS)
def test_lattice_start_and_energy_match_numpy(g, M, k, nc, rho):
    p = flex.Params(n_molecules=M, temperature=2.0, geometry=g, colours_per_axis=k, cells_per_side=nc,
                    density=rho, seed=3)
    s = flex.System(p)
    st = s.get_state()
    side = flex.oracle.bond_length_star()
    ref = bf.lattice(p, s.box, side)
    d = st["pos"] - ref
    d -= s.box * np.round(d / s.box)
    assert np.max(np.abs(d)) < 1e-12
    n = flex.SITES[g]
    assert np.array_equal(st["types"], np.tile(np.arange(n), M))
    e = bf.energy(st["pos"], st["types"], s.box, g, _sigma(g))
    assert s.energy() == pytest.approx(e, rel=1e-12)


def test_ideal_triangle_intramolecular_energy_closed_form():
    # one molecule alone: E = sum over its three bonds of WCA + FENE at b*
    # (sigma_ij = 0.95, 1.0, 1.05 for AB, AC, BC)
    p = flex.Params(n_molecules=1, temperature=1.0, density=0.001, colours_per_axis=2, cells_per_side=2)
    s = flex.System(p)
    b = flex.oracle.bond_length_star()
    e = sum(flex.oracle.wca(b * b, sij) + flex.oracle.fene(b, sij) for sij in (0.95, 1.0, 1.05))
    assert s.energy() == pytest.approx(e, rel=1e-13)
    assert s.energy_inter() == 0.0


def _replay(p, n_sweeps, schedule="checkerboard"):
    s = flex.System(p)
    rp = bf.Replayer(p, s.box)
    st = s.get_state()
    pos, types = st["pos"].copy(), st["types"].copy()
    e = rp.energy(pos, types)
    checked = flips = inf = 0
    for sw in range(n_sweeps):
        log = s.sweep_checkerboard(1, log=True) if schedule == "checkerboard" else s.sweep_random(1, log=True)
        for rec in log[np.argsort(log["seq"], kind="stable")]:
            a = int(rec["atom"])
            if schedule == "random":
                g = rp.draw(int(rec["slot"]), sw, 4)
                assert a == min(int(s.N * bf.uniform53_left(g[0], g[1])), s.N - 1)
            move, new, u_acc, changed, kind = rp.propose(pos, types, a, int(rec["slot"]), sw,
                                                         schedule == "checkerboard")
            assert rec["move"] == move and rec["kind"] == kind
            assert rec["t_log_u"] == pytest.approx(p.temperature * math.log(u_acc), rel=1e-14)
            if new is None:
                assert rec["exited"] == 1 and rec["accepted"] == 0
                continue
            assert rec["exited"] == 0
            e_new = rp.energy(*new)
            de = e_new - e
            if math.isinf(e_new):
                assert math.isinf(rec["delta_e"]) and rec["accepted"] == 0
                inf += 1
                continue
            tol = 1e-10 * (abs(rec["scale"]) + 1e-3 * abs(e)) + 1e-10
            assert abs(rec["delta_e"] - de) <= tol, (sw, a, move)
            assert rec["pair_terms"] == rp.terms(pos, types, changed) + rp.terms(*new, changed)
            accept = de <= 0 or p.temperature * math.log(u_acc) < -de
            if abs(de + p.temperature * math.log(u_acc)) > 1e-7 * (abs(rec["scale"]) + 1.0):
                assert bool(rec["accepted"]) == accept
            if rec["accepted"]:
                pos, types = new
                e = e_new
            checked += 1
            flips += move == 2
        st = s.get_state()
        assert np.array_equal(st["types"], types)
        d = st["pos"] - pos
        d -= s.box * np.round(d / s.box)
        assert np.max(np.abs(d)) < 1e-12
        assert st["e_acc"] == pytest.approx(e, rel=1e-9, abs=1e-9)
    return checked, flips, inf


@pytest.mark.parametrize("g,M,k,nc,rho", GEOMS)
def test_replay_checkerboard_every_attempt(g, M, k, nc, rho):
    # every attempt's proposal, cell exit, dE, pair-term count and decision
    # against the numpy replay from the definitions, from the lattice start
    p = flex.Params(n_molecules=M, temperature=2.0, geometry=g, colours_per_axis=k, cells_per_side=nc,
                    density=rho, seed=7)
    checked, flips, _ = _replay(p, 2 if g == flex.TRIANGLE else 1)
    assert checked > 300 and flips > 50


def test_replay_random_schedule():
    p = flex.Params(n_molecules=125, temperature=2.0, colours_per_axis=3, cells_per_side=3, seed=9)
    checked, _, _ = _replay(p, 2, schedule="random")
    assert checked > 500


def test_energy_invariant_accumulated_equals_resum():
    p = flex.Params(n_molecules=125, temperature=1.0, colours_per_axis=3, cells_per_side=3, seed=4)
    s = flex.System(p)
    s.sweep_checkerboard(30)
    e = s.energy()
    assert s.get_state()["e_acc"] == pytest.approx(e, rel=1e-9)


def test_fene_wall_rejects_and_bonds_never_reach_it():
    # a stretched triangle: bond 0-1 at r = 1.5 with types B, C (limit
    # 1.5 * 1.05 = 1.575).  The flips that put A next to B or C on that bond
    # (limits 1.425, 1.5) reach the wall: infinite dE, always rejected.  Hot
    # translations (T = 1e6) accept almost every finite move; no bond ever
    # reaches its limit.
    p = flex.Params(n_molecules=1, temperature=1e6, density=0.001, p_flip=0.5, colours_per_axis=2,
                    cells_per_side=2, seed=5)
    s = flex.System(p, lattice=False)
    L = s.box
    pos = np.array([[L / 2, L / 2, L / 2], [L / 2 + 1.5, L / 2, L / 2], [L / 2 + 0.75, L / 2 + 0.9, L / 2]])
    s.set_state(pos, np.array([1, 2, 0], dtype=np.uint8), 0)
    inf_flips = 0
    for _ in range(200):
        log = s.sweep_checkerboard(1, log=True)
        walls = np.isinf(log["delta_e"])
        assert not np.any(log["accepted"][walls])
        inf_flips += int(np.sum(walls & (log["move"] == 2)))
        st = s.get_state()
        x, ty = st["pos"], st["types"]
        sg = np.array([0.9, 1.0, 1.1])[ty]
        for i, j in [(0, 1), (1, 2), (0, 2)]:
            d = x[i] - x[j]
            d -= L * np.round(d / L)
            assert np.linalg.norm(d) < 1.5 * 0.5 * (sg[i] + sg[j])
    assert inf_flips > 0


@pytest.mark.parametrize("g", [flex.TRIANGLE, flex.SQUARE, flex.TETRAHEDRON])
def test_flip_chain_samples_boltzmann_exactly(g):
    # two molecules at fixed, perturbed (not ideal) positions, flips only:
    # the type states the flips reach (6, 8 or 4 per molecule) must be visited
    # with the Boltzmann weights of the numpy energies (intramolecular WCA +
    # FENE terms change with the types), by independent chains
    from scipy.stats import chisquare

    T = 1.5
    n = flex.SITES[g]
    sigma = _sigma(g)
    rng = np.random.default_rng(g)
    perms = bf.flips(g)
    # the orbit of the start types under the flips
    start = tuple(range(n))
    orbit, frontier = {start}, [start]
    while frontier:
        t = frontier.pop()
        for pm in perms:
            u = tuple(t[pm[s]] for s in range(n))
            if u not in orbit:
                orbit.add(u)
                frontier.append(u)
    orbit = sorted(orbit)
    assert len(orbit) == {flex.TRIANGLE: 6, flex.SQUARE: 8, flex.TETRAHEDRON: 4}[g]
    states = [(a, c) for a in orbit for c in orbit]
    mk = lambda seed: flex.Params(n_molecules=2, temperature=T, geometry=g, density=0.002, p_flip=1.0,  # noqa: E731
                                  colours_per_axis=2, cells_per_side=2, seed=seed)
    s = flex.System(mk(1), lattice=False)
    box = s.box
    side = flex.oracle.bond_length_star()
    for _ in range(500):
        c = np.array([[2.0, 2.0, 2.0], [2.0 + rng.uniform(1.2, 1.8), 2.3, 2.1]])
        pos = []
        for m in range(2):
            q = rng.normal(size=4)
            q /= np.linalg.norm(q)
            R = bf.quat_to_matrix(q)
            pos.append(c[m] + (bf.body(g, side) + rng.uniform(-0.08, 0.08, size=(n, 3))) @ R.T)
        pos = np.mod(np.concatenate(pos), box)
        E = np.array([bf.energy(pos, np.array(a + c, dtype=np.uint8), box, g, sigma) for a, c in states])
        if np.all(np.isfinite(E)) and T < np.ptp(E) < 8 * T:
            break
    else:
        pytest.fail("no suitable configuration")
    for i, (a, c) in enumerate(states):
        s.set_state(pos, np.array(a + c, dtype=np.uint8), 0)
        assert s.energy() == pytest.approx(E[i], rel=1e-12)
    pi = np.exp(-(E - E.min()) / T)
    pi /= pi.sum()
    idx = {st: i for i, st in enumerate(states)}
    n_chains = 3000
    counts = np.zeros(len(states))
    for ch_i in range(n_chains):
        ch = flex.System(mk(1000 + ch_i), lattice=False)
        ch.set_state(pos, np.array(orbit[0] + orbit[0], dtype=np.uint8), 0)
        ch.sweep_checkerboard(15)
        ty = ch.get_state()["types"]
        counts[idx[(tuple(ty[:n]), tuple(ty[n:]))]] += 1
    exp = pi * n_chains
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    stat, pval = chisquare(obs, ex * obs.sum() / ex.sum())
    assert pval > 1e-4, (stat, pval)


def test_invalid_parameters_are_rejected():
    # cells narrower than r_c + 2 sqrt(3) d = 1.58 (125 triangles: L = 6.79,
    # n_c = 6 gives 1.13): the 27 cells around an atom would miss partners
    with pytest.raises(ValueError):
        flex.System(flex.Params(n_molecules=125, temperature=1.0, colours_per_axis=3, cells_per_side=6))
    with pytest.raises(ValueError):
        flex.System(flex.Params(n_molecules=125, temperature=1.0, geometry=7))
    # same-colour cells closer than the worst-case reach 2 D + r_c are allowed:
    # the cells of a colour are then attempted in ascending index, and that
    # order defines the chain (125 squares at density 1.2: (k - 1) w = 4.98
    # below 2 * 3.2 + 1.23)
    p = flex.Params(n_molecules=125, temperature=1.0, geometry=flex.SQUARE, colours_per_axis=3, cells_per_side=3)
    s = flex.System(p)
    assert (3 - 1) * s.box / 3 < flex.reach(p)


def test_checkerboard_order_is_colour_cell_atom_ascending():
    # the attempt order that defines the chain when same-colour cells can
    # interact (125 squares at density 1.2, k = 3, n_c = 3: (k - 1) w below the
    # reach): colours in order, the cells of a colour in ascending index, the
    # atoms of a cell in ascending index, cells from the positions at the
    # sweep's start and the sweep's shift
    p = flex.Params(n_molecules=125, temperature=1.0, geometry=flex.SQUARE, colours_per_axis=3,
                    cells_per_side=3, density=1.2, seed=11)
    s = flex.System(p)
    rp = bf.Replayer(p, s.box)
    k = p.colours_per_axis
    nc = p.cells_per_side
    for sw in range(2):
        pos = s.get_state()["pos"].copy()
        h = rp.shift(sw)
        cells = np.array([rp.cell(pos[i], h) for i in range(s.N)])
        cx, cy, cz = cells % nc, (cells // nc) % nc, cells // (nc * nc)
        colour = (cx % k) + k * (cy % k) + k * k * (cz % k)
        want = np.lexsort((np.arange(s.N), cells, colour))
        log = s.sweep_checkerboard(1, log=True)
        got = log["atom"][np.argsort(log["seq"], kind="stable")]
        assert np.array_equal(got, want)
