"""Pins of the oracle's self-intermediate scattering functions F_s(q, t) and
F_s^cm(q, t) (Sec. III.B, Eqs. 5 and 6) and of the unwrapped positions they
are built on.  None of these needs a GPU."""
import math

import numpy as np
import pytest


def _sphere_average(d, q, n_mu=64, n_phi=128):
    # Mean over the unit sphere of exp(i q n . d), for every row of d, by a
    # Gauss-Legendre rule in cos(theta) times the trapezoid rule in phi (both
    # spectrally accurate for this entire integrand); then the mean over rows.
    mu, w = np.polynomial.legendre.leggauss(n_mu)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1 - mu ** 2)
    n = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(mu, np.ones(n_phi))], axis=-1).reshape(-1, 3)
    wt = np.repeat(w / 2, n_phi) / n_phi
    e = np.exp(1j * q * (np.asarray(d) @ n.T))
    return complex(np.mean(e @ wt))


@pytest.mark.parametrize("q", [5.1, 7.4])
def test_isotropic_average_equals_direction_average(oracle_mod, q):
    # The reading of "average over wavevectors of modulus q": the full
    # spherical average of exp(i q . d).  Brute force over directions.
    rng = np.random.default_rng(7)
    d = rng.normal(size=(40, 3)) * rng.uniform(0, 1.2, size=(40, 1))
    d[0] = 0.0
    ref = _sphere_average(d, q)
    assert abs(ref.imag) < 1e-13
    assert oracle_mod.fs_isotropic(d, q) == pytest.approx(ref.real, abs=1e-12)


def test_fs_is_one_at_the_origin(oracle_mod):
    p = oracle_mod.Params(n_molecules=64, temperature=3.0, seed=3)
    s = oracle_mod.System(p)
    s.sweep_checkerboard(5)
    ref = s.unwrapped()
    assert s.fs(ref) == (1.0, 1.0)


def test_common_translation_closed_form(oracle_mod):
    # Every centre moved by the same vector delta: both functions equal
    # sin(q |delta|) / (q |delta|), the sites moving with their centre.
    p = oracle_mod.Params(n_molecules=27, temperature=3.0, colours_per_axis=3, cells_per_side=3)
    s = oracle_mod.System(p)
    st = s.get_state()
    ref = s.unwrapped()
    delta = np.array([0.11, -0.23, 0.05])
    s.set_state(st["com"] + delta, st["quat"], st["types"], 0)
    x = np.linalg.norm(delta)
    fs, fs_cm = s.fs(ref, q=7.4, q_cm=5.1)
    assert fs == pytest.approx(math.sin(7.4 * x) / (7.4 * x), abs=1e-14)
    assert fs_cm == pytest.approx(math.sin(5.1 * x) / (5.1 * x), abs=1e-14)


def test_common_rotation_closed_form(oracle_mod):
    # Every molecule in the body frame (a triangle in the xy plane centred on
    # its centre of mass, circumradius R = b / sqrt 3), then turned by theta
    # about z: each site moves along a chord 2 R sin(theta / 2) and the
    # centres stay, so F_s = sinc(q * chord) and F_s^cm = 1.
    M = 27
    p = oracle_mod.Params(n_molecules=M, temperature=3.0, colours_per_axis=3, cells_per_side=3)
    s = oracle_mod.System(p)
    st = s.get_state()
    s.set_state(st["com"], np.tile([1.0, 0, 0, 0], (M, 1)), st["types"], 0)
    ref = s.unwrapped()
    theta = 0.9
    s.set_state(st["com"], np.tile([math.cos(theta / 2), 0, 0, math.sin(theta / 2)], (M, 1)),
                st["types"], 0)
    chord = 2 * oracle_mod.bond_length_star() / math.sqrt(3) * math.sin(theta / 2)
    fs, fs_cm = s.fs(ref, q=7.4)
    assert fs_cm == 1.0
    assert fs == pytest.approx(math.sin(7.4 * chord) / (7.4 * chord), abs=1e-14)


def test_flips_move_no_site(oracle_mod):
    # A flip exchanges the types of two sites but not their indices, so a run
    # of flips alone leaves both functions at exactly 1.
    p = oracle_mod.Params(n_molecules=64, temperature=3.0, p_flip=1.0, p_translate=0.0)
    s = oracle_mod.System(p)
    ref = s.unwrapped()
    t0 = s.get_state()["types"].copy()
    s.sweep_checkerboard(10)
    assert s.counters()["accepts"][oracle_mod.FLIP] > 100
    assert not np.array_equal(s.get_state()["types"], t0)
    assert s.fs(ref) == (1.0, 1.0)


def test_unwrapped_centres_follow_every_translation(oracle_mod):
    # Sweep by sweep, with steps far below L / 2: the unwrapped displacement of
    # each centre is the minimum image of its wrapped displacement, and the
    # unwrapped centre wraps back onto the stored one.  Many centres cross the
    # boundary, so a wrong sign or a missing image count fails here.
    p = oracle_mod.Params(n_molecules=64, temperature=1e6, seed=5, p_flip=0.0, p_translate=1.0,
                          max_displacement=0.35)
    s = oracle_mod.System(p)
    L = s.box
    prev_w = s.get_state()["com"].copy()
    prev_u = s.unwrapped()[0]
    crossed = 0
    for _ in range(30):
        s.sweep_random(1)
        w = s.get_state()["com"]
        u = s.unwrapped()[0]
        dw = w - prev_w
        np.testing.assert_allclose(u - prev_u, dw - L * np.rint(dw / L), atol=1e-12)
        np.testing.assert_allclose(u - L * np.floor(u / L), w, atol=1e-12)
        crossed += int(np.sum(np.abs(dw) > L / 2))
        prev_w, prev_u = w.copy(), u
    assert crossed >= 20
    ref_u = s.unwrapped()
    fs, fs_cm = s.fs(ref_u)
    assert (fs, fs_cm) == (1.0, 1.0)


def test_moment_helpers_are_library_statistics(oracle_mod):
    rng = np.random.default_rng(3)
    x, y = rng.normal(size=500), rng.normal(size=500)
    y = 0.6 * x + 0.8 * y
    assert oracle_mod.chi4_self(x) == pytest.approx(np.var(x), rel=1e-12)
    assert oracle_mod.pearson(x, y) == pytest.approx(np.corrcoef(x, y)[0, 1], rel=1e-12)
    assert oracle_mod.chi4(x, 64) == pytest.approx(64 * np.var(x), rel=1e-12)


@pytest.mark.parametrize("same", [True, False])
def test_two_populations_closed_forms(oracle_mod, same):
    # Even molecules turned by theta about the triangle's normal; odd ones (or,
    # when `same`, the even ones too) moved by delta.  Each contribution then
    # takes two values, so the per-particle variance is (a - b)^2 / 4 and the
    # Pearson coefficient of Eq. 13 is +1 (same molecules rotate and move) or
    # -1 (the movers are the molecules that did not rotate).
    M = 64
    p = oracle_mod.Params(n_molecules=M, temperature=3.0, colours_per_axis=2, cells_per_side=2)
    s = oracle_mod.System(p)
    st = s.get_state()
    ident = np.tile([1.0, 0, 0, 0], (M, 1))
    s.set_state(st["com"], ident, st["types"], 0)
    ref = s.unwrapped()
    u0, kref = s.orientation_ref()
    theta, delta = 0.8, np.array([0.2, 0.1, -0.3])
    even = np.arange(M) % 2 == 0
    quat = ident.copy()
    quat[even] = [math.cos(theta / 2), 0, 0, math.sin(theta / 2)]
    com = st["com"].copy()
    com[even if same else ~even] += delta
    s.set_state(com, quat, st["types"], 0)
    c2_i, fcm_i, fs_i = s.particle_terms(ref, u0, kref, q=7.4, q_cm=5.1)
    p2 = 0.5 * (3 * math.cos(theta) ** 2 - 1)
    x = 5.1 * np.linalg.norm(delta)
    fd = math.sin(x) / x
    assert oracle_mod.chi4_self(c2_i) == pytest.approx((1 - p2) ** 2 / 4, abs=1e-14)
    assert oracle_mod.chi4_self(fcm_i) == pytest.approx((1 - fd) ** 2 / 4, abs=1e-14)
    assert oracle_mod.pearson(c2_i, fcm_i) == pytest.approx(1.0 if same else -1.0, abs=1e-12)
    assert len(fs_i) == 3 * M and np.all(fs_i <= 1.0)
