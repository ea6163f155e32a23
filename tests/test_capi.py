"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/flipmc.h declares, and rejects bad parameters with a
status code and a message before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2506_21290_amd import flipmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "flipmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcf?_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "mc_init_system" in names and "mc_sweep" in names
    assert "mc_energy" in names and "mc_observables" in names
    L = C.CDLL(flipmc.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(flipmc.EXPORTED)


def test_params_default_matches_the_paper():
    p = flipmc.mc_params_default()
    assert list(p.sigma) == [0.9, 1.0, 1.1]  # Sec. II.A
    assert p.density == 1.2 and p.p_flip == 0.2
    assert p.p_translate == 0.4 and p.max_displacement == 0.1 and p.max_rotation == 0.2


def test_geometry_choices():
    # (k - 1) w must reach W = 2^(1/6) 1.1 + 2 b*/sqrt(3) ~ 2.3443
    for M in [64, 216, 512, 1000, 1728, 8000, 27000]:
        p = flipmc.mc_params_default(n_molecules=M)
        L, k, nc = flipmc.mc_geometry(p)
        assert L == pytest.approx((3 * M / 1.2) ** (1 / 3), rel=1e-14)
        assert nc % k == 0 and (k - 1) * L / nc >= 2.3442
    p = flipmc.mc_params_default(n_molecules=1000, colours_per_axis=3, cells_per_side=9)
    assert flipmc.mc_geometry(p)[1:] == (3, 9)


@pytest.mark.parametrize(
    "kw,code",
    [
        (dict(n_molecules=0), flipmc.MC_EINVAL),
        (dict(temperature=-1.0), flipmc.MC_EINVAL),
        (dict(precision=7), flipmc.MC_EINVAL),
        (dict(p_flip=0.8, p_translate=0.4), flipmc.MC_EINVAL),
        (dict(n_molecules=1000, colours_per_axis=2, cells_per_side=6), flipmc.MC_EGEOM),
        (dict(n_molecules=1000, colours_per_axis=3, cells_per_side=8), flipmc.MC_EGEOM),
        (dict(n_molecules=1000, colours_per_axis=4, cells_per_side=8), flipmc.MC_EGEOM),
        (dict(n_molecules=8, density=1.2), flipmc.MC_EGEOM),
    ],
)
def test_invalid_parameters(kw, code):
    p = flipmc.mc_params_default(**kw)
    with pytest.raises(flipmc.McError) as e:
        flipmc.mc_required_bytes(p)
    assert e.value.code == code
    assert len(flipmc.lib().mc_last_error()) > 0


def test_init_rejects_bad_buffers_without_a_device():
    L = flipmc.lib()
    p = flipmc.mc_params_default(n_molecules=64)
    h = C.c_void_p()
    assert L.mc_init_system(C.byref(p), None, None, None, None, 0, None, C.byref(h)) == flipmc.MC_EINVAL
    nbytes = flipmc.mc_required_bytes(p)
    fake = C.c_void_p(0x100000)
    rc = L.mc_init_system(C.byref(p), None, None, None, fake, nbytes - 1, None, C.byref(h))
    assert rc == flipmc.MC_ENOMEM
    p2 = flipmc.mc_params_default(n_molecules=100)  # not a cube: no lattice start
    assert L.mc_init_system(C.byref(p2), None, None, None, fake, 1 << 30, None, C.byref(h)) == flipmc.MC_EINVAL
    assert b"n^3" in L.mc_last_error()


def test_required_bytes_grows_with_state():
    a = flipmc.mc_required_bytes(flipmc.mc_params_default(n_molecules=1000))
    b = flipmc.mc_required_bytes(flipmc.mc_params_default(n_molecules=1000, flags=flipmc.MC_FLAG_HBM_STATE))
    c = flipmc.mc_required_bytes(flipmc.mc_params_default(n_molecules=8000))
    assert a < b < c
    assert a < 1 << 20


def test_box_must_hold_twice_the_reach():
    # The engine forms pair terms from the nearest image of two centres plus
    # the site offsets; that is every site pair's nearest image only when
    # L >= 2 (W + 2 d_max), W = 2^(1/6) 1.1 + 2 b*/sqrt(3).  27 molecules at
    # density 1.2 (L = 4.07, which k = 3, n_c = 3 would otherwise accept) and
    # 48 (L = 4.93) are rejected; 56 (L = 5.19) and 64 (L = 5.43) are not.
    W = 2 ** (1 / 6) * 1.1 + 2 * 0.9608971989592554 / 3 ** 0.5
    for M, ok in [(27, False), (48, False), (56, True), (64, True)]:
        L = (3 * M / 1.2) ** (1 / 3)
        assert (L >= 2 * (W + 0.2)) == ok
        p = flipmc.mc_params_default(n_molecules=M, colours_per_axis=3, cells_per_side=3)
        if ok:
            assert flipmc.mc_geometry(p)[0] == pytest.approx(L, rel=1e-14)
        else:
            with pytest.raises(flipmc.McError) as e:
                flipmc.mc_geometry(p)
            assert e.value.code == flipmc.MC_EGEOM


def test_noalloc_size_query_and_limit_without_a_device():
    # the state part of the buffer (the work arrays go to the static scratch),
    # and a clear MC_ENOMEM when the work arrays would exceed the scratch
    L = flipmc.lib()
    p = flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=1000)
    need = C.c_size_t()
    assert L.mcf_init_system_noalloc(C.byref(p), None, None, None, 0, C.byref(need), None, None) == 0
    assert 0 < need.value < flipmc.mcf_required_bytes(p)
    big = flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=100 ** 3)
    rc = L.mcf_init_system_noalloc(C.byref(big), None, None, None, 0, C.byref(need), None, None)
    assert rc == flipmc.MC_ENOMEM and b"static scratch" in L.mc_last_error()


def test_flexible_placement_without_a_device():
    # the paper's 1000 molecules (3000 or 4000 atoms) fit one workgroup's LDS
    # (160 KiB on gfx950, the fallback when no device answers); MC_FLAG_HBM_STATE
    # and 8000 triangles (24000 atoms) keep the state in the buffer
    for g in (flipmc.MC_TRIANGLE, flipmc.MC_SQUARE, flipmc.MC_TETRAHEDRON):
        res, lds = flipmc.mcf_placement(flipmc.mcf_params_default(g, n_molecules=1000))
        assert res and 3 * 8 * 1000 * flipmc.SITES[g] < lds < 160 * 1024
    res, lds = flipmc.mcf_placement(flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=1000,
                                                              flags=flipmc.MC_FLAG_HBM_STATE))
    assert not res and lds == 0
    assert not flipmc.mcf_placement(flipmc.mcf_params_default(flipmc.MC_TRIANGLE, n_molecules=8000))[0]


def test_flexible_sweep_many_rejects_empty_lists_without_a_device():
    L = flipmc.lib()
    assert L.mcf_sweep_many(None, 0, 1) == flipmc.MC_EINVAL
    arr = (C.c_void_p * 2)(None, None)
    assert L.mcf_sweep_many(arr, 2, 1) == flipmc.MC_EINVAL
    assert b"null system" in L.mc_last_error()


def test_batch_setters_reject_a_null_batch_without_a_device():
    L = flipmc.lib()
    assert L.mc_batch_set_workgroups(None, 8) == flipmc.MC_EINVAL
    assert L.mc_batch_set_hbm_stream(None, None) == flipmc.MC_EINVAL
    assert b"null batch" in L.mc_last_error()
