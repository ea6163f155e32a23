"""ctypes wrapper around the serial FP64 oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library; the C source is ``flipmc_oracle.c`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FLIPMC_ORACLE_SANITIZE=1 builds and loads a copy instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer (a process that loads it
# needs the ASan runtime preloaded; tests/test_sanitizers.py does that).
SANITIZE = os.environ.get("FLIPMC_ORACLE_SANITIZE") == "1"
LIB_PATH = os.path.join(HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")
SRC_PATH = os.path.join(HERE, "flipmc_oracle.c")
SOURCES = [SRC_PATH, os.path.join(HERE, "flex_oracle.c")]

TRANSLATE, ROTATE, FLIP = 0, 1, 2

RECORD_DTYPE = np.dtype(
    [
        ("delta_e", "<f8"),
        ("scale", "<f8"),
        ("t_log_u", "<f8"),
        ("sweep", "<u8"),
        ("molecule", "<u4"),
        ("slot", "<u4"),
        ("move", "u1"),
        ("accepted", "u1"),
        ("exited", "u1"),
        ("axis", "u1"),
        ("pair_terms", "<u4"),
        ("seq", "<u4"),
        ("pad", "<u4"),
    ]
)
assert RECORD_DTYPE.itemsize == 56


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (serial, FP64, no FMA contraction)."""
    stale = not os.path.exists(LIB_PATH) or any(
        os.path.getmtime(LIB_PATH) < os.path.getmtime(f)
        for f in SOURCES + [os.path.join(HERE, "flipmc_oracle.h"), os.path.join(HERE, "flex_oracle.h")])
    if force or stale:
        san = (["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"] if SANITIZE else [])
        subprocess.check_call(
            [
                "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", *san,
                "-fPIC", "-shared", *SOURCES, "-o", LIB_PATH, "-lm",
            ]
        )
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [
        ("n_molecules", C.c_uint32),
        ("density", C.c_double),
        ("temperature", C.c_double),
        ("sigma", C.c_double * 3),
        ("bond_length", C.c_double),
        ("p_flip", C.c_double),
        ("p_translate", C.c_double),
        ("max_displacement", C.c_double),
        ("max_rotation", C.c_double),
        ("seed", C.c_uint64),
        ("colours_per_axis", C.c_uint32),
        ("cells_per_side", C.c_uint32),
    ]


@dataclass
class Params:
    """Model and schedule parameters (Sec. II of the paper, plus the readings
    for the rigid body, the move set and the checkerboard)."""

    n_molecules: int
    temperature: float
    density: float = 1.2
    sigma: tuple = (0.9, 1.0, 1.1)
    bond_length: float = 0.0  # 0 -> b*, the minimum of WCA + FENE
    p_flip: float = 0.2
    p_translate: float = 0.4
    max_displacement: float = 0.1
    max_rotation: float = 0.2
    seed: int = 1
    colours_per_axis: int = 2
    cells_per_side: int = 2

    def to_c(self) -> _Params:
        p = _Params()
        p.n_molecules = self.n_molecules
        p.density = self.density
        p.temperature = self.temperature
        p.sigma = (C.c_double * 3)(*self.sigma)
        p.bond_length = self.bond_length
        p.p_flip = self.p_flip
        p.p_translate = self.p_translate
        p.max_displacement = self.max_displacement
        p.max_rotation = self.max_rotation
        p.seed = self.seed
        p.colours_per_axis = self.colours_per_axis
        p.cells_per_side = self.cells_per_side
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_u32.restype = C.c_double
        L.or_u32.argtypes = [C.c_uint32]
        L.or_u53.restype = C.c_double
        L.or_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.or_u53_left.restype = C.c_double
        L.or_u53_left.argtypes = [C.c_uint32, C.c_uint32]
        L.or_bond_length_star.restype = C.c_double
        L.or_wca.restype = C.c_double
        L.or_wca.argtypes = [C.c_double, C.c_double]
        L.or_fene.restype = C.c_double
        L.or_fene.argtypes = [C.c_double, C.c_double]
        L.or_box_length.restype = C.c_double
        L.or_box_length.argtypes = [C.c_uint32, C.c_double]
        L.or_stencil_reach.restype = C.c_double
        L.or_stencil_reach.argtypes = [dp, C.c_double]
        L.or_rotation_matrix.argtypes = [dp, dp]
        L.or_body_frame.argtypes = [C.c_double, dp]
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(_Params), C.c_char_p]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_init_lattice.argtypes = [C.c_void_p]
        L.or_set_state.argtypes = [C.c_void_p, dp, dp, u8p, C.c_uint64, C.c_double]
        L.or_get_state.argtypes = [C.c_void_p, dp, dp, u8p, u64p, dp]
        L.or_box.restype = C.c_double
        L.or_box.argtypes = [C.c_void_p]
        L.or_cell_width.restype = C.c_double
        L.or_cell_width.argtypes = [C.c_void_p]
        L.or_sites.argtypes = [C.c_void_p, dp]
        L.or_energy.restype = C.c_double
        L.or_energy.argtypes = [C.c_void_p]
        L.or_energy_intra.restype = C.c_double
        L.or_energy_intra.argtypes = [C.c_void_p]
        L.or_sweep_checkerboard.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64]
        L.or_sweep_random.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p]
        L.or_cell_of.argtypes = [C.c_void_p, dp, C.c_uint64]
        L.or_shift.argtypes = [C.c_void_p, C.c_uint64, dp]
        L.or_counters.argtypes = [C.c_void_p, u64p, u64p, u64p, u64p]
        L.or_gofr_bins.argtypes = [C.c_double, C.c_double, dp]
        L.or_gofr_accumulate.argtypes = [C.c_void_p, C.c_double, C.c_int, u64p, u64p]
        L.or_orientation_ref.argtypes = [C.c_void_p, dp, u8p]
        L.or_c2.restype = C.c_double
        L.or_c2.argtypes = [C.c_void_p, dp, u8p]
        L.or_unwrapped.argtypes = [C.c_void_p, dp, dp]
        L.or_c2_terms.argtypes = [C.c_void_p, dp, u8p, dp]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def u32(w):
    return lib().or_u32(int(w))


def u53(lo, hi):
    return lib().or_u53(int(lo), int(hi))


def u53_left(lo, hi):
    return lib().or_u53_left(int(lo), int(hi))


def bond_length_star():
    return lib().or_bond_length_star()


def wca(r2, sigma_ij):
    return lib().or_wca(float(r2), float(sigma_ij))


def fene(r, sigma_ij):
    return lib().or_fene(float(r), float(sigma_ij))


def box_length(m, density=1.2):
    return lib().or_box_length(int(m), float(density))


def stencil_reach(sigma=(0.9, 1.0, 1.1), bond_length=None):
    s = np.asarray(sigma, dtype=np.float64)
    b = bond_length_star() if bond_length is None else bond_length
    return lib().or_stencil_reach(_p(s, C.c_double), float(b))


def rotation_matrix(q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    r = np.zeros(9)
    lib().or_rotation_matrix(_p(q, C.c_double), _p(r, C.c_double))
    return r.reshape(3, 3)


def body_frame(bond_length=None):
    b = bond_length_star() if bond_length is None else bond_length
    out = np.zeros(9)
    lib().or_body_frame(float(b), _p(out, C.c_double))
    return out.reshape(3, 3)


def gofr_bins(box, dr=0.02):
    rm = C.c_double()
    n = lib().or_gofr_bins(float(box), float(dr), C.byref(rm))
    return n, rm.value


def gofr_normalise(counts, frames, n_sites, box, dr):
    """Eq. (3): g(r_b) = counts_b / (frames N rho (4 pi / 3)(r_{b+1}^3 - r_b^3)),
    rho = N / L^3, bin b = [b dr, (b + 1) dr); zeros without frames."""
    counts = np.asarray(counts, dtype=np.float64)
    if frames == 0:
        return np.zeros_like(counts)
    r = np.arange(len(counts) + 1) * dr
    shell = 4.0 * np.pi / 3.0 * (r[1:] ** 3 - r[:-1] ** 3)
    rho = n_sites / box ** 3
    return counts / (frames * n_sites * rho * shell)


class System:
    """One oracle Markov chain."""

    def __init__(self, params: Params, lattice: bool = True):
        self.params = params
        err = C.create_string_buffer(256)
        self._cp = params.to_c()
        h = lib().or_create(C.byref(self._cp), err)
        if not h:
            raise ValueError(err.value.decode())
        self.h = h
        self.M = params.n_molecules
        if lattice:
            rc = lib().or_init_lattice(self.h)
            if rc != 0:
                raise ValueError("lattice start needs M = n^3")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().or_destroy(h)
            self.h = None

    @property
    def box(self):
        return lib().or_box(self.h)

    @property
    def cell_width(self):
        return lib().or_cell_width(self.h)

    def get_state(self):
        M = self.M
        com = np.zeros(3 * M)
        quat = np.zeros(4 * M)
        types = np.zeros(3 * M, dtype=np.uint8)
        sweep = C.c_uint64()
        e = C.c_double()
        lib().or_get_state(
            self.h, _p(com, C.c_double), _p(quat, C.c_double), _p(types, C.c_uint8),
            C.byref(sweep), C.byref(e),
        )
        return {
            "com": com.reshape(M, 3), "quat": quat.reshape(M, 4),
            "types": types.reshape(M, 3), "sweep": sweep.value, "e_acc": e.value,
        }

    def set_state(self, com, quat, types, sweep, e_acc=None):
        com = np.ascontiguousarray(com, dtype=np.float64).reshape(-1)
        quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1)
        types = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
        assert com.size == 3 * self.M and quat.size == 4 * self.M and types.size == 3 * self.M
        lib().or_set_state(
            self.h, _p(com, C.c_double), _p(quat, C.c_double), _p(types, C.c_uint8),
            int(sweep), 0.0,
        )
        if e_acc is None:
            e_acc = self.energy()
        lib().or_set_state(
            self.h, _p(com, C.c_double), _p(quat, C.c_double), _p(types, C.c_uint8),
            int(sweep), float(e_acc),
        )

    def sites(self):
        out = np.zeros(9 * self.M)
        lib().or_sites(self.h, _p(out, C.c_double))
        return out.reshape(self.M, 3, 3)

    def energy(self):
        return lib().or_energy(self.h)

    def energy_intra(self):
        return lib().or_energy_intra(self.h)

    def sweep_checkerboard(self, n=1, log=False, cell_order_seed=0):
        rec = np.zeros(n * self.M, dtype=RECORD_DTYPE) if log else None
        ptr = rec.ctypes.data if log else None
        lib().or_sweep_checkerboard(self.h, int(n), ptr, int(cell_order_seed))
        return rec

    def sweep_random(self, n=1, log=False):
        rec = np.zeros(n * self.M, dtype=RECORD_DTYPE) if log else None
        ptr = rec.ctypes.data if log else None
        lib().or_sweep_random(self.h, int(n), ptr)
        return rec

    def shift(self, sweep):
        h = np.zeros(3)
        lib().or_shift(self.h, int(sweep), _p(h, C.c_double))
        return h

    def cell_of(self, c, sweep):
        c = np.ascontiguousarray(c, dtype=np.float64)
        return lib().or_cell_of(self.h, _p(c, C.c_double), int(sweep))

    def counters(self):
        a = np.zeros(3, dtype=np.uint64)
        b = np.zeros(3, dtype=np.uint64)
        e = C.c_uint64()
        t = C.c_uint64()
        lib().or_counters(self.h, _p(a, C.c_uint64), _p(b, C.c_uint64), C.byref(e), C.byref(t))
        return {"attempts": a, "accepts": b, "exits": e.value, "pair_terms": t.value}

    def gofr_accumulate(self, counts_all, counts_inter, dr=0.02):
        assert counts_all.dtype == np.uint64 and counts_inter.dtype == np.uint64
        lib().or_gofr_accumulate(
            self.h, float(dr), int(counts_all.size), _p(counts_all, C.c_uint64),
            _p(counts_inter, C.c_uint64),
        )

    def orientation_ref(self):
        u0 = np.zeros(3 * self.M)
        k = np.zeros(self.M, dtype=np.uint8)
        lib().or_orientation_ref(self.h, _p(u0, C.c_double), _p(k, C.c_uint8))
        return u0, k

    def c2(self, u0, kref):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        kref = np.ascontiguousarray(kref, dtype=np.uint8)
        return lib().or_c2(self.h, _p(u0, C.c_double), _p(kref, C.c_uint8))

    def unwrapped(self):
        """(centres (M, 3), sites (3M, 3)) followed through the periodic
        boundaries since the last lattice start or set_state."""
        com = np.zeros(3 * self.M)
        site = np.zeros(9 * self.M)
        lib().or_unwrapped(self.h, _p(com, C.c_double), _p(site, C.c_double))
        return com.reshape(self.M, 3), site.reshape(3 * self.M, 3)

    def fs(self, ref, q=7.4, q_cm=5.1):
        """(F_s(q, t), F_s^cm(q_cm, t)) from the reference ``ref`` =
        ``unwrapped()`` at t = 0; see ``fs_isotropic``."""
        com, site = self.unwrapped()
        return fs_isotropic(site - ref[1], q), fs_isotropic(com - ref[0], q_cm)


    def c2_terms(self, u0, kref):
        out = np.zeros(self.M)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        kref = np.ascontiguousarray(kref, dtype=np.uint8)
        lib().or_c2_terms(self.h, _p(u0, C.c_double), _p(kref, C.c_uint8), _p(out, C.c_double))
        return out

    def particle_terms(self, ref, u0, kref, q=7.4, q_cm=5.1):
        """Per-particle contributions (Sec. V.A) since the reference
        (``ref`` = unwrapped(), ``u0, kref`` = orientation_ref() at t = 0):
        C_2^i per molecule, F_s^cm,i per molecule and F_s^i per site, the
        last two direction-averaged like ``fs_isotropic``."""
        com, site = self.unwrapped()
        return (self.c2_terms(u0, kref), sinc_terms(com - ref[0], q_cm),
                sinc_terms(site - ref[1], q))


def sinc_terms(d, q):
    """sin(q |d|) / (q |d|) of each row of d: the mean of exp(i q . d) over
    all directions of a wavevector of modulus q."""
    x = q * np.sqrt(np.sum(np.asarray(d, dtype=np.float64) ** 2, axis=1))
    return np.sinc(x / np.pi)


def chi4_self(c_i):
    """Self part of the four-point susceptibility (Sec. V.B, Eq. 11): the
    variance of the per-particle contributions."""
    c_i = np.asarray(c_i, dtype=np.float64)
    return float(np.mean(c_i ** 2) - np.mean(c_i) ** 2)


def pearson(c2_i, fcm_i):
    """Pearson coefficient of Eq. 13 between C_2^i and F_s^cm,i."""
    c2_i = np.asarray(c2_i, dtype=np.float64)
    fcm_i = np.asarray(fcm_i, dtype=np.float64)
    cov = np.mean(c2_i * fcm_i) - np.mean(c2_i) * np.mean(fcm_i)
    return float(cov / np.sqrt(chi4_self(c2_i) * chi4_self(fcm_i)))


def chi4(c_hat, n):
    """Four-point susceptibility (Sec. V.B, Eq. 10) from the instantaneous
    values c_hat of one correlation in independent runs: n times their
    variance, n = M for a molecular correlation, 3M for sites."""
    c_hat = np.asarray(c_hat, dtype=np.float64)
    return float(n * (np.mean(c_hat ** 2) - np.mean(c_hat) ** 2))


def relaxation_time(t, c, level=float(np.exp(-1.0))):
    """Sec. III.C: the time at which a correlation c(t), sampled at times t,
    first falls to `level` (1/e), linear in ln t between the two samples
    around the crossing; None if it never falls that far."""
    for i in range(1, len(t)):
        if c[i] <= level < c[i - 1]:
            x0, x1 = np.log(float(t[i - 1])), np.log(float(t[i]))
            return float(np.exp(x0 + (x1 - x0) * (c[i - 1] - level) / (c[i - 1] - c[i])))
    return None


def fs_isotropic(d, q):
    """Self-intermediate scattering function (Sec. III.B, Eqs. 5 and 6) of the
    displacements d (n, 3), averaged over every direction of a wavevector of
    modulus q: the mean over a sphere of exp(i q . d) is sin(q |d|) / (q |d|),
    so F_s is the mean of that over the n particles.  The paper averages over
    wavevectors whose modulus is near q; the full spherical average at exactly
    q is the reading taken here."""
    return float(np.mean(sinc_terms(d, q)))
