"""ctypes wrapper around the flexible-molecule oracle (``flex_oracle.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may import it.  It shares no code with the
HIP library.  The model is the paper's own molecule (Sec. II.A: atoms joined by
FENE bonds, WCA between all atoms) and the other bodies of its outlook
(Sec. VII); see ``flex_oracle.h``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from . import oracle

TRIANGLE, SQUARE, TETRAHEDRON = 0, 1, 2
TRANSLATE, FLIP = 0, 2
SITES = {TRIANGLE: 3, SQUARE: 4, TETRAHEDRON: 4}
# four types of diameters evenly spaced over the paper's [0.9, 1.1]
SIGMA4 = (0.9, 0.9 + 0.2 / 3, 0.9 + 0.4 / 3, 1.1)

RECORD_DTYPE = np.dtype(
    [
        ("delta_e", "<f8"), ("scale", "<f8"), ("t_log_u", "<f8"), ("sweep", "<u8"),
        ("atom", "<u4"), ("slot", "<u4"), ("move", "u1"), ("accepted", "u1"), ("exited", "u1"),
        ("kind", "u1"), ("pair_terms", "<u4"), ("seq", "<u4"), ("pad", "<u4"),
    ]
)
assert RECORD_DTYPE.itemsize == 56


class _Params(C.Structure):
    _fields_ = [
        ("geometry", C.c_uint32),
        ("n_molecules", C.c_uint32),
        ("density", C.c_double),
        ("temperature", C.c_double),
        ("sigma", C.c_double * 4),
        ("bond_length", C.c_double),
        ("p_flip", C.c_double),
        ("max_displacement", C.c_double),
        ("seed", C.c_uint64),
        ("colours_per_axis", C.c_uint32),
        ("cells_per_side", C.c_uint32),
    ]


@dataclass
class Params:
    n_molecules: int
    temperature: float
    geometry: int = TRIANGLE
    density: float = 1.2
    sigma: tuple = None
    bond_length: float = 0.0
    p_flip: float = 0.2
    max_displacement: float = 0.1
    seed: int = 1
    colours_per_axis: int = 3
    cells_per_side: int = 3

    def to_c(self) -> _Params:
        p = _Params()
        p.geometry = self.geometry
        p.n_molecules = self.n_molecules
        p.density = self.density
        p.temperature = self.temperature
        sg = self.sigma or ((0.9, 1.0, 1.1, 0.0) if self.geometry == TRIANGLE else SIGMA4)
        p.sigma = (C.c_double * 4)(*(list(sg) + [0.0] * (4 - len(sg))))
        p.bond_length = self.bond_length
        p.p_flip = self.p_flip
        p.max_displacement = self.max_displacement
        p.seed = self.seed
        p.colours_per_axis = self.colours_per_axis
        p.cells_per_side = self.cells_per_side
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = oracle.lib()
        dp, u8p, u64p = C.POINTER(C.c_double), C.POINTER(C.c_uint8), C.POINTER(C.c_uint64)
        L.fx_sites.restype = C.c_uint32
        L.fx_sites.argtypes = [C.c_uint32]
        L.fx_flip_kinds.restype = C.c_uint32
        L.fx_flip_kinds.argtypes = [C.c_uint32]
        L.fx_box_length.restype = C.c_double
        L.fx_box_length.argtypes = [C.c_uint32, C.c_uint32, C.c_double]
        L.fx_reach.restype = C.c_double
        L.fx_reach.argtypes = [C.POINTER(_Params)]
        L.fx_create.restype = C.c_void_p
        L.fx_create.argtypes = [C.POINTER(_Params), C.c_char_p]
        L.fx_destroy.argtypes = [C.c_void_p]
        L.fx_init_lattice.argtypes = [C.c_void_p]
        L.fx_set_state.argtypes = [C.c_void_p, dp, u8p, C.c_uint64, C.c_double]
        L.fx_get_state.argtypes = [C.c_void_p, dp, u8p, u64p, dp]
        L.fx_box.restype = C.c_double
        L.fx_box.argtypes = [C.c_void_p]
        L.fx_energy.restype = C.c_double
        L.fx_energy.argtypes = [C.c_void_p]
        L.fx_energy_inter.restype = C.c_double
        L.fx_energy_inter.argtypes = [C.c_void_p]
        L.fx_sweep_checkerboard.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64]
        L.fx_sweep_random.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p]
        L.fx_counters.argtypes = [C.c_void_p, u64p, u64p, u64p, u64p]
        L.fx_gofr_accumulate.argtypes = [C.c_void_p, C.c_double, C.c_int, u64p, u64p]
        L.fx_orientation_ref.argtypes = [C.c_void_p, dp, u8p]
        L.fx_c2_terms.argtypes = [C.c_void_p, dp, u8p, dp]
        L.fx_unwrapped.argtypes = [C.c_void_p, dp, dp]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def box_length(geometry, m, density=1.2):
    return lib().fx_box_length(geometry, m, density)


def reach(params: Params):
    return lib().fx_reach(C.byref(params.to_c()))


class System:
    """One oracle Markov chain of flexible molecules."""

    def __init__(self, params: Params, lattice: bool = True):
        self.params = params
        err = C.create_string_buffer(256)
        self._c = params.to_c()
        h = lib().fx_create(C.byref(self._c), err)
        if not h:
            raise ValueError(err.value.decode())
        self.h = h
        self.n = SITES[params.geometry]
        self.M = params.n_molecules
        self.N = self.n * self.M
        if lattice and lib().fx_init_lattice(self.h) != 0:
            raise ValueError("lattice start needs n_molecules = n^3")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().fx_destroy(h)
            self.h = None

    @property
    def box(self):
        return lib().fx_box(self.h)

    def get_state(self):
        pos = np.zeros(3 * self.N)
        types = np.zeros(self.N, dtype=np.uint8)
        sweep, e = C.c_uint64(), C.c_double()
        lib().fx_get_state(self.h, _p(pos, C.c_double), _p(types, C.c_uint8), C.byref(sweep),
                           C.byref(e))
        return {"pos": pos.reshape(self.N, 3), "types": types, "sweep": sweep.value, "e_acc": e.value}

    def set_state(self, pos, types, sweep, e_acc=None):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
        types = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
        assert pos.size == 3 * self.N and types.size == self.N
        lib().fx_set_state(self.h, _p(pos, C.c_double), _p(types, C.c_uint8), int(sweep),
                           float("nan") if e_acc is None else float(e_acc))

    def energy(self):
        return lib().fx_energy(self.h)

    def energy_inter(self):
        return lib().fx_energy_inter(self.h)

    def sweep_checkerboard(self, n=1, log=False, cell_order_seed=0):
        rec = np.zeros(n * self.N, dtype=RECORD_DTYPE) if log else None
        ptr = rec.ctypes.data_as(C.c_void_p) if log else None
        lib().fx_sweep_checkerboard(self.h, int(n), ptr, int(cell_order_seed))
        return rec

    def sweep_random(self, n=1, log=False):
        rec = np.zeros(n * self.N, dtype=RECORD_DTYPE) if log else None
        ptr = rec.ctypes.data_as(C.c_void_p) if log else None
        lib().fx_sweep_random(self.h, int(n), ptr)
        return rec

    def counters(self):
        a = np.zeros(3, dtype=np.uint64)
        b = np.zeros(3, dtype=np.uint64)
        e, t = C.c_uint64(), C.c_uint64()
        lib().fx_counters(self.h, _p(a, C.c_uint64), _p(b, C.c_uint64), C.byref(e), C.byref(t))
        return {"attempts": a, "accepts": b, "exits": e.value, "pair_terms": t.value}

    def gofr_accumulate(self, counts_all, counts_inter, dr=0.02):
        lib().fx_gofr_accumulate(self.h, float(dr), int(counts_all.size), _p(counts_all, C.c_uint64),
                                 _p(counts_inter, C.c_uint64))

    def orientation_ref(self):
        u0 = np.zeros(3 * self.M)
        k = np.zeros(self.M, dtype=np.uint8)
        lib().fx_orientation_ref(self.h, _p(u0, C.c_double), _p(k, C.c_uint8))
        return u0, k

    def c2_terms(self, u0, kref):
        out = np.zeros(self.M)
        lib().fx_c2_terms(self.h, _p(np.ascontiguousarray(u0), C.c_double),
                          _p(np.ascontiguousarray(kref, dtype=np.uint8), C.c_uint8),
                          _p(out, C.c_double))
        return out

    def c2(self, u0, kref):
        return float(np.mean(self.c2_terms(u0, kref)))

    def unwrapped(self):
        atoms = np.zeros(3 * self.N)
        centres = np.zeros(3 * self.M)
        lib().fx_unwrapped(self.h, _p(atoms, C.c_double), _p(centres, C.c_double))
        return atoms.reshape(self.N, 3), centres.reshape(self.M, 3)
