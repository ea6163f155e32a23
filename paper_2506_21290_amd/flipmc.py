"""Python binding of the flip Monte Carlo C ABI (``include/flipmc.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libflipmc.so``.  PyTorch provides the device buffers and the streams.
The functions keep the C names; ``System`` and ``Batch`` are thin owners of
a handle plus its torch buffer.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflipmc.so")

MC_OK, MC_EINVAL, MC_ENOMEM, MC_EDEVICE, MC_EGEOM, MC_ENONFINITE, MC_EBUSY, MC_ENOTIMPL = (
    0, -1, -2, -3, -4, -5, -6, -7)
MC_FP64, MC_FP32_DE = 0, 1
MC_TRANSLATE, MC_ROTATE, MC_FLIP = 0, 1, 2
MC_FLAG_HBM_STATE, MC_FLAG_SINGLE_WORKGROUP, MC_FLAG_SERIAL_CELLS = 1, 2, 4
MC_ENGINE_LDS, MC_ENGINE_HBM, MC_ENGINE_SPREAD = 0, 1, 2
MC_GOFR_MAX_BINS = 256
MC_C2_MAX = 32

EXPORTED = [
    "mc_params_default", "mc_geometry", "mc_placement", "mc_engine", "mc_required_bytes",
    "mc_init_system", "mc_sweep",
    "mc_energy", "mc_observables", "mc_samples", "mc_reset_observables", "mc_get_state",
    "mc_set_state", "mc_decision_log", "mc_timing_enable", "mc_timing_read", "mc_destroy",
    "mc_last_error", "mc_batch_required_bytes", "mc_batch_create",
    "mc_batch_add", "mc_batch_run", "mc_batch_poll", "mc_batch_cancel", "mc_batch_destroy",
    "mc_batch_set_workgroups", "mc_batch_set_hbm_stream", "mc_dynamics",
    "mcf_params_default", "mcf_geometry", "mcf_placement", "mcf_required_bytes", "mcf_init_system",
    "mcf_sweep", "mcf_sweep_many",
    "mcf_energy", "mcf_observables", "mcf_reset_observables", "mcf_get_state", "mcf_set_state",
    "mcf_decision_log", "mcf_destroy", "mcf_init_system_noalloc", "mcf_dynamics",
]
MC_TRIANGLE, MC_SQUARE, MC_TETRAHEDRON = 0, 1, 2
SITES = {MC_TRIANGLE: 3, MC_SQUARE: 4, MC_TETRAHEDRON: 4}


class McError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"flipmc error {code}: {msg}")
        self.code = code


class mc_params(C.Structure):
    _fields_ = [
        ("n_molecules", C.c_uint32),
        ("precision", C.c_uint32),
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
        ("resum_interval", C.c_uint32),
        ("obs_interval", C.c_uint32),
        ("gofr_interval", C.c_uint32),
        ("obs_start", C.c_uint32),
        ("max_samples", C.c_uint32),
        ("flags", C.c_uint32),
        ("gofr_dr", C.c_double),
        ("barrier_polls", C.c_uint32),
        ("workgroups", C.c_uint32),
        ("fs_q", C.c_double),
        ("fs_q_cm", C.c_double),
    ]


class mc_obs(C.Structure):
    _fields_ = [
        ("sweep", C.c_uint64),
        ("attempts", C.c_uint64 * 3),
        ("accepts", C.c_uint64 * 3),
        ("exits", C.c_uint64),
        ("pair_terms", C.c_uint64),
        ("pair_tests", C.c_uint64),
        ("near_overflows", C.c_uint64),
        ("e_acc", C.c_double),
        ("e_resum", C.c_double),
        ("drift", C.c_double),
        ("max_abs_drift", C.c_double),
        ("resum_sweep", C.c_uint64),
        ("n_energy_samples", C.c_uint32),
        ("n_drift_samples", C.c_uint32),
        ("energy_sum", C.c_double),
        ("energy_sumsq", C.c_double),
        ("n_gofr_frames", C.c_uint32),
        ("gofr_nbins", C.c_uint32),
        ("gofr_dr", C.c_double),
        ("gofr_rmax", C.c_double),
        ("gofr_all", C.c_uint64 * MC_GOFR_MAX_BINS),
        ("gofr_inter", C.c_uint64 * MC_GOFR_MAX_BINS),
        ("n_c2", C.c_uint32),
        ("pad", C.c_uint32),
        ("c2_sweep", C.c_uint64 * MC_C2_MAX),
        ("c2", C.c_double * MC_C2_MAX),
        ("fs", C.c_double * MC_C2_MAX),
        ("fs_cm", C.c_double * MC_C2_MAX),
        ("c2_sq", C.c_double * MC_C2_MAX),
        ("fs_cm_sq", C.c_double * MC_C2_MAX),
        ("c2_fs_cm", C.c_double * MC_C2_MAX),
        ("fs_sq", C.c_double * MC_C2_MAX),
        ("gofr_norm_all", C.c_double * MC_GOFR_MAX_BINS),
        ("gofr_norm_inter", C.c_double * MC_GOFR_MAX_BINS),
    ]


class mcf_params(C.Structure):
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
        ("resum_interval", C.c_uint32),
        ("obs_interval", C.c_uint32),
        ("gofr_interval", C.c_uint32),
        ("obs_start", C.c_uint32),
        ("max_samples", C.c_uint32),
        ("flags", C.c_uint32),
        ("gofr_dr", C.c_double),
        ("fs_q", C.c_double),
        ("fs_q_cm", C.c_double),
    ]


class mc_dyn(C.Structure):
    _fields_ = [
        ("n_times", C.c_uint32),
        ("n_runs", C.c_uint32),
        ("t", C.c_uint64 * MC_C2_MAX),
        ("c2", C.c_double * MC_C2_MAX), ("fs", C.c_double * MC_C2_MAX),
        ("fs_cm", C.c_double * MC_C2_MAX),
        ("chi4_c2", C.c_double * MC_C2_MAX), ("chi4_fs", C.c_double * MC_C2_MAX),
        ("chi4_fs_cm", C.c_double * MC_C2_MAX),
        ("chi4s_c2", C.c_double * MC_C2_MAX), ("chi4s_fs", C.c_double * MC_C2_MAX),
        ("chi4s_fs_cm", C.c_double * MC_C2_MAX),
        ("rho", C.c_double * MC_C2_MAX),
        ("tau_c2", C.c_double), ("tau_fs", C.c_double), ("tau_fs_cm", C.c_double),
    ]


MOVE_RECORD_DTYPE = np.dtype(
    [
        ("delta_e", "<f8"), ("scale", "<f8"), ("t_log_u", "<f8"), ("sweep", "<u8"),
        ("molecule", "<u4"), ("move", "u1"), ("accepted", "u1"), ("exited", "u1"),
        ("axis", "u1"), ("pair_terms", "<u4"), ("pad", "<u4"),
    ]
)
assert MOVE_RECORD_DTYPE.itemsize == 48

_lib = None


def lib():
    """Load libflipmc.so; fails loudly when the HIP extension is missing."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime with the same soname as the system
        # one; loading torch first makes this library bind to that runtime, so
        # torch's streams and buffers and these kernels share one HIP instance
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')"
            )
        L = C.CDLL(LIB_PATH)
        vp, dp, u8p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint8)
        u32p, u64p, szp = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_size_t)
        pp = C.POINTER(mc_params)
        L.mc_params_default.argtypes = [pp]
        L.mc_params_default.restype = None
        L.mc_geometry.argtypes = [pp, dp, u32p, u32p]
        L.mc_placement.argtypes = [pp, C.POINTER(C.c_int), szp]
        L.mc_engine.argtypes = [pp, C.POINTER(C.c_int), u32p]
        L.mc_required_bytes.argtypes = [pp, szp]
        L.mc_init_system.argtypes = [pp, dp, dp, u8p, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.mc_sweep.argtypes = [vp, C.c_uint64]
        L.mc_energy.argtypes = [vp, dp, dp, dp]
        L.mc_observables.argtypes = [vp, C.POINTER(mc_obs)]
        L.mc_samples.argtypes = [vp, dp, dp, C.c_size_t, szp, szp]
        L.mc_reset_observables.argtypes = [vp]
        L.mc_get_state.argtypes = [vp, dp, dp, u8p, u64p, dp]
        L.mc_set_state.argtypes = [vp, dp, dp, u8p, C.c_uint64, C.c_double]
        L.mc_decision_log.argtypes = [vp, vp, C.c_size_t]
        L.mc_timing_enable.argtypes = [vp, C.c_int]
        L.mc_timing_read.argtypes = [vp, dp, u64p, dp, u64p]
        L.mc_destroy.argtypes = [vp]
        L.mc_destroy.restype = None
        L.mc_last_error.restype = C.c_char_p
        L.mc_batch_required_bytes.argtypes = [C.c_uint32, szp]
        L.mc_batch_create.argtypes = [C.c_uint32, C.c_uint32, vp, C.c_size_t, vp, vp, C.POINTER(vp)]
        L.mc_batch_add.argtypes = [vp, vp, C.c_uint64, u32p]
        L.mc_batch_run.argtypes = [vp, C.c_uint64, u32p]
        L.mc_batch_poll.argtypes = [vp, u32p, C.POINTER(vp), C.c_size_t, szp]
        L.mc_batch_cancel.argtypes = [vp, C.c_uint32]
        L.mc_batch_set_workgroups.argtypes = [vp, C.c_uint32]
        L.mc_batch_set_hbm_stream.argtypes = [vp, vp]
        L.mc_batch_destroy.argtypes = [vp]
        L.mc_batch_destroy.restype = None
        L.mc_dynamics.argtypes = [C.POINTER(mc_obs), C.c_size_t, C.c_uint32, C.POINTER(mc_dyn)]
        L.mcf_dynamics.argtypes = [C.POINTER(mc_obs), C.c_size_t, C.c_uint32, C.c_uint32, C.POINTER(mc_dyn)]
        fp = C.POINTER(mcf_params)
        L.mcf_params_default.argtypes = [fp, C.c_uint32]
        L.mcf_params_default.restype = None
        L.mcf_geometry.argtypes = [fp, dp, u32p, u32p]
        L.mcf_placement.argtypes = [fp, C.POINTER(C.c_int), szp]
        L.mcf_required_bytes.argtypes = [fp, szp]
        L.mcf_init_system.argtypes = [fp, dp, u8p, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.mcf_sweep.argtypes = [vp, C.c_uint64]
        L.mcf_sweep_many.argtypes = [C.POINTER(vp), C.c_uint32, C.c_uint64]
        L.mcf_energy.argtypes = [vp, dp, dp, dp]
        L.mcf_observables.argtypes = [vp, C.POINTER(mc_obs)]
        L.mcf_reset_observables.argtypes = [vp]
        L.mcf_get_state.argtypes = [vp, dp, u8p, u64p, dp]
        L.mcf_set_state.argtypes = [vp, dp, u8p, C.c_uint64, C.c_double]
        L.mcf_decision_log.argtypes = [vp, vp, C.c_size_t]
        L.mcf_init_system_noalloc.argtypes = [fp, dp, u8p, vp, C.c_size_t, szp, vp, C.POINTER(vp)]
        L.mcf_destroy.argtypes = [vp]
        L.mcf_destroy.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc != MC_OK:
        raise McError(rc, lib().mc_last_error().decode())


# Systems and batches still open at interpreter exit are closed by one atexit
# hook, registered after torch is imported (atexit runs last-in first-out, so
# the hook runs before torch's own and before the HIP runtime is torn down):
# batches first, then systems, newest first.  Each object holds its own
# reference to the library, so closing never depends on module globals that
# interpreter shutdown may already have cleared.
_live = []
_hook = []


def _track(obj):
    if not _hook:
        atexit.register(_close_all)
        _hook.append(True)
    _live.append(weakref.ref(obj))


def _close_all():
    objs = [r() for r in reversed(_live)]
    for o in objs:
        if isinstance(o, Batch):
            o.close()
    for o in objs:
        if isinstance(o, (System, FlexSystem)):
            o.close()
    _live.clear()


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ------------------------------------------------------------------ C names --

def mc_params_default(**overrides) -> mc_params:
    p = mc_params()
    lib().mc_params_default(C.byref(p))
    for k, v in overrides.items():
        if k == "sigma":
            p.sigma = (C.c_double * 3)(*v)
        else:
            setattr(p, k, v)
    return p


def mc_geometry(p: mc_params):
    box, k, nc = C.c_double(), C.c_uint32(), C.c_uint32()
    _check(lib().mc_geometry(C.byref(p), C.byref(box), C.byref(k), C.byref(nc)))
    return box.value, k.value, nc.value


def mc_placement(p: mc_params):
    """(resident in LDS?, dynamic LDS bytes per launch)"""
    r, n = C.c_int(), C.c_size_t()
    _check(lib().mc_placement(C.byref(p), C.byref(r), C.byref(n)))
    return bool(r.value), n.value


def mc_engine(p: mc_params):
    """(MC_ENGINE_*, workgroups per launch) that mc_sweep uses for p"""
    e, w = C.c_int(), C.c_uint32()
    _check(lib().mc_engine(C.byref(p), C.byref(e), C.byref(w)))
    return e.value, w.value


def mc_required_bytes(p: mc_params) -> int:
    n = C.c_size_t()
    _check(lib().mc_required_bytes(C.byref(p), C.byref(n)))
    return n.value


def mc_dynamics(runs, n_molecules, atoms_per_molecule=None) -> dict:
    """Ensemble means, chi_4 (Eq. 10), chi_4^self (Eq. 11), rho (Eq. 13) and
    the 1/e relaxation times of independent runs (mc_obs structures) of rigid
    molecules (mc_dynamics), or of flexible ones with atoms_per_molecule
    given (mcf_dynamics)."""
    arr = (mc_obs * len(runs))(*runs)
    d = mc_dyn()
    if atoms_per_molecule is None:
        _check(lib().mc_dynamics(arr, len(runs), int(n_molecules), C.byref(d)))
    else:
        _check(lib().mcf_dynamics(arr, len(runs), int(n_molecules), int(atoms_per_molecule), C.byref(d)))
    n = d.n_times
    out = {"t": np.array(d.t[:n], dtype=np.uint64), "n_runs": d.n_runs}
    for k in ("c2", "fs", "fs_cm", "chi4_c2", "chi4_fs", "chi4_fs_cm", "chi4s_c2", "chi4s_fs",
              "chi4s_fs_cm", "rho"):
        out[k] = np.array(getattr(d, k)[:n])
    for k in ("tau_c2", "tau_fs", "tau_fs_cm"):
        v = getattr(d, k)
        out[k] = None if math.isnan(v) else v
    return out


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream), stream


class System:
    """One Markov chain whose state lives in a torch-owned device buffer."""

    def __init__(self, params: mc_params, com=None, quat=None, types=None, stream=None, device="cuda"):
        import torch

        self.params = params
        self.M = params.n_molecules
        nbytes = mc_required_bytes(params)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._stream_handle, self.stream = _stream_handle(stream)
        h = C.c_void_p()
        if com is None:
            args = (None, None, None)
        else:
            com = np.ascontiguousarray(com, dtype=np.float64).reshape(-1)
            quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1)
            types = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
            args = (_ptr(com, C.c_double), _ptr(quat, C.c_double), _ptr(types, C.c_uint8))
        self._lib = lib()
        _check(self._lib.mc_init_system(C.byref(params), *args, C.c_void_p(self.buffer.data_ptr()),
                                        nbytes, self._stream_handle, C.byref(h)))
        self.h = h
        self._log = None
        _track(self)

    def close(self):
        """Wait for the system's kernels, release its handle, then its buffer."""
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.mc_destroy(h)  # synchronises its stream (and its batch's)
        self.h = None
        self.buffer = None
        self._log = None

    def __del__(self):
        self.close()

    def sweep(self, n=1):
        _check(lib().mc_sweep(self.h, int(n)))

    def energy(self):
        e, em, d = C.c_double(), C.c_double(), C.c_double()
        _check(lib().mc_energy(self.h, C.byref(e), C.byref(em), C.byref(d)))
        return e.value, em.value, d.value

    def obs_struct(self) -> mc_obs:
        """The accumulators as the C structure (the input of mc_dynamics)."""
        o = mc_obs()
        _check(self._lib.mc_observables(self.h, C.byref(o)))
        return o

    def observables(self) -> dict:
        o = self.obs_struct()
        nb = o.gofr_nbins
        return {
            "sweep": o.sweep,
            "attempts": np.array(o.attempts[:], dtype=np.uint64),
            "accepts": np.array(o.accepts[:], dtype=np.uint64),
            "exits": o.exits,
            "pair_terms": o.pair_terms,
            "pair_tests": o.pair_tests,
            "near_overflows": o.near_overflows,
            "e_acc": o.e_acc,
            "e_resum": o.e_resum,
            "drift": o.drift,
            "max_abs_drift": o.max_abs_drift,
            "resum_sweep": o.resum_sweep,
            "n_energy_samples": o.n_energy_samples,
            "n_drift_samples": o.n_drift_samples,
            "energy_sum": o.energy_sum,
            "energy_sumsq": o.energy_sumsq,
            "n_gofr_frames": o.n_gofr_frames,
            "gofr_dr": o.gofr_dr,
            "gofr_rmax": o.gofr_rmax,
            "gofr_all": np.array(o.gofr_all[:nb], dtype=np.uint64),
            "gofr_inter": np.array(o.gofr_inter[:nb], dtype=np.uint64),
            "gofr_norm_all": np.array(o.gofr_norm_all[:nb]),
            "gofr_norm_inter": np.array(o.gofr_norm_inter[:nb]),
            "c2_sweep": np.array(o.c2_sweep[: o.n_c2], dtype=np.uint64),
            "c2": np.array(o.c2[: o.n_c2]),
            "fs": np.array(o.fs[: o.n_c2]),
            "fs_cm": np.array(o.fs_cm[: o.n_c2]),
            "c2_sq": np.array(o.c2_sq[: o.n_c2]),
            "fs_cm_sq": np.array(o.fs_cm_sq[: o.n_c2]),
            "c2_fs_cm": np.array(o.c2_fs_cm[: o.n_c2]),
            "fs_sq": np.array(o.fs_sq[: o.n_c2]),
        }

    def samples(self, cap=None):
        cap = cap or self.params.max_samples
        e = np.zeros(cap)
        d = np.zeros(cap)
        ne, nd = C.c_size_t(), C.c_size_t()
        _check(lib().mc_samples(self.h, _ptr(e, C.c_double), _ptr(d, C.c_double), cap,
                                C.byref(ne), C.byref(nd)))
        return e[: ne.value], d[: nd.value]

    def reset_observables(self):
        _check(lib().mc_reset_observables(self.h))

    def get_state(self):
        M = self.M
        com, quat = np.zeros(3 * M), np.zeros(4 * M)
        types = np.zeros(3 * M, dtype=np.uint8)
        sweep, e = C.c_uint64(), C.c_double()
        _check(lib().mc_get_state(self.h, _ptr(com, C.c_double), _ptr(quat, C.c_double),
                                  _ptr(types, C.c_uint8), C.byref(sweep), C.byref(e)))
        return {"com": com.reshape(M, 3), "quat": quat.reshape(M, 4), "types": types.reshape(M, 3),
                "sweep": sweep.value, "e_acc": e.value}

    def set_state(self, com, quat, types, sweep, e_acc=math.nan):
        com = np.ascontiguousarray(com, dtype=np.float64).reshape(-1)
        quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1)
        types = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
        _check(lib().mc_set_state(self.h, _ptr(com, C.c_double), _ptr(quat, C.c_double),
                                  _ptr(types, C.c_uint8), int(sweep), float(e_acc)))

    def decision_log(self, n_sweeps):
        """Record the next n_sweeps sweeps; returns a torch buffer of records."""
        import torch

        if n_sweeps <= 0:
            _check(lib().mc_decision_log(self.h, None, 0))
            self._log = None
            return None
        cap = n_sweeps * self.M
        buf = torch.zeros(cap * MOVE_RECORD_DTYPE.itemsize, dtype=torch.uint8, device=self.buffer.device)
        _check(lib().mc_decision_log(self.h, C.c_void_p(buf.data_ptr()), cap))
        self._log = buf
        return buf

    def timing_enable(self, on=True):
        _check(lib().mc_timing_enable(self.h, 1 if on else 0))

    def timing_read(self):
        a, b = C.c_double(), C.c_double()
        na, nb = C.c_uint64(), C.c_uint64()
        _check(lib().mc_timing_read(self.h, C.byref(a), C.byref(na), C.byref(b), C.byref(nb)))
        return {"sweep_ms": a.value, "sweep_launches": na.value, "event_ms": b.value,
                "event_launches": nb.value}

    def read_log(self):
        if self._log is None:
            return None
        self.stream.synchronize()
        return np.frombuffer(self._log.cpu().numpy().tobytes(), dtype=MOVE_RECORD_DTYPE).copy()


class Batch:
    """Several systems advanced together, one time slice per run: one workgroup
    each, spare workgroups to the large systems with the most work left."""

    def __init__(self, max_slots, precision=MC_FP32_DE, stream=None, aux_stream=None,
                 hbm_stream=None, device="cuda"):
        import torch

        self._stream_handle, self.stream = _stream_handle(stream)
        # the multi-workgroup launches overlap the others on a second stream,
        # and the one-workgroup launch of systems with their state in HBM the
        # LDS class's on a third (default priority, like every stream here)
        self.aux_stream = aux_stream if aux_stream is not None else torch.cuda.Stream()
        self.hbm_stream = hbm_stream if hbm_stream is not None else torch.cuda.Stream()
        self._lib = lib()
        n = C.c_size_t()
        _check(self._lib.mc_batch_required_bytes(int(max_slots), C.byref(n)))
        self.buffer = torch.empty(n.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(self._lib.mc_batch_create(int(max_slots), int(precision),
                                         C.c_void_p(self.buffer.data_ptr()), n.value,
                                         self._stream_handle, C.c_void_p(self.aux_stream.cuda_stream),
                                         C.byref(h)))
        self.h = h
        _check(self._lib.mc_batch_set_hbm_stream(h, C.c_void_p(self.hbm_stream.cuda_stream)))
        self.max_slots = max_slots
        self.members = {}
        _track(self)

    def close(self):
        """Wait for the batch's streams and release it (its systems stay open)."""
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.mc_batch_destroy(h)
        self.h = None
        self.buffer = None

    def __del__(self):
        self.close()

    def add(self, system: System, n_sweeps) -> int:
        slot = C.c_uint32()
        _check(lib().mc_batch_add(self.h, system.h, int(n_sweeps), C.byref(slot)))
        self.members[slot.value] = system
        return slot.value

    def set_workgroups(self, max_workgroups=0):
        """At most max_workgroups workgroups at once (0 = one per compute unit)."""
        _check(lib().mc_batch_set_workgroups(self.h, int(max_workgroups)))

    def run(self, max_moves_per_slot=0) -> int:
        n = C.c_uint32()
        _check(lib().mc_batch_run(self.h, int(max_moves_per_slot), C.byref(n)))
        return n.value

    def poll(self):
        cap = self.max_slots
        slots = np.zeros(cap, dtype=np.uint32)
        systems = (C.c_void_p * cap)()
        n = C.c_size_t()
        _check(lib().mc_batch_poll(self.h, _ptr(slots, C.c_uint32), systems, cap, C.byref(n)))
        done = []
        for i in range(n.value):
            done.append((int(slots[i]), self.members.pop(int(slots[i]))))
        return done

    def cancel(self, slot):
        _check(lib().mc_batch_cancel(self.h, int(slot)))
        return self.members.pop(int(slot))


# ------------------------------------------------------ flexible molecules --

def mcf_params_default(geometry=MC_TRIANGLE, **overrides) -> mcf_params:
    p = mcf_params()
    lib().mcf_params_default(C.byref(p), int(geometry))
    for k, v in overrides.items():
        if k == "sigma":
            p.sigma = (C.c_double * 4)(*(list(v) + [0.0] * (4 - len(v))))
        else:
            setattr(p, k, v)
    return p


def mcf_geometry(p: mcf_params):
    box, k, nc = C.c_double(), C.c_uint32(), C.c_uint32()
    _check(lib().mcf_geometry(C.byref(p), C.byref(box), C.byref(k), C.byref(nc)))
    return box.value, k.value, nc.value


def mcf_placement(p: mcf_params):
    """(positions, types and cell lists resident in LDS?, dynamic LDS bytes)"""
    r, n = C.c_int(), C.c_size_t()
    _check(lib().mcf_placement(C.byref(p), C.byref(r), C.byref(n)))
    return bool(r.value), n.value


def mcf_required_bytes(p: mcf_params) -> int:
    n = C.c_size_t()
    _check(lib().mcf_required_bytes(C.byref(p), C.byref(n)))
    return n.value


class FlexSystem:
    """One Markov chain of flexible molecules (atoms as the moving unit) in a
    torch-owned device buffer."""

    def __init__(self, params: mcf_params, pos=None, types=None, stream=None, device="cuda",
                 no_alloc=False):
        """no_alloc: create it with mcf_init_system_noalloc (the work arrays
        in the library's static scratch, the buffer holds the state only)."""
        import torch

        self.params = params
        self.n = SITES[params.geometry]
        self.M = params.n_molecules
        self.N = self.n * self.M
        self._lib = lib()
        if pos is None:
            args = (None, None)
        else:
            pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
            types = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
            args = (_ptr(pos, C.c_double), _ptr(types, C.c_uint8))
        if no_alloc:
            need = C.c_size_t()
            _check(self._lib.mcf_init_system_noalloc(C.byref(params), *args, None, 0, C.byref(need),
                                                     None, None))
            nbytes = need.value
        else:
            nbytes = mcf_required_bytes(params)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._stream_handle, self.stream = _stream_handle(stream)
        h = C.c_void_p()
        if no_alloc:
            _check(self._lib.mcf_init_system_noalloc(C.byref(params), *args,
                                                     C.c_void_p(self.buffer.data_ptr()), nbytes, None,
                                                     self._stream_handle, C.byref(h)))
        else:
            _check(self._lib.mcf_init_system(C.byref(params), *args, C.c_void_p(self.buffer.data_ptr()),
                                             nbytes, self._stream_handle, C.byref(h)))
        self.h = h
        self._log = None
        _track(self)

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.mcf_destroy(h)
        self.h = None
        self.buffer = None
        self._log = None

    def __del__(self):
        self.close()

    def sweep(self, n=1):
        _check(self._lib.mcf_sweep(self.h, int(n)))

    def energy(self):
        e, em, d = C.c_double(), C.c_double(), C.c_double()
        _check(self._lib.mcf_energy(self.h, C.byref(e), C.byref(em), C.byref(d)))
        return e.value, em.value, d.value

    def obs_struct(self) -> mc_obs:
        o = mc_obs()
        _check(self._lib.mcf_observables(self.h, C.byref(o)))
        return o

    def observables(self) -> dict:
        o = self.obs_struct()
        nb = o.gofr_nbins
        return {
            "sweep": o.sweep, "attempts": np.array(o.attempts[:], dtype=np.uint64),
            "accepts": np.array(o.accepts[:], dtype=np.uint64), "exits": o.exits,
            "pair_terms": o.pair_terms, "e_acc": o.e_acc, "e_resum": o.e_resum, "drift": o.drift,
            "max_abs_drift": o.max_abs_drift, "n_energy_samples": o.n_energy_samples,
            "energy_sum": o.energy_sum, "energy_sumsq": o.energy_sumsq,
            "n_gofr_frames": o.n_gofr_frames, "gofr_dr": o.gofr_dr,
            "gofr_all": np.array(o.gofr_all[:nb], dtype=np.uint64),
            "gofr_inter": np.array(o.gofr_inter[:nb], dtype=np.uint64),
            "gofr_norm_all": np.array(o.gofr_norm_all[:nb]),
            "gofr_norm_inter": np.array(o.gofr_norm_inter[:nb]),
            "c2_sweep": np.array(o.c2_sweep[: o.n_c2], dtype=np.uint64),
            "c2": np.array(o.c2[: o.n_c2]), "fs": np.array(o.fs[: o.n_c2]),
            "fs_cm": np.array(o.fs_cm[: o.n_c2]),
            "c2_sq": np.array(o.c2_sq[: o.n_c2]), "fs_cm_sq": np.array(o.fs_cm_sq[: o.n_c2]),
            "c2_fs_cm": np.array(o.c2_fs_cm[: o.n_c2]), "fs_sq": np.array(o.fs_sq[: o.n_c2]),
        }

    def reset_observables(self):
        _check(self._lib.mcf_reset_observables(self.h))

    def get_state(self):
        pos = np.zeros(3 * self.N)
        types = np.zeros(self.N, dtype=np.uint8)
        sweep, e = C.c_uint64(), C.c_double()
        _check(self._lib.mcf_get_state(self.h, _ptr(pos, C.c_double), _ptr(types, C.c_uint8),
                                       C.byref(sweep), C.byref(e)))
        return {"pos": pos.reshape(self.N, 3), "types": types, "sweep": sweep.value, "e_acc": e.value}

    def set_state(self, pos, types, sweep, e_acc=math.nan):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
        types = np.ascontiguousarray(types, dtype=np.uint8).reshape(-1)
        _check(self._lib.mcf_set_state(self.h, _ptr(pos, C.c_double), _ptr(types, C.c_uint8),
                                       int(sweep), float(e_acc)))

    def decision_log(self, n_sweeps):
        import torch

        if n_sweeps <= 0:
            _check(self._lib.mcf_decision_log(self.h, None, 0))
            self._log = None
            return None
        cap = n_sweeps * self.N
        buf = torch.zeros(cap * MOVE_RECORD_DTYPE.itemsize, dtype=torch.uint8, device=self.buffer.device)
        _check(self._lib.mcf_decision_log(self.h, C.c_void_p(buf.data_ptr()), cap))
        self._log = buf
        return buf

    def read_log(self):
        if self._log is None:
            return None
        self.stream.synchronize()
        return np.frombuffer(self._log.cpu().numpy().tobytes(), dtype=MOVE_RECORD_DTYPE).copy()


def flex_sweep_many(systems, n=1):
    """n timesteps of each FlexSystem in `systems`, one workgroup per system
    (mcf_sweep_many); all must share one stream."""
    arr = (C.c_void_p * len(systems))(*[x.h for x in systems])
    _check(lib().mcf_sweep_many(arr, len(systems), int(n)))
