"""ctypes mirror of include/iat.h and the loader of libiat.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiat.so")

IAT_EINVAL, IAT_EHIP, IAT_EWORKSPACE, IAT_ENOTSUP = -1, -2, -3, -4
ST_COMPLEX, ST_BOUND_SEEN, ST_EXITED = 1 << 0, 1 << 1, 1 << 2
ST_TMAX, ST_H_UNDERFLOW, ST_NONFINITE, ST_MAX_STEPS = 1 << 8, 1 << 9, 1 << 10, 1 << 11
ST_R_UNDERFLOW, ST_WARN_R0, ST_ADJ_SKIPPED = 1 << 12, 1 << 13, 1 << 14
MAX_SPECIES = 8
NOALLOC_MAX_N = 65536
N_STATS, N_PHASES = 11, 5
GEN_ARRAYS, GEN_GRID, GEN_SWEEP, GEN_THERMAL = 0, 1, 2, 3
KERNEL_PLAIN, KERNEL_PERSISTENT = 1, 2
REDUCE_CELLS, REDUCE_W0_HIST, REDUCE_BOXCOUNT, REDUCE_LIFETIME, REDUCE_W0_HIST_BOUND = 1, 2, 3, 4, 5
W0_BINS, HEAT_BINS, LIFE_BINS, LIFE_SLOT = 64, 256, 96, 98

EXPORTS = ["iat_integrate", "iat_integrate_noalloc", "iat_integrate_tangent", "iat_adjoint", "iat_reduce", "iat_adjoint_workspace_bytes",
           "iat_workspace_bytes", "iat_fp64_peak", "iat_last_error", "iat_version", "iat_release"]
WS_INTEGRATE, WS_REDUCE, WS_ADJOINT = 1, 2, 3

_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class Species(ctypes.Structure):
    _fields_ = [("m_atom", _d), ("C4", _d)]


class System(ctypes.Structure):
    _fields_ = [("m_ion", _d), ("omega_rf", _d), ("a_x", _d), ("q_x", _d), ("a_ratio", _d * 3),
                ("q_ratio", _d * 3), ("E", _d), ("De", _d), ("phase0", _d), ("species", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("r0", _d), ("t_max", _d), ("rtol", _d), ("atol", _d),
                ("h0", _d), ("hmax", _d), ("hmin", _d), ("r_bounce_over_rm", _d), ("max_steps", ctypes.c_int64)]


class Gen(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("n_species", ctypes.c_int32), ("species", ctypes.c_int32 * 8), ("n_E", ctypes.c_int32),
                ("n_q", ctypes.c_int32), ("n_De", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("E", _d * 8), ("q", _d * 8), ("De", _d * 8), ("E_lo", _d), ("E_hi", _d), ("q_lo", _d),
                ("q_hi", _d), ("De_lo", _d), ("De_hi", _d), ("seed", ctypes.c_uint64), ("id0", ctypes.c_int64),
                ("T_ion", _d)]


class Batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("theta", _vp), ("phi", _vp), ("E", _vp), ("q_x", _vp), ("De", _vp),
                ("phase0", _vp), ("species", _vp), ("y0", _vp), ("id0_dev", _vp), ("gen", Gen)]


class Obs(ctypes.Structure):
    _fields_ = [("angle", _vp), ("q_transfer", _vp), ("dE_ion", _vp), ("t_dwell", _vp),
                ("t_bounce_first", _vp), ("t_bounce_last", _vp), ("n_bounce", _vp), ("status", _vp),
                ("n_accept", _vp), ("n_reject", _vp), ("n_rhs", _vp), ("y_final", _vp)]


class Launch(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("refill_every", ctypes.c_int32), ("step_budget", ctypes.c_int32),
                ("max_suspended", ctypes.c_int32), ("tail_budget", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("stats", _vp), ("kernel_ms", _vp)]


_P = ctypes.POINTER
_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load libiat.so (built in-tree by __graft_entry__.build()); fail loudly when absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; "
                             f"g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    L.iat_integrate.argtypes = [_P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs), _P(Launch), _vp,
                                ctypes.c_size_t, _vp]
    L.iat_integrate.restype = ctypes.c_int
    L.iat_integrate_noalloc.argtypes = [_P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs), _P(Launch), _vp]
    L.iat_integrate_noalloc.restype = ctypes.c_int
    L.iat_reduce.argtypes = [_P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs), ctypes.c_int, _vp, _vp]
    L.iat_reduce.restype = ctypes.c_int
    L.iat_integrate_tangent.argtypes = [_P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs), _vp, _vp,
                                        _vp, _vp, _P(Launch), _vp]
    L.iat_integrate_tangent.restype = ctypes.c_int
    L.iat_adjoint.argtypes = [_P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs), _vp, _vp, _vp, _vp,
                              ctypes.c_size_t, _P(Launch), _vp]
    L.iat_adjoint.restype = ctypes.c_int
    L.iat_adjoint_workspace_bytes.argtypes = [_P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs),
                                              _P(ctypes.c_size_t), _vp]
    L.iat_adjoint_workspace_bytes.restype = ctypes.c_int
    L.iat_workspace_bytes.argtypes = [ctypes.c_int, _P(System), _P(Species), ctypes.c_int, _P(Batch), _P(Obs),
                                      _P(Launch), ctypes.c_int, _P(ctypes.c_size_t), _vp]
    L.iat_workspace_bytes.restype = ctypes.c_int
    L.iat_fp64_peak.argtypes = [_vp, ctypes.c_int64, ctypes.c_int, _P(ctypes.c_double), _vp]
    L.iat_fp64_peak.restype = ctypes.c_int
    L.iat_last_error.restype = ctypes.c_char_p
    L.iat_version.restype = ctypes.c_char_p
    L.iat_release.restype = None
    _lib = L
    return L


class IatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libiat error {code}: {msg}")
        self.code = code


def check(rc: int):
    if rc != 0:
        raise IatError(rc, load().iat_last_error().decode())
