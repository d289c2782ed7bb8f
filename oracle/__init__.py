"""ctypes front end of the CPU oracle (liboracle.so, built from oracle/*.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline
leg are the only users.  Nothing here imports the HIP library package, and the
library never imports this.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# Round-off twin: the same sources compiled with FMA contraction.  Its spread from the main
# build measures how strongly a trajectory amplifies round-off (its conditioning).
TWIN_PATH = os.path.join(HERE, "liboracle_twin.so")
SOURCES = ["iat_oracle.c", "iat_oracle_tangent.c"]

COMPLEX, BOUND_SEEN, EXITED = 1 << 0, 1 << 1, 1 << 2
TMAX, H_UNDERFLOW, NONFINITE, MAX_STEPS, R_UNDERFLOW, WARN_R0 = (1 << 8, 1 << 9, 1 << 10, 1 << 11,
                                                                1 << 12, 1 << 13)

PROBLEM = np.dtype([
    ("m_ion", "f8"), ("m_atom", "f8"), ("C4", "f8"), ("De", "f8"), ("omega", "f8"),
    ("a", "f8", 3), ("q", "f8", 3), ("phase0", "f8"), ("r0", "f8"), ("t_max", "f8"),
    ("rtol", "f8"), ("atol", "f8"), ("h0", "f8"), ("hmax", "f8"), ("hmin", "f8"),
    ("r_bounce_over_rm", "f8"), ("max_steps", "i8"), ("y0", "f8", 12), ("exit_centre", "i8")])
RESULT = np.dtype([
    ("angle", "f8"), ("q_transfer", "f8"), ("dE_ion", "f8"), ("t_dwell", "f8"),
    ("t_first", "f8"), ("t_last", "f8"), ("n_bounce", "i4"), ("status", "u4"),
    ("n_accept", "i8"), ("n_reject", "i8"), ("n_rhs", "i8"), ("tau_final", "f8"),
    ("y_final", "f8", 12)])


class _Sweep(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_species", ctypes.c_int32), ("n_E", ctypes.c_int32),
                ("n_q", ctypes.c_int32), ("n_De", ctypes.c_int32), ("species", ctypes.c_int32 * 8),
                ("E", ctypes.c_double * 8), ("q", ctypes.c_double * 8), ("De", ctypes.c_double * 8),
                ("E_lo", ctypes.c_double), ("E_hi", ctypes.c_double), ("q_lo", ctypes.c_double),
                ("q_hi", ctypes.c_double), ("De_lo", ctypes.c_double), ("De_hi", ctypes.c_double)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain IEEE FP64: no fast-math, no FMA contraction) and
    its round-off twin liboracle_twin.so (identical sources, FMA contraction on)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not force and os.path.exists(LIB_PATH) and os.path.exists(TWIN_PATH):
        return LIB_PATH
    base = ["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math"]
    for path, extra in ((LIB_PATH, ["-ffp-contract=off"]), (TWIN_PATH, ["-mfma", "-ffp-contract=fast"])):
        subprocess.check_call(base + extra + ["-o", path + ".tmp", *srcs, "-lm"])
        os.replace(path + ".tmp", path)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.orc_integrate.argtypes = [vp, vp]
        L.orc_integrate_record.argtypes = [vp, vp, dp, ctypes.c_int64]
        L.orc_integrate_batch.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_int]
        L.orc_headon_state.argtypes = [ctypes.c_double] * 5 + [dp]
        L.orc_grid_angles.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_thermal_normals.argtypes = [ctypes.c_int64, ctypes.c_uint64, dp]
        L.orc_sweep_draw.argtypes = [ctypes.c_int64, ctypes.POINTER(_Sweep), dp, dp, dp, dp, dp, dp,
                                     ctypes.POINTER(ctypes.c_int32)]
        L.orc_observables.argtypes = [vp, dp, dp, ctypes.c_double, dp, dp, dp]
        L.orc_ion_energy.argtypes = [vp, dp, ctypes.c_double]
        L.orc_ion_energy.restype = ctypes.c_double
        L.orc_tableau.argtypes = [dp, dp, dp, dp]
        L.orc_rhs_au.argtypes = [vp, ctypes.c_double, dp, dp]
        L.orc_fixed_step_error.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_fixed_step_error.restype = ctypes.c_double
        if hasattr(L, "orc_tangent"):
            L.orc_tangent.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
            L.orc_fd.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp,
                                 ctypes.c_double, dp]
            L.orc_fd_richardson.argtypes = L.orc_fd.argtypes
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------- problems
def base_problem(system, species_entry, qx: Optional[float] = None, De: Optional[float] = None,
                 phase0: Optional[float] = None) -> np.ndarray:
    """One orc_problem (numpy record) from a workloads.System and (m_atom, C4)."""
    p = np.zeros((), dtype=PROBLEM)
    qx = system.q_x if qx is None else qx
    p["m_ion"] = system.m_ion
    p["m_atom"], p["C4"] = species_entry
    p["De"] = system.De if De is None else De
    p["omega"] = system.omega_rf
    p["a"] = [system.a_x * r for r in system.a_ratio]
    p["q"] = [qx * r for r in system.q_ratio]
    p["phase0"] = system.phase0 if phase0 is None else phase0
    p["r0"] = system.r0
    p["t_max"] = system.t_max
    p["rtol"], p["atol"] = system.rtol, system.atol
    p["h0"], p["hmax"], p["hmin"] = system.h0, system.hmax, system.hmin
    p["r_bounce_over_rm"] = system.r_bounce_over_rm
    p["max_steps"] = system.max_steps
    return p


def headon_state(theta, phi, E, m_atom, r0) -> np.ndarray:
    y = np.zeros(12)
    lib().orc_headon_state(theta, phi, E, m_atom, r0, _dptr(y))
    return y


def grid_angles(ids, n_theta, n_phi):
    th = ctypes.c_double()
    ph = ctypes.c_double()
    out = np.zeros((len(ids), 2))
    for i, gid in enumerate(ids):
        lib().orc_grid_angles(int(gid), n_theta, n_phi, ctypes.byref(th), ctypes.byref(ph))
        out[i] = th.value, ph.value
    return out


def _sweep_struct(gen) -> _Sweep:
    s = _Sweep()
    s.seed = gen.seed
    s.n_species = len(gen.species)
    for i, v in enumerate(gen.species):
        s.species[i] = v
    s.n_E, s.n_q, s.n_De = len(gen.E_list), len(gen.q_list), len(gen.De_list)
    for i, v in enumerate(gen.E_list):
        s.E[i] = v
    for i, v in enumerate(gen.q_list):
        s.q[i] = v
    for i, v in enumerate(gen.De_list):
        s.De[i] = v
    if gen.E_range:
        s.E_lo, s.E_hi = gen.E_range
    if gen.q_range:
        s.q_lo, s.q_hi = gen.q_range
    if gen.De_range:
        s.De_lo, s.De_hi = gen.De_range
    return s


def sweep_draw(gid: int, gen):
    s = _sweep_struct(gen)
    vals = [ctypes.c_double() for _ in range(6)]
    sp = ctypes.c_int32()
    lib().orc_sweep_draw(int(gid), ctypes.byref(s), *[ctypes.byref(v) for v in vals], ctypes.byref(sp))
    ct, ph, ph0, E, qx, De = [v.value for v in vals]
    return dict(cos_theta=ct, phi=ph, phase0=ph0, E=E, q_x=qx, De=De, species=sp.value)


K_IN_EH = 3.1668115634556e-6      # k_B x 1 K in hartree (CODATA 2018)


def thermal_normals(gid: int, seed: int) -> np.ndarray:
    z = np.zeros(10)
    lib().orc_thermal_normals(int(gid), int(seed), _dptr(z))
    return z[:9]


def thermal_state(system, gen, d, m_atom, gid) -> np.ndarray:
    """Start state (a.u.) of a thermal run (Fig. 3 text): atom on the r0 sphere with Gaussian velocity
    components at the bath temperature (E = k_B T), turned inward; ion Gaussian at T_ion in the
    isotropic harmonic trap omega = q_x Omega / 2^(3/2)."""
    z = thermal_normals(gid, gen.seed)
    st = math.sqrt(max(0.0, 1.0 - d["cos_theta"] ** 2))
    n = np.array([st * math.cos(d["phi"]), st * math.sin(d["phi"]), d["cos_theta"]])
    v = math.sqrt(d["E"] / m_atom) * z[0:3]
    if v @ n >= 0.0:
        v = -v
    omega = d["q_x"] * system.omega_rf / (2.0 * math.sqrt(2.0))
    kT = gen.T_ion * K_IN_EH
    sv = math.sqrt(kT / system.m_ion)
    y = np.zeros(12)
    y[0:3] = system.r0 * n
    y[6:9] = v
    y[3:6] = sv / omega * z[3:6]
    y[9:12] = sv * z[6:9]
    return y


def problems_for(workload, ids) -> np.ndarray:
    """orc_problem records for global trajectory ids of a workloads.Workload."""
    ids = np.asarray(ids, dtype=np.int64)
    sys_ = workload.system
    spec = workload.species()
    gen = workload.gen
    out = np.zeros(len(ids), dtype=PROBLEM)
    for i, gid in enumerate(ids):
        if gen.kind == "grid":
            th, ph = grid_angles([gid], gen.n_theta, gen.n_phi)[0]
            p = base_problem(sys_, spec[sys_.species])
            p["y0"] = headon_state(th, ph, sys_.E, p["m_atom"], sys_.r0)
        elif gen.kind == "sweep":
            d = sweep_draw(gid, gen)
            p = base_problem(sys_, spec[d["species"]], qx=d["q_x"], De=d["De"], phase0=d["phase0"])
            th = math.acos(d["cos_theta"])
            p["y0"] = headon_state(th, d["phi"], d["E"], p["m_atom"], sys_.r0)
        elif gen.kind == "thermal":
            d = sweep_draw(gid, gen)
            p = base_problem(sys_, spec[d["species"]], qx=d["q_x"], De=d["De"], phase0=d["phase0"])
            p["y0"] = thermal_state(sys_, gen, d, p["m_atom"], gid)
            p["exit_centre"] = 1
        else:
            raise ValueError(gen.kind)
        out[i] = p
    return out


_twin = None


def twin_lib():
    global _twin
    if _twin is None:
        if not os.path.exists(TWIN_PATH):
            build(force=True)
        T = ctypes.CDLL(TWIN_PATH)
        T.orc_integrate_batch.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        _twin = T
    return _twin


def integrate(problems: np.ndarray, nthreads: int = 0, twin: bool = False) -> np.ndarray:
    """Integrate a batch of orc_problem records (OpenMP over trajectories).  twin=True runs the
    round-off twin build instead."""
    problems = np.ascontiguousarray(problems, dtype=PROBLEM)
    res = np.zeros(len(problems), dtype=RESULT)
    if nthreads <= 0:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    L = twin_lib() if twin else lib()
    L.orc_integrate_batch(len(problems), _ptr(problems), _ptr(res), nthreads)
    return res


def integrate_one(problem, record_cap: int = 0):
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    r = np.zeros(1, dtype=RESULT)
    if record_cap:
        h = np.zeros(record_cap)
        rc = lib().orc_integrate_record(_ptr(p), _ptr(r), _dptr(h), record_cap)
        if rc != 0:
            raise RuntimeError("step record overflow")
        return r[0], h[: r[0]["n_accept"]]
    lib().orc_integrate(_ptr(p), _ptr(r))
    return r[0]


def observables(problem, y_init, y_fin, t_fin):
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    yi = np.ascontiguousarray(y_init, dtype=np.float64)
    yf = np.ascontiguousarray(y_fin, dtype=np.float64)
    a, q, e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_observables(_ptr(p), _dptr(yi), _dptr(yf), t_fin, ctypes.byref(a), ctypes.byref(q),
                          ctypes.byref(e))
    return a.value, q.value, e.value


def rhs_au(problem, t, y):
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    yy = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.zeros(12)
    lib().orc_rhs_au(_ptr(p), t, _dptr(yy), _dptr(dy))
    return dy


def ion_energy(problem, y, t):
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    yy = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_ion_energy(_ptr(p), _dptr(yy), t)


def tableau():
    A, b, bh, c = np.zeros(49), np.zeros(7), np.zeros(7), np.zeros(7)
    lib().orc_tableau(_dptr(A), _dptr(b), _dptr(bh), _dptr(c))
    return A.reshape(7, 7), b, bh, c


def fixed_step_error(kind, lam, t_end, n_steps):
    return lib().orc_fixed_step_error(kind, lam, t_end, n_steps)


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def tangent(problem, theta, phi, E, q_ratio, twin: bool = False):
    """d(angle, q, dE)/d(theta, phi, E, q_x, De), Phi(t_f, 0) and the FTLE (internal time).
    twin=True runs the round-off twin build."""
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    qr = np.ascontiguousarray(q_ratio, dtype=np.float64)
    d = np.zeros(15)
    Phi = np.zeros(144)
    ftle = ctypes.c_double()
    L = lib()
    if twin:
        T = twin_lib()
        T.orc_tangent.argtypes = L.orc_tangent.argtypes
        T.orc_tangent.restype = L.orc_tangent.restype
        L = T
    rc = L.orc_tangent(_ptr(p), theta, phi, E, _dptr(qr), _dptr(d), _dptr(Phi), ctypes.byref(ftle))
    if rc != 0:
        raise RuntimeError(f"orc_tangent failed ({rc})")
    return d.reshape(3, 5), Phi.reshape(12, 12), ftle.value


def lyapunov_spectrum(Phi, m_atom, m_ion, t_f):
    """Finite-time Lyapunov spectrum ln sigma_i(D Phi D^-1) / t_f, descending (a.u. time).
    D = sqrt(mass) on each coordinate of the (r_atom, r_ion, v_atom, v_ion) state: the canonical
    scaling q = sqrt(m) r, p = sqrt(m) v, in which the stability matrix of the Hamiltonian flow of
    Eq. (1) is symplectic in the standard form, so its singular values come in pairs s, 1/s."""
    d = np.sqrt(np.array([m_atom] * 3 + [m_ion] * 3 + [m_atom] * 3 + [m_ion] * 3))
    Pt = (d[:, None] * np.asarray(Phi)) / d[None, :]
    return np.log(np.linalg.svd(Pt, compute_uv=False)) / t_f


def fd(problem, theta, phi, E, q_ratio, rel_h=1e-6):
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    qr = np.ascontiguousarray(q_ratio, dtype=np.float64)
    d = np.zeros(15)
    rc = lib().orc_fd(_ptr(p), theta, phi, E, _dptr(qr), rel_h, _dptr(d))
    if rc != 0:
        raise RuntimeError(f"orc_fd failed ({rc})")
    return d.reshape(3, 5)


def fd_richardson(problem, theta, phi, E, q_ratio, rel_h=2e-6):
    """Frozen-step central differences of the observables, replayed in extended precision (long
    double) at steps h and h/2 and Richardson-extrapolated: (4 D(h/2) - D(h)) / 3, error O(h^4)."""
    p = np.ascontiguousarray(np.asarray(problem, dtype=PROBLEM).reshape(1))
    qr = np.ascontiguousarray(q_ratio, dtype=np.float64)
    d = np.zeros(15)
    rc = lib().orc_fd_richardson(_ptr(p), theta, phi, E, _dptr(qr), rel_h, _dptr(d))
    if rc != 0:
        raise RuntimeError(f"orc_fd_richardson failed ({rc})")
    return d.reshape(3, 5)
