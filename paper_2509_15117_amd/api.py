"""Python front end of libiat: marshals arguments to the C ABI; torch provides device memory and
streams.  Every step of the computation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _abi

KERNELS = {"plain": _abi.KERNEL_PLAIN, "persistent": _abi.KERNEL_PERSISTENT}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def system_struct(s) -> _abi.System:
    """From any object with the fields of workloads.System (atomic units)."""
    o = _abi.System()
    o.m_ion, o.omega_rf, o.a_x, o.q_x = s.m_ion, s.omega_rf, s.a_x, s.q_x
    for k in range(3):
        o.a_ratio[k] = s.a_ratio[k]
        o.q_ratio[k] = s.q_ratio[k]
    o.E, o.De, o.phase0, o.species = s.E, s.De, s.phase0, int(s.species)
    o.r0, o.t_max, o.rtol, o.atol = s.r0, s.t_max, s.rtol, s.atol
    o.h0, o.hmax, o.hmin = s.h0, s.hmax, s.hmin
    o.r_bounce_over_rm, o.max_steps = s.r_bounce_over_rm, int(s.max_steps)
    return o


def species_array(species: Sequence) -> "ctypes.Array":
    """[(m_atom in m_e, C4 in a.u.), ...] -> iat_species[]"""
    arr = (_abi.Species * max(1, len(species)))()
    for i, (m, c4) in enumerate(species):
        arr[i].m_atom, arr[i].C4 = m, c4
    return arr


def gen_struct(g, id0: Optional[int] = None) -> _abi.Gen:
    """From any object with the fields of workloads.Generator."""
    o = _abi.Gen()
    kinds = {"arrays": _abi.GEN_ARRAYS, "grid": _abi.GEN_GRID, "sweep": _abi.GEN_SWEEP}
    o.kind = kinds[g.kind]
    o.n_theta, o.n_phi = int(g.n_theta), int(g.n_phi)
    o.n_species = len(g.species)
    for i, v in enumerate(g.species):
        o.species[i] = int(v)
    o.n_E, o.n_q, o.n_De = len(g.E_list), len(g.q_list), len(g.De_list)
    for i, v in enumerate(g.E_list):
        o.E[i] = v
    for i, v in enumerate(g.q_list):
        o.q[i] = v
    for i, v in enumerate(g.De_list):
        o.De[i] = v
    if g.E_range:
        o.E_lo, o.E_hi = g.E_range
    if g.q_range:
        o.q_lo, o.q_hi = g.q_range
    if g.De_range:
        o.De_lo, o.De_hi = g.De_range
    o.seed = int(g.seed)
    o.id0 = int(g.id0 if id0 is None else id0)
    return o


OBS_FIELDS = {"angle": torch.float64, "q_transfer": torch.float64, "dE_ion": torch.float64,
              "t_dwell": torch.float64, "t_bounce_first": torch.float64, "t_bounce_last": torch.float64,
              "n_bounce": torch.int32, "status": torch.int32, "n_accept": torch.int64,
              "n_reject": torch.int64, "n_rhs": torch.int64}


def alloc_obs(n: int, device, y_final: bool = False, counters: bool = True) -> Dict[str, torch.Tensor]:
    out = {}
    for k, dt in OBS_FIELDS.items():
        if not counters and k in ("n_accept", "n_reject", "n_rhs", "t_bounce_first", "t_bounce_last"):
            continue
        out[k] = torch.empty(n, dtype=dt, device=device)
    if y_final:
        out["y_final"] = torch.empty(12, n, dtype=torch.float64, device=device)
    return out


def obs_struct(out: Dict[str, torch.Tensor]) -> _abi.Obs:
    o = _abi.Obs()
    for k in ("angle", "q_transfer", "dE_ion", "t_dwell", "t_bounce_first", "t_bounce_last", "n_bounce",
              "status", "n_accept", "n_reject", "n_rhs", "y_final"):
        setattr(o, k, _ptr(out.get(k)))
    return o


def batch_struct(n: int, gen, arrays: Optional[Dict[str, torch.Tensor]] = None,
                 y0: Optional[torch.Tensor] = None, id0: Optional[int] = None) -> _abi.Batch:
    b = _abi.Batch()
    b.n = int(n)
    arrays = arrays or {}
    for k in ("theta", "phi", "E", "q_x", "De", "phase0", "species"):
        setattr(b, k, _ptr(arrays.get(k)))
    b.y0 = _ptr(y0)
    b.gen = gen_struct(gen, id0)
    return b


def launch_struct(kernel="persistent", block=0, blocks_per_cu=0, refill_every=0, step_budget=0,
                  stats: Optional[torch.Tensor] = None) -> _abi.Launch:
    L = _abi.Launch()
    L.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    L.block, L.blocks_per_cu, L.refill_every = block, blocks_per_cu, refill_every
    L.step_budget = step_budget
    L.stats = _ptr(stats)
    return L


def integrate(system, species, gen, n: int, *, arrays=None, y0=None, id0=None, kernel="persistent", block=0,
              blocks_per_cu=0, refill_every=0, step_budget=0, y_final=False, counters=True, stats=None, out=None,
              stream=None, device=None) -> Dict[str, torch.Tensor]:
    """Integrate n trajectories on the current GPU; returns device tensors of the observables.

    system / gen: objects with the fields of workloads.System / workloads.Generator.
    species: [(m_atom, C4)] in atomic units.  stats: optional uint64[8] device counters (int64 tensor)."""
    L = _abi.load()
    device = device or torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = alloc_obs(n, device, y_final=y_final, counters=counters)
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, y0, id0)
    o = obs_struct(out)
    la = launch_struct(kernel, block, blocks_per_cu, refill_every, step_budget, stats)
    rc = L.iat_integrate(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o), ctypes.byref(la),
                         None, 0, _stream_handle(stream))
    _abi.check(rc)
    return out


def integrate_workload(w, n=None, id0=None, **kw):
    """Convenience: integrate the first n ids (from id0) of a workloads.Workload."""
    n = w.n if n is None else n
    return integrate(w.system, w.species(), w.gen, n, id0=id0, **kw)
