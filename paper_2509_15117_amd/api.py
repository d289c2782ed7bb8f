"""Python front end of libiat: marshals arguments to the C ABI; torch provides device memory and
streams.  Every step of the computation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _abi

KERNELS = {"plain": _abi.KERNEL_PLAIN, "persistent": _abi.KERNEL_PERSISTENT}
_K_IN_EH = 3.1668115634556e-6        # k_B x 1 K in hartree (CODATA 2018): Generator.T_ion is in kelvin


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
    kinds = {"arrays": _abi.GEN_ARRAYS, "grid": _abi.GEN_GRID, "sweep": _abi.GEN_SWEEP, "thermal": _abi.GEN_THERMAL}
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
    o.T_ion = float(getattr(g, "T_ion", 0.0)) * _K_IN_EH
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
                 y0: Optional[torch.Tensor] = None, id0: Optional[int] = None,
                 id0_dev: Optional[torch.Tensor] = None) -> _abi.Batch:
    b = _abi.Batch()
    b.n = int(n)
    arrays = arrays or {}
    for k in ("theta", "phi", "E", "q_x", "De", "phase0", "species"):
        setattr(b, k, _ptr(arrays.get(k)))
    b.y0 = _ptr(y0)
    if id0_dev is not None and (id0_dev.dtype != torch.int64 or not id0_dev.is_cuda or id0_dev.numel() != 1):
        raise ValueError("id0_dev must be a device int64 tensor of one element")
    b.id0_dev = _ptr(id0_dev)
    b.gen = gen_struct(gen, id0)
    return b


def launch_struct(kernel="persistent", block=0, blocks_per_cu=0, refill_every=0, step_budget=0,
                  stats: Optional[torch.Tensor] = None, kernel_ms=None, max_suspended=0,
                  tail_budget=0) -> _abi.Launch:
    """stats: optional device int64 tensor of at least 11 counters; kernel_ms: optional host
    ctypes float[5] for the phase durations (the call then waits).  Both are checked for size here,
    since the library writes all of their entries."""
    if stats is not None and (stats.numel() < _abi.N_STATS or stats.dtype != torch.int64 or not stats.is_cuda
                              or not stats.is_contiguous()):
        raise ValueError(f"stats must be a contiguous device int64 tensor of >= {_abi.N_STATS} entries")
    if kernel_ms is not None and len(kernel_ms) < _abi.N_PHASES:
        raise ValueError(f"kernel_ms must hold >= {_abi.N_PHASES} floats")
    L = _abi.Launch()
    L.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    L.block, L.blocks_per_cu, L.refill_every = block, blocks_per_cu, refill_every
    L.step_budget = step_budget
    L.max_suspended = max_suspended
    L.tail_budget = tail_budget
    L.stats = _ptr(stats)
    L.kernel_ms = None if kernel_ms is None else ctypes.cast(kernel_ms, ctypes.c_void_p)
    return L


def phase_ms():
    """A host buffer for the phase durations of one call: setup, main, tail, solo, observables."""
    return (ctypes.c_float * _abi.N_PHASES)()


def new_stats(device=None) -> torch.Tensor:
    """Zeroed device counters for launch.stats (see include/iat.h for the entries)."""
    return torch.zeros(_abi.N_STATS, dtype=torch.int64, device=device or "cuda")


def longest_of(stats) -> tuple:
    """(attempted steps, global id) of the longest trajectory recorded in stats[10] (0, 0 if none)."""
    v = int(stats[10]) & 0xFFFFFFFFFFFFFFFF
    return v >> 34, v & ((1 << 34) - 1)


def integrate(system, species, gen, n: int, *, arrays=None, y0=None, id0=None, kernel="persistent", block=0,
              blocks_per_cu=0, refill_every=0, step_budget=0, y_final=False, counters=True, stats=None, out=None,
              stream=None, device=None, kernel_ms=None, max_suspended=0, tail_budget=0,
              noalloc=False, id0_dev=None) -> Dict[str, torch.Tensor]:
    """Integrate n trajectories on the current GPU; returns device tensors of the observables.

    system / gen: objects with the fields of workloads.System / workloads.Generator.
    species: [(m_atom, C4)] in atomic units.  stats: optional uint64[11] device counters (new_stats();
    entry 10 packs the call's longest trajectory, see longest_of()).
    kernel_ms: optional phase_ms() buffer receiving the phase durations (setup, main, tail, solo,
    observables) measured with HIP events on the stream; the call then waits for completion.
    noalloc=True calls iat_integrate_noalloc (the library's fixed workspace; n <= NOALLOC_MAX_N, no
    kernel_ms; pass `out` to keep the call itself free of allocations).  id0_dev: optional device int64
    tensor of one element added to the first id when the kernels run (graph replays over chunks)."""
    L = _abi.load()
    device = device or torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = alloc_obs(n, device, y_final=y_final, counters=counters)
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, y0, id0, id0_dev)
    o = obs_struct(out)
    la = launch_struct(kernel, block, blocks_per_cu, refill_every, step_budget, stats, kernel_ms, max_suspended,
                       tail_budget)
    if noalloc:
        rc = L.iat_integrate_noalloc(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o),
                                     ctypes.byref(la), _stream_handle(stream))
    else:
        rc = L.iat_integrate(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o),
                             ctypes.byref(la), None, 0, _stream_handle(stream))
    _abi.check(rc)
    return out


def integrate_workload(w, n=None, id0=None, **kw):
    """Convenience: integrate the first n ids (from id0) of a workloads.Workload."""
    n = w.n if n is None else n
    return integrate(w.system, w.species(), w.gen, n, id0=id0, **kw)


def tangent(system, species, gen, n: int, *, arrays=None, id0=None, phi=False, lyap=False, out=None, stream=None,
            device=None) -> Dict[str, torch.Tensor]:
    """Observables plus their sensitivities d(angle, q_transfer, dE_ion)/d(theta, phi, E, q_x, De)
    (key 'dobs_dp', shape n x 3 x 5), the finite-time Lyapunov exponent per a.u. time ('ftle'),
    with lyap=True the finite-time Lyapunov spectrum of the canonically scaled stability matrix
    ('lyap', n x 12, descending) and, with phi=True, the 12 x 12 stability matrix of the internal
    state ('Phi')."""
    L = _abi.load()
    device = device or torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = alloc_obs(n, device, counters=True)
    out["dobs_dp"] = torch.empty(n, 3, 5, dtype=torch.float64, device=device)
    out["ftle"] = torch.empty(n, dtype=torch.float64, device=device)
    if phi:
        out["Phi"] = torch.empty(n, 12, 12, dtype=torch.float64, device=device)
    if lyap:
        out["lyap"] = torch.empty(n, 12, dtype=torch.float64, device=device)
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, None, id0)
    o = obs_struct(out)
    la = launch_struct()
    rc = L.iat_integrate_tangent(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o),
                                 _ptr(out["dobs_dp"]), _ptr(out["ftle"]), _ptr(out.get("lyap")), _ptr(out.get("Phi")),
                                 ctypes.byref(la),
                                 _stream_handle(stream))
    _abi.check(rc)
    return out


def n_cells(gen) -> int:
    """Number of sweep cells (species x E x q_x x De lists; a range counts as one)."""
    return max(1, len(gen.species)) * max(1, len(gen.E_list)) * max(1, len(gen.q_list)) * max(1, len(gen.De_list))


def _reduce(kind, system, species, gen, n, obs, out, id0, arrays, stream, id0_dev=None):
    L = _abi.load()
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, None, id0, id0_dev)
    o = obs_struct(obs)
    rc = L.iat_reduce(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o), kind, _ptr(out),
                      _stream_handle(stream))
    _abi.check(rc)
    return out


def reduce_cells(system, species, gen, n, obs, *, id0=None, arrays=None, out=None, stream=None, id0_dev=None):
    """Per sweep cell (count, complex count, sum dE_ion, sum dE_ion^2, sum n_bounce), shape n_cells x 5.
    Passing the previous chunk's out accumulates."""
    dev = obs["status"].device
    if out is None:
        out = torch.zeros(n_cells(gen), 5, dtype=torch.float64, device=dev)
    return _reduce(_abi.REDUCE_CELLS, system, species, gen, n, obs, out, id0, arrays, stream, id0_dev)


def reduce_hist(system, species, gen, n, obs, *, id0=None, arrays=None, out=None, stream=None, flag="complex",
                id0_dev=None):
    """Complex/total counts over log10(E/W0) per species slot (n_slots x 64 x 2) and the heating histogram
    (256,) in one flat tensor; use split_hist() to view them.  Passing the previous out accumulates.
    flag="bound" counts the trajectories that reached the negative-energy bound state in the second
    column instead of the complex flag."""
    dev = obs["status"].device
    slots = len(gen.species) if gen.kind in ("sweep", "thermal") else 1
    if out is None:
        out = torch.zeros(slots * 2 * _abi.W0_BINS + _abi.HEAT_BINS, dtype=torch.float64, device=dev)
    kind = {"complex": _abi.REDUCE_W0_HIST, "bound": _abi.REDUCE_W0_HIST_BOUND}[flag]
    return _reduce(kind, system, species, gen, n, obs, out, id0, arrays, stream, id0_dev)


def split_hist(flat: torch.Tensor):
    slots = (flat.numel() - _abi.HEAT_BINS) // (2 * _abi.W0_BINS)
    return flat[: slots * 2 * _abi.W0_BINS].view(slots, _abi.W0_BINS, 2), flat[slots * 2 * _abi.W0_BINS:]


def reduce_lifetime(system, species, gen, n, obs, *, id0=None, arrays=None, out=None, stream=None):
    """Complex lifetimes per species slot (n_slots x 98: 96 log10(t/us) bins over [-2, 4], censored
    count, spare) followed by the survival power-law exponent per slot; obs needs t_bounce_first/last.
    Passing the previous out accumulates the counts (the exponents are refitted)."""
    dev = obs["status"].device
    slots = len(gen.species) if gen.kind in ("sweep", "thermal") else 1
    if out is None:
        out = torch.zeros(slots * _abi.LIFE_SLOT + slots, dtype=torch.float64, device=dev)
    return _reduce(_abi.REDUCE_LIFETIME, system, species, gen, n, obs, out, id0, arrays, stream)


def split_lifetime(flat: torch.Tensor):
    """(histograms n_slots x 96, censored n_slots, exponents n_slots) views of reduce_lifetime's output."""
    slots = flat.numel() // (_abi.LIFE_SLOT + 1)
    h = flat[: slots * _abi.LIFE_SLOT].view(slots, _abi.LIFE_SLOT)
    return h[:, : _abi.LIFE_BINS], h[:, _abi.LIFE_BINS], flat[slots * _abi.LIFE_SLOT:]


def boxcount(system, species, gen, obs, *, stream=None):
    """Box-counting dimensions of the complex-forming set of a whole square power-of-two GRID batch:
    {'D_boundary', 'D_set', 'N_set' (per level k, boxes of 2^k cells), 'N_boundary'}."""
    side = gen.n_theta
    levels = side.bit_length()
    out = torch.zeros(2 + 2 * levels, dtype=torch.float64, device=obs["status"].device)
    _reduce(_abi.REDUCE_BOXCOUNT, system, species, gen, gen.n_theta * gen.n_phi, obs, out, 0, None, stream)
    h = out.cpu()
    return {"D_boundary": float(h[0]), "D_set": float(h[1]), "N_set": h[2::2].long().tolist(),
            "N_boundary": h[3::2].long().tolist()}


def adjoint(system, species, gen, n: int, obs: Dict[str, torch.Tensor], obs_bar: torch.Tensor, *, arrays=None,
            id0=None, ws: Optional[torch.Tensor] = None, y0_bar: bool = False, stream=None):
    """p_bar (n x 5) = d/d(theta, phi, E, q_x, De) of sum_k obs_bar[:, k] obs_k, obs = (angle, q_transfer,
    dE_ion), by the discrete adjoint.  obs: the outputs of integrate() on the same batch with counters
    (n_accept); obs['status'] gains ADJ_SKIPPED where the gradient is NaN.  ws: optional uint8 device
    workspace of adjoint_workspace_bytes() bytes (else allocated by the library).  With y0_bar=True
    returns (p_bar, y0_bar), y0_bar (n x 12) the gradient with respect to the start state in a.u."""
    L = _abi.load()
    obs_bar = obs_bar.contiguous()
    if obs_bar.shape != (n, 3) or obs_bar.dtype != torch.float64:
        raise ValueError("obs_bar must be a float64 tensor of shape (n, 3)")
    if "n_accept" not in obs:
        raise ValueError("obs must come from integrate(..., counters=True) of the same batch")
    p_bar = torch.empty(n, 5, dtype=torch.float64, device=obs_bar.device)
    yb = torch.empty(n, 12, dtype=torch.float64, device=obs_bar.device) if y0_bar else None
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, None, id0)
    o = obs_struct(obs)
    la = launch_struct()
    rc = L.iat_adjoint(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o), _ptr(obs_bar),
                       _ptr(p_bar), _ptr(yb), _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(),
                       ctypes.byref(la), _stream_handle(stream))
    _abi.check(rc)
    return (p_bar, yb) if y0_bar else p_bar


def adjoint_workspace_bytes(system, species, gen, n: int, obs, *, arrays=None, id0=None, stream=None) -> int:
    L = _abi.load()
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, None, id0)
    o = obs_struct(obs)
    out = ctypes.c_size_t(0)
    rc = L.iat_adjoint_workspace_bytes(ctypes.byref(sysv), sp, len(species), ctypes.byref(b), ctypes.byref(o),
                                       ctypes.byref(out), _stream_handle(stream))
    _abi.check(rc)
    return int(out.value)


def workspace_bytes(which: str, system, species, gen, n: int, *, arrays=None, id0=None, reduce_kind="w0_hist",
                    obs=None, stream=None, **launch) -> int:
    """Device bytes that one call over ids [id0, id0 + n) needs: which = 'integrate' (what iat_integrate
    allocates for this launch shape; launch keyword arguments as for integrate()), 'reduce' (what
    iat_reduce of reduce_kind allocates: 'cells', 'w0_hist', 'w0_hist_bound', 'boxcount', 'lifetime')
    or 'adjoint' (as adjoint_workspace_bytes; needs obs of the forward run)."""
    kinds = {"integrate": _abi.WS_INTEGRATE, "reduce": _abi.WS_REDUCE, "adjoint": _abi.WS_ADJOINT}
    reduces = {"cells": _abi.REDUCE_CELLS, "w0_hist": _abi.REDUCE_W0_HIST, "w0_hist_bound": _abi.REDUCE_W0_HIST_BOUND,
               "boxcount": _abi.REDUCE_BOXCOUNT, "lifetime": _abi.REDUCE_LIFETIME}
    L = _abi.load()
    sysv = system_struct(system)
    sp = species_array(species)
    b = batch_struct(n, gen, arrays, None, id0)
    o = obs_struct(obs) if obs is not None else None
    la = launch_struct(**launch)
    out = ctypes.c_size_t(0)
    rc = L.iat_workspace_bytes(kinds[which], ctypes.byref(sysv), sp, len(species), ctypes.byref(b),
                               ctypes.byref(o) if o is not None else None, ctypes.byref(la), reduces[reduce_kind],
                               ctypes.byref(out), _stream_handle(stream) if which == "adjoint" else None)
    _abi.check(rc)
    return int(out.value)


class ScatteringObservables(torch.autograd.Function):
    """obs = (angle, q_transfer, dE_ion) per trajectory as a differentiable function of per-trajectory
    (theta, phi, E, q_x, De) tensors (float64, device, length n); the backward pass is the library's
    discrete adjoint.  Usage: ScatteringObservables.apply(theta, phi, E, q_x, De, system, species, gen)
    with gen.kind == 'arrays' (species / phase0 from the system, or gen-level arrays via `extra`)."""

    @staticmethod
    def forward(ctx, theta, phi, E, q_x, De, system, species, gen, extra=None):
        arrays = {"theta": theta.contiguous(), "phi": phi.contiguous(), "E": E.contiguous(),
                  "q_x": q_x.contiguous(), "De": De.contiguous()}
        if extra:
            arrays.update({k: v.contiguous() for k, v in extra.items()})
        n = theta.numel()
        out = integrate(system, species, gen, n, arrays=arrays, counters=True)
        ctx.save_for_backward(*arrays.values())
        ctx.keys = list(arrays.keys())
        ctx.cfg = (system, species, gen, n)
        ctx.obs = out
        return torch.stack([out["angle"], out["q_transfer"], out["dE_ion"]], dim=1)

    @staticmethod
    def backward(ctx, grad):
        system, species, gen, n = ctx.cfg
        arrays = dict(zip(ctx.keys, ctx.saved_tensors))
        p_bar = adjoint(system, species, gen, n, ctx.obs, grad.to(torch.float64).contiguous(), arrays=arrays)
        return p_bar[:, 0], p_bar[:, 1], p_bar[:, 2], p_bar[:, 3], p_bar[:, 4], None, None, None, None


def run_chunks(w, *, n: Optional[int] = None, chunk: int = 1 << 22, n_streams: int = 4, kernel="persistent",
               cells: bool = False, hist: bool = False, hist_bound: bool = False,
               stats: Optional[torch.Tensor] = None, progress=None, sample=None, graph: bool = False, **launch):
    """Integrate ids [0, n) of a workloads.Workload in chunks of `chunk` ids spread round-robin over
    `n_streams` streams (default priority), reducing each chunk on its stream: per-cell sums (cells=True,
    sweeps), the W0 / heating histograms (hist=True) and the W0 histogram of the bound-state flag
    (hist_bound=True, res['hist_bound']).  Only the reductions are kept.  While one
    chunk's long-lived complexes finish in its tail kernel, the next chunks run on the other streams.
    Returns {'cells': (n_cells, 5), 'hist': flat histogram} (device tensors, summed over streams).
    progress(c, n_chunks): called on the host as chunk c completes (in chunk order).
    sample: optional sorted global ids whose per-trajectory outputs (with step counters and final
    states) are copied out of their chunk before its buffers are reused: res['sample'].
    graph=True: each stream captures its chunk's calls (integration and reductions) once in a HIP graph,
    with the chunk's first id read from a device scalar (iat_batch.id0_dev), and replays it for every
    later full chunk after writing that id; the first chunk runs eagerly (code objects, pools) and so
    does a shorter last chunk.  The bits are those of the eager calls (not with sample)."""
    want = sample is not None
    if graph and want:
        raise ValueError("run_chunks: graph replay does not copy out samples")
    if graph and w.gen.kind == "thermal":
        # the one large run that replayed thermal chunks from a graph faulted the GPU, cause not found
        raise ValueError("run_chunks: graph replay is not available for thermal batches")
    n = w.n if n is None else n
    dev = torch.device("cuda", torch.cuda.current_device())
    cur = torch.cuda.current_stream()
    streams = [torch.cuda.Stream(device=dev) for _ in range(max(1, n_streams))]
    m = min(chunk, n)
    bufs = [alloc_obs(m, dev, counters=want, y_final=want) for _ in streams]
    if want:
        ids_h = torch.as_tensor(sample, dtype=torch.int64).cpu()
        if len(ids_h) and (bool((ids_h[1:] < ids_h[:-1]).any()) or int(ids_h[0]) < 0 or int(ids_h[-1]) >= n):
            raise ValueError("sample must be sorted ids in [0, n)")
        ids_d = ids_h.to(dev)
        s_out = {k: torch.empty((12, len(ids_h)) if k == "y_final" else (len(ids_h),), dtype=v.dtype, device=dev)
                 for k, v in bufs[0].items()}
    slots = len(w.gen.species) if w.gen.kind in ("sweep", "thermal") else 1
    c_out = [torch.zeros(n_cells(w.gen), 5, dtype=torch.float64, device=dev) for _ in streams] if cells else None
    h_out = ([torch.zeros(slots * 2 * _abi.W0_BINS + _abi.HEAT_BINS, dtype=torch.float64, device=dev)
              for _ in streams] if hist else None)
    hb_out = ([torch.zeros(slots * 2 * _abi.W0_BINS + _abi.HEAT_BINS, dtype=torch.float64, device=dev)
               for _ in streams] if hist_bound else None)
    for s in streams:
        s.wait_stream(cur)
    offs = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in streams] if graph else None
    graphs = [None] * len(streams)

    def calls(k, cnt, id0, id0_dev):
        obs = {key: v[:cnt] for key, v in bufs[k].items()}
        integrate(w.system, w.species(), w.gen, cnt, id0=id0, out=obs, stream=streams[k], kernel=kernel, stats=stats,
                  id0_dev=id0_dev, **launch)
        if cells:
            reduce_cells(w.system, w.species(), w.gen, cnt, obs, id0=id0, out=c_out[k], stream=streams[k],
                         id0_dev=id0_dev)
        if hist:
            reduce_hist(w.system, w.species(), w.gen, cnt, obs, id0=id0, out=h_out[k], stream=streams[k],
                        id0_dev=id0_dev)
        if hist_bound:
            reduce_hist(w.system, w.species(), w.gen, cnt, obs, id0=id0, out=hb_out[k], stream=streams[k],
                        flag="bound", id0_dev=id0_dev)
        return obs

    done = []
    for c, id0 in enumerate(range(0, n, chunk)):
        k = c % len(streams)
        cnt = min(chunk, n - id0)
        if graph and c > 0 and cnt == m:
            with torch.cuda.stream(streams[k]):
                if graphs[k] is None:
                    streams[k].synchronize()
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=streams[k]):
                        calls(k, cnt, 0, offs[k])
                    graphs[k] = g
                offs[k].fill_(id0)
                graphs[k].replay()
            obs = {key: v[:cnt] for key, v in bufs[k].items()}
        else:
            obs = calls(k, cnt, id0, None)
        if want:
            a = int(torch.searchsorted(ids_h, torch.tensor(id0)))
            b = int(torch.searchsorted(ids_h, torch.tensor(id0 + cnt)))
            if b > a:
                with torch.cuda.stream(streams[k]):
                    loc = ids_d[a:b] - id0
                    for key, v in obs.items():
                        if key == "y_final":
                            s_out[key][:, a:b] = v.index_select(1, loc)
                        else:
                            s_out[key][a:b] = v.index_select(0, loc)
        if progress is not None:
            ev = torch.cuda.Event()
            ev.record(streams[k])
            done.append(ev)
    for c, ev in enumerate(done):
        ev.synchronize()
        progress(c, len(done))
    for s in streams:
        cur.wait_stream(s)
    res = {}
    if cells:
        res["cells"] = torch.stack(c_out).sum(0)
    if hist:
        res["hist"] = torch.stack(h_out).sum(0)
    if hist_bound:
        res["hist_bound"] = torch.stack(hb_out).sum(0)
    if want:
        res["sample"] = s_out
        for v in s_out.values():
            for s in streams:
                v.record_stream(s)
    for b in bufs:               # the buffers were used on the side streams
        for v in b.values():
            for s in streams:
                v.record_stream(s)
    if graph:
        for o in offs:
            for s in streams:
                o.record_stream(s)
        res["graphs"] = graphs   # keep the captured graphs (and their memory) alive with the results
    return res


def autotune(w, *, n: int = 1 << 20, id0: int = 0, cache: Optional[str] = None, blocks=(64, 128, 256),
             refills=(1, 4, 16, 64), blocks_per_cu=(0, 1), step_budget: int = 20000,
             verbose: bool = False) -> Dict[str, int]:
    """Pick the persistent kernel's launch shape for a workload (block size, refill granularity,
    resident blocks per compute unit; 0 = as many as fit) by the main kernel's throughput: the RHS
    evaluations it performed over its event-timed duration.  The sample is ids [id0, id0 + n) of a
    random sweep (independent draws), or for a grid n / 16 ids at each of 16 places spread over it.
    For these runs the accepted-step cap is lowered to twice the step budget, so the latency-bound
    four-lane and solo levels, which the shape does not change, stay short; the main kernel's work up
    to the budget is the same.  The winner is cached in a JSON file keyed by the workload, n and the
    budget.  Returns keyword arguments for integrate() / run_chunks(); every candidate gives the same
    bits, only the time differs."""
    import copy
    import json
    import os
    key = f"{w.name}:{n}:{step_budget}"
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(key)
            if hit:
                return {k: v for k, v in hit.items() if k in ("block", "refill_every", "blocks_per_cu", "step_budget")}
        except (OSError, ValueError, AttributeError):
            pass
    wt = copy.deepcopy(w)
    wt.system.max_steps = 2 * step_budget
    if w.gen.kind == "grid":
        total = int(w.gen.n_theta) * int(w.gen.n_phi)
        parts = 16 if total >= 16 else 1
        m = max(1, min(n, total) // parts)
        starts = [(total - m) * k // max(parts - 1, 1) for k in range(parts)]
    else:
        m, starts = n, [id0]
    dev = torch.device("cuda", torch.cuda.current_device())
    out = alloc_obs(m, dev, counters=False)
    stats = new_stats(dev)

    def rate(cfg):
        stats.zero_()
        main_ms = 0.0
        for s0 in starts:
            ms = phase_ms()
            integrate_workload(wt, n=m, id0=s0, out=out, stats=stats, kernel_ms=ms, kernel="persistent",
                               step_budget=step_budget, **cfg)
            main_ms += ms[1]
        st = stats.cpu().tolist()
        return (st[0] - st[6] - st[8]) / max(main_ms * 1e-3, 1e-9), main_ms

    rate(dict(block=256, refill_every=1, blocks_per_cu=0))          # warm-up (code objects, pools)
    best, best_r, table = None, -1.0, []
    for blk in blocks:
        for rf in refills:
            for pc in blocks_per_cu:
                cfg = dict(block=blk, refill_every=rf, blocks_per_cu=pc)
                r, main_ms = rate(cfg)
                table.append(dict(cfg, rhs_per_s=r, main_ms=main_ms))
                if verbose:
                    print(f"autotune {key}: {cfg} main kernel {main_ms:.1f} ms, {r:.3e} RHS/s", flush=True)
                if r > best_r:
                    best, best_r = cfg, r
    best = dict(best, step_budget=step_budget)
    if cache:
        data = {}
        if os.path.exists(cache):
            try:
                with open(cache) as f:
                    data = json.load(f)
            except (OSError, ValueError):
                data = {}
        data[key] = dict(best, rhs_per_s=best_r, candidates=table)
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return best


def fp64_peak(n_threads: int = 256 * 2048, iters: int = 20000, stream=None) -> float:
    """Measured FP64 FMA rate of this GPU in TFLOP/s (see iat_fp64_peak)."""
    L = _abi.load()
    scratch = torch.empty(n_threads, dtype=torch.float64, device=torch.device("cuda", torch.cuda.current_device()))
    out = ctypes.c_double(0.0)
    _abi.check(L.iat_fp64_peak(_ptr(scratch), n_threads, iters, ctypes.byref(out), _stream_handle(stream)))
    return out.value
