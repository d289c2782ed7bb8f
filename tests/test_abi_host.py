"""Host-only checks of the C ABI: the library loads, exports what include/iat.h declares, and its
argument validation rejects bad input before touching the GPU."""
import ctypes
import os
import re

import pytest

import workloads as W
from paper_2509_15117_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "iat.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(iat_\w+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = _abi.load()
    declared = header_functions()
    assert set(declared) == set(_abi.EXPORTS), declared
    for name in declared:
        assert hasattr(L, name), name
    assert b"gfx950" in L.iat_version()


def test_struct_layouts_match_header_sizes():
    # sizes implied by the header's field lists (LP64)
    assert ctypes.sizeof(_abi.System) == 8 * 21 + 8 + 8
    assert ctypes.sizeof(_abi.Gen) == 64 + 8 * 30 + 16 + 8
    assert ctypes.sizeof(_abi.Obs) == 12 * 8
    assert ctypes.sizeof(_abi.Launch) == 8 * 4 + 8 * 2
    # n, seven per-trajectory arrays, y0 and the device-side id offset, then the generator
    assert ctypes.sizeof(_abi.Batch) == 8 + 9 * 8 + ctypes.sizeof(_abi.Gen)
    assert _abi.Batch.gen.offset == 80 and _abi.Batch.id0_dev.offset == 72


def _call(system=None, species=None, n_species=None, batch=None, obs=None, launch=None):
    from paper_2509_15117_amd import api  # noqa: F401  (torch import is fine on CPU)
    w = W.config1()
    sysv = system or api.system_struct(w.system)
    sp = species or api.species_array(w.species())
    b = batch or api.batch_struct(0, w.gen)
    o = obs if obs is not None else _abi.Obs()
    la = launch or _abi.Launch()
    rc = _abi.load().iat_integrate(ctypes.byref(sysv), sp, 1 if n_species is None else n_species, ctypes.byref(b),
                                   ctypes.byref(o), ctypes.byref(la), None, 0, None)
    return rc, _abi.load().iat_last_error().decode()


def _obs_dummy():
    o = _abi.Obs()
    for k in ("angle", "q_transfer", "dE_ion", "t_dwell", "n_bounce", "status"):
        setattr(o, k, ctypes.c_void_p(0x1000))  # never dereferenced: n == 0 or rejected first
    return o


def test_validation_rejects_bad_arguments_without_gpu():
    from paper_2509_15117_amd import api
    w = W.config1()
    ok, _ = _call(obs=_obs_dummy())
    assert ok == 0                                   # n == 0: valid and nothing to do
    ok, _ = _call(obs=_abi.Obs())
    assert ok == 0                                   # n == 0 needs no output buffers
    rc, msg = _call(batch=api.batch_struct(4, w.gen), obs=_abi.Obs())
    assert rc == _abi.IAT_EINVAL and "obs" in msg
    s = api.system_struct(w.system)
    s.rtol = 0.0
    rc, msg = _call(system=s, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "rtol" in msg
    rc, msg = _call(n_species=0, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "n_species" in msg
    b = api.batch_struct(65, w.gen)                  # 8x8 grid holds 64 ids
    rc, msg = _call(batch=b, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "grid" in msg
    la = api.launch_struct("plain", block=100)
    rc, msg = _call(launch=la, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "block" in msg
    la = api.launch_struct(tail_budget=-2)
    rc, msg = _call(launch=la, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "tail_budget" in msg
    la = api.launch_struct()
    la.reserved = 1
    rc, msg = _call(launch=la, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "reserved" in msg
    g = W.Generator(kind="sweep", species=[0, 7], E_range=(1e-12, 1e-11), q_range=(0.1, 0.2),
                    De_range=(1e-6, 1e-5))
    rc, msg = _call(batch=api.batch_struct(0, g), obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "species" in msg
    th = W.fig3_thermal().gen
    g = W.Generator(kind="thermal", species=[0], E_list=[1e-12], q_list=[0.2], De_list=[1e-6], T_ion=-1e-6)
    rc, msg = _call(batch=api.batch_struct(0, g), obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "T_ion" in msg
    g = W.Generator(kind="thermal", species=[0], E_list=[1e-12], q_list=[0.0], De_list=[1e-6])
    rc, msg = _call(batch=api.batch_struct(0, g), obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "q_x" in msg
    b = api.batch_struct(0, th)
    b.y0 = 0x1000                                    # a device address the check never dereferences
    rc, msg = _call(batch=b, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "y0" in msg
    five = W.fig3_thermal().species()
    rc, msg = _call(species=api.species_array(five), n_species=5, batch=api.batch_struct(0, th), obs=_obs_dummy())
    assert rc == 0, msg
    s = api.system_struct(w.system)
    s.hmax = 1.0                                     # > pi/4: beyond an eighth of the RF period
    rc, msg = _call(system=s, obs=_obs_dummy())
    assert rc == _abi.IAT_EINVAL and "hmax" in msg
    # the accepted-step cap must fit the device's step counters
    limit = 1 << 28
    txt = open(os.path.join(ROOT, "include", "iat.h")).read()
    assert "#define IAT_MAX_STEPS_LIMIT (1LL << 28)" in txt
    for cap, want in ((limit, 0), (limit + 1, _abi.IAT_EINVAL), (1 << 40, _abi.IAT_EINVAL), (0, 0)):
        s = api.system_struct(w.system)
        s.max_steps = cap
        rc, msg = _call(system=s, obs=_obs_dummy())
        assert rc == want and (want == 0 or "max_steps" in msg), (cap, rc, msg)


def test_derivatives_reject_thermal_and_explicit_starts_without_gpu():
    """Tangent and adjoint differentiate with respect to (theta, phi, E) of a head-on start: thermal
    batches and caller-given start states are refused before the GPU is touched."""
    from paper_2509_15117_amd import api
    L = _abi.load()
    th = W.fig3_thermal()
    sysv = api.system_struct(th.system)
    sp = api.species_array(th.species())
    o = _obs_dummy()
    rc = L.iat_integrate_tangent(ctypes.byref(sysv), sp, 5, ctypes.byref(api.batch_struct(4, th.gen)), ctypes.byref(o),
                                 ctypes.c_void_p(0x1000), None, None, None, None, None)
    assert rc == _abi.IAT_ENOTSUP and "thermal" in L.iat_last_error().decode()
    rc = L.iat_adjoint(ctypes.byref(sysv), sp, 5, ctypes.byref(api.batch_struct(4, th.gen)), ctypes.byref(o),
                       None, None, None, None, 0, None, None)
    assert rc == _abi.IAT_ENOTSUP and "thermal" in L.iat_last_error().decode()
    w = W.config1()
    b = api.batch_struct(4, W.Generator(kind="arrays"))
    b.y0 = 0x1000
    rc = L.iat_integrate_tangent(ctypes.byref(api.system_struct(w.system)), api.species_array(w.species()), 1,
                                 ctypes.byref(b), ctypes.byref(o), ctypes.c_void_p(0x1000), None, None, None, None, None)
    assert rc == _abi.IAT_ENOTSUP and "y0" in L.iat_last_error().decode()


def test_launch_buffers_are_size_checked_before_the_call():
    """The library writes all 11 entries of launch.stats (device) and all 5 phase durations of
    launch.kernel_ms (host); the binding refuses smaller or misplaced buffers before any call."""
    torch = pytest.importorskip("torch")
    from paper_2509_15117_amd import api
    assert (_abi.N_STATS, _abi.N_PHASES) == (11, 5)
    txt = open(os.path.join(ROOT, "include", "iat.h")).read()
    assert "device uint64[11]" in txt and "HOST float[5]" in txt
    with pytest.raises(ValueError, match="stats"):
        api.launch_struct(stats=torch.zeros(10, dtype=torch.int64))         # too short (and on the host)
    with pytest.raises(ValueError, match="stats"):
        api.launch_struct(stats=torch.zeros(11, dtype=torch.int64))         # host memory, not device
    with pytest.raises(ValueError, match="kernel_ms"):
        api.launch_struct(kernel_ms=(ctypes.c_float * 4)())
    la = api.launch_struct(kernel_ms=api.phase_ms(), tail_budget=-1, step_budget=7, max_suspended=5)
    assert (la.tail_budget, la.step_budget, la.max_suspended, la.reserved) == (-1, 7, 5, 0)
    assert len(api.phase_ms()) == 5


def test_noalloc_refuses_oversized_batches_and_timing_without_gpu():
    """The allocation-free entry point holds its workspace in a fixed array: a batch above its limit
    and phase timing (events and a wait) are refused before the GPU is touched."""
    from paper_2509_15117_amd import api
    L = _abi.load()
    w = W.config5()
    txt = open(os.path.join(ROOT, "include", "iat.h")).read()
    assert f"#define IAT_NOALLOC_MAX_N {_abi.NOALLOC_MAX_N}" in txt
    sysv = api.system_struct(w.system)
    sp = api.species_array(w.species())

    def call(n, launch):
        b = api.batch_struct(n, w.gen)
        rc = L.iat_integrate_noalloc(ctypes.byref(sysv), sp, 3, ctypes.byref(b), ctypes.byref(_obs_dummy()),
                                     ctypes.byref(launch), None)
        return rc, L.iat_last_error().decode()

    rc, msg = call(_abi.NOALLOC_MAX_N + 1, _abi.Launch())
    assert rc == _abi.IAT_EINVAL and "limit" in msg and str(_abi.NOALLOC_MAX_N) in msg, msg
    rc, msg = call(1 << 40, _abi.Launch())
    assert rc == _abi.IAT_EINVAL, msg
    rc, msg = call(4, api.launch_struct(kernel_ms=api.phase_ms()))
    assert rc == _abi.IAT_EINVAL and "kernel_ms" in msg, msg
    rc, msg = call(0, _abi.Launch())
    assert rc == 0, msg                              # nothing to do: no GPU call
    la = api.launch_struct(block=100)
    rc, msg = call(4, la)
    assert rc == _abi.IAT_EINVAL and "block" in msg, msg


def test_boxcount_refuses_a_device_id_offset_without_gpu():
    """Box counting needs the whole grid from id 0; a batch whose first id is only known on the device
    (graph replays over chunks) is refused before the GPU is touched."""
    from paper_2509_15117_amd import api
    L = _abi.load()
    w = W.config1()
    b = api.batch_struct(64, w.gen)
    b.id0_dev = 0x1000                               # never dereferenced: refused first
    rc = L.iat_reduce(ctypes.byref(api.system_struct(w.system)), api.species_array(w.species()), 1, ctypes.byref(b),
                      ctypes.byref(_obs_dummy()), _abi.REDUCE_BOXCOUNT, ctypes.c_void_p(0x1000), None)
    assert rc == _abi.IAT_EINVAL and "BOXCOUNT" in L.iat_last_error().decode()


def test_run_chunks_refuses_graph_replay_of_thermal_batches_without_gpu():
    """Graph replay of chunks is switched off for thermal batches (refused before any device call)."""
    from paper_2509_15117_amd import api
    with pytest.raises(ValueError, match="thermal"):
        api.run_chunks(W.fig3_thermal(), n=64, chunk=32, graph=True, cells=True)
    with pytest.raises(ValueError, match="samples"):
        api.run_chunks(W.config3(), n=64, chunk=32, graph=True, sample=[1, 2])


def test_workspace_bytes_of_integrate_and_reduce_on_the_host():
    """iat_workspace_bytes sizes the calls without a GPU: iat_integrate's workspace is 256 B of counters,
    the work buffer (22 doubles and 5 ints per trajectory, rounded up to 256 B) and 248 B per
    continuation record of the tail and solo levels (one of each per trajectory for small batches; none
    for the plain kernel or without a step budget); iat_reduce allocates per-cell partial sums for
    CELLS (64 slices of 5 doubles), level flags for BOXCOUNT and nothing for the histograms."""
    from paper_2509_15117_amd import api
    w = W.config1()
    sysv, sp = w.system, w.species()

    def ws(which, wl=w, n=64, **kw):
        return api.workspace_bytes(which, wl.system, wl.species(), wl.gen, n, **kw)

    def ceil256(x):
        return -(-x // 256) * 256
    s3 = W.config3()
    for n in (1, 64, 1000):
        work = 256 + ceil256(n * (22 * 8 + 5 * 4))
        assert ws("integrate", wl=s3, n=n) == work + 2 * n * 248
        assert ws("integrate", wl=s3, n=n, kernel="plain") == work
        assert ws("integrate", wl=s3, n=n, step_budget=-1) == work
        assert ws("integrate", wl=s3, n=n, max_suspended=5) == work + 2 * min(n, 5) * 248
    assert ws("integrate", n=0) == 0
    with pytest.raises(_abi.IatError, match="exceed"):        # the call's own validation: 1000 ids of an 8x8 grid
        ws("integrate", n=1000)
    assert ws("reduce", wl=s3, n=1000, reduce_kind="cells") == 225 * 64 * 5 * 8
    for k in ("w0_hist", "w0_hist_bound", "lifetime"):
        assert ws("reduce", n=64, reduce_kind=k) == 0
    assert ws("reduce", n=64, reduce_kind="boxcount") == 256 + 64 + 64 // 4 + 1
    L = _abi.load()
    b = api.batch_struct(64, w.gen)
    out = ctypes.c_size_t(7)
    args = (ctypes.byref(api.system_struct(sysv)), api.species_array(sp), 1, ctypes.byref(b), None,
            ctypes.byref(_abi.Launch()))
    assert L.iat_workspace_bytes(9, *args, 0, ctypes.byref(out), None) == _abi.IAT_EINVAL
    assert b"unknown workspace kind" in L.iat_last_error()
    assert L.iat_workspace_bytes(_abi.WS_REDUCE, *args, 99, ctypes.byref(out), None) == _abi.IAT_EINVAL
    assert L.iat_workspace_bytes(_abi.WS_INTEGRATE, *args, 0, None, None) == _abi.IAT_EINVAL
    assert out.value == 7


def test_workspace_bytes_refuses_what_the_reduction_refuses():
    from paper_2509_15117_amd import api
    g = W.config1()
    with pytest.raises(_abi.IatError, match="CELLS needs a SWEEP"):
        api.workspace_bytes("reduce", g.system, g.species(), g.gen, 64, reduce_kind="cells")
    with pytest.raises(_abi.IatError, match="whole GRID"):
        api.workspace_bytes("reduce", g.system, g.species(), g.gen, 32, reduce_kind="boxcount")
    s3 = W.config3()
    with pytest.raises(_abi.IatError, match="whole GRID"):
        api.workspace_bytes("reduce", s3.system, s3.species(), s3.gen, 64, reduce_kind="boxcount")
    assert api.workspace_bytes("reduce", g.system, g.species(), g.gen, 0, reduce_kind="cells") == 0
