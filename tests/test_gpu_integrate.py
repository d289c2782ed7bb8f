"""GPU parity of iat_integrate (plain and persistent kernels) against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests import _parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_15117_amd as iat  # noqa: E402
from paper_2509_15117_amd import api  # noqa: E402

KERNELS = ["plain", "persistent"]


def run(w, n=None, id0=0, **kw):
    out = api.integrate_workload(w, n=n, id0=id0, y_final=True, **kw)
    torch.cuda.synchronize()
    return PT.to_numpy(out)


def oracle_run(w, ids):
    P = oracle.problems_for(w, ids)
    return P, oracle.integrate(P)


def assert_parity(P, ref, got, name, min_direct=1, wide_frac=PT.WIDE_FRAC):
    direct, rest, _ = PT.check_parity(P, ref, got, name, min_direct=min_direct, wide_frac=wide_frac)
    return direct, rest


@pytest.mark.parametrize("kernel", KERNELS)
def test_config1_grid_parity(kernel):
    w = W.config1()
    got = run(w, kernel=kernel)
    P, ref = oracle_run(w, range(64))
    print(f"config1 {kernel}: n_bounce {got['n_bounce'].tolist()}", flush=True)
    direct, rest = assert_parity(P, ref, got, f"config1/{kernel}", min_direct=16)
    assert len(direct) + len(rest) == 64


@pytest.mark.parametrize("kernel", KERNELS)
def test_sweep_parity_ragged(kernel):
    """1000 sweep ids of the 5-species workload (ragged: not a multiple of 64), id0 offset."""
    w = W.config3()
    id0 = 1_234_567
    got = run(w, n=1000, id0=id0, kernel=kernel)
    P, ref = oracle_run(w, np.arange(id0, id0 + 1000))
    assert_parity(P, ref, got, f"sweep/{kernel}", min_direct=400)


def test_thermal_start_states_match_the_oracle():
    """Thermal-run starts (Fig. 3): after a 1 ns run (two steps) the GPU state equals the oracle's
    to the last bits -- the Philox blocks, the Box-Muller normals and the state built from them."""
    w = W.fig3_thermal()
    w.system.t_max = W.seconds(1e-9)
    id0, n = 987_654, 1000
    got = run(w, n=n, id0=id0)
    P, ref = oracle_run(w, np.arange(id0, id0 + n))
    assert np.all(got["status"] & oracle.TMAX) and np.all(ref["status"] & oracle.TMAX)
    assert np.array_equal(got["n_accept"], ref["n_accept"])
    yr = np.stack(ref["y_final"], axis=1)
    scale = np.abs(yr).max(axis=1, keepdims=True)
    err = np.abs(got["y_final"] - yr) / scale
    print(f"thermal starts: n={n}, max |gpu - oracle| / component scale {err.max():.1e}", flush=True)
    assert err.max() < 1e-13


@pytest.mark.parametrize("kernel", KERNELS)
def test_thermal_parity_ragged(kernel):
    """1000 thermal-run ids (ragged, id0 offset): direct trajectories one by one, the rest in
    ensemble; the exit is the sphere about the trap centre."""
    w = W.fig3_thermal()
    w.system.max_steps = 2_000_000
    id0 = 31_337
    got = run(w, n=1000, id0=id0, kernel=kernel)
    P, ref = oracle_run(w, np.arange(id0, id0 + 1000))
    r_atom = np.linalg.norm(got["y_final"][0:3], axis=0)
    ex = (got["status"].astype(np.int64) & oracle.EXITED) != 0
    assert np.all(np.abs(r_atom[ex] - w.system.r0) < 1e-8 * w.system.r0)
    assert_parity(P, ref, got, f"thermal/{kernel}", min_direct=400)


def test_fig4_energy_sweep_parity_ragged():
    """Fig. 4 runs: r0 = 20,000 a0, collision energies log-uniform over 0.1 uK - 1 mK, random RF
    phase, five atoms; 700 ids from an offset."""
    w = W.fig4_energy()
    w.system.max_steps = 2_000_000
    id0 = 4_000_321
    got = run(w, n=700, id0=id0)
    P, ref = oracle_run(w, np.arange(id0, id0 + 700))
    assert np.all(P["r0"] == 20_000.0)
    assert_parity(P, ref, got, "fig4", min_direct=300)


def test_plain_and_persistent_are_bitwise_identical():
    """Same ids -> same bits, whichever kernel, lane or launch shape; a small step budget sends
    most trajectories through the four-lanes-per-trajectory kernel, so it is checked too."""
    thermal = W.fig3_thermal()
    thermal.system.max_steps = 2_000_000
    for w, n in ((W.config1(), 64), (W.config3(), 3001), (thermal, 2001)):
        a = run(w, n=n, kernel="plain")
        for kw in (dict(block=256), dict(block=64, refill_every=4), dict(block=128, blocks_per_cu=1),
                   dict(step_budget=-1), dict(step_budget=7), dict(step_budget=500, refill_every=3),
                   dict(step_budget=7, max_suspended=5),            # most cannot be suspended
                   dict(step_budget=7, tail_budget=11),             # most finish in the solo kernel
                   dict(step_budget=5, tail_budget=3, max_suspended=40),   # solo records run out
                   dict(step_budget=7, tail_budget=-1)):
            b = run(w, n=n, kernel="persistent", **kw)
            for k in a:
                assert np.array_equal(a[k], b[k], equal_nan=True), (w.name, kw, k)


def test_full_size_grid_sampled_against_oracle():
    """1024x1024 grid in the benchmark's launch configuration; sampled ids checked one by one."""
    w = W.config2()
    stats = api.new_stats()
    out = api.integrate_workload(w, y_final=True, stats=stats)
    torch.cuda.synchronize()
    got = PT.to_numpy(out)
    st = got["status"].astype(np.int64)
    ends = st & (oracle.EXITED | oracle.TMAX | oracle.H_UNDERFLOW | oracle.NONFINITE | oracle.MAX_STEPS)
    assert np.all(ends != 0), "every trajectory must end with a stop reason"
    assert np.all((got["angle"] >= 0) & (got["angle"] <= math.pi))
    # RHS evaluations: the first stage, 6 per attempted step, 4 x 5 for the exit re-steps
    ran = (st & (oracle.EXITED | oracle.TMAX)) != 0
    expect = 1 + 6 * (got["n_accept"] + got["n_reject"]) + np.where(st & oracle.EXITED, 20, 0)
    assert np.array_equal(got["n_rhs"][ran], expect[ran])
    s = stats.cpu().numpy()
    assert s[3] == w.n and s[0] == got["n_rhs"].sum() and s[1] == got["n_accept"].sum()
    # every attempted step is counted once, whichever of the three kernels ran it
    assert s[5] == (got["n_accept"] + got["n_reject"]).sum()
    # (the step budget counts attempted steps; a trajectory whose exit search starts on the budget's
    # own step is suspended with exactly that many)
    att = got["n_accept"] + got["n_reject"]
    assert int((att > 20000).sum()) <= s[7] + s[9] <= int((att >= 20000).sum())
    # the last survivors of the four-lane tail move to the solo level once they fit its waves (four
    # per compute unit): at most that many finish there; stats[10] names the longest trajectory
    n_solo = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    assert 0 < s[9] <= n_solo, (s[9], n_solo)
    steps_max, gid_max = api.longest_of(stats.cpu())
    assert steps_max == int(att.max()) and att[gid_max] == steps_max
    assert 0 < s[8] and s[6] + s[8] < s[0]
    rng = np.random.default_rng(11)
    ids = np.sort(rng.choice(w.n, size=96, replace=False))
    P, ref = oracle_run(w, ids)
    sub = {k: (v[:, ids] if k == "y_final" else v[ids]) for k, v in got.items()}
    assert_parity(P, ref, sub, "config2-sampled", min_direct=10)


@pytest.mark.parametrize("which", ["sweep_1.2e7", "stream_1e8", "fig4_5e6"])
def test_full_size_chunked_sampled_against_oracle(which):
    """The 1.2e7 sweep and the 5e6 Fig. 4 energy sweep (r0 = 20,000 a0) in the benchmark's launch
    configuration (the job split over two streams, reductions on the device), and the whole 1e8 stream
    in the same chunked form: 96 seeded ids copied out of their chunks and checked one by one (direct)
    or in ensemble; the reductions count every trajectory once."""
    sweep = which.startswith("sweep")
    w = {"sweep_1.2e7": W.config3, "stream_1e8": W.config5, "fig4_5e6": W.fig4_energy}[which]()
    n = w.n
    seed = {"sweep_1.2e7": 3, "stream_1e8": 5, "fig4_5e6": 44}[which]
    ids = np.sort(np.random.default_rng(seed).choice(n, size=96, replace=False))
    print(f"{w.name}: n={n} in two chunks on two streams, 96 sampled ids", flush=True)
    res = api.run_chunks(w, n=n, chunk=-(-n // 2), n_streams=2, cells=sweep, hist=not sweep, sample=ids)
    got = PT.to_numpy(res["sample"])
    if sweep:
        assert res["cells"][:, 0].sum().item() == n
    else:
        assert api.split_hist(res["hist"])[1].sum().item() == n
    # the oracle stops at 2e6 accepted steps (the library runs to the workloads' cap of 2e7): the few
    # sampled complexes that live longer are left out on both sides
    P = oracle.problems_for(w, ids)
    P["max_steps"] = 2_000_000
    ref = oracle.integrate(P)
    keep = np.where((got["n_accept"] < 2_000_000) & ((ref["status"] & oracle.MAX_STEPS) == 0))[0]
    print(f"{w.name}: {96 - len(keep)} sampled complexes beyond 2e6 steps left out", flush=True)
    assert len(keep) >= 90
    sub = {k: (v[:, keep] if k == "y_final" else v[keep]) for k, v in got.items()}
    assert_parity(P[keep], ref[keep], sub, f"{w.name}-sampled", min_direct=10)


def test_stream_batch_in_bench_configuration_sampled_against_oracle():
    """The stream's timed batch exactly as the benchmark runs it: 20 chunks of 2^22 ids after one warm-up
    chunk (ids 2^22 .. 21 * 2^22 - 1) in one iat_integrate call with the stream's step budget and the
    recorded launch shape, then the on-device W0 and heating histograms.  96 seeded ids are gathered on
    the device and checked one by one (direct) or in ensemble; the histograms and the counters count
    every trajectory of the batch once."""
    import bench
    w = W.config5()
    C = bench.STREAM_CHUNK
    n, id0 = 20 * C, C
    launch = dict(block=128, refill_every=16, step_budget=bench.STREAM_STEP_BUDGET)
    dev = torch.device("cuda", 0)
    print(f"stream batch: n={n} from id {id0}, launch {launch}, 96 sampled ids", flush=True)
    out = api.alloc_obs(n, dev, y_final=True, counters=True)
    stats = api.new_stats()
    api.integrate(w.system, w.species(), w.gen, n, id0=id0, out=out, stats=stats, **launch)
    hist = api.reduce_hist(w.system, w.species(), w.gen, n, out, id0=id0)
    torch.cuda.synchronize()
    hw, hh = api.split_hist(hist)
    assert hw[..., 0].sum().item() == n and hh.sum().item() == n
    s = stats.cpu().tolist()
    assert s[3] == n
    # every trajectory ends with a stop reason; every RHS evaluation and attempted step is counted once
    ends = oracle.EXITED | oracle.TMAX | oracle.H_UNDERFLOW | oracle.NONFINITE | oracle.MAX_STEPS
    assert int(((out["status"].to(torch.int64) & ends) == 0).sum().item()) == 0
    na, nr = out["n_accept"].to(torch.int64), out["n_reject"].to(torch.int64)
    assert s[1] == int(na.sum().item()) and s[5] == int((na + nr).sum().item())
    assert s[0] == int(out["n_rhs"].to(torch.int64).sum().item())
    del na, nr
    longest, gid = api.longest_of(stats)
    print(f"stream batch: longest trajectory {gid} with {longest} attempted steps; solo trajectories {s[9]}",
          flush=True)
    ids = np.sort(np.random.default_rng(55).choice(n, size=96, replace=False))
    loc = torch.as_tensor(ids, device=dev)
    got = PT.to_numpy({k: (v.index_select(1, loc) if k == "y_final" else v.index_select(0, loc))
                       for k, v in out.items()})
    del out
    # as in the chunked test: the oracle stops at 2e6 accepted steps, and the few sampled complexes that
    # live longer are left out on both sides
    P = oracle.problems_for(w, ids + id0)
    P["max_steps"] = 2_000_000
    ref = oracle.integrate(P)
    keep = np.where((got["n_accept"] < 2_000_000) & ((ref["status"] & oracle.MAX_STEPS) == 0))[0]
    print(f"stream batch: {96 - len(keep)} sampled complexes beyond 2e6 steps left out", flush=True)
    assert len(keep) >= 90
    sub = {k: (v[:, keep] if k == "y_final" else v[keep]) for k, v in got.items()}
    assert_parity(P[keep], ref[keep], sub, "stream-batch-sampled", min_direct=10)


def _edge_system(**over):
    w = W.config1()
    for k, v in over.items():
        setattr(w.system, k, v)
    return w


def test_edge_cases_status_flags():
    w = W.config1()
    # empty batch: nothing launched, nothing written
    out = api.integrate_workload(w, n=0)
    assert all(v.numel() == 0 for v in out.values())
    # a single trajectory, and a ragged batch
    for n in (1, 65 - 1):
        got = run(w, n=n)
        P, ref = oracle_run(w, range(n))
        assert np.array_equal(got["n_bounce"], ref["n_bounce"])
    # tiny t_max -> TMAX + COMPLEX at exactly tau_max
    wt = _edge_system(t_max=w.system.t_max * 1e-3)
    got = run(wt, n=8)
    assert np.all(got["status"] & oracle.TMAX) and np.all(got["status"] & oracle.COMPLEX)
    P, ref = oracle_run(wt, range(8))
    assert np.allclose(got["t_dwell"], ref["t_dwell"], rtol=1e-15, atol=0)
    assert np.array_equal(got["n_accept"], ref["n_accept"])
    # hmin above h0 -> H_UNDERFLOW before any step
    got = run(_edge_system(hmin=1.0), n=4)
    assert np.all(got["status"] & oracle.H_UNDERFLOW) and np.all(got["n_accept"] == 0)
    # accepted-step cap
    got = run(_edge_system(max_steps=10), n=4)
    assert np.all(got["status"] & oracle.MAX_STEPS) and np.all(got["n_accept"] == 10)
    # Cs at 1 uK violates 10|V(r0)| < E: warning bit, run proceeds
    cs = W.Workload("cs", 2, W.System(E=W.kelvin(1e-6), max_steps=50), ["Cs133"],
                    W.Generator(kind="grid", n_theta=1, n_phi=2))
    got = run(cs)
    assert np.all(got["status"] & oracle.WARN_R0)
    # non-finite start state through y0: flagged, no step taken
    y0 = torch.zeros(12, 3, dtype=torch.float64, device="cuda")
    y0[:, 0] = float("nan")
    y0[0, 1:] = 5000.0
    y0[6, 1:] = -7.7e-9
    g = W.Generator(kind="arrays")
    out = api.integrate(w.system, w.species(), g, 3, y0=y0, counters=True)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert st[0] & oracle.NONFINITE and out["n_rhs"][0].item() == 0
    assert st[1] & oracle.EXITED and st[2] & oracle.EXITED


def test_arrays_mode_matches_grid_mode():
    w = W.config1()
    th_ph = oracle.grid_angles(range(64), 8, 8)
    arrays = {"theta": torch.tensor(th_ph[:, 0], device="cuda"), "phi": torch.tensor(th_ph[:, 1], device="cuda")}
    g = W.Generator(kind="arrays")
    a = PT.to_numpy(api.integrate(w.system, w.species(), g, 64, arrays=arrays, y_final=True))
    b = run(w)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_trap_off_two_body_invariants_on_the_gpu():
    """Independent of the oracle: with the trap off (a = q = 0) the ion-atom pair is an isolated
    two-body system, so the GPU's final states must conserve the energy (kinetic + C8/r^8 - C4/r^4),
    the angular momentum and the uniform motion of the centre of mass, here at rtol 1e-12 to 1e-10
    of the well depth and of m_a r0 v0, for head-on and off-axis starts."""
    w = W.config1()
    w.system.q_x = 0.0
    w.system.a_x = 0.0
    w.system.rtol, w.system.atol = 1e-12, 1e-14
    m_a, C4 = w.species()[0]
    m_i, De, r0 = w.system.m_ion, w.system.De, w.system.r0
    C8 = C4 * C4 / (4.0 * De)
    v0 = math.sqrt(2.0 * w.system.E / m_a)
    bs = [0.0, 300.0, 700.0, 1500.0, 3000.0, 4500.0]
    y0 = np.zeros((12, len(bs)))
    for j, b in enumerate(bs):
        y0[0:3, j] = [b, 0.0, math.sqrt(r0 ** 2 - b ** 2)]
        y0[6:9, j] = [0.0, 0.0, -v0]
    out = api.integrate(w.system, w.species(), W.Generator(kind="arrays"), len(bs),
                        y0=torch.from_numpy(y0).to("cuda"), y_final=True)
    torch.cuda.synchronize()
    got = PT.to_numpy(out)
    assert np.all(got["status"].astype(np.int64) & oracle.EXITED)

    def energy(y):
        d = y[0:3] - y[3:6]
        r2 = d @ d
        return 0.5 * m_a * y[6:9] @ y[6:9] + 0.5 * m_i * y[9:12] @ y[9:12] + C8 / r2 ** 4 - C4 / r2 ** 2

    def angmom(y):
        return m_a * np.cross(y[0:3], y[6:9]) + m_i * np.cross(y[3:6], y[9:12])

    M = m_a + m_i
    for j in range(len(bs)):
        a, f = y0[:, j], got["y_final"][:, j]
        dE = abs(energy(f) - energy(a)) / De
        dL = np.abs(angmom(f) - angmom(a)).max() / (m_a * r0 * v0)
        V = (m_a * a[6:9] + m_i * a[9:12]) / M
        R = (m_a * f[0:3] + m_i * f[3:6]) / M - (m_a * a[0:3] + m_i * a[3:6]) / M - V * got["t_dwell"][j]
        print(f"b = {bs[j]:6.0f} a0: bounces {got['n_bounce'][j]}, energy drift {dE:.1e} De, "
              f"angular momentum {dL:.1e}, centre of mass {np.abs(R).max() / r0:.1e} r0", flush=True)
        assert dE < 1e-10 and dL < 1e-10 and np.abs(R).max() < 1e-9 * r0


@pytest.mark.parametrize("kernel", KERNELS)
def test_linear_trap_parity(kernel):
    """The linear trap of the Fig. 1 discussion (q_y = -q_x, no RF along z): the whole 8x8 grid and a
    ragged slice of the 64x64 grid, direct trajectories one by one, the rest in ensemble."""
    for side, id0, n, min_direct in ((8, 0, 64, 8), (64, 1000, 777, 100)):
        w = W.headon_grid(side, f"yb_rb_headon_grid_{side}x{side}_linear")
        w.system.a_ratio, w.system.q_ratio = W.LINEAR
        w.system.max_steps = 2_000_000
        got = run(w, n=n, id0=id0, kernel=kernel)
        P, ref = oracle_run(w, np.arange(id0, id0 + n))
        assert np.all(P["q"][:, 1] == -P["q"][:, 0]) and np.all(P["q"][:, 2] == 0.0)
        assert_parity(P, ref, got, f"linear{side}/{kernel}", min_direct=min_direct, wide_frac=PT.WIDE_FRAC_LINEAR)
