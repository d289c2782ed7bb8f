"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: order conditions
and convergence order of the Dormand-Prince pair, the gradient of the Eq. (1)
Hamiltonian written out independently here, two-body invariants with the trap off,
closed-form head-on kinematics, the classical deflection integral, Floquet theory of
the Mathieu equation (Hill determinant), time reversibility, the rotational symmetry
of the ring trap, numpy's Philox4x64-10 and hand-made final states.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.linalg import eigh_tridiagonal
from scipy.optimize import brentq

import oracle
import workloads as W

oracle.build()


# ----------------------------------------------------------------------------- helpers
def rb_problem(**over):
    w = W.config1()
    p = oracle.base_problem(w.system, w.species()[0])
    for k, v in over.items():
        p[k] = v
    return p


def trap_off(p):
    p["a"] = 0.0
    p["q"] = 0.0
    return p


def potential(p, r):
    C8 = p["C4"] ** 2 / (4 * p["De"])
    return C8 / r ** 8 - p["C4"] / r ** 4


# ----------------------------------------------------------------------------- tableau
def test_tableau_order_conditions():
    A, b, bh, c = oracle.tableau()
    # row sums c_i = sum_j a_ij, FSAL: last row of A equals b
    assert np.allclose(A.sum(1), c, atol=1e-15, rtol=0)
    assert np.allclose(A[6, :6], b[:6], atol=0, rtol=0)
    assert b[6] == 0.0
    e = np.ones(7)
    Ac = A @ c
    conds5 = [
        (e, 1.0), (c, 1 / 2), (c ** 2, 1 / 3), (Ac, 1 / 6),
        (c ** 3, 1 / 4), (c * Ac, 1 / 8), (A @ c ** 2, 1 / 12), (A @ Ac, 1 / 24),
        (c ** 4, 1 / 5), (c ** 2 * Ac, 1 / 10), (c * (A @ c ** 2), 1 / 15), (c * (A @ Ac), 1 / 30),
        (Ac ** 2, 1 / 20), (A @ c ** 3, 1 / 20), (A @ (c * Ac), 1 / 40), (A @ (A @ c ** 2), 1 / 60),
        (A @ (A @ Ac), 1 / 120),
    ]
    for v, target in conds5:
        assert abs(b @ v - target) < 1e-15
    for v, target in conds5[:8]:
        assert abs(bh @ v - target) < 1e-15
    # the embedded solution is genuinely fourth order: it misses a fifth-order condition
    assert max(abs(bh @ v - t) for v, t in conds5[8:]) > 1e-6


@pytest.mark.parametrize("kind,lam,t_end", [(0, -1.0, 2.0), (1, 0.0, 2 * math.pi)])
def test_fixed_step_convergence_order_five(kind, lam, t_end):
    errs = [abs(oracle.fixed_step_error(kind, lam, t_end, n)) for n in (20, 40, 80)]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for s in slopes:
        assert 4.8 < s < 5.3, slopes


# ----------------------------------------------------------------------------- forces
def hamiltonian(p, y, t):
    """Eq. (1) written out in atomic units."""
    ra, ri, va, vi = y[0:3], y[3:6], y[6:9], y[9:12]
    r = np.linalg.norm(ra - ri)
    h = 0.5 * p["m_atom"] * va @ va + 0.5 * p["m_ion"] * vi @ vi + potential(p, r)
    for k in range(3):
        h += (p["a"][k] + 2 * p["q"][k] * math.cos(p["omega"] * t + p["phase0"])) * \
            p["m_ion"] * p["omega"] ** 2 * ri[k] ** 2 / 8
    return h


def fd_accelerations(p, y, t, rel=1e-6):
    acc = np.zeros(6)
    for j in range(6):
        step = rel * max(1.0, abs(y[j]))
        yp, ym = y.copy(), y.copy()
        yp[j] += step
        ym[j] -= step
        dH = (hamiltonian(p, yp, t) - hamiltonian(p, ym, t)) / (2 * step)
        acc[j] = -dH / (p["m_atom"] if j < 3 else p["m_ion"])
    return acc


@pytest.mark.parametrize("sep", [55.0, 70.0, 140.0, 600.0])
def test_interaction_force_is_minus_gradient_of_eq1(sep):
    p = rb_problem(phase0=0.3)
    rng = np.random.default_rng(7)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    y = np.zeros(12)
    y[3:6] = [3.0, -2.0, 1.0]
    y[0:3] = y[3:6] + sep * n
    y[6:12] = rng.normal(size=6) * 1e-8
    t = 1.234e9
    dy = oracle.rhs_au(p, t, y)
    assert np.allclose(dy[0:6], y[6:12], rtol=0, atol=0)
    ref = fd_accelerations(p, y, t)
    scale = np.abs(ref).max()
    assert np.abs(dy[6:12] - ref).max() < 1e-7 * scale


@pytest.mark.parametrize("phase0,t", [(0.0, 0.0), (0.7, 3.1e9), (2.0, 1.0e10)])
def test_trap_force_is_minus_gradient_of_eq1(phase0, t):
    p = rb_problem(phase0=phase0)
    p["a"] = [0.01, 0.01, -0.02]
    y = np.zeros(12)
    y[0:3] = [0.0, 0.0, 1e7]           # atom far away: the ion feels the trap only
    y[3:6] = [120.0, -80.0, 45.0]
    dy = oracle.rhs_au(p, t, y)
    ref = fd_accelerations(p, y, t)
    assert np.abs(dy[9:12] - ref[3:6]).max() < 1e-8 * np.abs(ref[3:6]).max()
    # sign convention of Eq. (1): at RF phase 0 with a = 0 the x axis is restoring for q > 0
    p2 = rb_problem(phase0=0.0)
    d0 = oracle.rhs_au(p2, 0.0, y)
    assert d0[9] < 0 and d0[10] > 0 and d0[11] > 0


def test_potential_minimum_and_newton_third_law():
    p = trap_off(rb_problem())
    rm = (p["C4"] / (2 * p["De"])) ** 0.25
    assert abs(potential(p, rm) + p["De"]) < 1e-14 * p["De"]
    y = np.zeros(12)
    y[0:3] = [rm, 0.0, 0.0]
    dy = oracle.rhs_au(p, 0.0, y)
    y2 = y.copy()
    y2[0] = 0.9 * rm
    dy2 = oracle.rhs_au(p, 0.0, y2)
    assert abs(dy[6]) < 1e-12 * abs(dy2[6])          # no force at the well bottom
    assert dy2[6] > 0                                # repulsive inside r_m
    y3 = y.copy()
    y3[0:3] = [40.0, 70.0, -20.0]
    y3[3:6] = [1.0, 2.0, 3.0]
    d3 = oracle.rhs_au(p, 0.0, y3)
    fa = p["m_atom"] * d3[6:9]
    fi = p["m_ion"] * d3[9:12]
    assert np.abs(fa + fi).max() < 1e-14 * np.abs(fa).max()


# ----------------------------------------------------------------------------- invariants
def _energy(p, y):
    r = np.linalg.norm(y[0:3] - y[3:6])
    return (0.5 * p["m_atom"] * y[6:9] @ y[6:9] + 0.5 * p["m_ion"] * y[9:12] @ y[9:12] + potential(p, r))


def _angmom(p, y):
    return p["m_atom"] * np.cross(y[0:3], y[6:9]) + p["m_ion"] * np.cross(y[3:6], y[9:12])


@pytest.mark.parametrize("b", [30.0, 150.0, 900.0])
def test_two_body_invariants_trap_off(b):
    p = trap_off(rb_problem(rtol=1e-12, atol=1e-14))
    E = p["m_atom"] * 0 + W.kelvin(1.5e-6)
    v0 = math.sqrt(2 * E / p["m_atom"])
    r0 = p["r0"]
    y0 = np.zeros(12)
    y0[0:3] = [b, 0.0, math.sqrt(r0 ** 2 - b ** 2)]
    y0[6:9] = [0.0, 0.0, -v0]
    p["y0"] = y0
    res = oracle.integrate_one(p)
    assert res["status"] & oracle.EXITED
    yf = res["y_final"]
    # energy drift normalised by the largest kinetic energy on the path (~ the well depth)
    assert abs(_energy(p, yf) - _energy(p, y0)) / p["De"] < 1e-10
    L0 = _angmom(p, y0)
    assert np.abs(_angmom(p, yf) - L0).max() / (p["m_atom"] * r0 * v0) < 1e-10
    # centre of mass moves uniformly
    M = p["m_atom"] + p["m_ion"]
    R0 = (p["m_atom"] * y0[0:3] + p["m_ion"] * y0[3:6]) / M
    V0 = (p["m_atom"] * y0[6:9] + p["m_ion"] * y0[9:12]) / M
    Rf = (p["m_atom"] * yf[0:3] + p["m_ion"] * yf[3:6]) / M
    assert np.abs(Rf - (R0 + V0 * res["t_dwell"])).max() < 1e-9 * r0


def test_headon_trap_off_closed_forms():
    """Trap off, head on: one bounce, straight back-scatter, 2 mu v0 momentum transfer,
    recoil energy of the ion, and the dwell time from the 1-D quadrature of dr / rdot."""
    p = trap_off(rb_problem(rtol=1e-14, atol=1e-18))
    E = W.kelvin(1.5e-6)
    theta, phi = 0.7, 0.3
    p["y0"] = oracle.headon_state(theta, phi, E, p["m_atom"], p["r0"])
    res = oracle.integrate_one(p)
    ma, mi = p["m_atom"], p["m_ion"]
    M, mu = ma + mi, ma * mi / (ma + mi)
    v0 = math.sqrt(2 * E / ma)
    assert res["n_bounce"] == 1 and res["status"] & oracle.EXITED
    assert not res["status"] & oracle.COMPLEX
    assert abs(res["angle"] - math.pi) < 1e-9
    # the exit speed inherits the energy error, which is ~rtol relative to the well depth,
    # i.e. ~rtol * De / E relative to the collision energy (6e-7 at rtol 1e-12)
    assert abs(res["q_transfer"] - 2 * mu * v0) < 1e-7 * 2 * mu * v0
    dE = 2 * mi * ma ** 2 * v0 ** 2 / M ** 2
    assert abs(res["dE_ion"] - dE) < 2e-7 * dE
    # dwell time: t = 2 int_{r_t}^{r0} dr / sqrt(2 (E_rel - V(r)) / mu)
    r0 = p["r0"]
    E_rel = 0.5 * mu * v0 ** 2 + potential(p, r0)
    rm = (p["C4"] / (2 * p["De"])) ** 0.25
    rt = brentq(lambda r: potential(p, r) - E_rel, 0.5 * rm, rm, xtol=1e-14, rtol=1e-15)

    def integrand(s):
        r = rt + s * s
        return 2 * s / math.sqrt(max(2 * (E_rel - potential(p, r)) / mu, 1e-300))
    smax = math.sqrt(r0 - rt)
    pts = [math.sqrt(x) for x in (0.01, 0.1, 1.0, 10.0, 100.0, 1000.0) if x < r0 - rt]
    I, _ = quad(integrand, 0.0, smax, points=pts, limit=400, epsabs=0, epsrel=1e-13)
    # truncation error of the dwell time: 5e-8 at rtol 1e-13, 2e-8 at 1e-14 (converges to I)
    assert abs(res["t_dwell"] - 2 * I) < 5e-8 * 2 * I


def deflection_chi(p, b, E_cm):
    """Classical deflection function chi(b) = pi - 2 b int_0^{u_t} du / sqrt(G(u)),
    G(u) = 1 - b^2 u^2 - V(1/u)/E (u = 1/r)."""
    C4 = p["C4"]
    C8 = C4 ** 2 / (4 * p["De"])

    def G(u):
        return 1 - b * b * u * u - (C8 * u ** 8 - C4 * u ** 4) / E_cm
    # outermost turning point: first root of G moving inward from u = 0
    us = np.linspace(1e-12, 1.0 / 30.0, 200001)
    g = G(us)
    i = np.argmax(g <= 0)
    ut = brentq(G, us[i - 1], us[i], xtol=1e-18, rtol=1e-15)

    def f(w):
        u = ut * (1 - w * w)
        return 2 * ut * w / math.sqrt(max(G(u), 1e-300))
    I, _ = quad(f, 0.0, 1.0, limit=400, epsabs=0, epsrel=1e-13)
    return math.pi - 2 * b * I


@pytest.mark.parametrize("b", [700.0, 1200.0, 3000.0])
def test_deflection_against_classical_deflection_integral(b):
    p = trap_off(rb_problem(rtol=1e-12, atol=1e-14))
    E = W.kelvin(10e-3)
    ma, mi = p["m_atom"], p["m_ion"]
    mu = ma * mi / (ma + mi)
    v0 = math.sqrt(2 * E / ma)
    r0 = 1.0e6
    p["r0"] = r0
    y0 = np.zeros(12)
    y0[0:3] = [b, 0.0, math.sqrt(r0 ** 2 - b ** 2)]
    y0[6:9] = [0.0, 0.0, -v0]
    p["y0"] = y0
    res = oracle.integrate_one(p)
    assert res["status"] & oracle.EXITED
    E_cm = 0.5 * mu * v0 ** 2
    chi = deflection_chi(p, b, E_cm)
    lab = math.atan2(abs(math.sin(chi)), math.cos(chi) + ma / mi)
    assert abs(res["angle"] - lab) < 2e-7 * lab
    if b >= 3000.0:
        # small-angle limit of the C4 tail: |chi| ~ (3 pi / 4) C4 / (E_cm b^4)
        chi_sa = 0.75 * math.pi * p["C4"] / (E_cm * b ** 4)
        lab_sa = math.atan2(math.sin(chi_sa), math.cos(chi_sa) + ma / mi)
        assert abs(res["angle"] / lab_sa - 1) < 5 * chi_sa


# ----------------------------------------------------------------------------- Mathieu
def hill_beta(a, q, nmodes=40):
    """Characteristic exponent of x'' + (a - 2 q cos 2 xi) x = 0 from Hill's determinant:
    a is the lowest eigenvalue of the tridiagonal matrix diag((2n + beta)^2), off-diagonal q."""
    n = np.arange(-nmodes, nmodes + 1)

    def lam0(beta):
        return eigh_tridiagonal((2 * n + beta) ** 2, np.full(len(n) - 1, q), eigvals_only=True,
                                select="i", select_range=(0, 0))[0]
    return brentq(lambda bb: lam0(bb) - a, 1e-12, 1 - 1e-12, xtol=1e-15, rtol=1e-15)


def monodromy_trace(ax, qx, axis):
    """Trace of the one-RF-period monodromy matrix of the ion alone, from the oracle."""
    p = rb_problem(rtol=1e-13, atol=1e-16)
    p["a"] = [ax, ax, -2 * ax]
    p["q"] = [qx, qx, -2 * qx]
    p["r0"] = 1e9
    p["t_max"] = 2 * math.pi / p["omega"]
    cols = []
    for j in range(2):
        y0 = np.zeros(12)
        y0[0:3] = [0.0, 0.0, 1e8]
        if j == 0:
            y0[3 + axis] = 1.0
        else:
            y0[9 + axis] = p["omega"]       # unit velocity in internal units
        p["y0"] = y0
        res = oracle.integrate_one(p)
        assert res["status"] & oracle.TMAX
        cols.append((res["y_final"][3 + axis], res["y_final"][9 + axis] / p["omega"]))
    return cols[0][0] + cols[1][1]


@pytest.mark.parametrize("ax,qx", [(0.0, 0.05), (0.0, 0.2), (0.0, 0.35), (0.01, 0.2)])
def test_ion_alone_obeys_mathieu_floquet_theory(ax, qx):
    for axis, (a_k, q_k) in enumerate([(ax, qx), (ax, qx), (-2 * ax, -2 * qx)]):
        if axis == 1:
            continue
        tr = monodromy_trace(ax, qx, axis)
        beta = math.acos(tr / 2) / math.pi
        assert abs(beta - hill_beta(a_k, q_k)) < 1e-9


def test_secular_frequency_lowest_order_limit():
    """omega ~ (Omega/2) sqrt(a + q^2/2): holds to O(q^2) relative as q -> 0."""
    for qx in (0.02, 0.05, 0.1):
        beta = math.acos(monodromy_trace(0.0, qx, 0) / 2) / math.pi
        lowest = math.sqrt(qx * qx / 2)
        assert abs(beta / lowest - 1) < 0.25 * qx * qx


# ----------------------------------------------------------------------------- symmetry
def _one_bounce_problem(rtol=1e-12):
    w = W.config1()
    w.system.rtol = rtol
    w.system.atol = 1e-14
    return oracle.problems_for(w, [63])[0]


def test_time_reversibility_of_a_direct_collision():
    # velocities carry the energy error relative to the collision energy (~rtol De / E),
    # so reversal is checked at rtol 1e-14
    p = _one_bounce_problem(1e-14)
    fwd = oracle.integrate_one(p)
    assert fwd["n_bounce"] == 1 and fwd["status"] & oracle.EXITED
    yf = fwd["y_final"]
    q = p.copy()
    q["y0"] = np.concatenate([yf[0:6], -yf[6:12]])
    q["phase0"] = -(fwd["tau_final"] + p["phase0"])
    q["t_max"] = fwd["t_dwell"]
    q["r0"] = 1e12
    back = oracle.integrate_one(q)
    assert back["status"] & oracle.TMAX
    yb = back["y_final"]
    y0 = p["y0"]
    v0 = np.linalg.norm(y0[6:9])
    assert np.abs(yb[0:6] - y0[0:6]).max() < 1e-7 * p["r0"]
    assert np.abs(-yb[6:12] - y0[6:12]).max() < 1e-7 * v0


def test_ring_trap_rotational_symmetry():
    """q_y = q_x: rotating the start about z leaves every observable unchanged.

    Different azimuths take different step sequences, so the runs differ by truncation
    error.  The ion energy at the exit is compared at a common time: it swings with the
    micromotion, so an exit-time difference dt moves it by dE_ion/dt * dt."""
    w = W.config1()
    w.system.rtol, w.system.atol = 1e-12, 1e-14
    sp = w.species()[0]
    out, probs = [], []
    for phi in (0.1, 0.77, 1.3):
        p = oracle.base_problem(w.system, sp)
        p["y0"] = oracle.headon_state(1.45, phi, w.system.E, p["m_atom"], w.system.r0)
        out.append(oracle.integrate_one(p))
        probs.append(p)
    for r, p in zip(out[1:], probs[1:]):
        assert r["n_bounce"] == out[0]["n_bounce"] == 1
        for key in ("angle", "q_transfer", "t_dwell"):
            assert abs(r[key] - out[0][key]) < 1e-8 * abs(out[0][key])
        t_ref = out[0]["t_dwell"]
        y_al = r["y_final"] + oracle.rhs_au(p, r["t_dwell"], r["y_final"]) * (t_ref - r["t_dwell"])
        dE_al = oracle.ion_energy(p, y_al, t_ref) - oracle.ion_energy(p, p["y0"], 0.0)
        assert abs(dE_al - out[0]["dE_ion"]) < 1e-7 * abs(out[0]["dE_ion"])


# ----------------------------------------------------------------------------- observables
def test_observables_on_synthetic_final_states():
    p = rb_problem()
    E = W.kelvin(1.5e-6)
    y0 = oracle.headon_state(0.4, 1.1, E, p["m_atom"], p["r0"])
    v0 = math.sqrt(2 * E / p["m_atom"])
    back = y0.copy()
    back[6:9] = -y0[6:9]
    a, q, e = oracle.observables(p, y0, back, 0.0)
    assert abs(a - math.pi) < 1e-15 and abs(q - 2 * p["m_atom"] * v0) < 1e-15 * q
    a, q, e = oracle.observables(p, y0, y0, 0.0)
    assert a == 0.0 and q == 0.0 and e == 0.0
    side = y0.copy()
    side[6:9] = np.cross(y0[6:9], [0.0, 0.0, 1.0])
    side[6:9] *= v0 / np.linalg.norm(side[6:9])
    a, q, e = oracle.observables(p, y0, side, 0.0)
    assert abs(a - math.pi / 2) < 1e-15
    assert oracle.ion_energy(p, y0, 0.0) == 0.0
    # ion energy = Eq. (1) ion terms
    y = y0.copy()
    y[3:6] = [10.0, -20.0, 5.0]
    y[9:12] = [1e-9, 2e-9, -3e-9]
    t = 7.7e8
    ref = 0.5 * p["m_ion"] * y[9:12] @ y[9:12] + sum(
        (p["a"][k] + 2 * p["q"][k] * math.cos(p["omega"] * t + p["phase0"])) * p["m_ion"] *
        p["omega"] ** 2 * y[3 + k] ** 2 / 8 for k in range(3))
    assert abs(oracle.ion_energy(p, y, t) - ref) < 1e-14 * abs(ref)


def test_exit_is_located_on_the_sphere():
    w = W.config1()
    res = oracle.integrate(oracle.problems_for(w, range(0, 64, 9)), 4)
    for r in res:
        assert r["status"] & oracle.EXITED
        yf = r["y_final"]
        assert abs(np.linalg.norm(yf[0:3] - yf[3:6]) - w.system.r0) < 1e-9 * w.system.r0


# ----------------------------------------------------------------------------- status bits
def test_status_flags_forced_from_inputs():
    p = _one_bounce_problem(1e-10)
    q = p.copy()
    q["t_max"] = 1e-3 * p["t_max"]
    r = oracle.integrate_one(q)
    assert r["status"] & oracle.TMAX and r["status"] & oracle.COMPLEX
    assert r["tau_final"] == q["t_max"] * q["omega"]
    q = p.copy()
    q["hmin"] = 1.0
    r = oracle.integrate_one(q)
    assert r["status"] & oracle.H_UNDERFLOW and r["n_accept"] == 0
    q = p.copy()
    q["y0"][0] = float("nan")
    r = oracle.integrate_one(q)
    assert r["status"] & oracle.NONFINITE and r["n_rhs"] == 0
    q = p.copy()
    q["max_steps"] = 10
    r = oracle.integrate_one(q)
    assert r["status"] & oracle.MAX_STEPS and r["n_accept"] == 10
    r = oracle.integrate_one(p)
    assert not r["status"] & oracle.WARN_R0
    cs = W.Workload("cs", 1, W.System(E=W.kelvin(1e-6)), ["Cs133"], W.Generator(kind="grid", n_theta=1, n_phi=1))
    q = oracle.problems_for(cs, [0])[0]
    q["max_steps"] = 5
    assert oracle.integrate_one(q)["status"] & oracle.WARN_R0


# ----------------------------------------------------------------------------- generators
def test_philox4x64_matches_numpy():
    rng = np.random.default_rng(3)
    for _ in range(6):
        ctr = rng.integers(1, 2 ** 63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        # numpy increments the 256-bit counter before producing each block
        start = ctr.copy()
        start[0] -= np.uint64(1)
        ref = np.random.Philox(key=key, counter=start).random_raw(4).astype(np.uint64)
        assert np.array_equal(oracle.philox4x64_10(ctr, key), ref)
    zero = np.zeros(4, dtype=np.uint64)
    ref0 = np.random.Philox(key=np.array([5, 9], dtype=np.uint64),
                            counter=np.full(4, 2 ** 64 - 1, dtype=np.uint64)).random_raw(4)
    assert np.array_equal(oracle.philox4x64_10(zero, np.array([5, 9], dtype=np.uint64)), ref0)


def test_sweep_draws_follow_the_philox_stream_and_cell_digits():
    w = W.config3()
    g = w.gen
    for gid in (0, 1, 224, 225, 9_999_999):
        d = oracle.sweep_draw(gid, g)
        bg = np.random.Philox(key=np.array([g.seed, 0], dtype=np.uint64),
                              counter=np.array([2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1],
                                               dtype=np.uint64))
        bg.advance(gid)  # counter (gid, 0, 0, 0) after the pre-increment
        u = (bg.random_raw(4) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        assert d["cos_theta"] == 1 - 2 * u[0] and d["phi"] == 2 * math.pi * u[1]
        assert d["phase0"] == 2 * math.pi * u[2]
        c = gid % 225
        assert d["species"] == c // 45
        assert d["E"] == g.E_list[(c // 9) % 5] and d["q_x"] == g.q_list[(c // 3) % 3]
        assert d["De"] == g.De_list[c % 3]


def test_grid_is_cell_centred_on_the_octant():
    a = oracle.grid_angles([0, 1, 7, 8, 63], 8, 8)
    step = math.pi / 2 / 8
    assert np.allclose(a[0], [0.5 * step, 0.5 * step], rtol=0, atol=1e-16)
    assert np.allclose(a[1], [0.5 * step, 1.5 * step], rtol=0, atol=1e-16)
    assert np.allclose(a[3], [1.5 * step, 0.5 * step], rtol=0, atol=1e-16)
    assert np.allclose(a[4], [7.5 * step, 7.5 * step], rtol=0, atol=1e-16)
    assert np.allclose(oracle.grid_angles([0], 1, 1)[0], [math.pi / 4, math.pi / 4])
