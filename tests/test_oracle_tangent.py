"""Pins of the oracle's tangent-linear (internal differentiation of the accepted-step map).

* The stability matrix of a Hamiltonian flow is symplectic: Phi^T Omega Phi = Omega with the
  mass-weighted form Omega = [[0, M], [-M, 0]] of the (r, v) coordinates.  Every entry of the
  Jacobian (the force Hessian, mass factors, signs, the trap term) enters this identity.
* Observable sensitivities agree with frozen-step central differences of the oracle's own
  primal, entry by entry at the best of several steps.
* At the step h = 1e-6 relative, central differences agree in the norm of the
  parameter-scaled gradient only to a few 1e-3: the frozen-step map is strongly nonlinear in E
  (the recorded fine steps around the bounce stop fitting a trajectory whose bounce moves), so
  the difference quotient itself is off by O(h^2) = 2e-4 there; it falls to 2e-6 at h = 1e-7.
"""
import numpy as np
import pytest

import oracle
import workloads as W

oracle.build()

DIRECT_IDS = [40, 47, 51, 58, 63]      # one-bounce cells of the 8x8 grid


def _problem(gid, rtol=1e-10):
    w = W.config1()
    w.system.rtol = rtol
    p = oracle.problems_for(w, [gid])[0]
    th, ph = oracle.grid_angles([gid], 8, 8)[0]
    return w, p, th, ph


def _scales(w):
    return np.array([1.0, 1.0, w.system.E, w.system.q_x, w.system.De])


@pytest.mark.parametrize("gid", DIRECT_IDS[:3])
def test_stability_matrix_is_symplectic(gid):
    w, p, th, ph = _problem(gid)
    _, Phi, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    M = np.diag([p["m_atom"]] * 3 + [p["m_ion"]] * 3)
    Om = np.block([[np.zeros((6, 6)), M], [-M, np.zeros((6, 6))]])
    defect = Phi.T @ Om @ Phi - Om
    scale = np.abs(Phi.T) @ np.abs(Om) @ np.abs(Phi)
    assert (np.abs(defect) / scale).max() < 1e-7
    # and it is not trivially so: the collision stretches phase space by orders of magnitude
    assert np.linalg.svd(Phi, compute_uv=False)[0] > 100.0


@pytest.mark.parametrize("gid", DIRECT_IDS)
def test_lyapunov_spectrum_comes_in_opposite_pairs(gid):
    """A symplectic matrix has singular values in pairs (s, 1/s), so the finite-time Lyapunov
    spectrum of the canonically scaled stability matrix is symmetric: lambda_i + lambda_(13-i) = 0.
    The Dormand-Prince map is symplectic only up to its truncation error, so on these trajectories
    (s_max ~ 1e4) the pairs hold to ~3e-5 in ln(s s'), tested at 2e-4; without the sqrt(mass)
    scaling the pairing fails by more than 1e-2 (the masses differ by a factor two)."""
    w, p, th, ph = _problem(gid)
    _, Phi, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    t_f = oracle.integrate_one(p)["t_dwell"]
    lam = oracle.lyapunov_spectrum(Phi, p["m_atom"], p["m_ion"], t_f)
    assert np.all(np.diff(lam) <= 0) and lam[0] > 0
    pair = (lam + lam[::-1]) * t_f                      # ln(s_i s_(13-i))
    assert np.abs(pair).max() < 2e-4, pair
    s_raw = np.linalg.svd(Phi, compute_uv=False)
    assert np.abs(np.log(s_raw * s_raw[::-1])).max() > 1e-2


@pytest.mark.parametrize("gid", DIRECT_IDS)
def test_sensitivities_match_central_differences_entrywise(gid):
    """Each sizeable entry (>= 1% of the observable's largest parameter-scaled sensitivity)
    agrees to 1e-3 at the best of several difference steps (the differences themselves resolve
    some entries only to a few 1e-4).  Frozen steps limit the usable
    step from above (the recorded fine steps around the bounce stop fitting a perturbed
    trajectory) and round-off limits it from below, so the error curve has a minimum."""
    w, p, th, ph = _problem(gid)
    d, _, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    fds = [oracle.fd(p, th, ph, w.system.E, w.system.q_ratio, rh) for rh in (1e-5, 3e-6, 1e-6, 3e-7, 1e-7)]
    s = _scales(w)
    for k in range(3):
        g = d[k] * s
        big = np.abs(g) >= 0.01 * np.abs(g).max()
        best = np.min([np.abs(g - f[k] * s) for f in fds], axis=0)
        assert np.all(best[big] <= 1e-3 * np.abs(g[big])), (k, g, best)
    # the azimuthal derivative vanishes for the axially symmetric trap
    assert np.all(np.abs(d[:, 1] * s[1]) < 1e-6 * np.abs(d * s).max(axis=1))


@pytest.mark.parametrize("gid", DIRECT_IDS[:2])
def test_sensitivities_match_central_differences_at_1e_6(gid):
    w, p, th, ph = _problem(gid)
    d, _, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    f = oracle.fd(p, th, ph, w.system.E, w.system.q_ratio, 1e-6)
    s = _scales(w)
    for k in range(3):
        g, gf = d[k] * s, f[k] * s
        assert np.linalg.norm(g - gf) < 5e-3 * np.linalg.norm(gf)


def test_free_particle_limit():
    """Trap off and no interaction (C4 = 0): the flow is free flight, which every Runge-Kutta step
    integrates exactly, so the stability matrix at the exit is [[I, tau_f I], [0, I]] in the internal
    state (positions in a0, velocities per unit of tau = Omega t)."""
    w = W.config1()
    w.system.a_x, w.system.q_x = 0.0, 0.0
    m = w.species()[0][0]
    p = oracle.base_problem(w.system, (m, 0.0))
    th, ph = 0.7, 0.3
    _, Phi, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    p["y0"] = oracle.headon_state(th, ph, w.system.E, m, w.system.r0)
    r = oracle.integrate_one(p)
    assert r["status"] & oracle.EXITED and r["n_bounce"] == 0
    tau_f = r["tau_final"]
    v0 = np.sqrt(2.0 * w.system.E / m) / w.system.omega_rf
    assert tau_f == pytest.approx(2.0 * w.system.r0 / v0, rel=1e-9)
    ref = np.block([[np.eye(6), tau_f * np.eye(6)], [np.zeros((6, 6)), np.eye(6)]])
    assert np.abs(Phi - ref).max() <= 1e-12 * tau_f


@pytest.mark.parametrize("gid", DIRECT_IDS)
def test_tangent_against_extended_precision_richardson_differences(gid):
    """Frozen-step central differences replayed in extended precision and Richardson-extrapolated
    from h and h/2 (h = 1e-6 relative, the step of the differentiation workload) resolve the
    sensitivities far below the FP64 floor of plain differences: the parameter-scaled gradient of a
    random contraction agrees with the tangent within 1e-5 of its norm (observed 6e-8..3e-6, the
    tangent's own round-off, measured by its FMA twin at 3e-7..2e-6).  The remaining truncation is
    O(h^4): doubling h multiplies the difference by ~16 (not 4, as for plain central differences)."""
    w, p, th, ph = _problem(gid)
    s = _scales(w)
    g = np.random.default_rng(gid).normal(size=3)
    d, _, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    ref = (g[:, None] * d).sum(0) * s

    def err(h):
        r = oracle.fd_richardson(p, th, ph, w.system.E, w.system.q_ratio, h)
        return np.linalg.norm((g[:, None] * r).sum(0) * s - ref) / np.linalg.norm(ref)
    e1, e2, e4 = err(1e-6), err(2e-6), err(4e-6)
    print(f"gid {gid}: |tangent - Richardson FD| / |grad| at h = 1e-6, 2e-6, 4e-6: {e1:.1e} {e2:.1e} {e4:.1e}")
    assert e1 < 1e-5
    assert 10.0 < e4 / e2 < 25.0
