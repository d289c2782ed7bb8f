"""Pins of the oracle's bounce bookkeeping (bounce count, first and last bounce times) and of its
bound-state bit, against closed forms of the two-body problem with the trap off.

A bounce is a periapsis of the relative motion inside r_b = r_m (the short-range collision that the
Fig. 1 text counts); its time is the end of the accepted step across which the radial rate turns
from negative to positive, so the true periapsis lies inside that step.  Fig. 2's complex lifetimes
are differences of these times.  The bound-state bit records a negative relative energy (the
temporary bound state of the text after Eq. (2)).

* Head-on scattering: exactly one bounce, and the periapsis time from the quadrature of dr / rdot
  (half the dwell time) falls inside the step that recorded it.
* A bound radial oscillation (atom released at rest inside the well): the bounce count, first and
  last bounce times follow from the radial period, again a quadrature.
* Relative energies of +-2 % of |V| at the start, with the ion moving and the atom at rest: only the
  negative one sets the bit.  Using m_a instead of the reduced mass, the atom's velocity instead of
  the relative one, or a wrong sign of the C8 term would each flip one of the two cases.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle
import workloads as W

oracle.build()


def _problem(**over):
    w = W.config1()
    p = oracle.base_problem(w.system, w.species()[0])
    p["a"] = 0.0
    p["q"] = 0.0
    for k, v in over.items():
        p[k] = v
    return p


def _V(p, r):
    C8 = p["C4"] ** 2 / (4 * p["De"])
    return C8 / r ** 8 - p["C4"] / r ** 4


def _rm(p):
    return (p["C4"] / (2 * p["De"])) ** 0.25


def _mu(p):
    return p["m_atom"] * p["m_ion"] / (p["m_atom"] + p["m_ion"])


def _transit_time(p, E_rel, r_a, r_b):
    """int_{r_a}^{r_b} dr / sqrt(2 (E_rel - V(r)) / mu) with turning points allowed at either end:
    r = r_a + (r_b - r_a)(1 - cos u)/2 takes the inverse-square-root ends away."""
    mu = _mu(p)

    def f(u):
        r = r_a + (r_b - r_a) * (1 - math.cos(u)) / 2
        dr = (r_b - r_a) * math.sin(u) / 2
        return dr / math.sqrt(max(2 * (E_rel - _V(p, r)) / mu, 1e-300))
    val, _ = quad(f, 0.0, math.pi, limit=400, epsabs=0, epsrel=1e-13)
    return val


def _step_ends(h):
    """internal times at the ends of the recorded accepted steps (the oracle accumulates tau += h)"""
    return np.add.accumulate(h)


def test_headon_bounce_time_lies_in_the_step_of_the_periapsis():
    p = _problem(rtol=1e-14, atol=1e-18)
    E = W.kelvin(1.5e-6)
    p["y0"] = oracle.headon_state(0.7, 0.3, E, p["m_atom"], p["r0"])
    res, h = oracle.integrate_one(p, record_cap=4_000_000)
    assert res["n_bounce"] == 1 and res["status"] & oracle.EXITED
    assert res["t_first"] == res["t_last"] > 0
    assert not res["status"] & oracle.BOUND_SEEN
    W_ = p["omega"]
    mu, v0 = _mu(p), math.sqrt(2 * E / p["m_atom"])
    E_rel = 0.5 * mu * v0 ** 2 + _V(p, p["r0"])
    rt = brentq(lambda r: _V(p, r) - E_rel, 0.5 * _rm(p), _rm(p), xtol=1e-14, rtol=1e-15)
    t_peri = _transit_time(p, E_rel, rt, p["r0"]) * W_           # internal time of the periapsis
    ends = _step_ends(h)
    j = int(np.argmin(np.abs(ends - res["t_first"] * W_)))
    assert abs(ends[j] - res["t_first"] * W_) <= 1e-14 * ends[j]
    # timing slack: the integration's own timing error over the whole path, read off the exit time
    # against its quadrature (twice the periapsis time); far below the step through the periapsis
    slack = max(abs(res["t_dwell"] * W_ - 2 * t_peri), 1e-12 * t_peri)
    print(f"periapsis at tau {t_peri:.9f}; recording step ({ends[j] - h[j]:.9f}, {ends[j]:.9f}], "
          f"h = {h[j]:.2e}, timing slack {slack:.1e}")
    assert ends[j] - h[j] - slack < t_peri <= ends[j] + slack
    assert h[j] + 2 * slack < 1e-5 * t_peri


@pytest.mark.parametrize("n_expect", [1, 6])
def test_bound_radial_oscillation_bounce_count_and_times(n_expect):
    """Atom released at rest at 1.5 r_m from the ion (trap off): the pair oscillates between the
    release point and the inner turning point r_in < r_m with radial period T.  Periapses at
    T/2 + k T; t_max after n_expect of them.  The run ends at t_max as a complex with the bound
    state seen, never leaving."""
    p = _problem(rtol=1e-12, atol=1e-14)
    rm = _rm(p)
    r_s = 1.5 * rm
    y0 = np.zeros(12)
    y0[0:3] = [0.0, 0.0, r_s]
    p["y0"] = y0
    E_rel = _V(p, r_s)
    r_in = brentq(lambda r: _V(p, r) - E_rel, 0.5 * rm, rm, xtol=1e-14, rtol=1e-15)
    T = 2 * _transit_time(p, E_rel, r_in, r_s)                    # a.u. time
    p["t_max"] = (n_expect - 1 + 0.5 + 0.37) * T
    res, h = oracle.integrate_one(p, record_cap=4_000_000)
    W_ = p["omega"]
    st = int(res["status"])
    assert st & oracle.TMAX and st & oracle.BOUND_SEEN and not st & oracle.EXITED
    assert bool(st & oracle.COMPLEX) == True         # t_max reached (and >= 2 bounces when n_expect > 1)
    assert res["n_bounce"] == n_expect
    ends = _step_ends(h)
    hmax_bounce = 0.0
    for name, k in (("t_first", 0), ("t_last", n_expect - 1)):
        t_true = (0.5 + k) * T * W_
        j = int(np.argmin(np.abs(ends - res[name] * W_)))
        assert abs(ends[j] - res[name] * W_) <= 1e-14 * ends[j]
        slack = 1e-8 * t_true
        print(f"{name}: bounce {k + 1} at tau {t_true:.9e}, recording step ({ends[j] - h[j]:.9e}, {ends[j]:.9e}]")
        assert ends[j] - h[j] - slack < t_true <= ends[j] + slack
        hmax_bounce = max(hmax_bounce, h[j])
    assert hmax_bounce < 0.02 * T * W_


@pytest.mark.parametrize("frac,bound", [(0.98, True), (1.02, False)])
def test_bound_state_bit_follows_the_relative_energy(frac, bound):
    """Atom at rest at 1.5 r_m, ion moving away from it with relative kinetic energy frac |V|
    (trap off): relative energy -2 % or +2 % of |V|.  The bound pair turns around and bounces (t_max
    after a little over one radial period); the unbound one separates to r0 and exits."""
    p = _problem(rtol=1e-12, atol=1e-14)
    rm = _rm(p)
    r_s = 1.5 * rm
    V = _V(p, r_s)
    u = math.sqrt(2 * frac * abs(V) / _mu(p))
    y0 = np.zeros(12)
    y0[0:3] = [0.0, 0.0, r_s]
    y0[9:12] = [0.0, 0.0, -u]
    p["y0"] = y0
    if bound:
        E_rel = (frac - 1) * abs(V)
        r_out = brentq(lambda r: _V(p, r) - E_rel, r_s, 100 * rm, xtol=1e-10, rtol=1e-15)
        r_in = brentq(lambda r: _V(p, r) - E_rel, 0.5 * rm, rm, xtol=1e-14, rtol=1e-15)
        p["t_max"] = 1.2 * 2 * _transit_time(p, E_rel, r_in, r_out)
    res = oracle.integrate_one(p)
    st = int(res["status"])
    assert bool(st & oracle.BOUND_SEEN) == bound
    if bound:
        assert st & oracle.TMAX and res["n_bounce"] >= 1
    else:
        assert st & oracle.EXITED and res["n_bounce"] == 0
