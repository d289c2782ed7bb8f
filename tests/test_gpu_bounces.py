"""GPU bounce bookkeeping and bound-state bit against the oracle on starts whose answers are fixed
by closed forms (the oracle's pins in test_oracle_bounces.py): a bound radial oscillation with six
periapses, relative energies of -2 % and +2 % of |V| at the start, and head-on scattering, all with
the trap off.  Same accept/reject decisions, so the bounce count, status and step counts must be
identical; the first and last bounce times within max(1e-12, 10 x the oracle's round-off spread)
relative, the spread over its FMA twin and four one-ulp probes of the start positions.  The embedded
error estimate at rtol 1e-12 is a difference of nearly equal stage sums that keeps about seven digits,
so round-off moves every step size by ~1e-8 while the decisions stay the same: over the six periods of
the bound oscillation the bounce times of the oracle's probes spread by 6e-9..1.4e-8."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle
import workloads as W
from tests import _parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402


def _system():
    s = W.System(q_x=0.0, a_x=0.0, rtol=1e-12, atol=1e-14)
    return s


def _consts(s, sp):
    m_a, C4 = sp
    De = s.De
    C8 = C4 * C4 / (4 * De)
    rm = (C4 / (2 * De)) ** 0.25
    mu = m_a * s.m_ion / (m_a + s.m_ion)
    return m_a, C4, C8, rm, mu


def _cases():
    s = _system()
    sp = W.species_table(["Rb87"])[0]
    m_a, C4, C8, rm, mu = _consts(s, sp)

    def V(r):
        return C8 / r ** 8 - C4 / r ** 4

    def period(E_rel, r_a, r_b):
        def f(u):
            r = r_a + (r_b - r_a) * (1 - math.cos(u)) / 2
            return (r_b - r_a) * math.sin(u) / 2 / math.sqrt(max(2 * (E_rel - V(r)) / mu, 1e-300))
        return 2 * quad(f, 0.0, math.pi, limit=400, epsabs=0, epsrel=1e-13)[0]

    r_s = 1.5 * rm
    out = []
    # bound oscillation, six periapses
    y = np.zeros(12)
    y[2] = r_s
    E_rel = V(r_s)
    r_in = brentq(lambda r: V(r) - E_rel, 0.5 * rm, rm, xtol=1e-14, rtol=1e-15)
    out.append(("oscillation", y, 5.87 * period(E_rel, r_in, r_s)))
    for frac in (0.98, 1.02):
        u = math.sqrt(2 * frac * abs(E_rel) / mu)
        y = np.zeros(12)
        y[2] = r_s
        y[11] = -u
        out.append((f"relative energy {frac - 1:+.0%} |V|", y, 0.1 * s.t_max if frac > 1 else 4 * period(E_rel, r_in, r_s)))
    v0 = math.sqrt(2 * W.kelvin(1.5e-6) / m_a)
    y = np.zeros(12)
    n = np.array([math.sin(0.7) * math.cos(0.3), math.sin(0.7) * math.sin(0.3), math.cos(0.7)])
    y[0:3], y[6:9] = s.r0 * n, -v0 * n
    out.append(("head-on scattering", y, s.t_max))
    return s, sp, out


def test_bounces_and_bound_state_match_the_oracle_on_closed_form_starts():
    s, sp, cases = _cases()
    for name, y0, t_max in cases:
        s.t_max = t_max
        print(f"case: {name}", flush=True)
        got = PT.to_numpy(api.integrate(s, [sp], W.Generator(kind="arrays"), 1,
                                        y0=torch.from_numpy(y0.reshape(12, 1)).to("cuda"), y_final=True))
        p = oracle.base_problem(s, sp)
        p["y0"] = y0
        r = oracle.integrate_one(p)
        print(f"{name}: gpu n_bounce {got['n_bounce'][0]} status {int(got['status'][0]):#x} "
              f"t_first {got['t_bounce_first'][0]:.12e} t_last {got['t_bounce_last'][0]:.12e}; oracle "
              f"{r['n_bounce']} {int(r['status']):#x} {r['t_first']:.12e} {r['t_last']:.12e}", flush=True)
        assert got["n_bounce"][0] == r["n_bounce"]
        assert int(got["status"][0]) & 0xFFFF == int(r["status"])
        assert got["n_accept"][0] == r["n_accept"] and got["n_reject"][0] == r["n_reject"]
        P = np.array([p])
        runs = [oracle.integrate(P, twin=True)[0]]
        for sg in PT.PROBE_SIGNS:
            q = P.copy()
            q["y0"][:, 0:3] *= 1.0 + sg * 2.0 ** -52
            runs.append(oracle.integrate(q)[0])
        for gk, rk in (("t_bounce_first", "t_first"), ("t_bounce_last", "t_last")):
            spread = max(abs(x[rk] - r[rk]) for x in runs)
            bar = max(1e-12 * abs(r[rk]), 10.0 * spread)
            print(f"{name}: {gk} |gpu - oracle| / |oracle| = {abs(got[gk][0] - r[rk]) / max(abs(r[rk]), 1e-300):.2e}, "
                  f"spread {spread / max(abs(r[rk]), 1e-300):.2e}", flush=True)
            assert abs(got[gk][0] - r[rk]) <= bar, (name, gk)
            assert bar <= 1e-6 * abs(r[rk]), (name, gk)        # the bar stays meaningful
    # the cases cover what they are meant to: six bounces bound, the bit both ways
    assert [c[0] for c in cases][0] == "oscillation"
