"""GPU tangent-linear (iat_integrate_tangent) against the oracle's internal differentiation."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import _parity as PT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402

DIRECT = [40, 41, 47, 51, 55, 58, 63]


def _scales(w):
    return np.array([1.0, 1.0, w.system.E, w.system.q_x, w.system.De])


def tangent_spread(p, th, ph, w):
    """Round-off spread of the oracle's tangent for one trajectory: the worst difference, per
    observable (norm of the parameter-scaled gradient) and for Phi (max entry), between the oracle
    and five round-off probes of it (the FMA twin build and +-1 ulp in theta and phi).  The tangent
    is far worse conditioned than the final state: a collision that stretches phase space by 10^3
    turns a round-off shift of the trajectory into a relative change of Phi near 1e-6."""
    s = _scales(w)
    d, Phi, _ = oracle.tangent(p, th, ph, w.system.E, w.system.q_ratio)
    runs = PT.tangent_runs(p, th, ph, w.system.E, w.system.q_ratio)
    sd = np.zeros(3)
    sp = 0.0
    for d2, P2, _ in runs:
        for k in range(3):
            sd[k] = max(sd[k], np.linalg.norm((d2[k] - d[k]) * s))
        sp = max(sp, np.abs(P2 - Phi).max())
    return d, Phi, sd, sp


def test_tangent_matches_oracle_tangent_on_direct_trajectories():
    """Per direct trajectory: each observable's scaled gradient within max(1e-9 |g|, 10 x spread) of the
    oracle's, and Phi within max(1e-9 max|Phi|, 10 x spread) entrywise."""
    w = W.config1()
    out = PT.to_numpy(api.tangent(w.system, w.species(), w.gen, 64, phi=True))
    P = oracle.problems_for(w, range(64))
    ref = oracle.integrate(P)
    th_ph = oracle.grid_angles(range(64), 8, 8)
    s = _scales(w)
    for gid in DIRECT:
        assert ref[gid]["n_bounce"] == 1 and out["n_bounce"][gid] == 1
        d, Phi, sd, sp = tangent_spread(P[gid], th_ph[gid][0], th_ph[gid][1], w)
        g = out["dobs_dp"][gid]
        for k in range(3):
            a, b = g[k] * s, d[k] * s
            err = np.linalg.norm(a - b)
            bar = max(1e-9 * np.linalg.norm(b), 10.0 * sd[k])
            print(f"gid {gid} obs {k}: |dg|/|g| = {err / np.linalg.norm(b):.2e}, "
                  f"spread {sd[k] / np.linalg.norm(b):.2e}", flush=True)
            assert err <= bar, (gid, k, a, b, sd[k])
            assert bar <= 5e-4 * np.linalg.norm(b)      # the bar itself stays meaningful
        Pg = out["Phi"][gid]
        err = np.abs(Pg - Phi).max()
        assert err <= max(1e-9 * np.abs(Phi).max(), 10.0 * sp), (gid, err, sp)
    # the observables of the tangent run are those of iat_integrate
    plain = PT.to_numpy(api.integrate_workload(w, kernel="plain", y_final=True))
    for k in ("angle", "q_transfer", "dE_ion", "t_dwell", "n_bounce", "status"):
        assert np.array_equal(out[k], plain[k]), k


def test_stability_matrix_symplectic_and_ftle_consistent():
    w = W.config1()
    out = PT.to_numpy(api.tangent(w.system, w.species(), w.gen, 64, phi=True))
    sp = w.species()[0]
    M = np.diag([sp[0]] * 3 + [w.system.m_ion] * 3)
    Om = np.block([[np.zeros((6, 6)), M], [-M, np.zeros((6, 6))]])
    for gid in DIRECT:
        Phi = out["Phi"][gid]
        defect = Phi.T @ Om @ Phi - Om
        assert (np.abs(defect) / (np.abs(Phi.T) @ np.abs(Om) @ np.abs(Phi))).max() < 1e-7
        smax = np.linalg.svd(Phi, compute_uv=False)[0]
        assert abs(out["ftle"][gid] - np.log(smax) / out["t_dwell"][gid]) <= 1e-10 * abs(out["ftle"][gid])
    assert np.all(np.isfinite(out["ftle"])) and np.all(out["ftle"] > 0)


def test_lyapunov_spectrum_matches_oracle_and_pairs():
    """The finite-time Lyapunov spectrum of the canonically scaled stability matrix: per direct
    trajectory of the 8x8 grid, every exponent whose singular value is resolvable (s_k^2 above
    1e-12 s_max^2) equals the oracle's (numpy SVD of the oracle's Phi) in ln s_k within
    max(12e-9 s_max / s_k, 10 x the spread of the oracle's five round-off probes): the first term is
    the Phi test's entrywise bar (1e-9 max|Phi|) carried to s_k by Weyl's inequality
    (|d s_k| <= ||d Phi||_2 <= 12 max|d Phi_ij|).  Pairs whose smaller member is resolvable sum to
    zero within 2e-4 in ln(s s') (the Dormand-Prince map is symplectic up to its truncation error);
    below s_max * 1e-6 the normal matrix the library diagonalises holds the small singular values
    only to rounding, and their pairs are the reliable values."""
    w = W.config1()
    out = PT.to_numpy(api.tangent(w.system, w.species(), w.gen, 64, lyap=True))
    P = oracle.problems_for(w, range(64))
    ref = oracle.integrate(P)
    th_ph = oracle.grid_angles(range(64), 8, 8)
    m_a, m_i = P[0]["m_atom"], P[0]["m_ion"]
    for gid in DIRECT:
        t_f = ref[gid]["t_dwell"]
        lam = out["lyap"][gid]
        assert np.all(np.isfinite(lam)) and np.all(np.diff(lam) <= 0)
        _, Phi, _, _ = tangent_spread(P[gid], th_ph[gid][0], th_ph[gid][1], w)
        lo = oracle.lyapunov_spectrum(Phi, m_a, m_i, t_f)
        # the probes' spread of the oracle's spectrum, in ln s
        spread = np.zeros(12)
        q_runs = PT.tangent_runs(P[gid], th_ph[gid][0], th_ph[gid][1], w.system.E, w.system.q_ratio)
        for _, P2, _ in q_runs:
            spread = np.maximum(spread, np.abs(oracle.lyapunov_spectrum(P2, m_a, m_i, t_f) - lo) * t_f)
        ok = (lo - lo[0]) * t_f > 0.5 * np.log(1e-12)
        err = np.abs(lam - lo) * t_f
        bar = np.maximum(12e-9 * np.exp((lo[0] - lo) * t_f), 10.0 * spread)
        print(f"id {gid}: s_max {np.exp(lo[0] * t_f):.2e}, worst |ln s_gpu - ln s_oracle| {err[ok].max():.1e} "
              f"(bar {bar[ok].min():.1e}..{bar[ok].max():.1e}), resolvable pairs "
              f"{np.abs((lam + lam[::-1]) * t_f)[ok & ok[::-1]].max():.1e}",
              flush=True)
        assert np.all(err[ok] <= bar[ok]), (gid, err, bar)
        # pairs whose smaller member is resolvable through the normal matrix (s^2 above 1e-12 s_max^2)
        both = ok & ok[::-1]
        assert both.sum() >= 6 and np.abs((lam + lam[::-1]) * t_f)[both].max() < 2e-4
