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


def test_tangent_matches_oracle_tangent_on_direct_trajectories():
    w = W.config1()
    out = PT.to_numpy(api.tangent(w.system, w.species(), w.gen, 64, phi=True))
    P = oracle.problems_for(w, range(64))
    ref = oracle.integrate(P)
    th_ph = oracle.grid_angles(range(64), 8, 8)
    s = _scales(w)
    for gid in DIRECT:
        assert ref[gid]["n_bounce"] == 1 and out["n_bounce"][gid] == 1
        d, Phi, _ = oracle.tangent(P[gid], th_ph[gid][0], th_ph[gid][1], w.system.E, w.system.q_ratio)
        g = out["dobs_dp"][gid]
        for k in range(3):
            a, b = g[k] * s, d[k] * s
            assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b), (gid, k, a, b)
        Pg = out["Phi"][gid]
        assert np.abs(Pg - Phi).max() <= 1e-6 * np.abs(Phi).max(), gid
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
