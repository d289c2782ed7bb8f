"""Tangent and adjoint on a ragged slice of the 225-cell sweep: five species, three q_x, three well
depths and random directions and RF phases, so every parameter column (q_x and D_e forcing, the
species' masses and C4) is exercised, not only the Yb+-Rb grid.

* The GPU tangent lies within max(1e-9, 10 x spread) of the oracle's on the direct trajectories,
  spread = the oracle's own five-probe round-off spread (as for the grid).
* The GPU adjoint equals the GPU tangent's contraction within 1e-7 of the contributing terms.
"""
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

from paper_2509_15117_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)
N, ID0 = 96, 5003


def _setup():
    w = W.config3()
    w.system.max_steps = 2_000_000
    P = oracle.problems_for(w, range(ID0, ID0 + N))
    draws = [oracle.sweep_draw(i, w.gen) for i in range(ID0, ID0 + N)]
    return w, P, draws


def _scales(d):
    return np.array([1.0, 1.0, d["E"], d["q_x"], d["De"]])


def test_sweep_tangent_matches_oracle_on_direct_trajectories():
    w, P, draws = _setup()
    print(f"sweep tangent: n={N}, id0={ID0}", flush=True)
    out = PT.to_numpy(api.tangent(w.system, w.species(), w.gen, N, id0=ID0))
    ref = oracle.integrate(P)
    checked = 0
    for j in range(N):
        if not (ref[j]["n_bounce"] <= 1 and out["n_bounce"][j] <= 1 and ref[j]["status"] & oracle.EXITED):
            continue
        d = draws[j]
        th = math.acos(d["cos_theta"])
        qr = w.system.q_ratio
        g_or, _, _ = oracle.tangent(P[j], th, d["phi"], d["E"], qr)
        runs = [oracle.tangent(P[j], th, d["phi"], d["E"], qr, twin=True)]
        for sg in PT.PROBE_SIGNS:
            q = P[j].copy()
            q["y0"][0:3] *= 1.0 + sg * 2.0 ** -52
            runs.append(oracle.tangent(q, th, d["phi"], d["E"], qr))
        s = _scales(d)
        for k in range(3):
            b = g_or[k] * s
            if not np.all(np.isfinite(b)) or np.linalg.norm(b) == 0.0:
                continue
            spread = max(np.linalg.norm((r[0][k] - g_or[k]) * s) for r in runs)
            a = out["dobs_dp"][j][k] * s
            assert np.linalg.norm(a - b) <= max(1e-9 * np.linalg.norm(b), 10.0 * spread), (ID0 + j, k, a, b)
        checked += 1
    print(f"sweep tangent: {checked} direct trajectories checked", flush=True)
    assert checked >= 20


def _dy0(theta, phi, E, m, r0):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    n = np.array([st * cp, st * sp, ct])
    nt = np.array([ct * cp, ct * sp, -st])
    nph = np.array([-st * sp, st * cp, 0.0])
    v0 = np.sqrt(2.0 * E / m)
    d = np.zeros((3, 12))
    d[0, :3], d[0, 6:9] = r0 * nt, -v0 * nt
    d[1, :3], d[1, 6:9] = r0 * nph, -v0 * nph
    d[2, 6:9] = -v0 / (2.0 * E) * n
    return d


def test_sweep_adjoint_equals_tangent_contraction():
    w, P, draws = _setup()
    obs = api.integrate_workload(w, n=N, id0=ID0, counters=True)
    g = torch.from_numpy(np.random.default_rng(11).normal(size=(N, 3))).to(DEV)
    print(f"sweep adjoint: n={N}, id0={ID0}", flush=True)
    pb, yb = api.adjoint(w.system, w.species(), w.gen, N, obs, g, id0=ID0, y0_bar=True)
    tan = PT.to_numpy(api.tangent(w.system, w.species(), w.gen, N, id0=ID0))
    pb, yb, gn = pb.cpu().numpy(), yb.cpu().numpy(), g.cpu().numpy()
    ref = np.einsum("ik,ikp->ip", gn, tan["dobs_dp"])
    nb = obs["n_bounce"].cpu().numpy()
    spc = w.species()
    checked = 0
    for j in range(N):
        if nb[j] > 1 or not (np.all(np.isfinite(pb[j])) and np.all(np.isfinite(ref[j]))):
            continue
        d = draws[j]
        s = _scales(d)
        T = np.abs(ref[j] * s)
        T[:3] += np.abs(_dy0(math.acos(d["cos_theta"]), d["phi"], d["E"], spc[d["species"]][0], w.system.r0)
                        * yb[j][None, :]).sum(1) * s[:3]
        bar = 1e-7 * T + 1e-12 * np.linalg.norm(ref[j] * s)
        assert np.all(np.abs(pb[j] - ref[j]) * s <= bar), (ID0 + j, pb[j] * s, ref[j] * s, bar)
        checked += 1
    print(f"sweep adjoint: {checked} direct trajectories checked", flush=True)
    assert checked >= 20
