"""Pins of the oracle's thermal-run start (Fig. 3 text and caption) and of its exit sphere.

* The nine normals of a trajectory are Box-Muller pairs of the Philox4x64-10 blocks
  (id, 2..4, 0, 0): checked against numpy's Philox and numpy's own Box-Muller arithmetic, and,
  pooled over many ids, against the standard normal (Kolmogorov-Smirnov, moments, correlations).
* The start states: the atom on the r0 sphere about the trap centre, moving inward, with each
  velocity component's variance k_B T / m_a and a half-normal radial component; the ion with the
  equipartition variances of the isotropic trap omega = q_x Omega / 2^(3/2) (k_B T_ion / (m_i
  omega^2) per position component, k_B T_ion / m_i per velocity component); the direction
  uniform on the sphere.
* The exit: with the interaction switched off the atom flies straight through the sphere about the
  trap centre and leaves it after the chord time -2 (x0 . v) / |v|^2, wherever the ion is; the
  separation test of head-on runs would miss a grazing atom whose separation from the displaced
  ion starts above r0, which is why thermal runs use the centre sphere.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W

oracle.build()


def _philox_block(gid, word1, seed):
    """numpy's Philox4x64-10 block at counter (gid, word1, 0, 0), key (seed, 0)."""
    # numpy increments the 256-bit counter before each block: start one below
    c0, c1 = gid - 1, word1
    if gid == 0:
        c0, c1 = 2 ** 64 - 1, word1 - 1
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                          counter=np.array([c0, c1, 0, 0], dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("gid", [0, 1, 29, 30, 123_456_789])
def test_thermal_normals_are_box_muller_of_the_philox_blocks(gid):
    seed = W.fig3_thermal().gen.seed
    u = np.concatenate([(_philox_block(gid, 2 + b, seed) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
                        for b in range(3)])
    ref = []
    for m in range(5):
        r = np.sqrt(-2.0 * np.log1p(-u[2 * m]))
        ref += [r * np.cos(2.0 * np.pi * u[2 * m + 1]), r * np.sin(2.0 * np.pi * u[2 * m + 1])]
    z = oracle.thermal_normals(gid, seed)
    assert z.shape == (9,)
    np.testing.assert_allclose(z, ref[:9], rtol=1e-13, atol=1e-15)


def test_thermal_normals_are_standard_normal():
    n = 40_000
    Z = np.array([oracle.thermal_normals(i, 777) for i in range(n)])
    for k in range(9):
        assert stats.kstest(Z[:, k], "norm").pvalue > 1e-4, k
    assert np.all(np.abs(Z.mean(0)) < 5.0 / math.sqrt(n))
    assert np.all(np.abs(Z.var(0) - 1.0) < 5.0 * math.sqrt(2.0 / n))
    C = np.corrcoef(Z.T)
    assert np.all(np.abs(C[~np.eye(9, dtype=bool)]) < 5.0 / math.sqrt(n))


@pytest.fixture(scope="module")
def thermal_batch():
    w = W.fig3_thermal()
    n = 6000
    P = oracle.problems_for(w, range(n))
    draws = [oracle.sweep_draw(i, w.gen) for i in range(n)]
    return w, P, draws


def test_thermal_atom_starts_on_the_centre_sphere_moving_inward(thermal_batch):
    w, P, draws = thermal_batch
    y = P["y0"]
    r = np.linalg.norm(y[:, 0:3], axis=1)
    np.testing.assert_allclose(r, w.system.r0, rtol=1e-15)
    n = y[:, 0:3] / r[:, None]
    vr = np.einsum("ij,ij->i", n, y[:, 6:9])
    assert np.all(vr < 0.0)
    assert np.all(P["exit_centre"] == 1)
    # direction uniform on the sphere
    N = len(r)
    assert np.all(np.abs(n.mean(0)) < 5.0 / math.sqrt(3.0 * N))
    assert abs((n[:, 2] ** 2).mean() - 1.0 / 3.0) < 5.0 * math.sqrt(4.0 / 45.0 / N)
    # velocity components ~ N(0, k_B T / m_a) before the inward flip: the flip keeps the squares,
    # and the radial component is minus a half-normal
    m = P["m_atom"]
    T = np.array([d["E"] for d in draws])
    s2 = T / m
    zz = y[:, 6:9] ** 2 / s2[:, None]
    assert abs(zz.mean() - 1.0) < 5.0 * math.sqrt(2.0 / zz.size)
    zr = vr / np.sqrt(s2)
    assert abs(zr.mean() + math.sqrt(2.0 / math.pi)) < 5.0 * math.sqrt((1.0 - 2.0 / math.pi) / N)
    # tangential part: mean zero
    vt = y[:, 6:9] - vr[:, None] * n
    assert np.all(np.abs((vt / np.sqrt(s2)[:, None]).mean(0)) < 5.0 / math.sqrt(N))


def test_thermal_ion_has_the_equipartition_variances_of_the_isotropic_trap(thermal_batch):
    w, P, draws = thermal_batch
    y = P["y0"]
    kT = w.gen.T_ion * oracle.K_IN_EH
    q = np.array([d["q_x"] for d in draws])
    omega = q * w.system.omega_rf / 2.0 ** 1.5
    zx = y[:, 3:6] * (omega * np.sqrt(w.system.m_ion / kT))[:, None]
    zv = y[:, 9:12] * math.sqrt(w.system.m_ion / kT)
    for z in (zx, zv):
        assert np.all(np.abs(z.mean(0)) < 5.0 / math.sqrt(len(z)))
        assert np.all(np.abs(z.var(0) - 1.0) < 5.0 * math.sqrt(2.0 / len(z)))
    # 10 uK in a 2 MHz trap at q = 0.2 spreads the ion over a few hundred bohr
    assert 200.0 < np.sqrt(np.mean(y[:, 3:6] ** 2)) < 800.0


def _free_flight(exit_centre, ion_x, t_max_factor=3.0):
    """Atom at r0 z_hat moving nearly tangentially, interaction (C4 -> 0) and trap (a = q = 0)
    off, so the ion stays at rest at (ion_x, 0, 0).  Returns the problem and the chord time."""
    w = W.fig3_thermal()
    p = oracle.base_problem(w.system, (W.species_table(["Rb87"])[0][0], 1e-12), qx=0.2, De=W.kelvin(1.0))
    r0 = w.system.r0
    v0 = 2e-9
    v = v0 * np.array([1.0, 0.0, -0.05]) / math.sqrt(1.0 + 0.05 ** 2)
    p["y0"][:] = 0.0
    p["y0"][2] = r0
    p["y0"][6:9] = v
    p["y0"][3] = ion_x
    p["a"] = 0.0
    p["q"] = 0.0
    t_chord = -2.0 * (p["y0"][0:3] @ v) / (v @ v)
    p["t_max"] = t_max_factor * t_chord
    p["exit_centre"] = exit_centre
    return p, t_chord


def test_thermal_exit_is_the_chord_through_the_centre_sphere():
    for ion_x in (0.0, -600.0, 600.0):
        p, t_chord = _free_flight(1, ion_x)
        r = oracle.integrate_one(p)
        assert r["status"] & oracle.EXITED and r["n_bounce"] == 0, (ion_x, r["status"])
        assert abs(r["t_dwell"] - t_chord) < 1e-9 * t_chord, (ion_x, r["t_dwell"], t_chord)
        yf = r["y_final"]
        np.testing.assert_allclose(yf[0:3], p["y0"][0:3] + p["y0"][6:9] * r["t_dwell"], rtol=0, atol=1e-6)
        assert abs(np.linalg.norm(yf[0:3]) - p["r0"]) < 1e-9 * p["r0"]
        assert r["angle"] < 1e-12 and r["q_transfer"] < 1e-12 * p["m_atom"] * 2e-9


def test_separation_exit_misses_a_grazing_atom_when_the_ion_is_displaced():
    # ion 600 bohr away from the atom's side: the separation starts and stays above r0
    p, t_chord = _free_flight(0, -600.0)
    r = oracle.integrate_one(p)
    assert r["status"] & oracle.TMAX and not r["status"] & oracle.EXITED
    # with the ion at the centre both exits agree
    a = oracle.integrate_one(_free_flight(0, 0.0)[0])
    b = oracle.integrate_one(_free_flight(1, 0.0)[0])
    assert a["status"] & oracle.EXITED and b["status"] & oracle.EXITED
    assert abs(a["t_dwell"] - b["t_dwell"]) < 1e-9 * t_chord


def test_tangent_oracle_rejects_thermal_problems():
    p, _ = _free_flight(1, 0.0)
    with pytest.raises(Exception):
        oracle.tangent(p, 0.1, 0.2, 1e-12, (1.0, 1.0, -2.0))
