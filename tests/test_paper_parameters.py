"""The workloads against the parameters the paper prints (tests/golden/paper_parameters.json, each
entry citing its passage): the head-on runs of Figs. 1 and 2, the thermal runs of Fig. 3, the
energy sweep of Fig. 4, the model constants and the Eq. (2) scale."""
import json
import math
import os

import numpy as np

import oracle
import workloads as W
from oracle import reduce as R

G = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_parameters.json")))


def test_headon_runs_use_the_fig1_and_fig2_parameters():
    for key, w in (("headon_fig1", W.config1()), ("headon_fig1", W.config2()), ("lifetimes_fig2", W.fig2_survival())):
        g = G[key]
        assert w.system.r0 == g["r0_a0"]
        E = w.system.E if w.gen.kind == "grid" else w.gen.E_list[0]
        assert math.isclose(E, W.kelvin(g["E_uK"] * 1e-6), rel_tol=1e-15)
        De = w.system.De if w.gen.kind == "grid" else w.gen.De_list[0]
        assert math.isclose(De, W.kelvin(g["De_K"]), rel_tol=1e-15)
    assert W.config1().species_names[W.config1().system.species] == G["headon_fig1"]["atom"]


def test_thermal_runs_use_the_fig3_parameters():
    g = G["thermal_fig3"]
    w = W.fig3_thermal()
    assert w.system.r0 == g["r0_a0"] and w.gen.kind == "thermal"
    assert math.isclose(w.gen.T_ion, g["T_ion_uK"] * 1e-6, rel_tol=1e-15)
    assert sorted(w.gen.De_list) == [W.kelvin(x) for x in g["De_K"]]
    # the ion's trap frequency of the thermal draw: omega = q_x Omega / 2^(3/2)
    d = oracle.sweep_draw(0, w.gen)
    y = oracle.thermal_state(w.system, w.gen, d, w.species()[d["species"]][0], 0)
    z = oracle.thermal_normals(0, w.gen.seed)
    omega = g["omega_over_qx_Omega"] * d["q_x"] * w.system.omega_rf
    sv = math.sqrt(w.gen.T_ion * oracle.K_IN_EH / w.system.m_ion)
    np.testing.assert_allclose(y[3:6], sv / omega * z[3:6], rtol=1e-14)


def test_energy_sweep_uses_the_fig4_parameters():
    g = G["energy_sweep_fig4"]
    w = W.fig4_energy()
    assert w.system.r0 == g["r0_a0"] and w.gen.De_list == [W.kelvin(g["De_K"])]
    assert w.gen.kind == "sweep"          # random direction and RF phase per trajectory
    inset = W.fig4_inset()
    assert len(inset.gen.q_list) == g["inset_qx_values"] and inset.species_names[inset.gen.species[0]] == g["inset_atom"]
    assert inset.system.r0 == g["r0_a0"]
    # Fig. 4 runs 10^4 head-on collisions at each of 100 energies per species; the inset 10^4 per cell
    assert w.n == g["headon_per_energy"] * g["energies_per_species"] * len(w.gen.species)
    n_cells = len(inset.gen.q_list) * len(inset.gen.E_list)
    assert inset.n == g["headon_per_energy"] * n_cells
    # 1 uK bath <-> 1.5 uK collision energy through m v0^2 / 2 = 3 k_B T / 2
    assert math.isclose(W.kelvin(1e-6) * g["E_of_T"], W.kelvin(1.5e-6), rel_tol=1e-15)


def test_model_constants_and_eq2():
    g = G["model"]
    m, C4 = W.species_table(["Rb87"])[0]
    assert math.isclose(C4, g["C4_over_alpha"] * W.SPECIES["Rb87"][1], rel_tol=1e-15)
    e = G["eq2"]
    assert math.isclose(e["prefactor"], 8.0 / (3.0 * math.pi), rel_tol=1e-15)
    # the oracle's Eq. (2) has the printed prefactor and mass-ratio power: heavy-atom limit and scaling
    s = W.System()
    w0 = R.w0_eq2(m, s.m_ion, C4, s.omega_rf, 0.0, 0.2)
    om = 0.5 * s.omega_rf * math.sqrt(0.5 * 0.2 ** 2)
    ref = e["prefactor"] * (m / (s.m_ion + m)) ** e["mass_ratio_power"] * (s.m_ion ** 2 * om ** 4 * C4 / 0.2 ** 2) ** (1 / 3)
    assert math.isclose(float(w0), ref, rel_tol=1e-12)
