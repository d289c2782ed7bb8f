"""Seeded synthetic workloads: physical constants, species data and batch descriptions.

This module only describes inputs.  It holds none of the method's arithmetic (no
equations of motion, no integrator, no initial-condition geometry, no random
draws): both the CPU oracle and the HIP library receive these numbers and each
turns them into trajectories with its own code.

Units are atomic units throughout (a0, m_e, E_h, hbar/E_h); the helpers below
convert the laboratory quantities quoted in the paper (amu, kelvin, seconds, Hz).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

# CODATA 2018 conversion factors.
AMU_IN_ME = 1822.888486209          # unified atomic mass unit / electron mass
KELVIN_IN_EH = 3.1668115634556e-6   # k_B * 1 K / E_h
AU_TIME_IN_S = 2.4188843265857e-17  # hbar / E_h in seconds


def amu(m: float) -> float:
    return m * AMU_IN_ME


def kelvin(T: float) -> float:
    return T * KELVIN_IN_EH


def seconds(t: float) -> float:
    return t / AU_TIME_IN_S


def angular_hz(f: float) -> float:
    """2*pi*f expressed in inverse atomic time units."""
    return 2.0 * math.pi * f * AU_TIME_IN_S


# Species: (isotopic mass in amu, static dipole polarizability in a.u.).  Rb and the
# Yb+ ion mass are the values the workloads quote; the others are isotopic masses
# and the commonly tabulated static polarizabilities of the neutral atoms.
SPECIES = {
    "Li6": (6.0151229, 164.11),
    "Na23": (22.989769, 162.7),
    "K40": (39.963998, 289.7),
    "Rb87": (86.91, 319.0),
    "Cs133": (132.905452, 400.9),
}
SPECIES_ORDER = ["Li6", "Na23", "K40", "Rb87", "Cs133"]
YB174_ION_AMU = 173.94

RING = ((1.0, 1.0, -2.0), (1.0, 1.0, -2.0))     # (a ratios, q ratios): a_z=-2a_x, q_y=q_x, q_z=-2q_x
LINEAR = ((1.0, 1.0, -2.0), (1.0, -1.0, 0.0))   # q_y=-q_x, no RF along z


def species_table(names: List[str]):
    """[(m_atom in m_e, C4 = alpha/2 in a.u.)] for the given species names."""
    out = []
    for nm in names:
        m, alpha = SPECIES[nm]
        out.append((amu(m), 0.5 * alpha))
    return out


@dataclass
class System:
    """Trap, defaults and integrator settings shared by a whole batch (atomic units)."""
    m_ion: float = amu(YB174_ION_AMU)
    omega_rf: float = angular_hz(2.0e6)
    a_x: float = 0.0
    q_x: float = 0.2
    a_ratio: tuple = RING[0]
    q_ratio: tuple = RING[1]
    E: float = kelvin(1.5e-6)        # default collision energy
    De: float = kelvin(1.0)          # default well depth
    phase0: float = 0.0              # default RF phase at t = 0
    species: int = 0                 # default index into the species table
    r0: float = 5000.0
    t_max: float = seconds(10e-3)
    rtol: float = 1e-10
    atol: float = 1e-12
    h0: float = 0.0                  # 0 -> library default (internal time units)
    hmax: float = 0.0
    hmin: float = 0.0
    r_bounce_over_rm: float = 1.0
    # accepted-step cap (a numerical safety stop, status MAX_STEPS), given to the oracle and the
    # library alike: complexes in the deepest wells can take ~1e8 steps to reach t_max
    max_steps: int = 20_000_000


@dataclass
class Generator:
    """How trajectory ids map to per-trajectory parameters.

    kind = "grid":  cell-centred (theta, phi) grid on the octant, id = j*n_phi + k.
    kind = "sweep": counter-based random draws keyed by (seed, id): direction uniform
                    on the sphere, RF phase uniform; E, q, De either from lists (cell
                    digits of id mod the product of list lengths) or from ranges.
    kind = "thermal": as "sweep" for species, q, De, RF phase and the start point, with E the bath
                    energy k_B T; atom velocity Gaussian at T (turned inward), ion Gaussian at T_ion
                    in the isotropic trap omega = q Omega / 2^(3/2) (thermal runs of Fig. 3).
    kind = "arrays": explicit per-trajectory arrays supplied by the caller.
    """
    kind: str = "grid"
    n_theta: int = 8
    n_phi: int = 8
    seed: int = 0
    id0: int = 0
    species: List[int] = field(default_factory=lambda: [0])
    E_list: List[float] = field(default_factory=list)
    q_list: List[float] = field(default_factory=list)
    De_list: List[float] = field(default_factory=list)
    E_range: Optional[tuple] = None     # log-uniform
    T_ion: float = 10e-6                # kind = "thermal": ion temperature (K)
    q_range: Optional[tuple] = None     # uniform
    De_range: Optional[tuple] = None    # log-uniform


@dataclass
class Workload:
    name: str
    n: int
    system: System
    species_names: List[str]
    gen: Generator

    def species(self):
        return species_table(self.species_names)

    def with_n(self, n: int) -> "Workload":
        return replace(self, n=n)


SEED_BASE = 250915117000


def headon_grid(n_side: int, name: str) -> Workload:
    return Workload(name=name, n=n_side * n_side, system=System(), species_names=["Rb87"],
                    gen=Generator(kind="grid", n_theta=n_side, n_phi=n_side))


def config1() -> Workload:
    """Yb+ + Rb, 8x8 octant grid, D_e = 1 K, E = 1.5 uK, q = 0.2, r0 = 5000 a0."""
    return headon_grid(8, "yb_rb_headon_grid_8x8")


def config2() -> Workload:
    """The same system on a 1024x1024 octant grid (1,048,576 trajectories)."""
    return headon_grid(1024, "yb_rb_headon_grid_1024x1024")


def config3() -> Workload:
    """1.2e7-trajectory uneven sweep over 5 species x 5 E x 3 q x 3 De cells."""
    sys_ = System(phase0=0.0)
    gen = Generator(kind="sweep", seed=SEED_BASE + 3, species=[0, 1, 2, 3, 4],
                    E_list=[kelvin(x * 1e-6) for x in (1, 3, 10, 30, 100)],
                    q_list=[0.1, 0.2, 0.3],
                    De_list=[kelvin(x) for x in (0.1, 1.0, 10.0)])
    return Workload(name="sweep_5species_225cells", n=12_000_000, system=sys_,
                    species_names=list(SPECIES_ORDER), gen=gen)


def config4() -> Workload:
    """Differentiation workload: Yb+ + Rb on a 512x512 octant grid."""
    return headon_grid(512, "yb_rb_headon_grid_512x512_tangent")


def config5() -> Workload:
    """1e8-trajectory streaming sweep: Li6, K40, Cs133; E, q, De from ranges."""
    gen = Generator(kind="sweep", seed=SEED_BASE + 5, species=[0, 1, 2],
                    E_range=(kelvin(1e-6), kelvin(1e-3)), q_range=(0.05, 0.35),
                    De_range=(kelvin(0.01), kelvin(100.0)))
    return Workload(name="stream_li_k_cs_1e8", n=100_000_000, system=System(),
                    species_names=["Li6", "K40", "Cs133"], gen=gen)


def fig2_survival() -> Workload:
    """Complex lifetimes (Fig. 2): head-on collisions of the five atoms with Yb+ from random directions
    and RF phases, E = 1.5 uK, q = 0.2, D_e = 1 K; species = id mod 5."""
    gen = Generator(kind="sweep", seed=SEED_BASE + 12, species=[0, 1, 2, 3, 4], E_list=[kelvin(1.5e-6)],
                    q_list=[0.2], De_list=[kelvin(1.0)])
    return Workload(name="fig2_survival_5species", n=100_000, system=System(), species_names=list(SPECIES_ORDER),
                    gen=gen)


def fig3_thermal() -> Workload:
    """Thermal runs (Fig. 3): the five atoms with Yb+, bath at 1, 10 and 100 uK, ion at 10 uK,
    q = 0.2, D_e = 1 and 100 K, uniform RF phase; cell = id mod 30 (species slowest)."""
    gen = Generator(kind="thermal", seed=SEED_BASE + 13, species=[0, 1, 2, 3, 4],
                    E_list=[kelvin(x * 1e-6) for x in (1.0, 10.0, 100.0)], q_list=[0.2],
                    De_list=[kelvin(1.0), kelvin(100.0)], T_ion=10e-6)
    return Workload(name="fig3_thermal_5species", n=3_000_000, system=System(), species_names=list(SPECIES_ORDER),
                    gen=gen)


def fig4_energy(species=(0, 1, 2, 3, 4)) -> Workload:
    """Collision-energy sweep (Fig. 4): head-on collisions of each atom with Yb+ from r0 = 20,000 a0,
    q_x = 0.2, D_e = 1 K, random direction and RF phase, collision energy log-uniform over
    0.1 uK - 1 mK (the paper takes 100 fixed energies; a continuous draw binned on the device in
    log10(E / W0) is the same measurement on the axis of the threshold claim).  10^6 trajectories
    per species."""
    sys_ = System(r0=20_000.0)
    gen = Generator(kind="sweep", seed=SEED_BASE + 14, species=list(species),
                    E_range=(kelvin(0.1e-6), kelvin(1e-3)), q_list=[0.2], De_list=[kelvin(1.0)])
    return Workload(name=f"fig4_energy_sweep_{len(species)}species", n=1_000_000 * len(species),
                    system=sys_, species_names=list(SPECIES_ORDER), gen=gen)


def fig4_inset() -> Workload:
    """Fig. 4 inset: Yb+ - Li head-on at q_x = 0.1, 0.2, 0.3, 0.4 (Omega fixed) and eight collision
    energies 0.1 - 2 uK, r0 = 20,000 a0, D_e = 1 K, random direction and RF phase; 32 cells,
    10^4 trajectories each (cell = id mod 32, energy digit before q)."""
    sys_ = System(r0=20_000.0)
    gen = Generator(kind="sweep", seed=SEED_BASE + 15, species=[0],
                    E_list=[kelvin(x * 1e-6) for x in (0.1, 0.2, 0.3, 0.5, 0.7, 1.0, 1.5, 2.0)],
                    q_list=[0.1, 0.2, 0.3, 0.4], De_list=[kelvin(1.0)])
    return Workload(name="fig4_inset_li_4q_8E", n=320_000, system=sys_, species_names=list(SPECIES_ORDER),
                    gen=gen)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
