"""Plain reductions of a batch's observables (the ensemble figures of the paper): per-cell sums,
complex-formation histograms over log10(E / W0), the heating histogram, and box counting of the
complex-forming set.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle): used by the tests and the smoke check.  Every
function is the definition written out with numpy; nothing is blocked or reordered.

Readings fixed here (the paper draws these quantities but does not give binning details):
* cells: cell = id mod (number of sweep cells), the cell digits of the sweep generator.
* W0 histogram: 64 equal bins of log10(E / W0) over [-3, 3], values outside clamped to the end bins;
  one histogram per species slot of the sweep (slot 0 for a grid or explicit arrays).
* heating histogram: 256 equal bins of sign(dE) log10(1 + |dE| / (k_B x 1 nK)) over
  [-log10(1 + 1e8), +log10(1 + 1e8)], clamped.
* complex lifetimes (Fig. 2): t_last - t_first bounce of exited complexes, 96 bins of
  log10(t / 1 us) over [-2, 4] (clamped) per species slot; complexes still bound at t_max or at the
  step cap are censored (alive throughout); the survival S(t) at each bin's lower edge and its
  power-law exponent by least squares of log S against log t over edges t >= 20 us.
* box counting: boxes of s x s cells, s = 2^k; a box is "occupied" when it holds a complex-forming
  cell and on the "boundary" when it holds both kinds; dimensions are least-squares slopes of
  log N(s) against log(1/s) over s = 2 .. 64.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

K_NANOKELVIN = 3.1668115634556e-15      # k_B x 1 nK in hartree (CODATA 2018)
W0_BINS, W0_LO, W0_HI = 64, -3.0, 3.0
HEAT_BINS = 256
HEAT_X = math.log10(1.0 + 1.0e8)


def n_cells(gen) -> int:
    return max(1, len(gen.species)) * max(1, len(gen.E_list)) * max(1, len(gen.q_list)) * max(1, len(gen.De_list))


def reduce_cells(ids, gen, dE, n_bounce, status) -> np.ndarray:
    """Per cell: (count, complex count, sum dE, sum dE^2, sum n_bounce); sums by math.fsum (exactly
    rounded), so any summation order on the other side is within a few ulps of the total's scale."""
    ids = np.asarray(ids, dtype=np.int64)
    nc = n_cells(gen)
    cell = ids % nc
    out = np.zeros((nc, 5))
    for c in range(nc):
        m = cell == c
        e = np.asarray(dE)[m]
        out[c, 0] = m.sum()
        out[c, 1] = (np.asarray(status)[m] & oracle.COMPLEX != 0).sum()
        out[c, 2] = math.fsum(e.tolist())
        out[c, 3] = math.fsum((e * e).tolist())
        out[c, 4] = math.fsum(np.asarray(n_bounce)[m].astype(np.float64).tolist())
    return out


def w0_eq2(m_a, m_i, C4, Omega, a_x, q_x):
    """Eq. (2): the micromotion-heating energy scale W0 of Cetina et al., with the secular frequency
    omega = (Omega / 2) sqrt(a_x + q_x^2 / 2).  Atomic units (masses in m_e, energies in hartree)."""
    omega = 0.5 * Omega * np.sqrt(a_x + 0.5 * np.asarray(q_x) ** 2)
    return (8.0 / (3.0 * math.pi)) * (m_a / (m_i + m_a)) ** (5.0 / 3.0) * np.cbrt(
        m_i ** 2 * omega ** 4 * C4 / np.asarray(q_x) ** 2)


def w0_coordinate(E, W0):
    """Fractional bin coordinate of log10(E / W0) on the 64-bin axis (before clamping)."""
    return (np.log10(np.asarray(E) / W0) - W0_LO) / (W0_HI - W0_LO) * W0_BINS


def heat_coordinate(dE):
    """Fractional bin coordinate of the signed log heating on the 256-bin axis (before clamping)."""
    dE = np.asarray(dE)
    x = np.where(dE < 0.0, -1.0, 1.0) * np.log10(1.0 + np.abs(dE) / K_NANOKELVIN)
    return (x + HEAT_X) / (2.0 * HEAT_X) * HEAT_BINS


def _bin(coord, nbins):
    return np.clip(np.floor(coord), 0, nbins - 1).astype(np.int64)


def sweep_params(ids, workload):
    """(E, q_x, species slot, species index) per global id of a sweep workload, from the oracle's
    generator."""
    gen = workload.gen
    E = np.empty(len(ids))
    q = np.empty(len(ids))
    slot = np.empty(len(ids), dtype=np.int64)
    sp = np.empty(len(ids), dtype=np.int64)
    for i, gid in enumerate(ids):
        d = oracle.sweep_draw(int(gid), gen)
        E[i], q[i], sp[i] = d["E"], d["q_x"], d["species"]
        slot[i] = list(gen.species).index(d["species"])
    return E, q, slot, sp


def w0_hist(ids, workload, dE, status, flag=None):
    """Returns (hist (n_slots, 64, 2) of (total, flagged), heat (256,), w0 coordinate, heat coordinate)
    for a sweep workload; the coordinates let a comparison recognise values that sit on a bin edge.
    flag: the status bit counted in the second column, the complex flag by default (BOUND_SEEN: the
    negative-energy bound state of the Eq. (2) text)."""
    flag = oracle.COMPLEX if flag is None else flag
    sysw = workload.system
    spec = workload.species()
    if workload.gen.kind in ("sweep", "thermal"):      # thermal runs: E is the bath energy k_B T
        E, q, slot, sp = sweep_params(ids, workload)
        n_slots = len(workload.gen.species)
    else:
        E = np.full(len(ids), sysw.E)
        q = np.full(len(ids), sysw.q_x)
        slot = np.zeros(len(ids), dtype=np.int64)
        sp = np.full(len(ids), sysw.species)
        n_slots = 1
    m_a = np.array([spec[s][0] for s in sp])
    C4 = np.array([spec[s][1] for s in sp])
    W0 = w0_eq2(m_a, sysw.m_ion, C4, sysw.omega_rf, sysw.a_x, q)
    cw = w0_coordinate(E, W0)
    b = _bin(cw, W0_BINS)
    hist = np.zeros((n_slots, W0_BINS, 2))
    cpx = (np.asarray(status) & flag) != 0
    np.add.at(hist, (slot, b, 0), 1.0)
    np.add.at(hist, (slot[cpx], b[cpx], 1), 1.0)
    ch = heat_coordinate(dE)
    heat = np.bincount(_bin(ch, HEAT_BINS), minlength=HEAT_BINS).astype(np.float64)
    return hist, heat, cw, ch


def boxcount(mask: np.ndarray, kmin: int = 1, kmax: int = 6):
    """mask: side x side booleans (side a power of two), True = complex-forming.  Returns
    (D_boundary, D_set, N_set per level, N_boundary per level)."""
    side = mask.shape[0]
    assert mask.shape == (side, side) and side & (side - 1) == 0
    levels = side.bit_length()
    n_set, n_bnd = [], []
    for k in range(levels):
        s = 1 << k
        boxes = mask.reshape(side // s, s, side // s, s)
        any_ = boxes.any(axis=(1, 3))
        all_ = boxes.all(axis=(1, 3))
        n_set.append(int(any_.sum()))
        n_bnd.append(int((any_ & ~all_).sum()))
    dims = []
    for counts in (n_bnd, n_set):
        xs = [-k * math.log(2.0) for k in range(kmin, min(kmax, levels - 1) + 1) if counts[k] > 0]
        ys = [math.log(counts[k]) for k in range(kmin, min(kmax, levels - 1) + 1) if counts[k] > 0]
        dims.append(float(np.polyfit(xs, ys, 1)[0]) if len(xs) >= 2 else float("nan"))
    return dims[0], dims[1], n_set, n_bnd


AU_TIME_MICRO = 2.4188843265857e-11     # atomic unit of time in microseconds (CODATA 2018)
LIFE_BINS, LIFE_LO, LIFE_HI = 96, -2.0, 4.0
EXITED, TMAX, MAX_STEPS = 1 << 2, 1 << 8, 1 << 11


def life_coordinate(t_first, t_last):
    return (np.log10((np.asarray(t_last) - np.asarray(t_first)) * AU_TIME_MICRO) - LIFE_LO) / \
        (LIFE_HI - LIFE_LO) * LIFE_BINS


def lifetime_hist(slot, n_slots, t_first, t_last, n_bounce, status):
    """(hist (n_slots, 96), censored (n_slots,), coordinate of each finished complex or nan)."""
    status = np.asarray(status).astype(np.int64)
    cpx = (status & oracle.COMPLEX) != 0
    done = cpx & ((status & EXITED) != 0) & (np.asarray(n_bounce) >= 2)
    cens = cpx & ~done & ((status & (TMAX | MAX_STEPS)) != 0)
    coord = np.full(len(status), np.nan)
    coord[done] = life_coordinate(np.asarray(t_first)[done], np.asarray(t_last)[done])
    hist = np.zeros((n_slots, LIFE_BINS))
    np.add.at(hist, (np.asarray(slot)[done], _bin(coord[done], LIFE_BINS)), 1.0)
    censored = np.bincount(np.asarray(slot)[cens], minlength=n_slots).astype(np.float64)
    return hist, censored, coord


def survival(hist, censored):
    """S at the lower edge of every bin (alive = finished later, or censored)."""
    total = hist.sum() + censored
    alive = np.cumsum(hist[::-1])[::-1] + censored
    return alive / total if total > 0 else np.full(len(hist), np.nan)


def survival_exponent(hist, censored, t_min_us=20.0):
    edges = LIFE_LO + np.arange(LIFE_BINS) * (LIFE_HI - LIFE_LO) / LIFE_BINS
    S = survival(hist, censored)
    sel = (edges >= math.log10(t_min_us)) & (S > 0)
    if sel.sum() < 2:
        return float("nan")
    return float(-np.polyfit(edges[sel] * math.log(10.0), np.log(S[sel]), 1)[0])
