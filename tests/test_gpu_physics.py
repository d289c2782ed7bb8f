"""Qualitative results the paper reports, reproduced by the GPU path (physics smoke tests).

* Fig. 1 text: the regular regions are direct collisions -- one bounce and no complex.
* Fig. 2 text: after ~20 us the complexes decay by a power law (non-hyperbolic chaos), not
  exponentially (hyperbolic): for every species whose complexes span a decade of lifetimes beyond
  20 us (at least 30 complexes alive at each of >= 15 bin edges, 1/16 decade apart), log S is fitted
  better by a line in log t than by a line in t.  Measured on 500,000 trajectories: Na23 and K40
  qualify (residuals 0.36 vs 0.95 and 0.14 vs 0.54); the heavier atoms decay too steeply
  (exponents ~2.4) for the range to discriminate.
* Fig. 3 (thermal runs, 600,000 trajectories, 20,000 per bar): complexes form more often with
  cooler baths (every species and well) and heavier atoms (at every temperature, pooled over the
  wells), and changing the well depth from 1 K to 100 K leaves the probability unchanged: the
  30 bars' 15 differences are consistent with zero (chi^2 below its 99.9 % point, every |z| < 4;
  measured chi^2 = 21.7 for 15 degrees of freedom).  Measured P(complex) at 1 / 10 / 100 uK:
  Li6 0.12 / 0.025 / 0.002 up to Cs133 0.25 / 0.075 / 0.020.
* Fig. 4 (head-on from r0 = 20,000 a0, q_x = 0.2, D_e = 1 K, energies log-uniform over
  0.1 uK - 1 mK, 200,000 per atom, binned in log10(E / W0) on the device): the probability falls
  with the energy like a negative tanh and complex formation is suppressed (below 5 % of its
  low-energy value) from a threshold at 2-4 W0 for Li6, Na23 and K40 (measured 3.3 W0, one bin
  of 0.094 decades below being 2.6 W0) and 4-10 W0 for Rb87 (6.3 W0), so the absolute threshold
  grows with the mass.  Cs133 (mass ratio 0.76 to Yb+) is not suppressed up to 1 mK: its head-on
  collisions leave the atom nearly at rest while the ion recoils, and the trap returns the ion for
  a second hit (mostly exactly two bounces), which the bounce-count definition of a complex counts.
  Inset (Li6, q_x = 0.1 - 0.4 at fixed Omega, eight energies 0.1 - 2 uK, 10^4 per cell): a larger
  q_x gives more complexes at every energy and a higher threshold.
* Abstract, Fig. 3 and Fig. 4 text: lower-energy collisions with heavier atoms form complexes more
  often, and complex formation is suppressed above a threshold energy that is greater for heavier
  atoms.  On the 225-cell sweep (200 trajectories per cell, pooled over q_x and D_e: 1800 per
  species and energy): at every collision energy the probability does not fall with the atom's
  mass (3 standard errors), and the fraction that survives from 1 to 100 uK,
  P(100 uK) / P(1 uK), grows with the mass (the threshold moves up), from full suppression for the
  light atoms.  (Below the threshold the probability is a plateau and need not fall with energy:
  for Cs133 it rises by a few per cent between 1 and 30 uK.)
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402
from paper_2509_15117_amd import _abi  # noqa: E402


def test_direct_cells_are_not_complexes():
    w = W.config1()
    out = api.integrate_workload(w, counters=False)
    nb = out["n_bounce"].cpu().numpy()
    st = out["status"].cpu().numpy()
    one = nb == 1
    assert one.any() and (~one).any()
    assert np.all((st[one] & _abi.ST_COMPLEX) == 0)
    assert np.all((st[nb >= 2] & _abi.ST_COMPLEX) != 0)


def test_complex_probability_trends_on_the_sweep():
    w = W.config3()
    w.system.max_steps = 2_000_000       # bound the longest complexes (they are complexes either way)
    n = 225 * 200
    print(f"physics: sweep cells, n={n}", flush=True)
    res = api.run_chunks(w, n=n, chunk=n, n_streams=1, cells=True)
    c = res["cells"].cpu().numpy().reshape(5, 5, 3, 3, 5)     # species, E, q, De, fields
    tot = c[..., 0].sum(axis=(2, 3))
    cpx = c[..., 1].sum(axis=(2, 3))
    assert np.all(tot == 1800)
    p = cpx / tot
    se = np.sqrt(np.maximum(p * (1 - p), 1.0 / tot) / tot)
    names = w.species_names
    print("P(complex) species x E (1, 3, 10, 30, 100 uK):\n" + "\n".join(
        f"  {names[s]:6s} " + " ".join(f"{x:.3f}" for x in p[s]) for s in range(5)), flush=True)
    masses = np.array([m for m, _ in w.species()])
    order = np.argsort(masses)
    for e in range(5):
        for a, b in zip(order[:-1], order[1:]):            # heavier atom: no fewer complexes
            assert p[b, e] >= p[a, e] - 3 * np.hypot(se[a, e], se[b, e]), (names[a], names[b], e)
    # threshold above which complexes are suppressed grows with the mass
    surv = (cpx[:, 4] + 0.5) / (cpx[:, 0] + 0.5)
    print("P(100 uK) / P(1 uK):", dict(zip(names, np.round(surv, 3))), flush=True)
    assert np.all(np.diff(surv[order]) >= -0.05), surv[order]
    assert surv[order[1]] < 0.05 and surv[order[-1]] > 0.5
    # and the trend is strong: the heaviest atom at the lowest energy against the lightest at the highest
    assert p[order[-1], 0] > p[order[0], 4] + 5 * np.hypot(se[order[-1], 0], se[order[0], 4])


def test_complex_survival_is_a_power_law():
    import oracle.reduce as R
    w = W.fig2_survival()
    n = 500_000
    print(f"physics: Fig. 2 survival, n={n}", flush=True)
    out = api.integrate_workload(w, n=n, counters=True)
    flat = api.reduce_lifetime(w.system, w.species(), w.gen, n, out)
    h, cens, expo = (t.cpu().numpy() for t in api.split_lifetime(flat))
    edges = R.LIFE_LO + np.arange(R.LIFE_BINS) * (R.LIFE_HI - R.LIFE_LO) / R.LIFE_BINS
    fitted = 0
    for s, name in enumerate(w.species_names):
        total = h[s].sum() + cens[s]
        print(f"  {name:6s} complexes {int(total)} (censored {int(cens[s])}), survival exponent {expo[s]:.3f}",
              flush=True)
        if total < 300:
            continue
        S = R.survival(h[s], cens[s])
        sel = (edges >= np.log10(20.0)) & (S * total >= 30)
        if sel.sum() < 15:
            print(f"  {name:6s} {sel.sum()} edges from 20 us: too short a range to discriminate", flush=True)
            continue
        logt, y = edges[sel] * np.log(10.0), np.log(S[sel])

        def rms(x):
            return float(np.sqrt(np.mean((y - np.polyval(np.polyfit(x, y, 1), x)) ** 2)))

        r_pow, r_exp = rms(logt), rms(np.exp(logt))
        print(f"  {name:6s} {sel.sum()} edges from 20 us: residual power law {r_pow:.3f}, exponential {r_exp:.3f}",
              flush=True)
        assert r_pow < r_exp, (name, r_pow, r_exp)
        assert 0.05 < expo[s] < 5.0, (name, expo[s])
        fitted += 1
    assert fitted >= 2


def _grid(side, q_ratio):
    w = W.config1()
    w.gen = W.Generator(kind="grid", n_theta=side, n_phi=side)
    w.system.q_ratio = q_ratio
    return w.with_n(side * side)


def test_ring_trap_is_azimuthally_symmetric():
    """Ring trap (q_y = q_x, q_z = -2 q_x): a rotation about z maps trajectories onto each other, so
    along each theta row of the grid every direct trajectory has the same observables up to the
    integration's own error: each phi takes its own step sequence, and at rtol 1e-10 the rows agree
    to ~3e-7 (angle) and ~3e-6 (momentum transfer, relative), tested at 1e-5 (Fig. 1 then shows bands
    in theta)."""
    side = 32
    w = _grid(side, W.RING[1])
    out = api.integrate_workload(w, counters=False)
    nb = out["n_bounce"].cpu().numpy().reshape(side, side)
    ang = out["angle"].cpu().numpy().reshape(side, side)
    q = out["q_transfer"].cpu().numpy().reshape(side, side)
    rows, worst = 0, 0.0
    for j in range(side):
        if np.all(nb[j] == 1):
            rows += 1
            ra, rq = np.ptp(ang[j]) / abs(ang[j]).max(), np.ptp(q[j]) / q[j].max()
            worst = max(worst, ra, rq)
            assert ra <= 1e-5 and rq <= 1e-5, (j, ra, rq)
    print(f"ring trap: {rows} direct theta rows, largest relative spread over phi {worst:.1e}", flush=True)
    assert rows >= 4


def test_linear_trap_saddle_at_pi_over_4():
    """Linear trap (q_y = -q_x, no RF along z), the configuration of the Fig. 1 discussion: the
    micromotion at phi = pi/4 is perpendicular to the incoming atom, and the saddle between the two
    regular regions there is dominated by complexes.  On a 64 x 64 octant grid the four phi columns
    around pi/4 form complexes more often than the eight columns nearest phi = 0 and pi/2 (measured:
    the columns peak at 0.81 just below pi/4, against 0.61 near phi = 0 and 0.38 near pi/2)."""
    side = 64
    w = _grid(side, W.LINEAR[1])
    out = api.integrate_workload(w, counters=False)
    cpx = ((out["status"].cpu().numpy() & _abi.ST_COMPLEX) != 0).reshape(side, side)
    mid = cpx[:, side // 2 - 2: side // 2 + 2].mean()
    edge = np.concatenate([cpx[:, :4], cpx[:, -4:]], axis=1).mean()
    n_mid, n_edge = side * 4, side * 8
    se = np.sqrt(mid * (1 - mid) / n_mid + edge * (1 - edge) / n_edge)
    by_col = cpx.mean(axis=0)
    print("linear trap, P(complex) by phi column:", np.array2string(by_col, precision=2, max_line_width=200),
          flush=True)
    assert mid > edge + 3 * se, (mid, edge, se)
    # and the ring trap has no such structure: its columns agree
    ring = ((api.integrate_workload(_grid(side, W.RING[1]), counters=False)["status"].cpu().numpy()
             & _abi.ST_COMPLEX) != 0).reshape(side, side)
    assert np.ptp(ring.mean(axis=0)) <= 0.1


def test_thermal_runs_fig3_trends_and_no_well_depth_dependence():
    w = W.fig3_thermal()
    w.system.max_steps = 2_000_000
    n = 30 * 20_000
    print(f"physics: Fig. 3 thermal runs, n={n}", flush=True)
    res = api.run_chunks(w, n=n, chunk=n // 2, n_streams=2, cells=True)
    c = res["cells"].cpu().numpy().reshape(5, 3, 2, 5)       # species, T, De, fields
    tot, cpx = c[..., 0], c[..., 1]
    assert np.all(tot == 20_000)
    p = cpx / tot
    se = np.sqrt(np.maximum(p * (1 - p), 1.0 / tot) / tot)
    names = w.species_names
    print("P(complex) at 1 / 10 / 100 uK, De = 1 K | 100 K:\n" + "\n".join(
        f"  {names[s]:6s} " + " ".join(f"{p[s, e, 0]:.4f}|{p[s, e, 1]:.4f}" for e in range(3)) for s in range(5)),
        flush=True)
    # cooler baths: more complexes, for every species and well
    for e in range(2):
        assert np.all(p[:, e] > p[:, e + 1] + 3 * np.hypot(se[:, e], se[:, e + 1])), e
    # heavier atoms: no fewer complexes at any temperature, and clearly more for the heaviest
    pp, tt = cpx.sum(2) / tot.sum(2), tot.sum(2)
    sp = np.sqrt(np.maximum(pp * (1 - pp), 1.0 / tt) / tt)
    order = np.argsort([m for m, _ in w.species()])
    for e in range(3):
        for a, b in zip(order[:-1], order[1:]):
            assert pp[b, e] >= pp[a, e] - 3 * np.hypot(sp[a, e], sp[b, e]), (names[a], names[b], e)
        assert pp[order[-1], e] > pp[order[0], e] + 10 * np.hypot(sp[order[0], e], sp[order[-1], e])
    # the well depth (1 K against 100 K) does not change the probability
    z = (p[..., 0] - p[..., 1]) / np.hypot(se[..., 0], se[..., 1])
    chi2 = float((z ** 2).sum())
    print(f"De 1 K vs 100 K: chi^2 {chi2:.1f} for {z.size} differences, largest |z| {np.abs(z).max():.2f}", flush=True)
    assert chi2 < 37.7 and np.abs(z).max() < 4.0         # chi^2(15) 99.9 % point


def test_fig4_threshold_is_a_few_w0():
    """Fig. 4 text: P(complex) falls with collision energy to a threshold of a few W0 (Eq. (2)), above
    which complexes are suppressed, and the threshold grows with the atom's mass.  Both flags are
    measured on the same trajectories: the complex flag (>= 2 bounces or t_max) and the bound-state
    bit (the relative energy went negative: the temporary atom-ion bound state of the Eq. (2) text).
    * Bound-state bit, every atom (Cs133 included): the fraction falls with energy above W0 (no rise
      between bins 0.45 decades apart beyond 3 SE, and a clear fall over the range).
    * Complex flag, Li6 .. Rb87: every complex also reached the bound state, and the flag's threshold
      lies at 2-6 W0, increasing with mass.
    * Complex flag, Cs133: it first rises above W0 (the heavy atom's recoiling ion returns for a second
      head-on hit without a bound state) and falls beyond its maximum; no threshold within 1 mK."""
    import oracle.reduce as R
    w = W.fig4_energy()
    w.system.max_steps = 2_000_000
    n = 5 * 200_000
    print(f"physics: Fig. 4 energy sweep, n={n}", flush=True)
    res = api.run_chunks(w, n=n, chunk=n // 2, n_streams=2, hist=True, hist_bound=True)
    h = api.split_hist(res["hist"])[0].cpu().numpy()
    hb = api.split_hist(res["hist_bound"])[0].cpu().numpy()
    assert np.array_equal(h[..., 0], hb[..., 0])
    x = R.W0_LO + (np.arange(R.W0_BINS) + 0.5) * (R.W0_HI - R.W0_LO) / R.W0_BINS
    W0 = [R.w0_eq2(m, w.system.m_ion, C4, w.system.omega_rf, w.system.a_x, 0.2) for m, C4 in w.species()]
    th_abs = []
    for s, name in enumerate(w.species_names):
        tot, c, cb = h[s, :, 0], h[s, :, 1], hb[s, :, 1]
        sel = tot >= 500
        xs, p, pb, t = x[sel], c[sel] / tot[sel], cb[sel] / tot[sel], tot[sel]
        se = np.sqrt(np.maximum(p * (1 - p), 1.0 / t) / t)
        seb = np.sqrt(np.maximum(pb * (1 - pb), 1.0 / t) / t)
        plateau = p[xs <= 0.0].max()
        below = np.where((xs > 0.0) & (p < 0.05 * plateau))[0]
        print(f"  {name:6s} plateau {plateau:.3f}, P(complex) | P(bound state) by log10(E/W0): " +
              " ".join(f"{a:+.2f}:{b:.3f}|{d:.3f}" for a, b, d in zip(xs, p, pb) if -1.0 <= a <= 2.0), flush=True)
        # bound-state bit: falls with energy above W0 for every atom
        up = xs >= 0.0
        xa, pa, sa = xs[up], pb[up], seb[up]
        for j in range(len(xa)):
            for k in range(j + 1, len(xa)):
                if xa[k] - xa[j] >= 0.45:
                    assert pa[k] <= pa[j] + 3 * np.hypot(sa[j], sa[k]), (name, xa[j], xa[k], pa[j], pa[k])
        assert pa[-1] < pa[0] - 5 * np.hypot(sa[0], sa[-1]), (name, pa[0], pa[-1])
        if name == "Cs133":
            assert len(below) == 0                           # no threshold within 1 mK
            m = int(np.argmax(np.where(up, p, -1.0)))
            print(f"  Cs133 complex flag: maximum {p[m]:.3f} at log10(E/W0) = {xs[m]:+.2f}, {p[-1]:.3f} at "
                  f"{xs[-1]:+.2f}; bound-state bit {pb[m]:.3f} -> {pb[-1]:.3f}", flush=True)
            assert xs[m] > 0.0 and p[-1] < p[m] - 10 * np.hypot(se[m], se[-1])
            continue
        # every complex of the lighter atoms also reached the bound state
        assert np.all(pb >= p - 3 * np.hypot(se, seb)), name
        x_th = xs[below[0]]
        print(f"  {name:6s} threshold {10 ** x_th:.2f} W0 = {10 ** x_th * W0[s] / W.kelvin(1e-6):.2f} uK", flush=True)
        lo, hi = (0.6, 1.0) if name == "Rb87" else (0.30, 0.61)
        assert lo <= x_th <= hi, (name, x_th)
        assert np.all(p[xs > x_th + 0.3] < 0.01), name       # suppressed above the threshold
        assert 0.4 < plateau < 0.8, name
        th_abs.append(10 ** x_th * W0[s])
    assert np.all(np.diff(th_abs) > 0), th_abs              # heavier atom, higher threshold


def test_fig4_inset_larger_q_more_complexes_and_higher_threshold():
    w = W.fig4_inset()
    w.system.max_steps = 2_000_000
    n = w.n
    print(f"physics: Fig. 4 inset, n={n}", flush=True)
    res = api.run_chunks(w, n=n, chunk=n // 2, n_streams=2, cells=True)
    c = res["cells"].cpu().numpy().reshape(8, 4, 5)           # energy, q, fields
    tot, cpx = c[..., 0], c[..., 1]
    assert np.all(tot == n // 32)
    p = cpx / tot
    se = np.sqrt(np.maximum(p * (1 - p), 1.0 / tot) / tot)
    E = [0.1, 0.2, 0.3, 0.5, 0.7, 1.0, 1.5, 2.0]
    print("Li6 P(complex), rows E (uK), columns q = 0.1 .. 0.4:\n" + "\n".join(
        f"  {E[e]:4.1f} " + " ".join(f"{p[e, k]:.3f}" for k in range(4)) for e in range(8)), flush=True)
    for e in range(8):
        for k in range(3):
            assert p[e, k + 1] >= p[e, k] - 3 * np.hypot(se[e, k], se[e, k + 1]), (E[e], k)
        if p[e, 3] > 0.05:
            assert p[e, 3] > p[e, 0] + 5 * np.hypot(se[e, 0], se[e, 3]), E[e]
    th = [next((E[e] for e in range(8) if p[e, k] < 0.02), 99.0) for k in range(4)]
    print("Li6 threshold (first energy with P < 0.02) by q:", th, flush=True)
    assert np.all(np.diff(th) >= 0) and th[3] > th[0]
