"""Pins of the oracle's reductions (box counting, Eq. (2), histogram axes, cell mapping).

* Box counting: sets whose dimensions are known exactly -- a filled square (2), a straight
  boundary (1, horizontal or diagonal), the Sierpinski gasket of Pascal's triangle mod 2
  (log2 3), and i.i.d. noise whose boundary fills the plane (2).
* Eq. (2): the paper states that W0 grows as q_x^(2/3) at fixed Omega with a_x = 0 (Sec. on Fig. 4).
  The rest of the formula is pinned through its exponents (omega^(4/3), C4^(1/3)), the heavy-atom
  limit of its mass factor, and a_x entering the secular frequency.
* Heating axis: zero heating sits on the middle edge, the axis is odd, and values built at a known
  coordinate land in the predicted bin.
* Cells: the cell a reduction assigns to an id (id mod number of cells) is the cell whose list
  values the sweep generator draws for that id.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import reduce as R

oracle.build()


def test_boxcount_filled_square():
    Db, Ds, n_set, n_bnd = R.boxcount(np.ones((256, 256), bool))
    assert Ds == pytest.approx(2.0, abs=1e-12)
    assert math.isnan(Db) and all(v == 0 for v in n_bnd)
    assert n_set == [(256 >> k) ** 2 for k in range(9)]


@pytest.mark.parametrize("diagonal", [False, True])
def test_boxcount_straight_boundary(diagonal):
    side = 512
    i, j = np.indices((side, side))
    mask = (j < i) if diagonal else (j < side // 2 + 3)
    Db, Ds, n_set, n_bnd = R.boxcount(mask)
    assert Db == pytest.approx(1.0, abs=0.03)
    if diagonal:   # the staircase boundary crosses exactly side/s boxes at every scale
        assert n_bnd[1:] == [side >> k for k in range(1, 10)]
        assert n_set == [(side >> k) * ((side >> k) + 1) // 2 - (side >> k if k == 0 else 0) for k in range(10)]
    else:          # column boundary at x = side/2 + 3
        w = side // 2 + 3
        assert n_set == [(side >> k) * (-(-w // (1 << k))) for k in range(10)]
        assert n_bnd == [0] + [side >> k for k in range(1, 10)]


def test_boxcount_sierpinski_gasket():
    side = 1024
    i, j = np.indices((side, side))
    mask = (i & j) == 0          # Pascal's triangle mod 2
    Db, Ds, n_set, _ = R.boxcount(mask)
    assert n_set == [3 ** (10 - k) for k in range(11)]
    assert Ds == pytest.approx(math.log2(3.0), abs=1e-12)
    assert Db == pytest.approx(math.log2(3.0), abs=0.05)


def test_boxcount_noise_boundary_fills_the_plane():
    mask = np.random.default_rng(7).random((512, 512)) < 0.5
    Db, Ds, _, n_bnd = R.boxcount(mask)
    # a 2x2 box is uniform with probability 2 / 16; from 4x4 boxes on, every box is mixed
    n1 = (512 >> 1) ** 2
    assert abs(n_bnd[1] - 7 / 8 * n1) < 5 * math.sqrt(n1 * 7 / 64)
    assert n_bnd[2:7] == [(512 >> k) ** 2 for k in range(2, 7)]
    assert 1.95 < Db < 2.0


def test_w0_scales_as_q_to_two_thirds():
    s = W.System()
    m_a, C4 = W.species_table(["Rb87"])[0]
    q = np.array([0.05, 0.1, 0.2, 0.4])
    w = R.w0_eq2(m_a, s.m_ion, C4, s.omega_rf, 0.0, q)
    assert np.allclose(w / w[0], (q / q[0]) ** (2.0 / 3.0), rtol=1e-13)


def test_w0_dependences():
    s = W.System()
    m_a, C4 = W.species_table(["Rb87"])[0]
    w = lambda **k: float(R.w0_eq2(k.get("m_a", m_a), k.get("m_i", s.m_ion), k.get("C4", C4),
                                   k.get("Om", s.omega_rf), k.get("a", 0.0), k.get("q", 0.2)))
    base = w()
    # omega^(4/3) and C4^(1/3)
    assert w(Om=2 * s.omega_rf) / base == pytest.approx(2 ** (4 / 3), rel=1e-13)
    assert w(C4=8 * C4) / base == pytest.approx(2.0, rel=1e-13)
    # heavy-atom limit m_a >> m_i: the mass ratio tends to 1 and W0 -> (8/3pi)(m_i^2 omega^4 C4/q^2)^(1/3)
    lim = w(m_a=1e12 * s.m_ion)
    om = 0.5 * s.omega_rf * math.sqrt(0.5 * 0.2 ** 2)
    assert lim == pytest.approx(8 / (3 * math.pi) * (s.m_ion ** 2 * om ** 4 * C4 / 0.04) ** (1 / 3), rel=1e-10)
    # secular frequency: a_x adds to q_x^2 / 2 under the square root
    assert w(a=0.02, q=0.2) / w(a=0.0, q=0.2) == pytest.approx(((0.02 + 0.02) / 0.02) ** (2 / 3), rel=1e-13)
    # at E = W0 the coordinate is the middle edge of the 64-bin axis
    assert R.w0_coordinate(base, base) == pytest.approx(32.0, abs=1e-12)


def test_heating_axis():
    assert R.heat_coordinate(0.0) == pytest.approx(128.0, abs=1e-12)
    x = np.array([1e-3, 0.7, 3.3, 7.9])
    dE = R.K_NANOKELVIN * (10.0 ** x - 1.0)
    c = R.heat_coordinate(dE)
    assert np.allclose(c, (x + R.HEAT_X) / (2 * R.HEAT_X) * 256, rtol=0, atol=1e-9)
    assert np.allclose(R.heat_coordinate(-dE), 256 - c, atol=1e-9)
    # clamped ends: heating beyond 1e8 nK (0.1 K) goes to the end bins
    big = np.array([-1.0, 1.0])
    _, heat, _, _ = R.w0_hist([0, 1], W.config1(), big, np.zeros(2, np.uint32))
    assert heat[0] == 1 and heat[255] == 1


def test_cells_follow_the_generator_digits():
    w = W.config3()
    nc = R.n_cells(w.gen)
    assert nc == 225
    ids = [0, 1, 7, 224, 225, 226, 10_000_003, 11_999_999]
    for gid in ids:
        d = oracle.sweep_draw(gid, w.gen)
        c = gid % nc
        # species slowest, De fastest
        De_i = c % 3
        q_i = (c // 3) % 3
        E_i = (c // 9) % 5
        sp_i = c // 45
        assert d["species"] == w.gen.species[sp_i]
        assert d["E"] == w.gen.E_list[E_i]
        assert d["q_x"] == w.gen.q_list[q_i]
        assert d["De"] == w.gen.De_list[De_i]


def test_cells_brute_force():
    rng = np.random.default_rng(3)
    w = W.config3()
    ids = np.arange(1000, 3000)
    dE = rng.normal(size=ids.size) * 1e-9
    nb = rng.integers(1, 50, ids.size)
    st = rng.integers(0, 2, ids.size).astype(np.uint32)
    out = R.reduce_cells(ids, w.gen, dE, nb, st)
    for c in (0, 17, 224):
        sel = [k for k in range(ids.size) if ids[k] % 225 == c]
        assert out[c, 0] == len(sel)
        assert out[c, 1] == sum(int(st[k]) for k in sel)
        assert out[c, 2] == pytest.approx(sum(dE[k] for k in sel), rel=1e-14, abs=1e-24)
        assert out[c, 4] == sum(int(nb[k]) for k in sel)
    assert out[:, 0].sum() == ids.size


def test_lifetime_axis_and_survival_of_a_power_law():
    """Pareto lifetimes S(t) = (t / 1 us)^-alpha: the histogram's survival fraction recovers alpha
    (statistical error ~1e-3 at 2e6 samples); lifetimes beyond the axis end (10 ms) count as censored,
    which leaves S unchanged below it."""
    rng = np.random.default_rng(9)
    alpha = 0.7
    n = 2_000_000
    t_us = rng.random(n) ** (-1.0 / alpha)                  # Pareto, t >= 1 us
    t_last = t_us / R.AU_TIME_MICRO
    t_first = np.zeros(n)
    st = np.full(n, oracle.COMPLEX | R.EXITED, dtype=np.int64)
    late = t_us > 1e4
    st[late] = oracle.COMPLEX | R.TMAX
    nb = np.full(n, 5)
    hist, cens, coord = R.lifetime_hist(np.zeros(n, np.int64), 1, t_first, t_last, nb, st)
    assert cens[0] == late.sum() and hist.sum() == n - late.sum()
    # bins below 1 us are empty; the coordinate of 1 us is the edge 32 (log10 1 = 0 on [-2, 4])
    assert hist[0, :32].sum() == 0
    assert R.life_coordinate(0.0, 1.0 / R.AU_TIME_MICRO) == pytest.approx(32.0, abs=1e-9)
    S = R.survival(hist[0], cens[0])
    edges = 10.0 ** (R.LIFE_LO + np.arange(96) * 6.0 / 96)
    sel = (edges >= 1.0) & (edges <= 1e3)
    assert np.allclose(S[sel], edges[sel] ** -alpha, rtol=0.05)
    assert R.survival_exponent(hist[0], cens[0]) == pytest.approx(alpha, abs=0.01)
    # not a complex, or a direct exit: not counted
    hist2, cens2, _ = R.lifetime_hist([0, 0], 1, [0.0, 0.0], [1e9, 1e9], [5, 1],
                                      [R.EXITED, oracle.COMPLEX | R.EXITED])
    assert hist2.sum() == 0 and cens2.sum() == 0


def test_w0_hist_flag_column_counts_the_chosen_status_bit():
    """The second column of the W0 histogram counts the complex flag by default and the bound-state
    bit when asked: brute-force counts per bin on a small status pattern."""
    w = W.config5()
    ids = np.arange(1000, 1400)
    st = np.zeros(len(ids), np.uint32)
    st[::3] |= oracle.COMPLEX
    st[::5] |= oracle.BOUND_SEEN
    dE = np.zeros(len(ids))
    hc, _, cw, _ = R.w0_hist(ids, w, dE, st)
    hb, _, _, _ = R.w0_hist(ids, w, dE, st, flag=oracle.BOUND_SEEN)
    _, _, slot, _ = R.sweep_params(ids, w)
    b = np.clip(np.floor(cw), 0, 63).astype(np.int64)
    for h, bit in ((hc, oracle.COMPLEX), (hb, oracle.BOUND_SEEN)):
        ref = np.zeros((3, 64))
        for s_, b_, flagged in zip(slot, b, (st & bit) != 0):
            ref[s_, b_] += flagged
        assert np.array_equal(h[..., 1], ref)
        assert np.array_equal(h[..., 0], hc[..., 0])
    assert hc[..., 1].sum() == len(ids[::3]) and hb[..., 1].sum() == len(ids[::5])
