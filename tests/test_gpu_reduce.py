"""GPU parity of iat_reduce (per-cell sums, W0 and heating histograms, box counting) against the
oracle's reductions of the same observables.

Integer results (counts, box counts) must be equal.  Sums run in a fixed order on the GPU and are
exactly rounded (fsum) in the oracle: they agree to n eps sum|x| with n the items per cell, tested
at 1e-12 sum|x|.  A histogram bin index is decided in FP64 on both sides from log10; a value within
1e-9 of a bin edge may fall on either side (the two log10 implementations differ in the last ulp),
so such items may move between the two adjacent bins and nothing else may differ."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import reduce as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)


def synthetic_obs(n, seed, p_complex=0.3):
    rng = np.random.default_rng(seed)
    dE = rng.normal(size=n) * 10.0 ** rng.uniform(-16, -6, n)
    dE[rng.random(n) < 0.01] = 0.0
    nb = rng.integers(1, 200, n).astype(np.int32)
    st = ((rng.random(n) < p_complex).astype(np.uint32) | (rng.integers(0, 2, n).astype(np.uint32) << 1)
          | (rng.integers(0, 2, n).astype(np.uint32) << 2) | (rng.integers(0, 2, n).astype(np.uint32) << 8))
    obs = {"dE_ion": torch.from_numpy(dE).to(DEV), "n_bounce": torch.from_numpy(nb).to(DEV),
           "status": torch.from_numpy(st.astype(np.int32)).to(DEV)}
    return obs, dE, nb, st


def test_reduce_cells_matches_oracle_and_accumulates():
    w = W.config3()
    n, id0 = 150_001, 987_654
    obs, dE, nb, st = synthetic_obs(n, 1)
    print(f"reduce CELLS: config3 generator, n={n}, id0={id0}", flush=True)
    got = api.reduce_cells(w.system, w.species(), w.gen, n, obs, id0=id0).cpu().numpy()
    ids = np.arange(id0, id0 + n)
    ref = R.reduce_cells(ids, w.gen, dE, nb, st)
    assert np.array_equal(got[:, [0, 1, 4]], ref[:, [0, 1, 4]])
    cell = ids % 225
    abs1 = np.bincount(cell, weights=np.abs(dE), minlength=225)
    abs2 = np.bincount(cell, weights=dE * dE, minlength=225)
    assert np.all(np.abs(got[:, 2] - ref[:, 2]) <= 1e-12 * abs1)
    assert np.all(np.abs(got[:, 3] - ref[:, 3]) <= 1e-12 * abs2)
    # chunks accumulate into the same output: two halves (the second ragged) give the same counts
    h = 70_000
    acc = torch.zeros(225, 5, dtype=torch.float64, device=DEV)
    api.reduce_cells(w.system, w.species(), w.gen, h, {k: v[:h] for k, v in obs.items()}, id0=id0, out=acc)
    api.reduce_cells(w.system, w.species(), w.gen, n - h, {k: v[h:] for k, v in obs.items()}, id0=id0 + h,
                     out=acc)
    acc = acc.cpu().numpy()
    assert np.array_equal(acc[:, [0, 1, 4]], ref[:, [0, 1, 4]])
    assert np.all(np.abs(acc[:, 2] - ref[:, 2]) <= 1e-12 * abs1)
    # fixed order: a second call is bitwise identical
    again = api.reduce_cells(w.system, w.species(), w.gen, n, obs, id0=id0).cpu().numpy()
    assert np.array_equal(again, got)


def test_reduce_on_a_thermal_generator():
    """Thermal runs (Fig. 3) share the sweep's cell digits and species slots; their W0 axis uses the
    bath energy k_B T in place of the collision energy."""
    w = W.fig3_thermal()
    n, id0 = 60_007, 424_242
    obs, dE, nb, st = synthetic_obs(n, 3)
    print(f"reduce CELLS and W0_HIST: thermal generator, n={n}, id0={id0}", flush=True)
    ids = np.arange(id0, id0 + n)
    got = api.reduce_cells(w.system, w.species(), w.gen, n, obs, id0=id0).cpu().numpy()
    ref = R.reduce_cells(ids, w.gen, dE, nb, st)
    assert got.shape == (30, 5) and np.array_equal(got[:, [0, 1, 4]], ref[:, [0, 1, 4]])
    abs1 = np.bincount(ids % 30, weights=np.abs(dE), minlength=30)
    assert np.all(np.abs(got[:, 2] - ref[:, 2]) <= 1e-12 * abs1)
    hw, hh = (t.cpu().numpy() for t in api.split_hist(api.reduce_hist(w.system, w.species(), w.gen, n, obs,
                                                                       id0=id0)))
    ref_w, ref_h, cw, ch = R.w0_hist(ids, w, dE, st)
    assert hw.shape == ref_w.shape == (5, 64, 2)
    _, _, slot, _ = R.sweep_params(ids, w)
    for s in range(5):
        for k in range(2):
            sel = slot == s if k == 0 else (slot == s) & ((st & 1) != 0)
            assert _hist_close(hw[s, :, k], ref_w[s, :, k], cw[sel], 64), (s, k)
    assert _hist_close(hh, ref_h, ch, 256)


def _hist_close(got, ref, coord, nbins, tol=1e-9):
    """got, ref: counts over the same axis; items whose coordinate lies within tol of an interior edge
    may sit in either adjacent bin."""
    diff = got - ref
    if not np.any(diff):
        return True
    frac = np.abs(coord - np.round(coord))
    edge = np.round(coord[(frac < tol) & (coord > 0.5) & (coord < nbins - 0.5)]).astype(np.int64)
    slack = np.zeros(nbins)
    np.add.at(slack, edge, 1.0)
    np.add.at(slack, edge - 1, 1.0)
    return diff.sum() == 0 and np.all(np.abs(diff) <= slack)


def test_reduce_hist_matches_oracle():
    w = W.config5()
    n, id0 = 120_003, 55_555_555
    obs, dE, nb, st = synthetic_obs(n, 2)
    print(f"reduce W0_HIST: config5 generator, n={n}, id0={id0}", flush=True)
    flat = api.reduce_hist(w.system, w.species(), w.gen, n, obs, id0=id0)
    hw, hh = (t.cpu().numpy() for t in api.split_hist(flat))
    ids = np.arange(id0, id0 + n)
    ref_w, ref_h, cw, ch = R.w0_hist(ids, w, dE, st)
    assert hw.shape == ref_w.shape == (3, 64, 2)
    assert hw[..., 0].sum() == n and hh.sum() == n
    _, _, slot, _ = R.sweep_params(ids, w)
    for s in range(3):
        for k in range(2):
            sel = slot == s if k == 0 else (slot == s) & ((st & 1) != 0)
            assert _hist_close(hw[s, :, k], ref_w[s, :, k], cw[sel], 64), (s, k)
    assert _hist_close(hh, ref_h, ch, 256)
    # Eq. (2) puts W0 below 1 uK for Li6 (every collision energy lies above it) and at a few to tens
    # of uK for K40 and Cs133, so those two populate both sides of E = W0
    assert hw[0, :32, 0].sum() == 0 and hw[0, 32:, 0].sum() > 0
    assert all(hw[s, :32, 0].sum() > 0 and hw[s, 32:, 0].sum() > 0 for s in (1, 2))
    # the bound-state variant: the same totals, the second column counting status bit 1
    fb = api.reduce_hist(w.system, w.species(), w.gen, n, obs, id0=id0, flag="bound")
    bw, bh = (t.cpu().numpy() for t in api.split_hist(fb))
    ref_b, _, _, _ = R.w0_hist(ids, w, dE, st, flag=oracle.BOUND_SEEN)
    assert np.array_equal(bw[..., 0], hw[..., 0]) and np.array_equal(bh, hh)
    for s in range(3):
        sel = (slot == s) & ((st & 2) != 0)
        assert _hist_close(bw[s, :, 1], ref_b[s, :, 1], cw[sel], 64), s
    assert 0 < bw[..., 1].sum() < n and bw[..., 1].sum() != hw[..., 1].sum()


def _grid_workload(side):
    w = W.config1()
    w.gen = W.Generator(kind="grid", n_theta=side, n_phi=side)
    return w.with_n(side * side)


@pytest.mark.parametrize("pattern", ["sierpinski", "diagonal", "noise", "empty"])
def test_boxcount_matches_oracle(pattern):
    side = 512
    i, j = np.indices((side, side))
    mask = {"sierpinski": (i & j) == 0, "diagonal": j < i,
            "noise": np.random.default_rng(5).random((side, side)) < 0.4,
            "empty": np.zeros((side, side), bool)}[pattern]
    w = _grid_workload(side)
    st = mask.reshape(-1).astype(np.int32) | (1 << 2)
    obs = {"status": torch.from_numpy(st).to(DEV), "dE_ion": torch.zeros(side * side, dtype=torch.float64,
                                                                            device=DEV),
           "n_bounce": torch.zeros(side * side, dtype=torch.int32, device=DEV)}
    print(f"reduce BOXCOUNT: {pattern} {side}x{side}", flush=True)
    got = api.boxcount(w.system, w.species(), w.gen, obs)
    Db, Ds, n_set, n_bnd = R.boxcount(mask)
    assert got["N_set"] == n_set and got["N_boundary"] == n_bnd
    for a, b in ((got["D_boundary"], Db), (got["D_set"], Ds)):
        assert (math.isnan(a) and math.isnan(b)) or abs(a - b) <= 1e-12
    if pattern == "sierpinski":
        assert got["D_set"] == pytest.approx(math.log2(3.0), abs=1e-12)


def test_reduce_rejects_bad_batches():
    w = W.config1()
    obs, _, _, _ = synthetic_obs(64, 3)
    with pytest.raises(api._abi.IatError):
        api.reduce_cells(w.system, w.species(), w.gen, 64, obs)          # CELLS needs a sweep
    w2 = _grid_workload(8)
    w2.gen = W.Generator(kind="grid", n_theta=8, n_phi=4)
    with pytest.raises(api._abi.IatError):
        api.boxcount(w2.system, w2.species(), w2.gen, obs)               # not square


def test_boxcount_of_the_integrated_grid():
    """The 1024 x 1024 head-on grid integrated on the GPU, its complex set box-counted on the GPU and by
    the oracle from the same mask (the dimensions themselves are reported, not pinned)."""
    w = W.config2()
    print("integrate + BOXCOUNT: 1024x1024 grid", flush=True)
    out = api.integrate_workload(w, counters=False)
    got = api.boxcount(w.system, w.species(), w.gen, out)
    mask = ((out["status"].cpu().numpy() & 1) != 0).reshape(1024, 1024)
    Db, Ds, n_set, n_bnd = R.boxcount(mask)
    print(f"D_boundary={got['D_boundary']:.4f} D_set={got['D_set']:.4f} P(complex)={mask.mean():.4f}", flush=True)
    assert got["N_set"] == n_set and got["N_boundary"] == n_bnd
    assert abs(got["D_boundary"] - Db) <= 1e-12 and abs(got["D_set"] - Ds) <= 1e-12
    assert 0.9 < got["D_boundary"] <= 2.0 and 1.0 < got["D_set"] <= 2.0
    # and the W0 / heating histogram of the same batch against the oracle's
    flat = api.reduce_hist(w.system, w.species(), w.gen, w.n, out)
    hw, hh = (t.cpu().numpy() for t in api.split_hist(flat))
    dE = out["dE_ion"].cpu().numpy()
    st = out["status"].cpu().numpy().astype(np.uint32)
    ref_w, ref_h, cw, ch = R.w0_hist(np.arange(w.n), w, dE, st)
    assert np.array_equal(hw, ref_w)          # one energy: a single bin, well inside the axis
    assert _hist_close(hh, ref_h, ch, 256)


def test_reduce_lifetime_matches_oracle():
    """Synthetic lifetimes spanning the axis (and beyond), a sweep generator for the species slots."""
    w = W.config3()
    n, id0 = 50_001, 123_456
    rng = np.random.default_rng(4)
    t_us = 10.0 ** rng.uniform(-3, 5, n)
    t_first = rng.uniform(0, 1e12, n)
    t_last = t_first + t_us / R.AU_TIME_MICRO
    nb = rng.integers(0, 6, n).astype(np.int32)
    st = (oracle.COMPLEX * (rng.random(n) < 0.7)) | np.where(rng.random(n) < 0.8, R.EXITED, R.TMAX)
    st = st.astype(np.int64)
    obs = {"status": torch.from_numpy(st.astype(np.int32)).to(DEV), "n_bounce": torch.from_numpy(nb).to(DEV),
           "dE_ion": torch.zeros(n, dtype=torch.float64, device=DEV),
           "t_bounce_first": torch.from_numpy(t_first).to(DEV), "t_bounce_last": torch.from_numpy(t_last).to(DEV)}
    print(f"reduce LIFETIME: config3 generator, n={n}, id0={id0}", flush=True)
    flat = api.reduce_lifetime(w.system, w.species(), w.gen, n, obs, id0=id0)
    h, cens, expo = (t.cpu().numpy() for t in api.split_lifetime(flat))
    _, _, slot, _ = R.sweep_params(np.arange(id0, id0 + n), w)
    ref_h, ref_c, coord = R.lifetime_hist(slot, 5, t_first, t_last, nb, st)
    assert np.array_equal(cens, ref_c)
    for s in range(5):
        assert _hist_close(h[s], ref_h[s], coord[(slot == s) & np.isfinite(coord)], 96), s
        ref_e = R.survival_exponent(ref_h[s], ref_c[s])
        assert abs(expo[s] - ref_e) <= 1e-9 * abs(ref_e), (s, expo[s], ref_e)
