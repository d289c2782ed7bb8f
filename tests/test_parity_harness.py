"""CPU checks of the parity harness itself (tests/_parity.py), with the oracle's FMA twin standing in
for the library: the twin is a legitimate arithmetic variant, so the harness must accept it; a planted
error in one field (on a copy of the twin's outputs, on the CPU) must be caught."""
import numpy as np

import oracle
import workloads as W
from tests import _parity as PT

oracle.build()


def _twin_outputs(P):
    g = PT.as_outputs(oracle.integrate(P, twin=True))
    return {k: np.array(v) for k, v in g.items()}


def test_harness_accepts_the_twin_on_the_grid_and_a_sweep_slice():
    for w, ids, min_direct in ((W.config1(), np.arange(64), 16),
                               (W.config3(), np.arange(1_234_567, 1_234_567 + 300), 100)):
        P = oracle.problems_for(w, ids)
        ref = oracle.integrate(P)
        got = _twin_outputs(P)
        direct, rest, rep = PT.check_parity(P, ref, got, w.name, min_direct=min_direct)
        assert rep["max_bar"] <= PT.MAX_BAR and len(direct) + len(rest) == len(ids)


def test_harness_catches_a_shifted_bounce_time_and_a_wrong_lifetime_distribution():
    w = W.config1()
    P = oracle.problems_for(w, np.arange(64))
    ref = oracle.integrate(P)
    got = _twin_outputs(P)
    direct, spread, rest = PT.classify(P, ref, got)
    i = int(direct[np.argmax(ref["n_bounce"][direct])])
    assert ref["n_bounce"][i] == 1
    bad = dict(got)
    bad["t_bounce_first"] = got["t_bounce_first"].copy()
    bad["t_bounce_first"][i] *= 1.0 + 1e-6
    hits = PT.bounce_time_mismatches(P, ref, bad, direct, spread)
    assert [h[:2] for h in hits] == [(i, "t_bounce_first")]
    # complexes whose lifetimes all collapse to zero: the survival check fails
    flat = dict(got)
    flat["t_bounce_last"] = got["t_bounce_first"].copy()
    flat["status"] = got["status"].copy()
    assert PT.survival_mismatches(ref, flat, rest)
    assert not PT.survival_mismatches(ref, got, rest)


def test_harness_sends_a_trajectory_the_oracle_does_not_fix_to_the_ensemble(monkeypatch):
    """A direct exit whose round-off probes spread by more than MAX_BAR / 10 is compared in ensemble
    (its bar would exceed MAX_BAR) and counts against the few direct exits that may drop out."""
    w = W.config1()
    P = oracle.problems_for(w, np.arange(64))
    ref = oracle.integrate(P)
    got = _twin_outputs(P)
    real = PT.classify
    direct0, spread0, _ = real(P, ref, got)

    def planted(k):
        def cls(P_, ref_, got_, step_rates=None):
            direct, spread, rest = real(P_, ref_, got_, step_rates)
            spread = spread.copy()
            spread[:k] = 2.0 * PT.MAX_BAR / 10.0
            return direct, spread, rest
        return cls

    monkeypatch.setattr(PT, "classify", planted(1))
    direct, rest, rep = PT.check_parity(P, ref, got, "planted-1", min_direct=10)
    assert len(direct) == len(direct0) - 1 and direct0[0] in rest
    assert rep["dropped_direct"] == 1 and rep["max_bar"] <= PT.MAX_BAR
    monkeypatch.setattr(PT, "classify", planted(3))
    try:
        PT.check_parity(P, ref, got, "planted-3", min_direct=10)
    except AssertionError as e:
        assert "dropped" in str(e)
    else:
        raise AssertionError("three of the oracle's direct exits dropped out without failing the bar")
