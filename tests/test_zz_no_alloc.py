"""iat_integrate_noalloc (the library's fixed workspace) against iat_integrate (a workspace allocated
per call).  Both run the same kernels, so every output of every trajectory must carry the same bits.
Two calls in a row on one GPU, the second with a smaller batch, so the second runs over what the
first left in the fixed array; small step budgets send most trajectories through the four-lane tail
and the solo level, whose continuation records live in that array."""
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)


def _bits(t):
    return t.view(torch.int64) if t.dtype == torch.float64 else t.to(torch.int64)


def _compare(w, n, id0, **launch):
    print(f"noalloc: {w.name} n={n} id0={id0} {launch}", flush=True)
    s_ref, s_got = api.new_stats(), api.new_stats()
    ref = api.integrate_workload(w, n=n, id0=id0, y_final=True, counters=True, stats=s_ref, **launch)
    out = api.alloc_obs(n, DEV, y_final=True, counters=True)
    for v in out.values():           # poison: an output the call does not write shows up
        v.fill_(-7)
    got = api.integrate_workload(w, n=n, id0=id0, out=out, stats=s_got, noalloc=True, **launch)
    torch.cuda.synchronize()
    for k in ref:
        same = torch.equal(_bits(ref[k]), _bits(got[k]))
        assert same, (k, int((_bits(ref[k]) != _bits(got[k])).sum()))
    a, b = s_ref.cpu().tolist(), s_got.cpu().tolist()
    # RHS, accepted, rejected, finished, useful slots, tail and solo counts (issued slots depend on
    # which trajectories shared a wave)
    for j in (0, 1, 2, 3, 5, 6, 7, 8, 9):
        assert a[j] == b[j], (j, a, b)
    print(f"noalloc: identical; finished in the tail {b[7]}, in the solo level {b[9]}", flush=True)
    return b


def test_noalloc_matches_integrate_twice_second_smaller():
    w = W.config1()
    b1 = _compare(w, 64, 0, step_budget=300, tail_budget=600)
    assert b1[7] + b1[9] > 0 and b1[9] > 0           # the fixed array's continuation records were used
    b2 = _compare(w, 40, 24, step_budget=150, tail_budget=2000, block=128, refill_every=4)
    assert b2[7] + b2[9] > 0
    # the plain kernel over the fixed work buffer
    _compare(w, 33, 5, kernel="plain")
