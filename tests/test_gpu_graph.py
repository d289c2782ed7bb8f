"""A persistent-kernel pass (counter reset, setup, refill kernel, tail, observables) and the
histogram reduction captured in a HIP graph: every replay gives the eager result bit for bit.  The
graph holds kernels and stream-ordered allocations only (counters are cleared by a kernel, not a
memset); the replays are separated by eager work of the program and synchronisations."""
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)


def test_graph_replays_match_eager():
    w = W.config1()
    n, id0 = 64, 0
    print(f"graph: 8x8 head-on grid, n={n}", flush=True)
    eager = api.integrate_workload(w, n=n, id0=id0, counters=False)
    cells_eager = api.reduce_hist(w.system, w.species(), w.gen, n, eager, id0=id0)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in eager.items()}
    out = api.alloc_obs(n, DEV, counters=False)
    cells = torch.zeros_like(cells_eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm the pools on the capturing stream's side
        api.integrate_workload(w, n=n, id0=id0, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.integrate_workload(w, n=n, id0=id0, out=out)
        api.reduce_hist(w.system, w.species(), w.gen, n, out, id0=id0, out=cells)
    for r in range(3):
        for v in out.values():             # eager work between replays: poison the outputs
            v.fill_(-1)
        cells.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"graph replay {r}", flush=True)
        for k in ref:
            assert torch.equal(out[k], ref[k]), (r, k)
        assert torch.equal(cells, cells_eager), r
    hw, hh = api.split_hist(cells)
    assert float(hw[..., 0].sum()) == n and float(hh.sum()) == n
