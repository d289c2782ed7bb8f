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


@pytest.mark.parametrize("which", ["sweep", "stream"])
def test_run_chunks_graph_replays_match_eager_chunks(which):
    """The chunked driver with graph replay: per stream one captured call sequence (integration and
    reductions) whose first id is read from a device scalar, replayed for every later full chunk.
    Per-cell sums, both W0 histograms and the counters must equal those of eager calls bit for bit
    (each chunk's work is integers and fixed-order sums), over several replays per stream and a
    shorter last chunk."""
    w = W.config3() if which == "sweep" else W.config5()
    w.system.max_steps = 200_000
    n, chunk = 5 * 6000 + 1234, 6000
    kw = dict(n=n, chunk=chunk, n_streams=2, cells=which == "sweep", hist=True, hist_bound=which == "stream")
    print(f"graph: run_chunks {which}, n={n}, chunk={chunk}", flush=True)
    s_e, s_g = api.new_stats(), api.new_stats()
    eager = api.run_chunks(w, stats=s_e, **kw)
    torch.cuda.synchronize()
    replay = api.run_chunks(w, stats=s_g, graph=True, **kw)
    torch.cuda.synchronize()
    assert replay["graphs"][0] is not None and replay["graphs"][1] is not None
    for key in ("cells", "hist", "hist_bound"):
        if key in eager:
            assert torch.equal(eager[key], replay[key]), key
    a, b = s_e.cpu().tolist(), s_g.cpu().tolist()
    for j in (0, 1, 2, 3, 5, 6, 7, 8, 9, 10):
        assert a[j] == b[j], (j, a, b)
    hw, _ = api.split_hist(replay["hist"])
    assert float(hw[..., 0].sum()) == n
