"""The launch-shape autotuner (api.autotune): it picks among shapes that all give the same bits, chosen
by the main kernel's measured throughput, and its cache round-trips: a second call returns the cached
shape without timing anything, and an unreadable cache file is ignored."""
import json

import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_15117_amd import api  # noqa: E402

SHAPE_KEYS = {"block", "refill_every", "blocks_per_cu", "step_budget"}


def _bits(t):
    return t.view(torch.int64) if t.dtype == torch.float64 else t.to(torch.int64)


def _same(a, b):
    for k in a:
        assert torch.equal(_bits(a[k]), _bits(b[k])), k


def test_autotuned_shape_gives_the_same_bits_and_the_cache_round_trips(tmp_path):
    w = W.config1()
    cache = str(tmp_path / "tune.json")
    print("autotune: 8x8 grid, 8 candidates", flush=True)
    best = api.autotune(w, n=64, cache=cache, blocks=(64, 256), refills=(1, 16), blocks_per_cu=(0, 1),
                        step_budget=300, verbose=True)
    assert set(best) == SHAPE_KEYS and best["step_budget"] == 300
    ref = api.integrate_workload(w, counters=True, y_final=True)
    got = api.integrate_workload(w, counters=True, y_final=True, **best)
    _same(ref, got)
    data = json.load(open(cache))
    key = f"{w.name}:64:300"
    assert len(data[key]["candidates"]) == 8 and data[key]["rhs_per_s"] > 0
    # a second call answers from the cache (the marker value below was never timed)
    data[key]["block"] = 192
    json.dump(data, open(cache, "w"))
    assert api.autotune(w, n=64, cache=cache, step_budget=300) == dict(best, block=192)
    # an unreadable cache is ignored and rewritten
    open(cache, "w").write("{not json")
    third = api.autotune(w, n=64, cache=cache, blocks=(64,), refills=(4,), blocks_per_cu=(0,), step_budget=300)
    assert third == {"block": 64, "refill_every": 4, "blocks_per_cu": 0, "step_budget": 300}
    assert f"{w.name}:64:300" in json.load(open(cache))


def test_autotune_on_a_stream_sample():
    w = W.config5()
    print("autotune: 2^16 ids of the stream", flush=True)
    best = api.autotune(w, n=1 << 16, id0=12_345, blocks=(128, 256), refills=(1, 4), blocks_per_cu=(0,))
    assert set(best) == SHAPE_KEYS and best["block"] in (128, 256) and best["refill_every"] in (1, 4)
    ref = api.integrate_workload(w, n=4096, id0=777, counters=True, y_final=True)
    got = api.integrate_workload(w, n=4096, id0=777, counters=True, y_final=True, **best)
    _same(ref, got)
