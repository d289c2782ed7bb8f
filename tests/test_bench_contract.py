"""The benchmark's output contract, checked on the recorded bench lines in profiles/ (no GPU): every
key the one-line JSON must carry, roofline and CPU-baseline objects included, and the traffic lookup
that only reports counters taken on the current kernel sources."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORDS = ["bench_yb_rb_grid1024.json", "bench_sweep_5species_225cells.json", "bench_stream_li_k_cs_1e8.json",
           "bench_fig3_thermal_5species.json", "bench_fig4_energy_sweep_5species.json"]


@pytest.mark.parametrize("name", RECORDS)
def test_recorded_bench_lines_follow_the_contract(name):
    d = json.load(open(os.path.join(ROOT, "profiles", name)))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["dtype"] == "f64" and d["data"] == "synthetic" and d["higher_is_better"] is True
    assert d["vs_baseline"] is None and d["value"] > 0 and "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.FP64_PEAK_TFLOPS
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert "traffic" in r
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path):
    tr = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    tr["sources"] = bench.sources_digest()
    p = tmp_path / "t.json"
    p.write_text(json.dumps(tr))
    assert tr["workloads"], "no workload in the traffic record"
    for wl, entry in tr["workloads"].items():
        for k, rec in entry["kernels"].items():
            assert bench.traffic_bytes(str(p), wl, k) == rec["bytes_per_launch"]
        assert bench.traffic_bytes(str(p), wl, "no_such_kernel") is None
    assert bench.traffic_bytes(str(p), "another_workload", "k_integrate_tail") is None
    wl = next(iter(tr["workloads"]))
    tr["sources"] = "0" * 64
    p.write_text(json.dumps(tr))
    assert bench.traffic_bytes(str(p), wl, "k_integrate_tail") is None
    assert bench.traffic_bytes(str(tmp_path / "missing.json"), wl, "k_integrate_tail") is None
    # the older one-workload layout is still read
    old = {"workload": "w", "sources": bench.sources_digest(), "kernels": {"k": {"bytes_per_launch": 7}}}
    p.write_text(json.dumps(old))
    assert bench.traffic_bytes(str(p), "w", "k") == 7


@pytest.mark.parametrize("name", RECORDS)
def test_roofline_names_the_dominant_kernel_of_the_three(name):
    """The refill pipeline has three integration kernels (persistent, four-lane tail, solo); each gets its
    own achieved FLOP rate from its own RHS count and event-timed duration, and the roofline object is
    the longest-running one."""
    d = json.load(open(os.path.join(ROOT, "profiles", name)))
    ks = {k["kernel"]: k for k in d["kernels"]}
    assert {"k_integrate_persistent", "k_integrate_tail", "k_integrate_solo"} <= set(ks)
    for k in ks.values():
        assert abs(k["flop_per_launch"] - bench.FLOP_PER_RHS * k["rhs_per_launch"]) <= 1e-6 * k["flop_per_launch"]
        assert abs(k["achieved"] - k["flop_per_launch"] / (k["avg_launch_ms"] * 1e-3) / 1e12) <= 1e-9 * k["achieved"]
    dom = max(ks.values(), key=lambda k: k["avg_launch_ms"])
    r = d["roofline"]
    assert r["kernel"] == dom["kernel"] and r["achieved"] == dom["achieved"] and r["traffic"] == dom["traffic"]


def test_grid_record_carries_the_solo_phase_and_its_traffic():
    d = json.load(open(os.path.join(ROOT, "profiles", "bench_yb_rb_grid1024.json")))
    assert set(d["phases_ms"]) == {"setup", "main", "tail", "solo", "observe"}
    assert 0 < d["solo_trajectories"] < d["tail_trajectories"] < d["config"]["trajectories"]
    # that line was taken while the PMC counters matched its kernel sources
    assert isinstance(d["roofline"]["traffic"], int) and d["roofline"]["traffic"] > 0
    cp = d["critical_path"]
    assert abs(cp["tail_ms"] - d["phases_ms"]["tail"] - d["phases_ms"]["solo"]) < 1e-6 * cp["tail_ms"]


@pytest.mark.parametrize("name", ["bench_stream_li_k_cs_1e8.json", "bench_stream_li_k_cs_1e8_profiled.json"])
def test_stream_headline_record(name):
    """The default line: the 1e8 Li/K/Cs stream, one step = one 2^22-id chunk, the timed chunks integrated
    as one batch; refill against plain on a matched chunk; the critical path of the batch's tail."""
    d = json.load(open(os.path.join(ROOT, "profiles", name)))
    c = d["config"]
    assert c["workload"] == "stream_li_k_cs_1e8" and c["trajectories_in_stream"] == 100_000_000
    assert c["chunk"] == 1 << 22 and d["steps"] == 20
    lo, hi = c["timed_ids"]
    assert hi - lo == d["steps"] * c["chunk"]
    assert abs(d["value"] - (hi - lo) / (d["ms_per_step"] * d["steps"] * 1e-3)) < 1e-6 * d["value"]
    assert set(c["launch"]) == {"block", "refill_every", "blocks_per_cu", "step_budget"}
    ph = d["phases_ms"]
    assert set(ph) == {"setup", "main", "tail", "solo", "observe"}
    assert sum(ph.values()) <= d["ms_per_step"] * d["steps"] * 1.001
    assert 0 < d["solo_trajectories"] < d["tail_trajectories"] < hi - lo
    cp = d["critical_path"]
    assert abs(cp["tail_ms"] - ph["tail"] - ph["solo"]) < 1e-6 * cp["tail_ms"]
    assert 0.5 < cp["frac_of_tail"] <= 1.0
    assert cp["trajectory_id"] == d["longest_trajectory"]["id"] and lo <= cp["trajectory_id"] < hi
    # refill against plain on the same chunk
    assert d["plain"]["sample"].startswith("one chunk") and d["speedup_vs_plain"] > 1.0
    assert set(d["p_complex_by_species"]) == {"Li6", "K40", "Cs133"}


def test_stream_trace_agrees_with_its_line():
    """profiles/k_integrate__stream_li_k_cs_1e8.md lists the timed batch's three dispatches from the
    kernel trace; each equals the phase the profiled bench line timed with HIP events."""
    import re
    d = json.load(open(os.path.join(ROOT, "profiles", "bench_stream_li_k_cs_1e8_profiled.json")))
    md = open(os.path.join(ROOT, "profiles", "k_integrate__stream_li_k_cs_1e8.md")).read()
    got = {}
    for m in re.finditer(r"\| \d+ \| `k_integrate_(persistent|tail|solo)<false>`[^|]*\| ([\d,.]+) \|", md):
        got[m.group(1)] = float(m.group(2).replace(",", ""))
    assert set(got) == {"persistent", "tail", "solo"}
    ph = d["phases_ms"]
    for k, phase in (("persistent", "main"), ("tail", "tail"), ("solo", "solo")):
        assert abs(got[k] - ph[phase]) < 0.1, (k, got[k], ph[phase])
    assert d["roofline"]["kernel"] == "k_integrate_solo"
    assert abs(d["roofline"]["avg_launch_ms"] - got["solo"]) < 0.1
