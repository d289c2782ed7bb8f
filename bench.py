"""Throughput benchmark: trajectories/s and RK stages/s of the persistent-refill kernel against the
plain one-launch-per-batch kernel, FP64 at rtol 1e-10, with the achieved fraction of the MI355X
FP64 vector peak and the CPU oracle timed on the host as a baseline.

Default workload: the 1e8-trajectory streaming sweep (Yb+ with Li6, K40 and Cs133, E log-uniform over
1 uK - 1 mK, q_x uniform over 0.05 - 0.35, De log-uniform over 0.01 - 100 K), keeping only on-device
histograms.  One "step" = one chunk of 2^22 ids of that stream: the K timed chunks (after W warm-up
chunks) are integrated as one batch by one iat_integrate call, whose refill queue runs over all of
them, and reduced to the W0 and heating histograms on the device.  Other workloads: one step = one
iat_integrate call over the whole workload.  Inputs are generated on the device from trajectory ids,
so nothing crosses PCIe inside the timed region.

    python bench.py [--steps K] [--warmup W] [--workload stream|grid1024|grid8|sweep|thermal|fig4|tangent|adjoint]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6           # MI355X dense FP64 vector peak (AMD spec)
# algorithmic FLOP, counting a division, a cosine or a power as one: 38 per right-hand-side evaluation
# and 966 per attempted Dormand-Prince step (six evaluations plus the stage sums, the error norm and
# the step control), i.e. 161 per evaluation
FLOP_PER_RHS = 161
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 chunks for stream, 3 passes otherwise)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stream",
                    choices=["grid1024", "grid8", "sweep", "stream", "stream-chunks", "thermal", "fig4", "tangent",
                             "adjoint"],
                    help="stream (default): the 1e8-trajectory Li/K/Cs sweep keeping only histograms, one step = "
                         "one 2^22-id chunk; stream-chunks: the same workload in chunks over several streams, one "
                         "step = the whole 1e8; grid1024: the 1024^2 head-on grid (one batch); sweep: the "
                         "1.2e7-trajectory 225-cell sweep with per-cell reductions; tangent / adjoint: the 512^2 "
                         "differentiation grid")
    ap.add_argument("--autotune", default="", metavar="CACHE.json",
                    help="cache file of the launch-shape autotuner (stream: it always runs, on the warm-up "
                         "ids; other workloads: only with this option)")
    ap.add_argument("--no-autotune", action="store_true", help="stream: keep the default launch shape")
    ap.add_argument("--step-budget", type=int, default=0,
                    help=f"stream: attempted steps before a trajectory leaves the one-lane kernel (0: "
                         f"{STREAM_STEP_BUDGET:,})")
    ap.add_argument("--graph", action="store_true",
                    help="chunked workloads (not thermal): replay one captured HIP graph per stream for the "
                         "later chunks instead of launching every chunk eagerly")
    ap.add_argument("--chunk", type=int, default=0, help="ids per chunk (default: the job split evenly over the streams)")
    ap.add_argument("--streams", type=int, default=2, help="streams the chunks are spread over")
    ap.add_argument("--n", type=int, default=0, help="run only the first N ids of the workload")
    ap.add_argument("--kernel", default="persistent", choices=["persistent", "plain"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--refill-every", type=int, default=0)
    ap.add_argument("--inflight", type=int, default=3,
                    help="also time this many whole passes in flight at once, one per stream (0: skip)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison run")
    ap.add_argument("--no-critical-path", action="store_true",
                    help="skip the longest trajectory's latency bound on the tail kernel")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--latency", type=int, default=-1, metavar="ID",
                    help="only time trajectory ID of the workload alone (four-lane tail and one-lane forms) "
                         "and print the per-step latency")
    ap.add_argument("--max-steps", type=int, default=0, help="accepted-step cap for --latency (0: the default)")
    ap.add_argument("--compare-solo", type=int, default=0, metavar="ROUNDS",
                    help="only time whole passes with the solo level (default tail budget) and without it "
                         "(tail budget -1), alternating, ROUNDS of each: the GPU clock under a lone wave "
                         "drifts between runs, so the two are compared pass by pass")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    return ap.parse_args()


def workload(name):
    import workloads as W
    return {"grid1024": W.config2, "grid8": W.config1, "sweep": W.config3, "stream": W.config5,
            "stream-chunks": W.config5, "thermal": W.fig3_thermal, "fig4": W.fig4_energy, "tangent": W.config4,
            "adjoint": W.config4}[name]()


# algorithmic FLOP of the differentiation (same canonical count as FLOP_PER_RHS): per attempted step of the
# primal 966; per tangent column and step 6 x 35 + 552 = 762; the adjoint per committed step recomputes
# the step (966) and applies one transposed column (762), after a checkpointing forward pass (966).
FLOP_PER_STEP, FLOP_PER_COLUMN_STEP = 966, 762


def main_diff(args):
    import numpy as np
    import torch
    from paper_2509_15117_amd import api
    torch.cuda.set_device(0)
    w = workload(args.workload)
    n = args.n or w.n
    cur = torch.cuda.current_stream()
    obs = api.integrate_workload(w, n=n, counters=True)       # primal counts (and the adjoint's input)
    torch.cuda.synchronize()
    rhs = float(obs["n_rhs"].sum())
    acc = float(obs["n_accept"].sum())
    steps = rhs / 6.0
    print(f"[bench] primal: {rhs:.3e} RHS evaluations", file=sys.stderr, flush=True)
    times = []
    for k in range(args.warmup + args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        if args.workload == "tangent":
            api.tangent(w.system, w.species(), w.gen, n)
            flop = steps * (FLOP_PER_STEP + 14 * FLOP_PER_COLUMN_STEP)
            kname = "k_tangent"
        else:
            g = torch.from_numpy(np.random.default_rng(k).normal(size=(n, 3))).to("cuda")
            api.adjoint(w.system, w.species(), w.gen, n, obs, g)
            flop = steps * FLOP_PER_STEP + acc * (FLOP_PER_STEP + FLOP_PER_COLUMN_STEP)
            kname = "k_adj_forward + k_adj_reverse"
        e1.record(cur)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        print(f"[bench] {args.workload} pass {k + 1}: {t:.2f} s", file=sys.stderr, flush=True)
        if k >= args.warmup:
            times.append(t)
    secs = sum(times) / len(times)
    tf = flop / secs / 1e12
    out = {
        "metric": "trajectories/s + RK stages/s (FP64, rtol 1e-10): refill kernel vs plain, % FP64 peak",
        "value": n / secs, "unit": "trajectories/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": secs * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name + ("" if args.workload == "tangent" else "_adjoint"), "trajectories": n,
                   "what": ("tangent-linear: 12x12 stability matrix + q_x, De columns, FTLE"
                            if args.workload == "tangent" else
                            "discrete adjoint of (angle, q, dE) w.r.t. (theta, phi, E, q_x, De), checkpoints "
                            "every 256 committed steps")},
        "primal_rk_stages": rhs,
        "roofline": {"bound": "alu", "kernel": kname, "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / FP64_PEAK_TFLOPS, "traffic": None, "avg_launch_ms": secs * 1e3,
                     "flop_per_launch": flop},
    }
    print(json.dumps(out), flush=True)


def chunked_job(api, torch, w, n, args, stats, kernel):
    """One pass over ids [0, n) in chunks on several streams, reductions on the device; HIP events on the
    current stream, which joins the side streams at the end of the pass."""
    # default: one chunk per stream, so every chunk's main kernel and long-lived tail run concurrently
    # (HBM holds a 1e8-trajectory job: ~240 B of work buffer and outputs per trajectory)
    chunk = args.chunk or -(-n // max(1, args.streams))
    cur = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    t0 = time.perf_counter()

    def progress(c, nc):
        print(f"[bench] {kernel}: chunk {c + 1}/{nc} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)

    res = api.run_chunks(w, n=n, chunk=chunk, n_streams=args.streams, kernel=kernel, graph=args.graph,
                         cells=args.workload in ("sweep", "thermal"),
                         hist=args.workload in ("stream", "stream-chunks", "fig4"), stats=stats,
                         progress=progress)
    e1.record(cur)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, res, chunk


def kernel_profile(api, torch, w, n, kernel):
    """Event-timed phases of one single-stream call on ids [0, n): the per-kernel roofline figures."""
    import ctypes
    stats = api.new_stats()
    out = api.alloc_obs(n, torch.device("cuda", 0), counters=False)
    ms = api.phase_ms()
    api.integrate_workload(w, n=n, out=out, stats=stats, kernel_ms=ms, kernel=kernel)
    s = stats.cpu().tolist()
    return list(ms), s


def main_chunked(args):
    import torch
    from paper_2509_15117_amd import api
    torch.cuda.set_device(0)
    w = workload(args.workload)
    n = args.n or w.n
    stats = api.new_stats()
    for _ in range(args.warmup):
        chunked_job(api, torch, w, n, args, None, args.kernel)
    secs, res = 0.0, None
    for k in range(args.steps):
        stats_k = stats if k == 0 else None
        t, res, chunk = chunked_job(api, torch, w, n, args, stats_k, args.kernel)
        secs += t
        print(f"[bench] pass {k + 1}/{args.steps}: {t:.2f} s", file=sys.stderr, flush=True)
    K = args.steps
    s = stats.cpu().tolist()
    traj_s = n * K / secs
    stages_s = s[0] / (secs / K)
    # per-kernel figures from one event-timed single-stream call on the first chunk
    print(f"[bench] kernel profile of the first {min(n, chunk)} ids", file=sys.stderr, flush=True)
    ms, ks = kernel_profile(api, torch, w, min(n, chunk), args.kernel)
    print(f"[bench] phases ms {[round(x, 1) for x in ms]}", file=sys.stderr, flush=True)
    main_name = "k_integrate_persistent" if args.kernel == "persistent" else "k_integrate_plain"
    kernels = []
    for name, secs_k, rhs in ((main_name, ms[1] / 1e3, ks[0] - ks[6] - ks[8]), ("k_integrate_tail", ms[2] / 1e3, ks[6]),
                              ("k_integrate_solo", ms[3] / 1e3, ks[8])):
        if secs_k > 0:
            tf = FLOP_PER_RHS * rhs / secs_k / 1e12
            kernels.append({"kernel": name, "avg_launch_ms": secs_k * 1e3, "rhs_per_launch": rhs,
                            "flop_per_launch": FLOP_PER_RHS * rhs, "achieved": tf, "frac": tf / FP64_PEAK_TFLOPS,
                            "traffic": traffic_bytes(args.traffic_file, w.name, name),
                            "launch": f"first chunk of {min(n, chunk)} ids, one stream"})
    dom = max(kernels, key=lambda k: k["avg_launch_ms"])
    out = {
        "metric": "trajectories/s + RK stages/s (FP64, rtol 1e-10): refill kernel vs plain, % FP64 peak",
        "value": traj_s, "unit": "trajectories/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "trajectories": n, "chunk": chunk, "streams": args.streams,
                   "kernel": args.kernel, "rtol": w.system.rtol, "atol": w.system.atol,
                   "reductions": ("per-cell sums" if args.workload in ("sweep", "thermal")
                                  else "W0 and heating histograms")},
        "rk_stages_per_s": stages_s, "accepted_steps_per_s": s[1] / (secs / K),
        "fp64_frac_peak": FLOP_PER_RHS * stages_s / (FP64_PEAK_TFLOPS * 1e12),
        "active_lane_fraction": s[5] / max(s[4], 1),
        "roofline": {"bound": "alu", "kernel": dom["kernel"], "achieved": dom["achieved"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": dom["frac"], "traffic": dom["traffic"],
                     "avg_launch_ms": dom["avg_launch_ms"], "flop_per_launch": dom["flop_per_launch"]},
        "kernels": kernels,
    }
    if args.workload in ("sweep", "thermal") and res is not None:
        c = res["cells"].cpu()
        out["p_complex_range"] = [float((c[:, 1] / c[:, 0]).min()), float((c[:, 1] / c[:, 0]).max())]
    if not args.no_plain and args.kernel != "plain":
        # plain vs refill on the same sample: the first 2^20 ids, one chunk per stream
        m = min(n, 1 << 20)
        sub = argparse.Namespace(**vars(args))
        sub.chunk = max(1, m // max(1, args.streams))
        tp, _, _ = chunked_job(api, torch, w, m, sub, None, "plain")
        tr, _, _ = chunked_job(api, torch, w, m, sub, None, "persistent")
        out["plain"] = {"trajectories_per_s": m / tp, "sample": f"first {m} ids in {args.streams} chunks",
                        "refill_same_sample": m / tr}
        out["speedup_vs_plain"] = tp / tr
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w.with_n(n), args.cpu_seconds)
    print(json.dumps(out), flush=True)


STREAM_CHUNK = 1 << 22
# step budget of the stream batch: whole batches of 20 chunks took 27.9 s at 10,000 attempted steps,
# 27.0-27.2 s at 20,000 (the library's default), 26.7 s at 40,000 and at 80,000 (a longer one-lane
# phase, a shorter four-lane tail)
STREAM_STEP_BUDGET = 40000


def main_stream(args):
    """The 1e8-trajectory Li/K/Cs stream, one step = one chunk of STREAM_CHUNK ids.  The W warm-up chunks
    (ids [0, W C)) and then the K timed chunks (ids [W C, (W + K) C)) are each integrated as one batch by
    one iat_integrate call (persistent refill over the whole batch; long-lived complexes continue in the
    four-lane tail and the solo level) and reduced on the device to the W0 and heating histograms; only
    those are kept.  Timed with HIP events on the launch stream, bracketed by device synchronisation."""
    import torch
    from paper_2509_15117_amd import api
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = workload("stream")
    C = args.chunk or STREAM_CHUNK
    K, Wu = args.steps, args.warmup
    sp = w.species()
    cur = torch.cuda.current_stream()

    budget = args.step_budget if args.step_budget > 0 else STREAM_STEP_BUDGET
    launch = {"step_budget": budget}

    def batch(n, id0, out, hist, **kw):
        api.integrate(w.system, sp, w.gen, n, id0=id0, out=out, counters=False, **launch, **kw)
        api.reduce_hist(w.system, sp, w.gen, n, out, id0=id0, out=hist)

    n = K * C
    id0 = Wu * C
    out = api.alloc_obs(n, dev, counters=False)
    if Wu > 0:
        m = Wu * C
        print(f"[bench] stream warm-up: {Wu} chunks ({m} ids)", file=sys.stderr, flush=True)
        wo = {k: v[:m] for k, v in out.items()} if m <= n else api.alloc_obs(m, dev, counters=False)
        batch(m, 0, wo, None)
        del wo
    if not args.no_autotune:
        # the main kernel's launch shape, timed on the warm-up range (outside the timed batch): a whole
        # chunk, so that the end of each trial launch is a small part of it, as in the batch
        launch = api.autotune(w, n=min(C, max(id0, 1 << 16)), id0=0, cache=args.autotune or None, step_budget=budget)
        print(f"[bench] autotuned launch {launch}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    hist = torch.zeros(len(w.gen.species) * 2 * 64 + 256, dtype=torch.float64, device=dev)
    stats = api.new_stats()
    ms = api.phase_ms()
    torch.cuda.synchronize()
    print(f"[bench] stream: {K} chunks of {C} ids (ids {id0} .. {id0 + n - 1}) as one batch", file=sys.stderr,
          flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(cur)
    batch(n, id0, out, hist, stats=stats, kernel_ms=ms)
    e1.record(cur)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    secs = e0.elapsed_time(e1) / 1e3
    s = stats.cpu().tolist()
    steps_max, gid_max = api.longest_of(stats.cpu())
    print(f"[bench] stream: {secs:.2f} s ({n / secs:.0f} trajectories/s), phases ms "
          f"{[round(x, 1) for x in ms]}, longest trajectory {gid_max} with {steps_max} attempted steps",
          file=sys.stderr, flush=True)
    kernels = []
    for name, ph, rhs in (("k_integrate_persistent", 1, s[0] - s[6] - s[8]), ("k_integrate_tail", 2, s[6]),
                          ("k_integrate_solo", 3, s[8])):
        secs_k = ms[ph] / 1e3
        if secs_k > 0:
            tf = FLOP_PER_RHS * rhs / secs_k / 1e12
            kernels.append({"kernel": name, "avg_launch_ms": secs_k * 1e3, "rhs_per_launch": rhs,
                            "flop_per_launch": FLOP_PER_RHS * rhs, "achieved": tf, "frac": tf / FP64_PEAK_TFLOPS,
                            "traffic": traffic_bytes(args.traffic_file, w.name, name),
                            "launch": f"one launch over the {n} ids of the timed batch"})
    dom = max(kernels, key=lambda k: k["avg_launch_ms"])
    h = api.split_hist(hist)[0].cpu()
    p_cx = [float(h[k, :, 1].sum() / max(h[k, :, 0].sum(), 1.0)) for k in range(h.shape[0])]
    out_line = {
        "metric": "trajectories/s + RK stages/s (FP64, rtol 1e-10): refill kernel vs plain, % FP64 peak",
        "value": n / secs, "unit": "trajectories/s", "n_gpus": 1, "steps": K, "warmup": Wu,
        "ms_per_step": secs * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "trajectories_in_stream": w.n, "chunk": C, "timed_ids": [id0, id0 + n],
                   "step": "one chunk of 2^22 ids; the K timed chunks integrated as one batch (one refill queue) "
                           "and reduced to on-device histograms", "kernel": "persistent",
                   "launch": launch or "default",
                   "rtol": w.system.rtol, "atol": w.system.atol, "max_steps": w.system.max_steps,
                   "reductions": "W0 (complex/total over log10(E/W0), per species) and heating histograms"},
        "rk_stages_per_s": s[0] / secs, "accepted_steps_per_s": s[1] / secs,
        "fp64_frac_peak": FLOP_PER_RHS * s[0] / secs / (FP64_PEAK_TFLOPS * 1e12),
        "active_lane_fraction": s[5] / max(s[4], 1),
        "roofline": {"bound": "alu", "kernel": dom["kernel"], "achieved": dom["achieved"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": dom["frac"], "traffic": dom["traffic"],
                     "avg_launch_ms": dom["avg_launch_ms"], "flop_per_launch": dom["flop_per_launch"]},
        "kernels": kernels,
        "phases_ms": {"setup": ms[0], "main": ms[1], "tail": ms[2], "solo": ms[3], "observe": ms[4]},
        "reduce_ms": secs * 1e3 - sum(ms),
        "tail_trajectories": s[7] + s[9], "solo_trajectories": s[9],
        "longest_trajectory": {"id": gid_max, "attempted_steps": steps_max},
        "p_complex_by_species": dict(zip(w.species_names, p_cx)),
        "host_wall_s": wall,
    }
    if not args.no_critical_path and steps_max > 0:
        out_line["critical_path"] = stream_critical_path(api, torch, w, gid_max, steps_max, ms[2] + ms[3])
    if not args.no_plain:
        # refill against plain on one matched chunk: the first timed chunk, each kernel in one call
        res = {}
        for kern in ("plain", "persistent"):
            o = {k: v[:C] for k, v in out.items()}
            st = api.new_stats()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(cur)
            api.integrate(w.system, sp, w.gen, C, id0=id0, out=o, counters=False, kernel=kern, stats=st,
                          **(launch if kern == "persistent" else {}))
            b.record(cur)
            torch.cuda.synchronize()
            t = a.elapsed_time(b) / 1e3
            sk = st.cpu().tolist()
            res[kern] = {"trajectories_per_s": C / t, "rk_stages_per_s": sk[0] / t, "seconds": t,
                         "fp64_frac_peak": FLOP_PER_RHS * sk[0] / t / (FP64_PEAK_TFLOPS * 1e12),
                         "active_lane_fraction": sk[5] / max(sk[4], 1)}
            print(f"[bench] matched chunk ({C} ids from {id0}), {kern}: {t:.2f} s", file=sys.stderr, flush=True)
        out_line["plain"] = dict(res["plain"], sample=f"one chunk of {C} ids from id {id0}")
        out_line["refill_same_chunk"] = res["persistent"]
        out_line["speedup_vs_plain"] = res["plain"]["seconds"] / res["persistent"]["seconds"]
    pk = api.fp64_peak()
    out_line["fp64_peak_measured_tflops"] = pk
    out_line["roofline"]["frac_of_measured_peak"] = out_line["roofline"]["achieved"] / pk
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out_line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out_line), flush=True)


def stream_critical_path(api, torch, w, gid, steps, tail_ms, cap=400_000):
    """The batch cannot end before its longest trajectory (found by the call's stats) has run its steps
    one after another.  A bounded prefix of that trajectory timed alone in the solo kernel gives the
    per-step latency; bound = its attempted steps x that latency, frac = bound / the tail phases."""
    import copy
    wl = copy.deepcopy(w)
    wl.system.max_steps = cap
    ms = api.phase_ms()
    r = api.integrate_workload(wl, n=1, id0=gid, counters=True, kernel="persistent", step_budget=1, tail_budget=1,
                               kernel_ms=ms)
    s1 = int(r["n_accept"].item() + r["n_reject"].item()) - 2
    us = ms[3] * 1e3 / max(s1, 1)
    bound_ms = steps * us / 1e3
    print(f"[bench] longest trajectory {gid}: {steps} attempted steps, {us:.3f} us per step alone", file=sys.stderr,
          flush=True)
    return {"trajectory_id": gid, "attempted_steps": steps, "lone_us_per_step": us, "lone_sample_steps": s1,
            "bound_ms": bound_ms, "tail_ms": tail_ms, "frac_of_tail": bound_ms / tail_ms if tail_ms > 0 else None}


def pipelined(api, torch, w, passes, launch):
    """`passes` independent whole passes over the workload, each on its own stream (default priority),
    all in flight at once: while one pass's long-lived complexes run out in its tail kernel, the
    others' main kernels fill the GPU.  The throughput of a stream of such jobs, not of one."""
    dev = torch.device("cuda", 0)
    outs = [api.alloc_obs(w.n, dev, counters=False) for _ in range(passes)]
    streams = [torch.cuda.Stream(device=dev) for _ in range(passes)]
    cur = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for st in streams:
        st.wait_stream(cur)
    for p, st in enumerate(streams):
        with torch.cuda.stream(st):
            api.integrate_workload(w, out=outs[p], **launch)
    for st in streams:
        cur.wait_stream(st)
    e1.record(cur)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    print(f"[bench] {passes} passes in flight: {secs:.2f} s", file=sys.stderr, flush=True)
    return {"passes": passes, "streams": passes, "seconds": secs, "trajectories_per_s": passes * w.n / secs,
            "what": "independent whole passes in flight at once, one per stream; value stays the one-pass figure"}


def critical_path(api, torch, w, tail_ms, budget=20000, cap=400_000):
    """The tail phase (four-lane tail kernel, then the solo kernel) is latency-bound: it cannot end
    before the longest trajectory has run its steps beyond the budget, one after another, at the
    per-step latency of a trajectory alone in its wave.  One more pass with step counters finds that
    trajectory; a bounded prefix of it (`cap` accepted steps) timed alone in the solo kernel gives the
    latency.  frac = that bound / the tail phase's duration."""
    import copy
    import ctypes
    o = api.integrate_workload(w, counters=True)
    steps = o["n_accept"].to(torch.int64) + o["n_reject"].to(torch.int64)
    i = int(torch.argmax(steps).item())
    n_steps = int(steps[i].item())
    wl = copy.deepcopy(w)
    wl.system.max_steps = cap
    ms = api.phase_ms()
    # one attempted step in the main kernel, one in the four-lane tail, the rest in the solo kernel
    r = api.integrate_workload(wl, n=1, id0=i, counters=True, kernel="persistent", step_budget=1, tail_budget=1,
                               kernel_ms=ms)
    s1 = int(r["n_accept"].item() + r["n_reject"].item()) - 2
    us = ms[3] * 1e3 / max(s1, 1)
    bound_ms = max(n_steps - budget, 0) * us / 1e3
    print(f"[bench] longest trajectory {i}: {n_steps} attempted steps, {us:.3f} us per step alone", file=sys.stderr,
          flush=True)
    return {"trajectory_id": i, "attempted_steps": n_steps, "lone_us_per_step": us,
            "lone_sample_steps": s1, "tail_bound_ms": bound_ms, "tail_ms": tail_ms,
            "frac": bound_ms / tail_ms if tail_ms > 0 else None}


def timed_runs(api, torch, w, out, stats, steps, warmup, **launch):
    """Warm up, then time `steps` full passes with HIP events on the launch stream.  Each pass also
    reports its phase durations (setup, main kernel, tail kernel, observables), which the library
    measures with HIP events recorded on the same stream between its kernels."""
    import ctypes
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        api.integrate_workload(w, out=out, **launch)
    torch.cuda.synchronize()
    stats.zero_()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    phases = []
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        ms = api.phase_ms()
        api.integrate_workload(w, out=out, stats=stats, kernel_ms=ms, **launch)
        phases.append(list(ms))
        print(f"[bench] pass {k + 1}/{steps} ({launch.get('kernel')}): phases ms "
              f"{[round(x, 3) for x in ms]}", file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    s = stats.cpu().tolist()
    avg = [sum(p[j] for p in phases) / len(phases) for j in range(len(phases[0]))]
    return dict(total_s=total_ms / 1e3, wall_s=wall, phase_ms=avg, rhs=s[0], acc=s[1], rej=s[2],
                done=s[3], issued=s[4], useful=s[5], tail_rhs=s[6], tail_done=s[7], solo_rhs=s[8], solo_done=s[9])


def cpu_baseline(w, target_s):
    """The oracle on a strided sample of the same ids, all host threads."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # size the sample to ~target_s of wall time: grow a calibration sample until it takes a second
    # (small samples are dominated by their longest trajectory), then scale
    n_cal = 256
    while True:
        ids = np.linspace(0, w.n - 1, n_cal).astype(np.int64)
        t = time.perf_counter()
        oracle.integrate(oracle.problems_for(w, ids), threads)
        dt = max(time.perf_counter() - t, 1e-3)
        if dt >= 1.0 or n_cal >= w.n or n_cal * 4 * 1.0 / dt > 400_000:
            break
        n_cal *= 4
    n = int(min(max(n_cal, n_cal * target_s / dt), 400_000, w.n))
    ids = np.linspace(0, w.n - 1, n).astype(np.int64)
    P = oracle.problems_for(w, ids)
    t = time.perf_counter()
    R = oracle.integrate(P, threads)
    el = time.perf_counter() - t
    # one thread on the first ids of the same sample, about a quarter of the all-thread time; the
    # heavy-tailed costs make RK stages/s the comparable figure between the two
    m = max(1, min(n, int(n * 0.25 / max(threads, 1))))
    t = time.perf_counter()
    R1 = oracle.integrate(P[:m], 1)
    el1 = time.perf_counter() - t
    return dict(value=n / el, unit="trajectories/s", cores=threads, kind="oracle",
                sample=f"{n} evenly strided ids of the {w.n}-trajectory workload, {el:.1f} s",
                rk_stages_per_s=float(R["n_rhs"].sum()) / el,
                single_core={"trajectories_per_s": m / el1, "rk_stages_per_s": float(R1["n_rhs"].sum()) / el1,
                             "sample": f"the first {m} ids of that sample, one thread, {el1:.1f} s"},
                host=host_description(), build="gcc -O3 -fno-fast-math -ffp-contract=off -fopenmp")


def host_description():
    """CPU model, logical CPUs and the CPUs this process may run on (lscpu when present)."""
    import shutil
    import subprocess
    d = {"logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}
    if shutil.which("lscpu"):
        try:
            txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
            for line in txt.splitlines():
                k, _, v = line.partition(":")
                if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                                 "CPU max MHz", "Hypervisor vendor"):
                    d[k.strip()] = v.strip()
        except (OSError, subprocess.SubprocessError):
            pass
    return d


def sources_digest():
    """sha256 over the sources of the integration kernels (names which build the counters were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("iat_device.h", "iat_host.h", "iat_integrate.hip"):
        h.update(f.encode())
        h.update(open(os.path.join(ROOT, "paper_2509_15117_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_bytes(path, workload_name, kernel):
    """HBM bytes per launch of `kernel` from PMC runs (FETCH_SIZE + WRITE_SIZE, scaled by a copy-kernel
    calibration), or None when absent or taken on other sources.  The file holds one entry per workload
    under "workloads" (or, in the older layout, one workload at the top level)."""
    try:
        tr = json.load(open(path))
    except (OSError, ValueError):
        return None
    if tr.get("sources") != sources_digest():
        return None
    entry = tr.get("workloads", {}).get(workload_name)
    if entry is None and tr.get("workload") == workload_name:
        entry = tr
    if entry is None:
        return None
    return entry.get("kernels", {}).get(kernel, {}).get("bytes_per_launch")


def calibrate_copy(nbytes, reps):
    """A plain device-to-device copy of known size: the reference for the PMC byte counters."""
    import torch
    torch.cuda.set_device(0)
    n = nbytes // 8
    a = torch.arange(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps}), flush=True)


def compare_solo(args):
    """Paired passes with and without the solo level (tail_budget 0 and -1), alternating which goes
    first; prints one JSON line with every pass's phase durations and the means."""
    import torch
    from paper_2509_15117_amd import api
    torch.cuda.set_device(0)
    w = workload(args.workload)
    out = api.alloc_obs(w.n, torch.device("cuda", 0), counters=False)
    api.integrate_workload(w, out=out)          # warm-up
    runs = {"solo": [], "no_solo": []}
    for k in range(args.compare_solo):
        order = (("no_solo", -1), ("solo", 0)) if k % 2 == 0 else (("solo", 0), ("no_solo", -1))
        for name, tb in order:
            ms = api.phase_ms()
            api.integrate_workload(w, out=out, kernel_ms=ms, tail_budget=tb)
            runs[name].append([float(x) for x in ms])
            print(f"[bench] round {k + 1}/{args.compare_solo} {name}: {sum(ms):.0f} ms", file=sys.stderr, flush=True)
    tot = {k: [sum(x) for x in v] for k, v in runs.items()}
    res = {"workload": w.name, "rounds": args.compare_solo, "passes_ms": runs,
           "mean_ms": {k: sum(v) / len(v) for k, v in tot.items()},
           "solo_faster_in": sum(a < b for a, b in zip(tot["solo"], tot["no_solo"]))}
    print(json.dumps(res), flush=True)


def lone_latency(args):
    """One trajectory alone on the GPU: the critical path of a batch is its longest trajectory's step
    count times this per-step latency."""
    import ctypes
    import torch
    from paper_2509_15117_amd import api
    torch.cuda.set_device(0)
    w = workload(args.workload)
    if args.max_steps:
        w.system.max_steps = args.max_steps
    api.integrate_workload(w, n=64)          # warm-up
    res = {"workload": w.name, "id": args.latency}
    # (step budget, tail budget, phase): the solo kernel, the four-lane tail kernel, the one-lane kernel
    for form, budget, budget2, ph in (("solo", 1, 1, 3), ("four_lane_tail", 1, -1, 2), ("one_lane", -1, 0, 1)):
        ms = api.phase_ms()
        o = api.integrate_workload(w, n=1, id0=args.latency, counters=True, kernel="persistent", step_budget=budget,
                                   tail_budget=budget2, kernel_ms=ms)
        steps = int(o["n_accept"].item() + o["n_reject"].item()) - (ph - 1)
        t = ms[ph]
        res[form] = {"attempted_steps": steps, "ms": t, "us_per_step": t * 1e3 / max(steps, 1),
                     "status": int(o["status"].item())}
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.steps is None:
        args.steps = 20 if args.workload == "stream" else 3
    if args.latency >= 0:
        return lone_latency(args)
    if args.compare_solo > 0:
        return compare_solo(args)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, 3)
        return
    if args.workload in ("tangent", "adjoint"):
        if args.gpus != 1:
            print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                              "n_gpus": args.gpus}))
            sys.exit(2)
        return main_diff(args)
    if args.workload == "stream":
        if args.gpus != 1:
            print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                              "n_gpus": args.gpus}))
            sys.exit(2)
        return main_stream(args)
    if args.workload in ("sweep", "stream-chunks", "thermal", "fig4"):
        if args.gpus != 1:
            print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                              "n_gpus": args.gpus}))
            sys.exit(2)
        return main_chunked(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2509_15117_amd import api
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    w = workload(args.workload)
    out = api.alloc_obs(w.n, torch.device("cuda", 0), counters=False)
    stats = api.new_stats()
    launch = dict(kernel=args.kernel, block=args.block, blocks_per_cu=args.blocks_per_cu,
                  refill_every=args.refill_every)
    if args.autotune and args.kernel == "persistent":
        best = api.autotune(w, n=min(w.n, 1 << 20), cache=args.autotune)
        print(f"[bench] autotuned launch {best}", file=sys.stderr, flush=True)
        launch.update(best)
    r = timed_runs(api, torch, w, out, stats, args.steps, args.warmup, **launch)
    K = args.steps
    traj_s = w.n * K / r["total_s"]
    stages_s = r["rhs"] / r["total_s"]
    # per kernel: algorithmic FLOP = 161 x the RHS evaluations it performed (the tail kernel counts its
    # own; the main kernel did the rest), over its event-timed average launch duration
    main_name = "k_integrate_persistent" if args.kernel == "persistent" else "k_integrate_plain"
    kernels = []
    for name, secs, rhs in ((main_name, r["phase_ms"][1] / 1e3, (r["rhs"] - r["tail_rhs"] - r["solo_rhs"]) / K),
                            ("k_integrate_tail", r["phase_ms"][2] / 1e3, r["tail_rhs"] / K),
                            ("k_integrate_solo", r["phase_ms"][3] / 1e3, r["solo_rhs"] / K)):
        if secs <= 0.0:
            continue
        tflops = FLOP_PER_RHS * rhs / secs / 1e12
        kernels.append({"kernel": name, "avg_launch_ms": secs * 1e3, "rhs_per_launch": rhs,
                        "flop_per_launch": FLOP_PER_RHS * rhs, "achieved": tflops,
                        "frac": tflops / FP64_PEAK_TFLOPS,
                        "traffic": traffic_bytes(args.traffic_file, w.name, name)})
    dom = max(kernels, key=lambda k: k["avg_launch_ms"])      # the dominant kernel by time
    res = {
        "metric": "trajectories/s + RK stages/s (FP64, rtol 1e-10): refill kernel vs plain, % FP64 peak",
        "value": traj_s,
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r["total_s"] * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "trajectories": w.n, "kernel": args.kernel, "rtol": w.system.rtol,
                   "atol": w.system.atol},
        "rk_stages_per_s": stages_s,
        "accepted_steps_per_s": r["acc"] / r["total_s"],
        "fp64_frac_peak": FLOP_PER_RHS * stages_s / (FP64_PEAK_TFLOPS * 1e12),
        "active_lane_fraction": r["useful"] / max(r["issued"], 1),
        "roofline": {"bound": "alu", "kernel": dom["kernel"], "achieved": dom["achieved"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": dom["frac"], "traffic": dom["traffic"],
                     "avg_launch_ms": dom["avg_launch_ms"], "flop_per_launch": dom["flop_per_launch"]},
        "kernels": kernels,
        "phases_ms": {"setup": r["phase_ms"][0], "main": r["phase_ms"][1], "tail": r["phase_ms"][2],
                      "solo": r["phase_ms"][3], "observe": r["phase_ms"][4]},
        "tail_trajectories": (r["tail_done"] + r["solo_done"]) / K,
        "solo_trajectories": r["solo_done"] / K,
    }
    if not args.no_plain and args.kernel != "plain":
        rp = timed_runs(api, torch, w, out, stats, 1, 0, **dict(launch, kernel="plain"))
        res["plain"] = {"trajectories_per_s": w.n / rp["total_s"], "rk_stages_per_s": rp["rhs"] / rp["total_s"],
                        "fp64_frac_peak": FLOP_PER_RHS * rp["rhs"] / rp["total_s"] / (FP64_PEAK_TFLOPS * 1e12),
                        "active_lane_fraction": rp["useful"] / max(rp["issued"], 1), "ms": rp["total_s"] * 1e3}
        res["speedup_vs_plain"] = traj_s / res["plain"]["trajectories_per_s"]
    if args.kernel == "persistent" and not args.no_critical_path:
        res["critical_path"] = critical_path(api, torch, w, r["phase_ms"][2] + r["phase_ms"][3])
    if args.inflight > 1:
        res["pipelined"] = pipelined(api, torch, w, args.inflight, launch)
    pk = api.fp64_peak()
    res["fp64_peak_measured_tflops"] = pk
    res["roofline"]["frac_of_measured_peak"] = res["roofline"]["achieved"] / pk
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
