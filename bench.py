"""Throughput benchmark: trajectories/s and RK stages/s of the persistent-refill kernel against the
plain one-launch-per-batch kernel, FP64 at rtol 1e-10, with the achieved fraction of the MI355X
FP64 vector peak and the CPU oracle timed on the host as a baseline.

One "step" = one iat_integrate call over the whole workload (every trajectory integrated from
its start to its exit or t_max, observables written).  Inputs are generated on the device from
trajectory ids, so nothing crosses PCIe inside the timed region.

    python bench.py [--steps K] [--warmup W] [--workload grid1024|grid8|sweep]
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
FLOP_PER_RHS = 161                # algorithmic FLOP per right-hand-side evaluation
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid1024", choices=["grid1024", "grid8", "sweep"])
    ap.add_argument("--kernel", default="persistent", choices=["persistent", "plain"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--refill-every", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return ap.parse_args()


def workload(name):
    import workloads as W
    if name == "grid1024":
        return W.config2()
    if name == "grid8":
        return W.config1()
    w = W.config3()
    return w


def timed_runs(api, torch, w, out, stats, steps, warmup, **launch):
    """Warm up, then time `steps` full passes with HIP events on the launch stream."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        api.integrate_workload(w, out=out, **launch)
    torch.cuda.synchronize()
    stats.zero_()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per = []
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        api.integrate_workload(w, out=out, stats=stats, **launch)
        e1.record(stream)
        per.append((e0, e1))
        print(f"[bench] launched pass {len(per)}/{steps} ({launch.get('kernel')})", file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    launch_ms = [a.elapsed_time(b) for a, b in per]
    s = stats.cpu().tolist()
    return dict(total_s=total_ms / 1e3, wall_s=wall, launch_ms=launch_ms, rhs=s[0], acc=s[1], rej=s[2],
                done=s[3], issued=s[4], useful=s[5])


def cpu_baseline(w, target_s):
    """The oracle on a strided sample of the same ids, all host threads."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on a small sample, then size the sample to ~target_s of wall time
    n_cal = 64
    ids = np.linspace(0, w.n - 1, n_cal).astype(np.int64)
    t = time.perf_counter()
    oracle.integrate(oracle.problems_for(w, ids), threads)
    dt = max(time.perf_counter() - t, 1e-3)
    n = int(min(max(n_cal, n_cal * target_s / dt), 200_000, w.n))
    ids = np.linspace(0, w.n - 1, n).astype(np.int64)
    P = oracle.problems_for(w, ids)
    t = time.perf_counter()
    R = oracle.integrate(P, threads)
    el = time.perf_counter() - t
    return dict(value=n / el, unit="trajectories/s", cores=threads, kind="oracle",
                sample=f"{n} evenly strided ids of the {w.n}-trajectory workload, {el:.1f} s",
                rk_stages_per_s=float(R["n_rhs"].sum()) / el)


def main():
    args = parse()
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
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    launch = dict(kernel=args.kernel, block=args.block, blocks_per_cu=args.blocks_per_cu,
                  refill_every=args.refill_every)
    r = timed_runs(api, torch, w, out, stats, args.steps, args.warmup, **launch)
    K = args.steps
    traj_s = w.n * K / r["total_s"]
    stages_s = r["rhs"] / r["total_s"]
    avg_launch_s = sum(r["launch_ms"]) / len(r["launch_ms"]) / 1e3
    flop_per_launch = FLOP_PER_RHS * r["rhs"] / K
    achieved = flop_per_launch / avg_launch_s / 1e12
    traffic = None
    if os.path.exists(args.traffic_file):
        try:
            tr = json.load(open(args.traffic_file))
            if tr.get("workload") == w.name and tr.get("kernel") == args.kernel:
                traffic = tr.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic},
    }
    if not args.no_plain and args.kernel != "plain":
        rp = timed_runs(api, torch, w, out, stats, 1, 0, **dict(launch, kernel="plain"))
        res["plain"] = {"trajectories_per_s": w.n / rp["total_s"], "rk_stages_per_s": rp["rhs"] / rp["total_s"],
                        "fp64_frac_peak": FLOP_PER_RHS * rp["rhs"] / rp["total_s"] / (FP64_PEAK_TFLOPS * 1e12),
                        "active_lane_fraction": rp["useful"] / max(rp["issued"], 1), "ms": rp["total_s"] * 1e3}
        res["speedup_vs_plain"] = traj_s / res["plain"]["trajectories_per_s"]
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
