"""Benchmark: RK4 Vlasov-Poisson steps of the two-stream workload
(1D+1V, uniform 4096 x 4096 cells, FP64) on one MI355X.

A step is one full RK4 step of the hot path (four fused stage kernels,
each with the flux divergence, the stage combination and the velocity
moment, plus four field solves) over the whole phase-space mesh, with the
state resident in HBM.  Prints one JSON line.

  value     cell-updates/s = cells * K / (time of K steps)
  roofline  the stage kernels: algorithmic bytes (16 state words per cell
            per RK4 step over the four stage launches) / their average
            launch duration measured with HIP events in a second pass of
            K steps, against the 8 TB/s HBM peak
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "phase-space cell-updates/s per RK4 step, % peak HBM GB/s; adjoint/forward ratio"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage1d_two_stream_4096.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--n", type=int, default=4096, help="cells per direction (default: the 4096^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline-pass", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-adjoint", action="store_true")
    return ap.parse_args()


def cpu_baseline(n, dt, seconds):
    """Oracle (FP64, OpenMP over rows) on the same workload: whole RK4
    steps of the n x n two-stream mesh until about `seconds` have passed."""
    import vp_inputs as I
    from oracle import oracle as O
    O.build(force=False)
    p = I.two_stream(n, n)
    f = p.initial_state()
    o = O.Oracle1D.from_problem(p)
    f = o.step(f, dt)                       # warm-up (page faults, factorisation)
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = o.step(f, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    return {"value": n * n * steps / el, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{steps} full RK4 steps of the {n}x{n} two-stream mesh, FP64, {el:.1f} s"}


def adjoint_ratio(steps=400, every=20):
    """Adjoint workload (Landau 512 x 512, FP64, 400 steps, checkpoint every
    20): wall time of the forward rollout and of the backward pass
    (segment recompute + discrete adjoint + field-energy gradient)."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import autograd as AG
    from paper_1204_3853_amd import vp
    prob, c, pvec = I.adjoint_setup(512, 512, seed=0)
    g = prob.veq[2:-2]
    dt = 1.531e-3
    plan = vp.Plan(prob)
    pt = torch.tensor(pvec, dtype=torch.float64, device="cuda", requires_grad=True)
    ct = torch.tensor(c, dtype=torch.float64, device="cuda")
    gt = torch.tensor(g, dtype=torch.float64, device="cuda")

    def run():
        pt.grad = None
        f0 = ((1.0 + ct + pt)[:, None] * gt[None, :]).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fT = AG.rollout(f0, plan, dt, steps, every)
        W = AG.field_energy(fT, plan)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        W.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    run()                                         # warm-up
    fw, bw = min(run() for _ in range(3))
    return {"workload": "Landau 1D+1V 512x512 FP64, 400 RK4 steps, checkpoint every 20, "
                        "gradient of 1/2 sum E^2 w.r.t. the 512-value initial profile",
            "forward_ms": round(fw * 1e3, 2), "backward_ms": round(bw * 1e3, 2), "ratio": round(bw / fw, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described in DESIGN.md, not launched)"}))
        sys.exit(2)
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp

    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    n = args.n
    p = I.two_stream(n, n)
    dt = 4.788e-4 * (4096 / n)
    plan = vp.Plan(p, dtype=dtype)
    f0 = torch.tensor(p.initial_state(), dtype=dtype, device="cuda")
    f = f0.clone()
    a = vp.field_of(plan, f)
    cells = n * n

    for _ in range(args.warmup):
        vp.rk4_step(plan, f, a, dt)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        vp.rk4_step(plan, f, a, dt)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ms_step = ms / args.steps
    value = cells * args.steps / (ms * 1e-3)

    esize = 8 if dtype == torch.float64 else 4
    bytes_step = 16 * esize * cells           # algorithmic bytes of the four stage launches
    roofline = None
    timing = None
    if not args.no_roofline_pass:
        plan.timing_enable(True)
        for _ in range(args.steps):
            vp.rk4_step(plan, f, a, dt)
        torch.cuda.synchronize()
        timing = plan.timing_read()
        plan.timing_enable(False)
        st_ms, st_n = timing["stage"]
        avg_ms = st_ms / st_n
        bytes_launch = bytes_step / 4.0
        achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            with open(TRAFFIC_FILE) as fh:
                tr = json.load(fh)
            if tr.get("n") == n and tr.get("dtype") == args.dtype:
                traffic = tr.get("bytes_per_launch")
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": "k_stage1d (4 launches per RK4 step)", "avg_launch_us": round(avg_ms * 1e3, 2),
                    "algorithmic_bytes_per_launch": bytes_launch,
                    "field_solve_us_per_launch": round(timing["field"][0] / max(timing["field"][1], 1) * 1e3, 2)}

    adj = None if args.no_adjoint else adjoint_ratio()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, dt, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"two-stream 1D+1V Vlasov-Poisson, uniform {n}x{n} cells, RK4, "
                               f"x in [0,10pi), v in [-8,8], dt={dt}", "cells": cells, "dt": dt},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "adjoint": adj,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
