"""Benchmark: RK4 Vlasov-Poisson steps of the two-stream workload
(1D+1V, uniform 4096 x 4096 cells, FP64) on one MI355X.

A step is one full RK4 step of the hot path (four fused stage kernels,
each with the flux divergence, the stage combination and the velocity
moment, plus four field solves) over the whole phase-space mesh, with the
state resident in HBM.  Prints one JSON line.

  value     cell-updates/s = cells * K / (time of K steps)
  roofline  the stage kernels: algorithmic bytes (12 state words per cell
            per RK4 step, 2 + 4 + 3 + 3 over the four stage launches of
            the lean stage schedule) / their average
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage1d_two_stream_4096_traffic.md")


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
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--amr-only", action="store_true", help="run only the two-level section (for profiling)")
    ap.add_argument("--no-4d", action="store_true")
    ap.add_argument("--no-limited", action="store_true")
    ap.add_argument("--no-regrid", action="store_true")
    ap.add_argument("--regrid-only", action="store_true", help="run only the regridding section (for profiling)")
    ap.add_argument("--no-amr-run", action="store_true")
    ap.add_argument("--no-species", action="store_true")
    ap.add_argument("--no-subcycle", action="store_true")
    ap.add_argument("--subcycle-only", action="store_true", help="run only the subcycled-stepping section")
    ap.add_argument("--species-only", action="store_true", help="run only the two-species section")
    ap.add_argument("--amr-run-only", action="store_true", help="run only the adaptive bump-on-tail section")
    ap.add_argument("--amr-run-t", type=float, default=22.5, help="end time of the adaptive bump-on-tail runs")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shape of the main workload")
    ap.add_argument("--tile-shape", default=None, metavar="T,W,R",
                    help="use this tile shape (threads, cells per thread, rows) instead of autotuning")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run three device-to-device copies of MIB MiB (reference for HBM traffic counters)")
    ap.add_argument("--4d-only", dest="fourd_only", action="store_true", help="run only the 2D+2V section")
    ap.add_argument("--limited-only", action="store_true", help="run only the limited-face section")
    ap.add_argument("--adjoint-only", action="store_true", help="run only the adjoint section")
    ap.add_argument("--amr4d-only", action="store_true", help="run only the two-level 2D+2V section")
    ap.add_argument("--no-amr4d", action="store_true")
    return ap.parse_args()


def read_traffic(n, dtype, shape):
    """HBM bytes per stage launch from the committed counter summary, when it
    covers this workload and tile shape (lines
    `traffic: n=<n> dtype=<dtype> shape=<T>x<W>x<R> bytes_per_launch=<B>`)."""
    if not os.path.exists(TRAFFIC_FILE) or shape is None:
        return None
    want = "x".join(str(v) for v in shape)
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if line.startswith("traffic:"):
                kv = dict(item.split("=") for item in line.split()[1:])
                if int(kv["n"]) == n and kv["dtype"] == dtype and kv.get("shape") == want:
                    return float(kv["bytes_per_launch"])
    return None


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
    cores = O.num_threads()
    value = n * n * steps / el
    # one thread: one step of the same mesh
    O.set_num_threads(1)
    t0 = time.perf_counter()
    f = o.step(f, dt)
    el1 = time.perf_counter() - t0
    O.set_num_threads(cores)
    return {"value": value, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full RK4 steps of the {n}x{n} two-stream mesh, FP64, {el:.1f} s",
            "single_thread": {"value": n * n / el1, "sample": f"1 step on 1 thread, {el1:.1f} s"}}


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
    # the forward tile shape for this mesh (on copies of the initial state)
    with torch.no_grad():
        f_tune = ((1.0 + ct + pt)[:, None] * gt[None, :]).contiguous()
        _, shape, _ = plan.autotune(f_tune, vp.field_of(plan, f_tune), dt, reps=5)

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
            "forward_tile_shape": {"threads": shape[0], "cells_per_thread": shape[1], "rows": shape[2]},
            "forward_ms": round(fw * 1e3, 2), "backward_ms": round(bw * 1e3, 2), "ratio": round(bw / fw, 3)}


def limited_bench(n=4096, steps=20, warmup=3):
    """The main workload with the limited face averages (section 2, eq.
    limitedFace): same bytes per step, more arithmetic per face."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    p = I.two_stream(n, n)
    dt = 4.788e-4 * (4096 / n)
    plan = vp.Plan(p)
    plan.set_face_scheme(vp.FACE_LIMITED)
    f = torch.tensor(p.initial_state(), dtype=torch.float64, device="cuda")
    a = vp.field_of(plan, f)
    _, shape, _ = plan.autotune(f, a, dt, reps=3)
    for _ in range(warmup):
        vp.rk4_step(plan, f, a, dt)
    st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    st.record()
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    sp.record()
    torch.cuda.synchronize()
    ms = st.elapsed_time(sp) / steps
    plan.timing_enable(True)
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    torch.cuda.synchronize()
    tm = plan.timing_read()
    plan.timing_enable(False)
    stage_us = tm["stage"][0] / tm["stage"][1] * 1e3
    bytes_launch = 12 * 8 * n * n / 4        # 12 state words per cell per step over 4 stage launches
    return {"workload": f"two-stream 1D+1V {n}x{n} FP64 with limited face averages, dt={dt}",
            "tile_shape": {"threads": shape[0], "cells_per_thread": shape[1], "rows": shape[2]},
            "ms_per_step": round(ms, 4), "cell_updates_per_s": n * n / (ms * 1e-3),
            "stage_kernel": {"avg_launch_us": round(stage_us, 2), "algorithmic_bytes_per_launch": bytes_launch,
                             "achieved_GBs": round(bytes_launch / (stage_us * 1e-6) / 1e9, 1)}}


def amr_dt(boxes, a, ncx=512, ncv=512, R=4, x_len=4 * math.pi, v_lo=-8.0, v_hi=8.0, cfl=0.5):
    """dt at CFL 0.5 with nu = dt (max face |v| / dx + max |a| / dv) on each
    level, the largest over the levels (the fine level, whose patches lie in
    |v| < 3, sets it)."""
    dxc, dvc = x_len / ncx, (v_hi - v_lo) / ncv
    dxf, dvf = dxc / R, dvc / R
    nu_c = max(abs(v_lo), abs(v_hi)) / dxc + abs(a[:ncx]).max() / dvc
    vmax_f = max(max(abs(v_lo + b["lo"][1] * dvf), abs(v_lo + (b["hi"][1] + 1) * dvf)) for b in boxes)
    nu_f = vmax_f / dxf + abs(a[ncx:]).max() / dvf
    return cfl / max(nu_c, nu_f)


def amr_bench(steps=100, warmup=3):
    """Two-level Landau hierarchy (coarse 512 x 512, ratio 4, 40 seeded
    patches of sides 16..128 inside |v| < 3; FP64): RK4 steps with the
    persistent tile-table launch (autotuned tile shape), the same steps
    captured in a HIP graph and replayed, and the per-patch launch
    baseline."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    boxes = I.amr_boxes(0)
    f0, veq_c, veq_f = I.amr_landau(boxes)
    spec = vp.two_level_spec(512, 512, 4 * math.pi, -8.0, 8.0, -1.0, 4, veq_c, veq_f)
    plan = vp.Plan(spec, boxes=boxes)
    f = torch.tensor(f0, dtype=torch.float64, device="cuda")
    a = vp.field_of(plan, f)
    dt = amr_dt(boxes, a.cpu().numpy())
    tuned, shape, _ = plan.autotune(f, a, dt, reps=5)

    def timed_steps(n):
        st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(warmup):
            vp.rk4_step(plan, f, a, dt)
        st.record()
        for _ in range(n):
            vp.rk4_step(plan, f, a, dt)
        sp.record()
        torch.cuda.synchronize()
        return st.elapsed_time(sp) / n

    plan.set_launch_mode(vp.LAUNCH_PERSISTENT)
    ms_persistent = timed_steps(steps)
    plan.timing_enable(True)
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    torch.cuda.synchronize()
    tm = plan.timing_read()
    plan.timing_enable(False)
    plan.set_launch_mode(vp.LAUNCH_PER_PATCH)
    ms_per_patch = timed_steps(steps)
    plan.set_launch_mode(vp.LAUNCH_PERSISTENT)

    # graph-captured step chain
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        vp.rk4_step(plan, f, a, dt)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        vp.rk4_step(plan, f, a, dt)
    for _ in range(warmup):
        g.replay()
    st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.record()
    for _ in range(steps):
        g.replay()
    sp.record()
    torch.cuda.synchronize()
    ms_graph = st.elapsed_time(sp) / steps

    # reduction alone, Sub-Patch (Alg. spreduce) vs Mask (Alg. mreduce)
    red = {}
    for name, alg in (("sub_patch", vp.REDUCE_SUBPATCH), ("mask", vp.REDUCE_MASK)):
        plan.set_reduction(alg)
        n_out = vp.reduce_moment(plan, f)
        plan.timing_enable(True)
        for _ in range(200):
            vp.reduce_moment(plan, f, n_out)
        torch.cuda.synchronize()
        t = plan.timing_read()["moment"]
        plan.timing_enable(False)
        red[name] = round(t[0] / t[1] * 1e3, 2)
    # the step with each reduction: the default takes the predictors' moments
    # from the stage kernels' row sums
    ms_by_reduction = {}
    for name, alg in (("sub_patch", vp.REDUCE_SUBPATCH), ("mask", vp.REDUCE_MASK), ("fused", vp.REDUCE_FUSED)):
        plan.set_reduction(alg)
        ms_by_reduction[name] = round(timed_steps(steps), 4)
    plan.set_reduction(vp.REDUCE_FUSED)

    # limited face averages on both levels (section 2, eq. limitedFace)
    plan.set_face_scheme(vp.FACE_LIMITED)
    ms_limited = timed_steps(steps)
    plan.set_face_scheme(vp.FACE_CENTERED)

    cells = plan.state_elems
    stage_ms, stage_n = tm["stage"]
    stage_us = stage_ms / stage_n * 1e3
    bytes_launch = 4 * 8 * cells            # 16 state words per cell per step over 4 stage launches
    per_launch = {k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in tm.items() if v[1]}
    return {"workload": "Landau 1D+1V two-level: coarse 512x512, ratio 4, 40 patches (seed 0, sides 16..128, "
                        "|v|<3), FP64, dt=%.4g" % dt,
            "cells": cells, "fine_cells": cells - 512 * 512,
            "tuned_shape": {"threads": shape[0], "cells_per_thread": shape[1], "rows": shape[2]},
            "ms_per_step_persistent": round(ms_persistent, 4),
            "ms_per_step_graph": round(ms_graph, 4),
            "ms_per_step_per_patch": round(ms_per_patch, 4),
            "ms_per_step_limited_faces": round(ms_limited, 4),
            "speedup_persistent_vs_per_patch": round(ms_per_patch / ms_persistent, 3),
            "speedup_graph_vs_per_patch": round(ms_per_patch / ms_graph, 3),
            "cell_updates_per_s_graph": cells / (ms_graph * 1e-3),
            "stage_kernel": {"avg_launch_us": round(stage_us, 2), "algorithmic_bytes_per_launch": bytes_launch,
                             "achieved_GBs": round(bytes_launch / (stage_us * 1e-6) / 1e9, 1)},
            "us_per_launch_by_class": per_launch,
            "reduction_us": {"sub_patch": red["sub_patch"], "mask": red["mask"],
                             "sub_patch_over_mask": round(red["sub_patch"] / red["mask"], 3)},
            "ms_per_step_by_reduction": ms_by_reduction}


def subcycle_bench(steps=40, warmup=3, cfl=0.5):
    """Subcycled against synchronous two-level stepping, each at its largest
    CFL-0.5 step, on two ratio-4 hierarchies over a 512 x 512 coarse Landau
    level (FP64): the 40 seeded patches inside |v| < 3, and one patch over
    the high-velocity band v in [4, 7.5) (every coarse column but the last).
    Synchronous: dt = cfl / max(nu_coarse, nu_fine).  Subcycled: the coarse
    step dt_c = cfl min(1 / nu_coarse, R / nu_fine) with R fine substeps.
    Reported: ms per step (the faster of eager launches and a replayed HIP
    graph) and simulated time per wall-clock second."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    ncx = ncv = 512
    R = 4
    dxc, dvc = 4 * math.pi / ncx, 16.0 / ncv
    layouts = {
        "core_40_patches_v_lt_3": I.amr_boxes(0),
        "band_v_4_to_7.5": [{"level": 1, "lo": [0, 12 * 32 * R], "hi": [(ncx - 1) * R - 1, int(15.5 * 32) * R - 1]}],
    }
    out = {}
    for name, boxes in layouts.items():
        f0, veq_c, veq_f = I.amr_landau(boxes)
        plan = vp.Plan(vp.two_level_spec(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, R, veq_c, veq_f), boxes=boxes)
        f = torch.tensor(f0, dtype=torch.float64, device="cuda")
        a = vp.field_of(plan, f)
        an = a.cpu().numpy()
        dxf, dvf = dxc / R, dvc / R
        nu_c = 8.0 / dxc + abs(an[:ncx]).max() / dvc
        vmax_f = max(max(abs(-8.0 + b["lo"][1] * dvf), abs(-8.0 + (b["hi"][1] + 1) * dvf)) for b in boxes)
        nu_f = vmax_f / dxf + abs(an[ncx:]).max() / dvf
        dt_sync = cfl / max(nu_c, nu_f)
        dt_sub = cfl * min(1.0 / nu_c, R / nu_f)
        _, shape, _ = plan.autotune(f.clone(), a.clone(), dt_sync, reps=5)     # tile shape for both

        def timed(fn, dt):
            g, ga = f.clone(), a.clone()
            for _ in range(warmup):
                fn(plan, g, ga, dt)
            st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            st.record()
            for _ in range(steps):
                fn(plan, g, ga, dt)
            sp.record()
            torch.cuda.synchronize()
            return st.elapsed_time(sp) / steps

        def timed_graph(fn, dt):
            g, ga = f.clone(), a.clone()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                fn(plan, g, ga, dt)
            torch.cuda.current_stream().wait_stream(s)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                fn(plan, g, ga, dt)
            for _ in range(warmup):
                graph.replay()
            st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            st.record()
            for _ in range(steps):
                graph.replay()
            sp.record()
            torch.cuda.synchronize()
            return st.elapsed_time(sp) / steps

        ms_sync = min(timed(vp.rk4_step, dt_sync), timed_graph(vp.rk4_step, dt_sync))
        ms_sub_eager = timed(vp.amr_subcycle_step, dt_sub)
        ms_sub_graph = timed_graph(vp.amr_subcycle_step, dt_sub)
        ms_sub = min(ms_sub_eager, ms_sub_graph)
        sim_sync = dt_sync / (ms_sync * 1e-3)
        sim_sub = dt_sub / (ms_sub * 1e-3)
        out[name] = {"coarse_cells": ncx * ncv, "fine_cells": plan.state_elems - ncx * ncv,
                     "tuned_shape": {"threads": shape[0], "cells_per_thread": shape[1], "rows": shape[2]},
                     "dt_sync": round(dt_sync, 7), "dt_subcycled": round(dt_sub, 7),
                     "ms_per_step_sync": round(ms_sync, 4), "ms_per_step_subcycled": round(ms_sub, 4),
                     "ms_per_step_subcycled_eager": round(ms_sub_eager, 4),
                     "ms_per_step_subcycled_graph": round(ms_sub_graph, 4),
                     "sim_time_per_s_sync": round(sim_sync, 3), "sim_time_per_s_subcycled": round(sim_sub, 3),
                     "subcycled_over_sync": round(sim_sub / sim_sync, 3)}
        del plan
    out["workload"] = ("Landau 1D+1V two-level, coarse 512x512, ratio 4, FP64: subcycled (coarse dt, 4 fine "
                       "substeps) vs synchronous steps, each at its largest CFL-0.5 step")
    return out


def regrid_bench(reps=50):
    """Regridding (section 3): the tagging kernel on the 4096 x 4096
    two-stream level (8 B read + 1 B written per cell) and on level 0 of the
    two-level Landau workload; on the latter also the host clustering, the
    creation of the new plan and the state transfer (prolongation + copy of
    old fine values)."""
    import torch
    import vp_inputs as I
    from paper_1204_3853_amd import vp

    def ev_time(fn, n):
        st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        st.record()
        for _ in range(n):
            fn()
        sp.record()
        torch.cuda.synchronize()
        return st.elapsed_time(sp) / n

    out = {}
    p = I.two_stream(4096, 4096)
    plan1 = vp.Plan(p)
    f1 = torch.tensor(p.initial_state(), dtype=torch.float64, device="cuda")
    tags1 = torch.empty((4096, 4096), dtype=torch.uint8, device="cuda")
    ms = ev_time(lambda: vp._check(vp.lib().vp_tag_cells(plan1.h, vp._ptr(f1), vp.ctypes.c_double(1e-6),
                                                         vp._ptr(tags1), None, vp._stream())), reps)
    cells = 4096 * 4096
    out["tag_4096"] = {"us": round(ms * 1e3, 2), "algorithmic_bytes": 9 * cells,
                       "achieved_GBs": round(9 * cells / (ms * 1e-3) / 1e9, 1)}
    del plan1, f1, tags1

    # the criterion summed over x, y, vx, vy on the 64^4 2D+2V mesh
    p4 = I.Problem2D(64, 64, 64, 64)
    plan4 = vp.Plan(p4)
    f4 = torch.tensor(p4.initial_state().ravel(), dtype=torch.float64, device="cuda")
    tags4 = torch.empty(64 ** 4, dtype=torch.uint8, device="cuda")
    ms = ev_time(lambda: vp._check(vp.lib().vp_tag_cells(plan4.h, vp._ptr(f4), vp.ctypes.c_double(1e-4),
                                                         vp._ptr(tags4), None, vp._stream())), reps)
    cells = 64 ** 4
    out["tag_2d2v_64"] = {"us": round(ms * 1e3, 2), "algorithmic_bytes": 9 * cells,
                          "achieved_GBs": round(9 * cells / (ms * 1e-3) / 1e9, 1)}
    del plan4, f4, tags4

    boxes = I.amr_boxes(0)
    f, veq_c, veq_f = I.amr_landau(boxes)
    spec = vp.two_level_spec(512, 512, 4 * math.pi, -8.0, 8.0, -1.0, 4, veq_c, veq_f)
    plan = vp.Plan(spec, boxes=boxes)
    fg = torch.tensor(f, dtype=torch.float64, device="cuda")
    tags, vals = vp.tag_cells(plan, fg, 0.0, values=True)
    tol = float(torch.quantile(vals.flatten().cpu(), 0.97))
    ms_tag = ev_time(lambda: vp.tag_cells(plan, fg, tol), reps)
    th = vp.tag_cells(plan, fg, tol).cpu()
    t0 = time.perf_counter()
    for _ in range(10):
        new_boxes = vp.cluster_tags(th, 4, 0.7, 2, 1)
    ms_cluster = (time.perf_counter() - t0) / 10 * 1e3
    t0 = time.perf_counter()
    new_plan = vp.Plan(spec, boxes=new_boxes)
    torch.cuda.synchronize()
    ms_plan = (time.perf_counter() - t0) * 1e3
    fn = torch.empty(new_plan.state_elems, dtype=torch.float64, device="cuda")
    ms_transfer = ev_time(lambda: vp.regrid_transfer(plan, fg, new_plan, fn), reps)
    out["amr"] = {"workload": "level 0 of the two-level Landau workload (512 x 512, ratio 4, 40 patches); "
                              "tolerance = 97th percentile of delta1 f + delta2 f",
                  "tagged_cells": int(th.sum()), "new_patches": len(new_boxes),
                  "new_fine_cells": int(new_plan.state_elems - 512 * 512),
                  "tag_us": round(ms_tag * 1e3, 2), "cluster_host_ms": round(ms_cluster, 3),
                  "plan_create_ms": round(ms_plan, 2), "transfer_us": round(ms_transfer * 1e3, 2)}
    return out


def linear_stability_courant():
    """RK4 on the centred fourth-order flux divergence: the largest Courant
    sum dt (|v|/dx + |a|/dv) of linear stability, 2 sqrt 2 over the peak of
    the divergence symbol (8 sin t - sin 2t)/6 (at cos t = 1 - sqrt(6)/2)."""
    c = 1.0 - math.sqrt(6.0) / 2.0
    return 2.0 * math.sqrt(2.0) / (math.sqrt(1.0 - c * c) * (4.0 - c) / 3.0)


# section 4, Table amr_param: largest patch per level (level 0 is one patch
# here whatever its limit), smallest patch, regrid interval, tag buffer
AMR_CASES = (
    ("amr1", dict(largest=[(32, 32), (64, 64), (64, 64), (64, 64)], smallest=4, interval=2, buffer=1)),
    ("amr2", dict(largest=[(16, 32), (32, 128), (128, 256), (128, 256)], smallest=8, interval=4, buffer=4)),
    ("amr3", dict(largest=[(16, 32), (32, 128), (128, 256), (128, 256)], smallest=8, interval=8, buffer=8)),
)


def amr_run_bench(t_end=22.5):
    """Adaptive bump-on-tail runs of section 4 as specified: level 0 16 x 32,
    refinement ratios [2,4], [4,2], [2,2] (up to four levels: the finest mesh
    is 256 x 512), initial refinement [(0,8),(15,24)], tol 0.01, dt =
    min(1.1 x previous, 0.5 x linear stability limit), first dt 0.01, the
    three parameter sets AMR1-3 of Table amr_param (the smallest patch size
    is taken as the smallest split part of the clustering, in cells of the
    level that is clustered: half the new level's size at ratio 2); each
    run to t_end; then the uniform 256 x 512 run to t_end with the same time
    step rule.  Reports wall time, regrid time, the deepest level reached,
    and the mean number of cells against the uniform mesh."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    coarse, ratios, tol = (16, 32), [(2, 4), (4, 2), (2, 2)], 0.01
    ncx, ncv = coarse
    boxes0 = [{"level": 1, "lo": [0, 32], "hi": [31, 99]}]
    f0, veqs = I.hier_state(I.bump_on_tail_profile, I.BUMP_X_LO, I.BUMP_X_LEN, I.BUMP_V_LO, I.BUMP_V_HI, 0.04, 0.3,
                            coarse, ratios, boxes0)
    spec = vp.hierarchy_spec(ncx, ncv, I.BUMP_X_LEN, I.BUMP_V_LO, I.BUMP_V_HI, -1.0, ratios, veqs, x_lo=I.BUMP_X_LO)
    fg = torch.tensor(f0, device="cuda")
    nxf, nvf = ncx, ncv
    for rx, rv in ratios:
        nxf, nvf = nxf * rx, nvf * rv
    uniform_cells = nxf * nvf
    out = {"workload": f"bump-on-tail (section 4), level 0 {ncx} x {ncv}, ratios {ratios}, up to "
                       f"{len(ratios) + 1} levels (finest {nxf} x {nvf}), tol {tol}, to t = {t_end}"}
    for name, c in AMR_CASES:
        minw = max(1, c["smallest"] // 2)
        run = vp.AmrRun(spec, boxes0, fg, tol, c["interval"], efficiency=0.7, min_width=minw, buffer=c["buffer"],
                        cfl=0.5, dt_growth=1.1, dt_initial=0.01, max_size=c["largest"])
        torch.cuda.synchronize()
        cell_steps, t0, deepest = 0, time.perf_counter(), 1
        info = run.info()
        while info["t"] < t_end:
            cells = info["state_elems"]
            run.advance(c["interval"])
            info = run.info()
            cell_steps += cells * c["interval"]
            deepest = max([deepest] + [b["level"] for b in run.boxes()])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"regrid_interval": c["interval"], "tag_buffer": c["buffer"], "largest_patch": c["largest"],
                     "smallest_patch": c["smallest"], "steps": info["steps"], "t_end": round(info["t"], 3),
                     "wall_s": round(wall, 3), "ms_per_step": round(wall / info["steps"] * 1e3, 3),
                     "regrids": info["regrids"], "regrid_s": round(info["regrid_seconds"], 3),
                     "final_patches": info["npatch"], "deepest_level": deepest,
                     "mean_cells": round(cell_steps / info["steps"]), "uniform_cells": uniform_cells,
                     "mean_reduction": round(1.0 - cell_steps / info["steps"] / uniform_cells, 3)}
        print(f"amr_run {name}: {out[name]}", file=sys.stderr, flush=True)
        del run
    # uniform 256 x 512 reference with the same time step rule
    prob = I.Problem1D(nx=nxf, nv=nvf, x_lo=I.BUMP_X_LO, x_len=I.BUMP_X_LEN, v_lo=I.BUMP_V_LO, v_hi=I.BUMP_V_HI,
                       profile="bump_on_tail", eps=0.04, k=0.3)
    plan = vp.Plan(prob)
    f = torch.tensor(prob.initial_state().ravel(), device="cuda")
    a = vp.field_of(plan, f)
    vmax = max(abs(I.BUMP_V_LO), abs(I.BUMP_V_HI))
    courant = linear_stability_courant()
    torch.cuda.synchronize()
    t, dt, steps, t0 = 0.0, None, 0, time.perf_counter()
    while t < t_end:
        lim = courant / (vmax / prob.dx + float(a.abs().max()) / prob.dv)
        dt = min(0.01 if dt is None else 1.1 * dt, 0.5 * lim)
        vp.rk4_step(plan, f, a, dt)
        t += dt
        steps += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["uniform"] = {"cells": nxf * nvf, "steps": steps, "t_end": round(t, 3), "wall_s": round(wall, 3),
                      "ms_per_step": round(wall / steps * 1e3, 3)}
    for name, _ in AMR_CASES:
        out[name]["speedup_vs_uniform"] = round(wall / out[name]["wall_s"], 3)
    return out


def species_bench(steps=20, warmup=3):
    """Two species on one configuration mesh: electrons (two-stream, 4096 x
    4096, v in [-8, 8]) and ions of mass ratio 100 (4096 x 1024, v in
    [-0.8, 0.8]), no background; RK4 steps of both with one field solve per
    stage from both moments."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    pe = I.two_stream(4096, 4096)
    vth = 0.1
    veq = I.cell_average_1d(lambda u: I.maxwellian(u / vth) / vth, -8 * vth, 8 * vth, 1024, first=-2, count=1028)
    pi_ = I.Problem1D(nx=4096, nv=1024, x_lo=pe.x_lo, x_len=pe.x_len, v_lo=-8 * vth, v_hi=8 * vth, qm=0.01,
                      eps=0.0, k=0.2, veq=veq)
    plans = [vp.Plan(pe), vp.Plan(pi_)]
    fs = [torch.tensor(p.initial_state().ravel(), device="cuda") for p in (pe, pi_)]
    g = vp.SpeciesGroup(plans, [-1.0, 1.0], 0.0)
    a = g.field(fs)
    dt = 4.788e-4
    for _ in range(warmup):
        g.rk4_step(fs, a, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.rk4_step(fs, a, dt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    cells = 4096 * 4096 + 4096 * 1024
    return {"workload": "electrons 4096 x 4096 (two-stream, v in [-8, 8]) + ions of mass ratio 100 "
                        "4096 x 1024 (v in [-0.8, 0.8]), FP64, dt=0.0004788",
            "cells": cells, "steps": steps, "ms_per_step": round(ms, 4),
            "cell_updates_per_s": cells / (ms * 1e-3),
            "algorithmic_GBs": round(12 * 8 * cells / (ms * 1e-3) / 1e9, 1)}


def fourd_bench(steps=50, warmup=3):
    """2D+2V 64^4 FP64 (x, y in [0, 4pi), v in [-6, 6]^2, Landau-type
    initial state): RK4 steps after the load-batch autotune."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    p = I.Problem2D(64, 64, 64, 64)
    plan = vp.Plan(p)
    f = torch.tensor(p.initial_state().ravel(), dtype=torch.float64, device="cuda")
    a = vp.field_of(plan, f)
    dt = 8.153e-3
    tuned, shape, _ = plan.autotune(f, a, dt, reps=3)
    for _ in range(warmup):
        vp.rk4_step(plan, f, a, dt)
    st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    st.record()
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    sp.record()
    torch.cuda.synchronize()
    ms = st.elapsed_time(sp) / steps
    plan.timing_enable(True)
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    torch.cuda.synchronize()
    tm = plan.timing_read()
    plan.timing_enable(False)
    cells = plan.state_elems
    stage_us = tm["stage"][0] / tm["stage"][1] * 1e3
    bytes_launch = 12 * 8 * cells / 4         # 12 state words per cell per step over 4 stage launches
    return {"workload": "2D+2V Vlasov-Poisson 64^4 FP64, x,y in [0,4pi), v in [-6,6]^2, dt=%g" % dt,
            "cells": cells, "steps": steps, "ms_per_step": round(ms, 4), "cell_updates_per_s": cells / (ms * 1e-3),
            "tuned_tile": {"threads": shape[0], "cells_x": shape[1], "cells_y": shape[2]},
            "stage_kernel": {"avg_launch_us": round(stage_us, 2), "algorithmic_bytes_per_launch": bytes_launch,
                             "achieved_GBs": round(bytes_launch / (stage_us * 1e-6) / 1e9, 1),
                             "frac_of_peak": round(bytes_launch / (stage_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
            "field_solve_us": round(tm["field"][0] / tm["field"][1] * 1e3, 2)}


def amr4d_bench(steps=20, warmup=3):
    """Two-level 2D+2V (the AMR of section 3 in the 2D+2V phase space):
    level 0 of 32^4 cells on x, y in [0, 4pi), v in [-6, 6]^2, ratio 2 in
    every direction (the fine mesh is 64^4), six seeded level-1 patches in
    the central half of the velocity box (the layout of the parity tests),
    Landau-type state, FP64: synchronous RK4 steps, against the uniform 64^4
    step of the same fine mesh."""
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp
    n, R = (32, 32, 32, 32), 2
    boxes = I.amr4d_boxes(0, n, R)
    f0, gxc, gyc, gxf, gyf = I.amr4d_state(n, R, boxes, eps=0.05)
    spec = vp.amr4d_spec(n, 4 * math.pi, 4 * math.pi, -6.0, 6.0, -1.0, R, (gxc, gyc, gxf, gyf))
    plan = vp.Plan(spec, boxes=boxes)
    f = torch.tensor(f0, dtype=torch.float64, device="cuda")
    a = vp.field_of(plan, f)
    dt = 0.01
    for _ in range(warmup):
        vp.rk4_step(plan, f, a, dt)
    st, sp = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    st.record()
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    sp.record()
    torch.cuda.synchronize()
    ms = st.elapsed_time(sp) / steps
    plan.timing_enable(True)
    for _ in range(steps):
        vp.rk4_step(plan, f, a, dt)
    torch.cuda.synchronize()
    tm = plan.timing_read()
    plan.timing_enable(False)
    cells = plan.state_elems
    coarse = n[0] * n[1] * n[2] * n[3]
    stage_us = tm["stage"][0] / tm["stage"][1] * 1e3
    # stage launches (face chunks included): 16 state words per cell and step over 4 launches
    bytes_launch = 16 * 8 * cells / 4
    per_launch = {k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in tm.items() if v[1]}
    # the uniform fine mesh
    pu = I.Problem2D(64, 64, 64, 64, eps=0.05)
    plan_u = vp.Plan(pu)
    fu = torch.tensor(pu.initial_state().ravel(), dtype=torch.float64, device="cuda")
    au = vp.field_of(plan_u, fu)
    for _ in range(warmup):
        vp.rk4_step(plan_u, fu, au, dt)
    torch.cuda.synchronize()
    st.record()
    for _ in range(steps):
        vp.rk4_step(plan_u, fu, au, dt)
    sp.record()
    torch.cuda.synchronize()
    ms_u = st.elapsed_time(sp) / steps
    return {"workload": "2D+2V two-level: level 0 32^4, ratio 2 (fine mesh 64^4), 6 seeded patches, FP64, dt=%g" % dt,
            "cells": cells, "coarse_cells": coarse, "fine_cells": cells - coarse,
            "uniform_fine_cells": 64 ** 4, "cell_fraction_of_uniform": round(cells / 64 ** 4, 4),
            "ms_per_step": round(ms, 4), "cell_updates_per_s": cells / (ms * 1e-3),
            "uniform_64_4_ms_per_step": round(ms_u, 4), "time_fraction_of_uniform": round(ms / ms_u, 3),
            "stage_kernel": {"avg_launch_us": round(stage_us, 2), "algorithmic_bytes_per_launch": bytes_launch,
                             "achieved_GBs": round(bytes_launch / (stage_us * 1e-6) / 1e9, 1)},
            "us_per_launch_by_class": per_launch}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is supported: run with --gpus 1 (the path is written "
                                   "for one device; sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch

    import vp_inputs as I
    from paper_1204_3853_amd import vp

    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.amr4d_only:
        print(json.dumps({"amr4d": amr4d_bench(steps=args.steps, warmup=args.warmup)}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_ratio()}), flush=True)
        return
    if args.limited_only:
        print(json.dumps({"limited": limited_bench(steps=args.steps, warmup=args.warmup)}), flush=True)
        return
    if args.fourd_only:
        print(json.dumps({"2d2v": fourd_bench(steps=args.steps, warmup=args.warmup)}), flush=True)
        return
    if args.amr_only:
        print(json.dumps({"amr": amr_bench(steps=args.steps, warmup=args.warmup)}), flush=True)
        return
    if args.regrid_only:
        print(json.dumps({"regrid": regrid_bench()}), flush=True)
        return
    if args.species_only:
        print(json.dumps({"species": species_bench(steps=args.steps, warmup=args.warmup)}), flush=True)
        return
    if args.amr_run_only:
        print(json.dumps({"amr_run": amr_run_bench(args.amr_run_t)}), flush=True)
        return
    if args.subcycle_only:
        print(json.dumps({"subcycle": subcycle_bench()}), flush=True)
        return
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    n = args.n
    p = I.two_stream(n, n)
    dt = 4.788e-4 * (4096 / n)
    plan = vp.Plan(p, dtype=dtype)
    f0 = torch.tensor(p.initial_state(), dtype=dtype, device="cuda")
    f = f0.clone()
    a = vp.field_of(plan, f)
    cells = n * n
    shapes = plan.tile_shapes()
    if args.tile_shape:
        shape = tuple(int(x) for x in args.tile_shape.split(","))
        plan.set_tile_shape(shapes.index(shape))
    elif not args.no_autotune:
        _, shape, _ = plan.autotune(f, a, dt, reps=5)     # on copies of (f, a); picks the tile shape
    else:
        shape = None

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
    bytes_step = 12 * esize * cells           # algorithmic bytes of the four stage launches
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
        traffic = read_traffic(n, args.dtype, shape)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": "k_stage1d (4 launches per RK4 step)", "avg_launch_us": round(avg_ms * 1e3, 2),
                    "algorithmic_bytes_per_launch": bytes_launch,
                    "field_solve_us_per_launch": round(timing["field"][0] / max(timing["field"][1], 1) * 1e3, 2)}
        if traffic:
            # HBM bytes the counters saw per launch, over the same launch time
            roofline["traffic_GBs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
            roofline["algorithmic_over_traffic"] = round(bytes_launch / traffic, 4)

    adj = None if args.no_adjoint else adjoint_ratio()
    amr = None if args.no_amr else amr_bench()
    fourd = None if args.no_4d else fourd_bench()
    amr4d = None if args.no_amr4d else amr4d_bench()
    limited = None if args.no_limited else limited_bench(n)
    regrid = None if args.no_regrid else regrid_bench()
    amr_run = None if args.no_amr_run else amr_run_bench(args.amr_run_t)
    species = None if args.no_species else species_bench(steps=args.steps, warmup=args.warmup)
    subcycle = None if args.no_subcycle else subcycle_bench()

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
                               f"x in [0,10pi), v in [-8,8], dt={dt}", "cells": cells, "dt": dt,
                   "tile_shape": None if shape is None else {"threads": shape[0], "cells_per_thread": shape[1],
                                                             "rows": shape[2]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "amr": amr,
        "2d2v": fourd,
        "amr4d": amr4d,
        "limited": limited,
        "regrid": regrid,
        "amr_run": amr_run,
        "species": species,
        "subcycle": subcycle,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
