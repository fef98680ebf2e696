#!/usr/bin/env python3
"""Benchmark of the ensemble-averaged RK stage on one MI355X.

Workload: the 2D 1024 x 1024 periodic case with 31 log-normal bins (sigma 0.5)
driven by a 1 atm plane sine wave, plain FP64, CFL time step computed on the
device.  A step is one SSP-RK3 step (three RK stages) of the whole grid; the
metric is cell-bin RK-stage updates per second, N * nb * 3 * steps / time.

Prints ONE JSON line.  `roofline` is the dominant kernel (the fused stage
kernel, timed with HIP events on its launch stream during the timed region)
against the 8 TB/s HBM peak with algorithmic bytes per launch (state read and
written by an RK stage: 16 nvar B/cell for stage 1, 24 nvar B/cell for stages
2 and 3).  `cpu_baseline` is the FP64 CPU oracle timed on this host for one
full RK3 step of the same grid.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--precision fp64|mixed] [--no-cpu-baseline]

Serving workload (--workload serving): the seeded stream of parameter-sweep
solves (Poisson arrivals; 70% 1D with 200-4000 cells, 25% 2D 64^2-512^2, 5% 3D
96^3; 11/21/31 bins; void fraction 1e-5..1e-3; 0.1-5 atm pulse; 50-500 steps)
served by the continuous-batching server in mixed precision, next to the same
stream solved one request at a time in plain FP64.  Reports solves/s and the
p50/p99 latency from arrival to result of both.

    python bench.py --workload serving [--requests 512] [--rate 20] [--budget-gib 64] [--no-sequential]

Other workloads: --workload collapse3d (256^3, 21 bins, 10 atm spherical pulse,
split mode; whole-step throughput in FP64 and mixed precision) and --workload
lagrangian (192^3 with 1e5 bubbles; bubble steps per second).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_WAVE_INSTS = 256 * 2.4e9       # 256 CUs x 2.4 GHz x one wave64 VALU instruction per CU per clock
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stage_2d1024_nb31_traffic.md")


# the sources that define the stage kernel's code (tile shapes are part of the kernel's name)
STAGE_SOURCES = ("device_common.hpp", "ee_kernels.hpp", "stage_kernel.hpp")


def kernel_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_21031_amd", "csrc")
    for name in STAGE_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_counters(precision: str, kernel: str):
    """Counter record of the committed rocprofv3 summary for this stage kernel, if it matches the sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    want = kernel_hash()
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_hash") == want and rec.get("precision") == precision and rec.get("kernel") == kernel:
                return rec
    return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case) -> dict:
    """The FP64 oracle on this host: one RK3 step of the full grid on every thread, and one RK3 step of a
    256 x 256 grid of the same recipe on one thread (a bounded sample; the full grid would take minutes)."""
    import oracle
    import workloads
    oracle.lib()
    threads = oracle.num_threads()
    pb = oracle.problem_from_case(case)
    q = oracle.init_state(pb, case.prim)
    dt = oracle.cfl_dt(pb, q)
    t0 = time.perf_counter()
    oracle.rk3_step(pb, q, dt)
    t = time.perf_counter() - t0
    import dataclasses
    small = dataclasses.replace(workloads.c2(n=256, nb=case.nb), gas=case.gas, contents=case.contents)
    pbs = oracle.problem_from_case(small)
    qs = oracle.init_state(pbs, small.prim)
    dts = oracle.cfl_dt(pbs, qs)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.rk3_step(pbs, qs, dts)
    t1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    N = case.ncells
    return {"value": 3 * N * case.nb / t, "unit": "cell·bin updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one SSP-RK3 step (3 stages) of the full {case.n[0]}x{case.n[1]} grid with {case.nb} bins "
                      f"on {threads} threads, {t:.1f} s",
            "cpu_model": cpu_model(),
            "one_thread": {"value": 3 * small.ncells * small.nb / t1, "unit": "cell·bin updates/s", "cores": 1,
                           "sample": f"one SSP-RK3 step of a {small.n[0]}x{small.n[1]} grid of the same recipe "
                                     f"({small.nb} bins) on one thread, {t1:.1f} s"}}


def serving(args):
    import torch
    import workloads
    import paper_2511_21031_amd as bub
    from paper_2511_21031_amd.serve import Server, run_sequential, summarize

    torch.cuda.set_device(0)
    reqs = workloads.c5_stream(count=args.requests, rate=args.rate)
    last = {"t": time.perf_counter()}

    def progress(tag):
        def f(done, total):
            now = time.perf_counter()
            if done == total or now - last["t"] > 10.0:
                last["t"] = now
                print(f"[{tag}] {done}/{total} solves done", file=sys.stderr, flush=True)
        return f

    # warm-up: code objects of every dimensionality and both precisions, on tiny solves
    warm = workloads.c5_stream(count=12, seed=5, scale=0.05)
    use_run = args.batch_mode == "run"
    Server(1 << 34, max_slots=8, chunk=2, use_run=use_run).run(warm, workloads.request_case, time_scale=0.0)
    run_sequential(warm[:3], workloads.request_case, bub.PREC_FP64, bub.BUBBLES_SPLIT, time_scale=0.0)
    torch.cuda.synchronize()

    budget = int(args.budget_gib * (1 << 30))
    srv = Server(budget, max_slots=args.slots, precision=bub.PREC_MIXED, bubble_mode=bub.BUBBLES_SPLIT, chunk=10,
                 lanes=args.lanes, use_run=use_run)
    ts = 0.0 if args.burst else 1.0
    recs = srv.run(reqs, workloads.request_case, time_scale=ts, progress=progress("served"))
    t_srv = max(r.finished for r in recs)
    s_srv = summarize(recs, t_srv)
    cell_bin_steps = sum(r.n[0] * r.n[1] * r.n[2] * r.nb * r.steps for r in reqs)
    out = {
        "metric": "batched solves/s with p50/p99 latency",
        "value": s_srv["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": len(warm),
        "ms_per_step": t_srv / len(reqs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"serving stream of {len(reqs)} ensemble-averaged solves, "
                               + ("all arriving at t=0" if args.burst else f"Poisson arrivals at {args.rate}/s")
                               + f" (70% 1D 200-4000 cells, 25% 2D 64^2-512^2, 5% 3D 96^3; 11/21/31 "
                               f"bins; 50-500 steps), split bubble sub-stepping, mixed precision",
                   "hbm_budget_gib": args.budget_gib, "max_slots": args.slots, "chunk": 10,
                   "batch_mode": args.batch_mode, "lanes": args.lanes,
                   "hw_queues": args.hw_queues or "HIP default",
                   "cell_bin_rk_steps": cell_bin_steps},
        "serving": {"p50_s": s_srv["p50_s"], "p99_s": s_srv["p99_s"], "mean_s": s_srv["mean_s"],
                    "wall_s": t_srv, "errors": s_srv["errors"], "peak_resident": srv.peak_active,
                    "peak_bytes": srv.peak_used, "step_calls": len(srv.chunks),
                    "cell_bin_stage_updates_per_s": 3 * cell_bin_steps / t_srv},
    }
    del srv
    torch.cuda.empty_cache()
    if not args.no_sequential:
        seq = run_sequential(reqs, workloads.request_case, bub.PREC_FP64, bub.BUBBLES_SPLIT, time_scale=ts,
                             progress=progress("sequential fp64"))
        t_seq = max(r.finished for r in seq)
        s_seq = summarize(seq, t_seq)
        out["sequential_fp64"] = {"solves_per_s": s_seq["solves_per_s"], "p50_s": s_seq["p50_s"],
                                  "p99_s": s_seq["p99_s"], "wall_s": t_seq, "errors": s_seq["errors"]}
        out["speedup_vs_sequential_fp64"] = s_srv["solves_per_s"] / s_seq["solves_per_s"]
    print(json.dumps(out), flush=True)


def collapse3d(args, quiet=False):
    """256^3, 21 bins, 10 atm spherical pulse, split mode: step throughput in FP64 and in the mixed form."""
    import torch
    import workloads
    import paper_2511_21031_amd as bub
    from paper_2511_21031_amd._binding import K_STAGE
    torch.cuda.set_device(0)
    case = workloads.c3()
    prim = torch.from_numpy(case.prim).cuda()
    res = {}
    for name, prec in (("fp64", bub.PREC_FP64), ("mixed", bub.PREC_MIXED)):
        ctx = bub.context_from_case(case, precision=prec, bubble_mode=bub.BUBBLES_SPLIT)
        q = ctx.init_state(prim)
        work = ctx.new_work()
        best, _ = ctx.autotune(q, work[:q.numel()].view_as(q), reps=2)
        for _ in range(args.warmup):
            ctx.rk3_step(q, work)
        torch.cuda.synchronize()
        ctx.profile_read(K_STAGE)
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.rk3_step(q, work)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.profile(False)
        code = ctx.last_error()[0]
        sms, sn = ctx.profile_read(K_STAGE)
        print(f"[collapse3d] {name}: {t / args.steps * 1e3:.1f} ms per step", file=sys.stderr, flush=True)
        res[name] = {"value": case.ncells * case.nb * 3 * args.steps / t, "ms_per_step": t / args.steps * 1e3,
                     "k_stage_avg_ms": sms / max(sn, 1), "tile": list(ctx.tiles()[best]), "device_error": code}
        del q, work, ctx
        torch.cuda.empty_cache()
    out = {"metric": "cell·bin RK-stage updates/s", "value": res["mixed"]["value"], "unit": "cell·bin updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["mixed"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
           "config": {"workload": "3D 256^3 reflective ensemble-averaged, 21 log-normal bins (sigma 0.3), 10 atm "
                                  "spherical pulse, split bubble sub-stepping (whole steps, bubble half-steps "
                                  "included)", "cells": case.ncells, "bins": case.nb},
           "fp64": res["fp64"], "mixed": res["mixed"], "mixed_over_fp64": res["mixed"]["value"] / res["fp64"]["value"]}
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


def lagrangian(args, quiet=False):
    """192^3 periodic, 1e5 bubbles, 2 atm plane wave: volume-averaged steps."""
    import torch
    import workloads
    import paper_2511_21031_amd as bub
    torch.cuda.set_device(0)
    lc = workloads.c4()
    ctx = bub.Context(3, lc.n, (lc.dx,) * 3, ((0, 0),) * 3, 1)
    bg = ctx.lagrangian_bubbles(torch.from_numpy(lc.bubbles).cuda())
    ql = ctx.lagrangian_init(torch.from_numpy(lc.prim).cuda())
    aD = ctx.lagrangian_smear(bg)
    work = ctx.lagrangian_work(lc.nbub)
    for _ in range(args.warmup):
        ctx.lagrangian_step(ql, bg, aD, work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.lagrangian_steps(ql, bg, aD, work, args.steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    code = ctx.last_error()[0]
    out = {"metric": "bubble steps/s", "value": lc.nbub * args.steps / t, "unit": "bubble·steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "volume-averaged 192^3 periodic, 1e5 bubbles in the central half box, R0 lognormal "
                                  "about 10 um (sigma 0.3), 2 atm plane wave, DP5(4) bubble sub-steps",
                      "cells": lc.ncells, "bubbles": lc.nbub},
           "cell_stage_updates_per_s": lc.ncells * 3 * args.steps / t, "device_error": code}
    if not quiet:
        print(json.dumps(out), flush=True)
    del ql, bg, aD, work, ctx
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed-run", action="store_true",
                    help="stage workload: skip the run in the other precision on the same grid")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--workload", choices=["stage", "serving", "collapse3d", "lagrangian"], default="stage")
    ap.add_argument("--no-extra", action="store_true",
                    help="stage: skip the shorter runs of the other workloads reported under extra_workloads")
    ap.add_argument("--tile", type=int, default=-1,
                    help="stage: tile shape index to use instead of the autotuner's choice (profiling runs)")
    ap.add_argument("--contents", choices=["polytropic", "transfer"], default="polytropic",
                    help="stage: bubble contents (transfer: gas and vapour with heat and vapour transfer)")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=20.0, help="serving: mean arrivals per second")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serving: HBM budget for resident solves")
    ap.add_argument("--slots", type=int, default=64, help="serving: batch slots (resident problems at most)")
    ap.add_argument("--no-sequential", action="store_true", help="serving: skip the sequential FP64 baseline")
    ap.add_argument("--burst", action="store_true", help="serving: every request arrives at t = 0")
    ap.add_argument("--lanes", type=int, default=4, help="serving: batch streams (lanes mode)")
    ap.add_argument("--batch-mode", choices=["run", "step"], default="run",
                    help="serving: chunks through bub_batch_run (step counts, completion flags) or bub_batch_step")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="serving: hardware queues per process (HIP GPU_MAX_HW_QUEUES, at most 32; 0 = HIP default)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X and the library has no "
              "multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        if args.hw_queues:
            if not 1 <= args.hw_queues <= 32:
                sys.exit("--hw-queues must be in 1..32")
            os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)   # read when HIP initialises
        serving(args)
        return
    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a 1 GiB device copy (1 GiB read, 1 GiB written) whose FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "collapse3d":
        collapse3d(args)
        return
    if args.workload == "lagrangian":
        lagrangian(args)
        return

    import workloads
    import paper_2511_21031_amd as bub
    case = workloads.c2()
    if args.contents == "transfer":
        import dataclasses
        case = dataclasses.replace(case, gas=dict(workloads.AIR_WITH_VAPOUR), contents=dict(workloads.AIR_VAPOUR))
    N, nb = case.ncells, case.nb
    first = args.precision
    runs = {first: stage_run(bub, torch, case, first, args)}
    if not args.no_mixed_run:
        other = "mixed" if first == "fp64" else "fp64"
        runs[other] = stage_run(bub, torch, case, other, args)
    r = runs[first]
    nvar = r["nvar"]
    # algorithmic bytes of an RK stage: 16 nvar B/cell for stage 1 (read u^k, write u^(k+1)), 24 nvar
    # for stages 2 and 3 (also read u^n); the fused stage kernel is the dominant kernel
    bytes_per_launch = (16 + 24 + 24) / 3.0 * nvar * N
    achieved = bytes_per_launch / (r["k_stage_avg_ms"] / 1e3) / 1e9
    bytes_per_step = (16 + 24 + 24) * nvar * N
    step_achieved = bytes_per_step / (r["ms_per_step"] / 1e3) / 1e9
    rec = measured_counters(first, r["kname"])
    traffic = rec["bytes_per_launch"] if rec else None
    out = {
        "metric": "cell·bin RK-stage updates/s",
        "value": r["value"],
        "unit": "cell·bin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if first == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "2D 1024x1024 periodic ensemble-averaged, 31 log-normal bins (sigma 0.5), "
                               "1 atm plane sine wave, CFL 0.3"
                               + (", gas and vapour contents with heat and vapour transfer (air/water vapour, "
                                  "20 C, transfer coefficients 5)" if args.contents == "transfer" else ""),
                   "cells": N, "bins": nb, "nvar": nvar, "precision": first,
                   "tile": r["tile"], "autotune_ms": r["autotune_ms"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        # every kernel of the step against the same algorithmic bytes (3 stages per step)
        "step_roofline": {"bytes_per_step": bytes_per_step, "achieved": step_achieved, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": step_achieved / HBM_PEAK_GBS},
        # the second roofline: VALU issue (one wave64 FP64 instruction per CU per clock at full rate)
        "valu": ({"wave_insts_per_launch": rec["valu_wave_insts_per_launch"],
                  "achieved": rec["valu_wave_insts_per_launch"] / (r["k_stage_avg_ms"] / 1e3),
                  "peak": VALU_PEAK_WAVE_INSTS, "unit": "wave-instructions/s",
                  "frac": rec["valu_wave_insts_per_launch"] / (r["k_stage_avg_ms"] / 1e3) / VALU_PEAK_WAVE_INSTS}
                 if rec else None),
        "kernels": {k: r[k] for k in ("k_stage_avg_ms", "k_stage_launches", "k_prim_avg_ms", "k_prim_launches",
                                      "other_avg_ms", "other_launches")},
    }
    for name, rr in runs.items():
        if name == first:
            continue
        out[name] = {"value": rr["value"], "ms_per_step": rr["ms_per_step"], "k_stage_avg_ms": rr["k_stage_avg_ms"],
                     "roofline_frac": bytes_per_launch / (rr["k_stage_avg_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "step_roofline_frac": bytes_per_step / (rr["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "tile": rr["tile"], "over_" + first: rr["value"] / r["value"]}
    if not args.no_extra and args.contents == "polytropic":
        out["extra_workloads"] = extra_workloads(args, bub, torch, workloads)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


def extra_workloads(args, bub, torch, workloads) -> dict:
    """Shorter runs of the other workloads, after the headline's timed steps, so that one benchmark line
    carries them: the 3D collapse (FP64 and mixed), the Lagrangian step, and the transfer contents on the
    headline grid."""
    import argparse
    import dataclasses
    sub = argparse.Namespace(**vars(args))
    sub.tile = -1                   # a forced tile shape is the headline grid's only
    sub.steps, sub.warmup = 5, 1
    c3 = collapse3d(sub, quiet=True)
    sub.steps, sub.warmup = 20, 3
    el = lagrangian(sub, quiet=True)
    tr_case = dataclasses.replace(workloads.c2(), gas=dict(workloads.AIR_WITH_VAPOUR),
                                  contents=dict(workloads.AIR_VAPOUR))
    tr = stage_run(bub, torch, tr_case, "fp64", sub)
    return {
        "collapse3d": {"config": c3["config"]["workload"], "steps": 5,
                       "fp64": {k: c3["fp64"][k] for k in ("value", "ms_per_step", "k_stage_avg_ms")},
                       "mixed": {k: c3["mixed"][k] for k in ("value", "ms_per_step", "k_stage_avg_ms")},
                       "unit": "cell·bin updates/s"},
        "lagrangian": {"config": el["config"]["workload"], "steps": 20, "value": el["value"], "unit": el["unit"],
                       "ms_per_step": el["ms_per_step"]},
        "transfer_contents": {"config": "the headline grid with gas and vapour contents (heat and vapour transfer)",
                              "steps": 20, "value": tr["value"], "unit": "cell·bin updates/s",
                              "ms_per_step": tr["ms_per_step"], "k_stage_avg_ms": tr["k_stage_avg_ms"]},
    }


def stage_run(bub, torch, case, precision, args) -> dict:
    """Autotune, warm up and time args.steps RK3 steps (one rk3_steps call) of `case` in one precision."""
    from paper_2511_21031_amd._binding import K_STAGE, K_PRIM, K_OTHER
    prec = bub.PREC_FP64 if precision == "fp64" else bub.PREC_MIXED
    ctx = bub.context_from_case(case, precision=prec)
    q = ctx.init_state(torch.from_numpy(case.prim).cuda())
    work = ctx.new_work()
    best, tile_ms = ctx.autotune(q, reps=10)        # project autotuner: fastest stage-kernel tile on this state
    if args.tile >= 0:                              # a fixed shape (after the same launches as a tuned run)
        ctx.tile = best = args.tile
    ctx.rk3_steps(q, work, args.warmup)
    torch.cuda.synchronize()
    for k in (K_STAGE, K_PRIM, K_OTHER):
        ctx.profile_read(k)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.rk3_steps(q, work, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    code, cell, b = ctx.last_error()
    if code != 0:
        print(f"device error {code} at cell {cell} bin {b}", file=sys.stderr)
        sys.exit(1)
    stage_ms, stage_n = ctx.profile_read(K_STAGE)
    prim_ms, prim_n = ctx.profile_read(K_PRIM)
    other_ms, other_n = ctx.profile_read(K_OTHER)
    elapsed = t1 - t0
    tx, ty, tz, blk = ctx.tiles()[best]
    tf = "double" if precision == "fp64" else "float"
    res = {"value": case.ncells * case.nb * 3 * args.steps / elapsed, "ms_per_step": elapsed / args.steps * 1e3,
           "k_stage_avg_ms": stage_ms / max(stage_n, 1), "k_stage_launches": stage_n,
           "k_prim_avg_ms": prim_ms / max(prim_n, 1), "k_prim_launches": prim_n,
           "other_avg_ms": other_ms / max(other_n, 1), "other_launches": other_n,
           "tile": [tx, ty, tz, blk], "autotune_ms": [round(m, 4) for m in tile_ms], "nvar": ctx.nvar,
           "kname": (f"void bub::k_stage<2, {tx}, {ty}, {tz}, {blk}, {tf}, true, 1>" if case.contents is None
                     else f"void bub::k_stage<2, {tx}, {ty}, {tz}, {blk}, {tf}, true, 2>")}
    print(f"[stage] {precision}: {res['ms_per_step']:.3f} ms per step, stage kernel {res['k_stage_avg_ms']:.3f} ms, "
          f"primitive pass {res['k_prim_avg_ms']:.3f} ms x {prim_n}", file=sys.stderr, flush=True)
    del q, work, ctx
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
