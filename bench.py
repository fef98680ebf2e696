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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stage_2d1024_nb31_traffic.md")


def kernel_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_21031_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(precision: str):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary, if it matches the sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    want = kernel_hash()
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_hash") == want and rec.get("precision") == precision:
                return rec["bytes_per_launch"]
    return None


def cpu_baseline(case) -> dict:
    import oracle
    pb = oracle.problem_from_case(case)
    q = oracle.init_state(pb, case.prim)
    dt = oracle.cfl_dt(pb, q)
    t0 = time.perf_counter()
    oracle.rk3_step(pb, q, dt)
    t = time.perf_counter() - t0
    N = case.ncells
    return {"value": 3 * N * case.nb / t, "unit": "cell·bin updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one SSP-RK3 step (3 stages) of the full {case.n[0]}x{case.n[1]} grid with {case.nb} bins, "
                      f"{t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X and this build has no "
              "multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2511_21031_amd as bub
    from paper_2511_21031_amd._binding import K_STAGE, K_PRIM, K_OTHER

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB read, 1 GiB written
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    case = workloads.c2()
    prec = bub.PREC_FP64 if args.precision == "fp64" else bub.PREC_MIXED
    ctx = bub.context_from_case(case, precision=prec)
    q = ctx.init_state(torch.from_numpy(case.prim).cuda())
    work = ctx.new_work()
    best, tile_ms = ctx.autotune(q, reps=5)     # project autotuner: fastest stage-kernel tile on this state
    for _ in range(args.warmup):
        ctx.rk3_step(q, work)
    torch.cuda.synchronize()
    for k in (K_STAGE, K_PRIM, K_OTHER):
        ctx.profile_read(k)
    ctx.profile(True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.rk3_step(q, work)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    code, cell, b = ctx.last_error()
    if code != 0:
        print(f"device error {code} at cell {cell} bin {b}", file=sys.stderr)
        sys.exit(1)

    stage_ms, stage_n = ctx.profile_read(K_STAGE)
    prim_ms, prim_n = ctx.profile_read(K_PRIM)
    elapsed = t1 - t0
    N, nb, nvar = case.ncells, case.nb, ctx.nvar
    updates = N * nb * 3 * args.steps
    value = updates / elapsed
    avg_stage_s = stage_ms / 1e3 / max(stage_n, 1)
    bytes_per_launch = (16 + 24 + 24) / 3.0 * nvar * N
    achieved = bytes_per_launch / avg_stage_s / 1e9
    traffic = measured_traffic(args.precision)
    out = {
        "metric": "cell·bin RK-stage updates/s",
        "value": value,
        "unit": "cell·bin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "2D 1024x1024 periodic ensemble-averaged, 31 log-normal bins (sigma 0.5), "
                               "1 atm plane sine wave, CFL 0.3",
                   "cells": N, "bins": nb, "nvar": nvar, "precision": args.precision,
                   "tile": list(ctx.tiles()[best]), "autotune_ms": [round(m, 4) for m in tile_ms]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "kernels": {"k_stage_avg_ms": stage_ms / max(stage_n, 1), "k_stage_launches": stage_n,
                    "k_prim_avg_ms": prim_ms / max(prim_n, 1), "k_prim_launches": prim_n,
                    "stage_share_of_gpu_time": stage_ms / max(stage_ms + prim_ms, 1e-30)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
