#!/usr/bin/env python3
"""Benchmark of the Hierarchical SUMMA local update on one MI355X.

One "step" is one pass of the whole hot path over the workload: all
k/b local updates of an HSUMMA product C = A x B (hsumma_run), with the
operands already resident in HBM.  Workload (the size the headline metric is
quoted at): n = 16384, 16 x 16 virtual grid, G = 16 groups (4 x 4 of 4 x 4),
b = M = 256, FP64 entries U[-1, 1] (seeded, synthetic).

Prints one JSON line.  `value` is FP64-accurate GFLOP/s = 2 n^3 / t of the
reported path.  `roofline` describes the dominant kernel (the update), whose
average launch duration is measured with HIP events on the stream it is
launched on.  `cpu_baseline` times the CPU oracle (plain FP64 triple loop)
on a bounded slice of the same product.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 MFMA
PEAK_BF16_TFLOPS = 2516.6    # MI355X dense BF16 MFMA
PEAK_FP8_TFLOPS = 5033.2     # MI355X dense FP8 MFMA
PEAK_HBM_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--P", type=int, default=16)
    ap.add_argument("--Q", type=int, default=16)
    ap.add_argument("--G", type=int, default=16)
    ap.add_argument("--b", type=int, default=256)
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--tile", type=str, default="")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--samples", type=int, default=256)
    return ap.parse_args()


def cpu_baseline(A, B, target_s):
    """Time the oracle's plain triple loop on the first r rows of the product."""
    from oracle import core
    core.build()
    n = B.shape[1]
    k = A.shape[1]
    r = 4
    t0 = time.perf_counter()
    core.gemm(A[:r], B)
    dt = time.perf_counter() - t0
    rows = int(max(r, min(A.shape[0], r * target_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    core.gemm(A[:rows], B)
    dt = time.perf_counter() - t0
    gflops = 2.0 * rows * n * k / dt / 1e9
    return {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": core.threads(),
            "kind": "oracle",
            "sample": "rows 0..%d of C (%d x %d x %d FP64 triple loop, %.1f s)" % (
                rows - 1, rows, k, n, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the local update of all "
              "virtual processors on a single MI355X (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1306_4161_amd import hsumma as hs
    from paper_1306_4161_amd import inputs

    n, P, Q, G, b, M = args.n, args.P, args.Q, args.G, args.b, args.M
    tile = {}
    if args.tile:
        tm, tn, kc = (int(x) for x in args.tile.split(","))
        tile = dict(tile_m=tm, tile_n=tn, kc=kc)
    log("generating operands n=%d" % n)
    A = inputs.uniform(n, n, inputs.SEED_A)
    B = inputs.uniform(n, n, inputs.SEED_B)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dC = torch.empty((n, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()

    plan = hs.Plan(n, P, Q, G, b, M, **tile)
    nouter = plan.num_outer_steps
    log("plan: groups=%r steps=%d outer=%d items=%d" % (plan.groups, plan.num_steps, nouter,
                                                         plan.num_items))
    ws = plan.workspace()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            plan.run(dA, dB, dC, ws=ws, stream=stream)
    torch.cuda.synchronize()
    log("warmup done")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev0.record(stream)
        for _ in range(args.steps):
            plan.run(dA, dB, dC, ws=ws, stream=stream)
        ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    log("timed %d steps: %.3f ms/step (wall %.3f s)" % (args.steps, ms, wall))
    flops = 2.0 * n * n * n
    gflops = flops / (ms * 1e-3) / 1e9
    # Dominant kernel: the update; one launch per outer step.
    launches = nouter
    per_launch_flops = 2.0 * n * n * M
    avg_launch_ms = ms / launches
    achieved = per_launch_flops / (avg_launch_ms * 1e-3) / 1e12

    # Accuracy on sampled entries (scaled error |c_hat - c| / (|A||B|)_ij).
    from oracle import core
    rows, cols = inputs.sample_entries(n, n, args.samples, inputs.SEED_SAMPLE)
    C = dC.cpu().numpy()
    cref, sref = core.sampled(A, B, rows, cols)
    got = C[rows, cols]
    scaled = float(np.max(np.abs(got - cref) / sref))
    pure = float(np.max(np.abs(got - cref) / np.abs(cref)))
    log("max scaled err %.3g, max pure rel err %.3g" % (scaled, pure))

    out = {
        "metric": "FP64-accurate GFLOP/s at n=16384: split-BF16/FP8 vs FP64-MFMA, % roofline",
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "path": "fp64-mfma",
        "config": {"workload": "HSUMMA local updates, n=%d, %dx%d grid, G=%d, b=%d, M=%d, "
                               "U[-1,1] FP64" % (n, P, Q, G, b, M),
                   "n": n, "P": P, "Q": Q, "G": G, "b": b, "M": M,
                   "tile": list(tile.values()) if tile else "default"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "fp64_update_kernel", "launches_per_step": launches,
                     "flops_per_launch": per_launch_flops},
        "accuracy": {"max_scaled_err": scaled, "max_pure_rel_err": pure,
                     "samples": int(rows.size)},
    }
    if not args.no_cpu:
        log("timing CPU oracle (~%.0f s)" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
