#!/usr/bin/env python3
"""Throughput of the ODC meshing path on one MI355X.

Workload: the MLP occupancy field at 256^3 (sigmoid(-20 sdf + 0.3 MLP),
32 seeded spheres, 6-band Fourier features, 4 x 256 ReLU layers; k = 15),
bf16-guarded precision.  One step = one full extraction (stages a-e, all
occupancy queries included) of that field with its inputs resident in HBM.
Metric: active cells meshed per second.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
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

import odc_inputs as I  # noqa: E402

MLP_FLOP_PER_QUERY = lambda f: 2 * (f.in_dim * f.width + (f.depth - 1) * f.width * f.width  # noqa: E731
                                    + f.width)
PEAK_FP32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2.5e15


def cpu_baseline(field, grid, seconds: float, sub: int = 16, seed: int = 0) -> dict:
    """The oracle, untuned, on sub-boxes of the same grid (same h, same field)
    centred on seeded points of the sdf spheres' surfaces, until `seconds` of
    CPU time have been spent.  Returns active cells per second."""
    from oracle import oracle as O
    O.build()
    rng = np.random.default_rng(seed)
    h = grid.size / grid.res
    cells = 0
    spent = 0.0
    boxes = 0
    while spent < seconds:
        s = field.spheres[rng.integers(len(field.spheres))].astype(np.float64)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        p = s[:3] + s[3] * d
        origin = np.clip(np.floor((p - np.asarray(grid.lo)) / h).astype(int) - sub // 2, 0,
                         grid.res - sub)
        lo = tuple(float(grid.lo[a] + origin[a] * h) for a in range(3))
        g2 = I.Grid(lo=lo, size=sub * h, res=sub, iters_1d=grid.iters_1d)
        t0 = time.perf_counter()
        m = O.Oracle(field, g2, mlp_tie_eps=1e-5).mesh()
        spent += time.perf_counter() - t0
        cells += len(m["cell_id"])
        boxes += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": cells / spent, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{boxes} sub-boxes of {sub}^3 cells at the benchmark's h around seeded "
                      f"sphere-surface points, {cells} active cells in {spent:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=("bf16", "fp32"), default="bf16")
    ap.add_argument("--res", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build meshes on one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_2409_13418_amd import odc

    field = I.mlp_field(3)
    grid = I.unit_grid(args.res, 15)
    prec = odc.PREC_BF16_GUARDED if args.precision == "bf16" else odc.PREC_FP32
    ctx = odc.Context(0)
    df = odc.DeviceField(field)
    params = odc.default_params(grid, prec)
    for _ in range(args.warmup):
        ctx.extract(df, params)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    step_ms = []
    stages = {k: 0.0 for k in odc.STAGES}
    counts = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        ctx.extract_async(df, params, cap_hint=(ctx.cap_v, ctx.cap_t))
        counts = ctx.sync()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        for k, v in ctx.stage_times().items():
            stages[k] += v
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    ms_per_step = total_s * 1e3 / args.steps
    cells = counts["n_active_cells"]
    value = cells / (ms_per_step / 1e3)
    for k in stages:
        stages[k] /= args.steps

    # roofline of the dominant kernel: the 2D-point search (fp32 matrix cores)
    per_query = MLP_FLOP_PER_QUERY(field)
    per_pair = 1 + (grid.lin1 + grid.bin1) + 2 * (grid.lin2 + grid.bin2)
    dom = max(("bisect", "search2d", "labels"), key=lambda k: stages[k])
    if dom == "search2d":
        flop = counts["n_pairs"] * per_pair * per_query
        peak = PEAK_FP32_MFMA
    elif dom == "bisect":
        flop = counts["n_active_edges"] * grid.iters_1d * per_query
        peak = PEAK_FP32_MFMA
    else:
        nc = (grid.res + 1) ** 3
        flop = nc * per_query
        peak = PEAK_BF16_MFMA if prec == odc.PREC_BF16_GUARDED else PEAK_FP32_MFMA
    achieved = flop / (stages[dom] / 1e3) / 1e12
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved * 1e12 / peak, "traffic": None}
    out = {
        "metric": "active cells meshed/sec at 256^3 MLP occupancy",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+fp32" if prec == odc.PREC_BF16_GUARDED else "fp32",
        "data": "synthetic",
        "config": {"workload": f"mlp{args.res}_{args.precision}", "res": args.res,
                   "field": "sigmoid(-20 sdf + 0.3 MLP): 32 spheres, 6 bands, 4x256 ReLU, seed 3",
                   "iters_1d": grid.iters_1d, "precision": args.precision},
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "counts": {k: counts[k] for k in ("n_active_cells", "n_active_edges", "n_pairs",
                                          "n_vertices", "n_triangles", "n_queries",
                                          "n_guard_corners", "n_fp64_cells")},
        "stages_ms": stages,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(field, grid, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
