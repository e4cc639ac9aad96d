#!/usr/bin/env python3
"""Throughput of the ODC meshing path on one MI355X.

Workload: the MLP occupancy field at 256^3 (sigmoid(-20 sdf + 0.3 MLP),
32 seeded spheres, 6-band Fourier features, 4 x 256 ReLU layers; k = 15),
bf16-guarded precision.  One step = one full extraction (stages a-e, all
occupancy queries included) of that field with its inputs resident in HBM.
Metric: active cells meshed per second.

Prints one JSON line (--jsonl PATH also appends it, after per-step records,
to a JSONL file).  --gpus above 1 is refused: the library meshes on one GPU.
Besides the timed steps, the line carries (all outside the timed region):
the dominant kernel's roofline; the plain fp32 path's throughput on the same
grid and whether its mesh equals the guarded path's (fp32_path); the same
with split-bf16 searches (x3_path: corner signs and cells equal to the
guarded path's, vertices to binary32 rounding of the searches) and with
coarse-to-fine corner evaluation (adaptive_path: 4-cell coarse grid); the paper's
quality measures of the mesh; a short Poisson serving trace through the
continuous-batching server (serve: p50/p99 latency, cells/s; --serve-requests-
default requests after --serve-warmup-default-s seconds of arrivals); the
Chamfer distance of both paths' meshes to the oracle's on sub-boxes; and the
oracle's own rate on all host threads and on one (cpu_baseline).

Other modes (not run by default):
  --mode batch  64 seeded shapes (32 CSG, 32 MLP fields; res uniform over
                {64, 96, 128, 192, 256}) meshed as one batch per step,
                graph-replayed with the autotuned launch shape; reported with
                the same batch under the default launch shape (the
                autotuner's gain) and the same shapes meshed one at a time
                on the plain fp32 path.
  --mode copy   a plain device-to-device copy of --copy-mib MiB, repeated
                --steps times: the reference kernel that scales the HBM byte
                counters (FETCH_SIZE, WRITE_SIZE) of a profile.
  --mode ablation  Table 3's rows (MDC, + 1D search, + 2D search, ODC; the last
                two also with 3D points clamped to their cells) on the same
                field: time, counts, manifold check, mean |phi - 1/2|,
                self-intersecting triangle pairs.
  --mode csg    the 72-primitive CSG field (48 boxes and 16 spheres, minus 8
                boxes; seed 2) at --res cells per axis, timed as the default
                line times the MLP field: cells/s, stage times, counts.
  --mode serve  Poisson arrivals (20 requests/s, 50/50 CSG/MLP, res 64/128/
                256/512 with weights .4/.3/.2/.1) through the continuous-
                batching server; p50/p99 latency (completion - arrival) and
                active cells/s over the requests after a 10 s warm-up;
                --serve-policy shortest admits the cheapest queued job first
                (a job older than --serve-age-ms goes first regardless);
                banded (the default) also keeps jobs estimated at more than
                --serve-band times a batch's first job out of that batch;
                fifo admits in arrival order.
"""
from __future__ import annotations

import argparse
import json
import math
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
ADAPTIVE_STEP = 4
PEAK_BF16_MFMA = 2.5e15


def _prec(odc, name: str) -> int:
    return {"bf16": odc.PREC_BF16_GUARDED, "fp32": odc.PREC_FP32,
            "x3": odc.PREC_BF16_X3}[name]


DTYPE = {"bf16": "bf16+fp32", "fp32": "fp32", "x3": "bf16+fp32"}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2409_13418_amd", "csrc")
    for fn in ("odc_kernels.hip", "odc_mlp.h", "odc_job.h", "odc_device.h", "odc_internal.h"):
        with open(os.path.join(src, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


PROFILE_OF = {"k_search2d_mlp": "search2d_mlp256_bf16.md",
              "k_search2d_x3": "search2d_x3_mlp256.md"}


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from its committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy), or None when
    there is none or the kernel sources changed after the counters were
    taken."""
    path = os.path.join(ROOT, "profiles", PROFILE_OF.get(kernel, "-"))
    if not os.path.exists(path):
        return None
    value, sha = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith(f"traffic_bytes_per_launch {kernel}:"):
                value = float(line.split(":")[1])
            if line.startswith("kernel_sources_sha256:"):
                sha = line.split(":", 1)[1].strip()
    return value if sha == kernel_sources_sha256() else None


def cpu_baseline(field, grid, seconds: float, sub: int = 16, seed: int = 0, chamfer=None,
                 threads: int = 0) -> dict:
    """The oracle, untuned, on sub-boxes of the same grid (same h, same field)
    centred on seeded points of the sdf spheres' surfaces, until `seconds` of
    wall time have been spent, on `threads` host threads (0 = all).  Returns
    active cells per second.  With `chamfer` = (context, device field,
    {name: precision}), the first sub-boxes are also meshed on the GPU at each
    precision and the Chamfer distance to the oracle's mesh is reported
    (outside the timed part)."""
    from oracle import oracle as O
    O.build()
    rng = np.random.default_rng(seed)
    h = grid.size / grid.res
    cells = 0
    spent = 0.0
    boxes = 0
    cham = {}
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
        m = O.Oracle(field, g2, mlp_tie_eps=1e-5, n_threads=threads).mesh()
        spent += time.perf_counter() - t0
        cells += len(m["cell_id"])
        boxes += 1
        if chamfer is not None and boxes <= 4 and len(m["tris"]):
            from paper_2409_13418_amd import odc
            sys.path.insert(0, os.path.join(ROOT, "tests"))
            from meshcheck import chamfer_h2
            ctx, df, precs = chamfer
            vo = np.asarray(g2.lo) + m["vert"] * h
            for name, prec in precs.items():
                r = ctx.extract(df, odc.default_params(g2, prec))
                cham.setdefault(name, []).append(
                    chamfer_h2(r["vertices"].cpu().numpy(), r["triangles"].cpu().numpy(), vo,
                               m["tris"], h, n=20000, seed=boxes))
    used = threads or int(os.environ.get("OMP_NUM_THREADS", "0")) or \
        len(os.sched_getaffinity(0))
    out = {"value": cells / spent, "unit": "cells/s", "cores": used, "kind": "oracle",
           "sample": f"{boxes} sub-boxes of {sub}^3 cells at the benchmark's h around seeded "
                     f"sphere-surface points, {cells} active cells in {spent:.1f} s"}
    if cham:
        out["chamfer_vs_oracle"] = {
            **{name: max(v) for name, v in cham.items()}, "unit": "h^2",
            "boxes": len(next(iter(cham.values()))),
            "method": "symmetric mean squared point-to-surface distance, 20k area samples per "
                      "mesh, GPU mesh of the same sub-box at each precision; max over boxes"}
    return out


def mesh_quality(ctx, df, grid, samples: int = 1000000, params=None) -> dict:
    """The paper's quality measures of the last mesh (Sec. 6, Table 3), outside
    the timed region: mean |phi - 1/2| at area-uniform surface samples (phi
    from the fp32 field evaluation on the GPU), self-intersecting triangle
    pairs (counted on the GPU) and the closed-manifold check."""
    from paper_2409_13418_amd import odc
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from meshcheck import is_closed_oriented_manifold, sample_surface
    r = ctx.extract(df, params if params is not None else odc.default_params(grid))
    v = r["vertices"].cpu().numpy().astype(np.float64)
    t = r["triangles"].cpu().numpy()
    ok, _ = is_closed_oriented_manifold(t, len(v))
    z = ctx.field_eval(df, sample_surface(v, t, samples, seed=5)).astype(np.float64)
    return {"abs_phi_minus_half": float(np.mean(np.abs(0.5 * np.tanh(0.5 * z)))),
            "self_intersecting_pairs": ctx.self_intersections(r["vertices"], r["triangles"], grid.h),
            "closed_manifold": bool(ok), "samples": samples}


def emit(out: dict, args, records=()) -> None:
    """Prints the result line; with --jsonl, also appends it (after any
    per-step records) to that file, one JSON object per line."""
    line = json.dumps(out)
    print(line, flush=True)
    if getattr(args, "jsonl", None):
        with open(args.jsonl, "a") as fh:
            for r in records:
                fh.write(json.dumps(r) + "\n")
            fh.write(line + "\n")


def _batch_mode(args):
    """64 shapes per step in one batched, graph-replayed launch."""
    import torch
    from paper_2409_13418_amd import odc

    cfgs = I.batch_configs(64, 4000)
    prec = _prec(odc, args.precision)
    dfs = [odc.DeviceField(f) for f, _ in cfgs]
    ps = [odc.default_params(g, prec if f.kind == odc.FIELD_MLP else odc.PREC_FP32)
          for f, g in cfgs]
    ctx = odc.Context(0)
    ctx.set_graph(True)
    caps = [(max(4096, 10 * g.res * g.res), max(8192, 20 * g.res * g.res)) for _, g in cfgs]

    def timed_batch():
        for _ in range(args.warmup):
            ctx.extract_batch(dfs, ps, caps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = ctx.extract_batch(dfs, ps, caps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, res

    # the default launch shape, then autotuned on the largest MLP shape
    ms_default, _ = timed_batch()
    big = max((k for k in range(len(cfgs)) if cfgs[k][0].kind == odc.FIELD_MLP),
              key=lambda k: cfgs[k][1].res)
    chosen = ctx.autotune(dfs[big], ps[big])
    ms, out = timed_batch()
    cells = sum(o["n_active_cells"] for o in out)
    # the same shapes one at a time, plain fp32 path, default launch shape
    ref = odc.Context(0)
    ps32 = [odc.default_params(g, odc.PREC_FP32) for _, g in cfgs]
    for k in range(len(cfgs)):
        ref.extract(dfs[k], ps32[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cells32 = 0
    for k in range(len(cfgs)):
        cells32 += ref.extract(dfs[k], ps32[k])["n_active_cells"]
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t1) * 1e3
    assert cells32 == cells, (cells32, cells)
    out = {
        "metric": "active cells meshed/sec, 64-shape batch",
        "value": cells / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "batch64", "shapes": 64, "seeds": "4000..4063",
                   "res": [g.res for _, g in cfgs], "precision_mlp": args.precision,
                   "launch_blocks": list(chosen), "graph": True},
        "active_cells": cells,
        "default_launch_shape": {"value": cells / (ms_default / 1e3), "unit": "cells/s",
                                 "ms_per_step": ms_default},
        "sequential_fp32": {"value": cells / (ms32 / 1e3), "unit": "cells/s", "ms": ms32},
    }
    emit(out, args)


def _serve_mode(args):
    """Poisson request trace through the serving loop."""
    emit(serve_run(args, args.serve_requests, args.serve_warmup_s), args)


def serve_run(args, n_requests: int, warm_s: float) -> dict:
    """Replays a seeded Poisson trace of n_requests (after warm_s seconds of
    warm-up arrivals) through the continuous-batching server; returns the
    latency percentiles (completion - submission) and active cells/s."""
    import threading

    import torch
    from paper_2409_13418_amd import odc

    rate = args.serve_rate
    n_warm = int(round(warm_s * rate))
    trace = I.serve_trace(n_warm + n_requests, rate, 5)
    prec = _prec(odc, args.precision)
    # a pool of seeded fields per kind (the trace's field seed modulo the pool)
    pool = 16
    fields = {}
    for kind, res, seed in {(k, r, s % pool) for _, k, r, s in trace}:
        if (kind, seed) not in fields:
            f = I.csg_random_field(6000 + seed) if kind == 0 else I.mlp_field(6100 + seed)
            fields[(kind, seed)] = odc.DeviceField(f)
    params = {}
    for _, kind, res, _ in trace:
        if (kind, res) not in params:
            params[(kind, res)] = odc.default_params(
                I.unit_grid(res, 15), prec if kind == 1 else odc.PREC_FP32)
    ctx = odc.Context(0)
    policy = {"fifo": odc.SERVE_FIFO, "shortest": odc.SERVE_SHORTEST,
              "banded": odc.SERVE_BANDED}[args.serve_policy]
    srv = odc.Server(ctx, int(args.serve_budget_gib * (1 << 30)), lanes=args.serve_lanes,
                     max_batch=16, policy=policy, age_ms=args.serve_age_ms,
                     band=args.serve_band)
    free_bufs = {}
    lock = threading.Lock()

    def take(res):
        with lock:
            lst = free_bufs.setdefault(res, [])
            if lst:
                return lst.pop()
        b = odc.OutputBuffers(max(4096, 10 * res * res), max(8192, 20 * res * res))
        torch.cuda.current_stream().synchronize()  # the allocation is usable by other streams
        return b

    tickets = []
    results = []
    done = threading.Event()

    def waiter():
        i = 0
        while True:
            with lock:
                if i >= len(tickets):
                    if done.is_set():
                        return
                    t = None
                else:
                    t, res, buf = tickets[i]
            if t is None:
                time.sleep(0.001)
                continue
            r = srv.wait(t)
            r["res"] = res
            results.append(r)
            with lock:
                free_bufs.setdefault(res, []).append(buf)
            i += 1

    th = threading.Thread(target=waiter)
    th.start()
    t_start = time.perf_counter()
    reset_done = False
    for i, (at, kind, res, seed) in enumerate(trace):
        if not reset_done and i == n_warm:
            srv.reset_stats()
            reset_done = True
        delay = at - (time.perf_counter() - t_start)
        if delay > 0:
            time.sleep(delay)
        buf = take(res)
        t = srv.submit(fields[(kind, seed % pool)], params[(kind, res)], buf)
        with lock:
            tickets.append((t, res, buf))
    done.set()
    th.join()
    st = srv.stats()
    wall = time.perf_counter() - t_start
    srv.close()
    bad = [r for r in results if r["status"] != odc.OK]
    by_res = {}
    for r in results[n_warm:]:
        by_res.setdefault(r["res"], []).append(r["latency_ms"])
    out = {
        "metric": "serve latency p50/p99 and active cells/sec",
        "value": st["cells_per_s"], "unit": "cells/s", "n_gpus": 1,
        "steps": n_requests, "warmup": n_warm, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": "serve_poisson", "rate_per_s": rate, "requests": n_requests,
                   "warmup_s": warm_s, "mix": "50/50 CSG/MLP", "res_weights":
                   {"64": 0.4, "128": 0.3, "256": 0.2, "512": 0.1}, "lanes": args.serve_lanes,
                   "budget_gib": args.serve_budget_gib, "field_pool": pool,
                   "policy": args.serve_policy,
                   "age_ms": args.serve_age_ms if args.serve_policy != "fifo" else None,
                   "band": args.serve_band if args.serve_policy == "banded" else None},
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
        "max_ms": st["max_ms"], "completed": st["completed"], "failed": len(bad),
        "batches": st["batches"], "window_s": st["window_s"], "wall_s": wall,
        "arena_peak_gib": st["arena_peak_bytes"] / (1 << 30),
        "p50_ms_by_res": {str(k): float(np.percentile(v, 50)) for k, v in sorted(by_res.items())},
        "p99_ms_by_res": {str(k): float(np.percentile(v, 99)) for k, v in sorted(by_res.items())},
    }
    return out


def _ablation_mode(args):
    """Table 3's structure on the benchmark field: Manifold Dual Contouring,
    + the 1D search, + the 2D search, + the intersection-free split (= ODC).
    Per row: extraction time, counts, the manifold check, and the fitting
    error mean |phi - 1/2| at area-uniform samples of the mesh (phi from the
    fp32 field evaluation on the GPU).  With --ablation-field sdf the input is
    a signed distance psi (the same zero set): the MDC row interpolates psi
    itself and the fitting error is mean |psi|, as for the paper's DeepSDF
    results."""
    import torch
    from paper_2409_13418_amd import odc
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from meshcheck import is_closed_oriented_manifold, sample_surface

    sdf = args.ablation_field == "sdf"
    field = I.sdf_mlp_field(3) if sdf else I.mlp_field(3)
    mdc = 7 | (I.ABL_SDF_INPUT if sdf else 0)
    prec = _prec(odc, args.precision)
    ctx = odc.Context(0)
    df = odc.DeviceField(field)
    rows = []
    for name, mode, clamp in (("MDC", mdc, 0), ("+ 1D search", 6, 0), ("+ 2D search", 4, 0),
                              ("+ IC (= ODC)", 0, 0), ("+ 2D search, 3D points clamped", 4, 1),
                              ("+ IC, 3D points clamped", 0, 1)):
        grid = I.unit_grid(args.res, 15)
        grid.ablation = mode
        grid.clamp = clamp
        params = odc.default_params(grid, prec)
        for _ in range(max(args.warmup, 1)):
            ctx.extract(df, params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.extract_async(df, params, cap_hint=(ctx.cap_v, ctx.cap_t))
            counts = ctx.sync()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        r = ctx.extract(df, params)
        v = r["vertices"].cpu().numpy().astype(np.float64)
        t = r["triangles"].cpu().numpy()
        ok, why = is_closed_oriented_manifold(t, len(v))
        pts = sample_surface(v, t, args.ablation_samples, seed=5)
        z = ctx.field_eval(df, pts).astype(np.float64)
        fit = float(np.mean(np.abs(z) if sdf else np.abs(0.5 * np.tanh(0.5 * z))))
        si = ctx.self_intersections(r["vertices"], r["triangles"], grid.h)
        rows.append({"row": name, "ablation": mode, "clamp_vertices": clamp, "ms": ms,
                     "cells_per_s": counts["n_active_cells"] / (ms / 1e3),
                     "n_vertices": counts["n_vertices"], "n_triangles": counts["n_triangles"],
                     "n_case3": r["n_case3"], ("abs_psi" if sdf else "abs_phi_minus_half"): fit,
                     "self_intersecting_pairs": si, "closed_manifold": bool(ok)})
        print(f"# {name}: {ms:.1f} ms, {'|psi|' if sdf else '|phi-1/2|'} {fit:.3e}, SI pairs {si}, "
              f"V {counts['n_vertices']}, "
              f"T {counts['n_triangles']}, manifold {ok}", file=sys.stderr, flush=True)
    emit({
        "metric": f"Table 3 ablation rows on the {args.res}^3 MLP "
                  f"{'signed-distance' if sdf else 'occupancy'} field", "n_gpus": 1,
        "dtype": DTYPE[args.precision], "data": "synthetic",
        "steps": args.steps,
        "config": {"workload": f"{'sdf' if sdf else 'mlp'}{args.res}_ablation", "res": args.res,
                   "samples": args.ablation_samples,
                   "fit": ("mean |psi| = mean |z| at area-uniform mesh samples" if sdf else
                           "mean |phi - 1/2| = mean |tanh(z/2)|/2 at area-uniform mesh samples"),
                   "self_intersections": "pairs of vertex-disjoint triangles that intersect"},
        "rows": rows}, args)


def _csg_mode(args):
    """The analytic CSG field through the same path and timing as the
    default line (its labels, bisection and searches run on the vector ALUs,
    one query per thread)."""
    from paper_2409_13418_amd import odc
    field = I.csg_random_field(2)
    grid = I.unit_grid(args.res, 15)
    ctx = odc.Context(0)
    df = odc.DeviceField(field)
    params = odc.default_params(grid, odc.PREC_BF16_GUARDED)
    ms_per_step, step_ms, stages, counts = _timed(ctx, df, params, args.steps, args.warmup)
    emit({"metric": f"active cells meshed/sec at {args.res}^3 CSG occupancy",
          "value": counts["n_active_cells"] / (ms_per_step / 1e3), "unit": "cells/s",
          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
          "data": "synthetic",
          "config": {"workload": f"csg{args.res}", "res": args.res,
                     "field": "union of 48 boxes and 16 spheres minus 8 boxes, seed 2",
                     "iters_1d": grid.iters_1d},
          "counts": {k: counts[k] for k in COUNT_KEYS}, "stages_ms": stages}, args,
         [{"step": i, "ms": t, "workload": f"csg{args.res}"} for i, t in enumerate(step_ms)])


def _copy_mode(args):
    import torch
    n = int(args.copy_mib) << 20
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    emit({"mode": "copy", "bytes_read": n, "bytes_written": n, "copies": args.steps,
          "GB_per_s": 2 * n / dt / 1e9}, args)


COUNT_KEYS = ("n_active_cells", "n_active_edges", "n_pairs", "n_vertices", "n_triangles",
              "n_queries", "n_search2d_queries", "n_search2d_needed", "n_corner_queries",
              "n_guard_corners", "n_fp64_cells")


def _timed(ctx, df, params, steps: int, warmup: int):
    """warmup untimed extractions, then `steps` timed ones (stage events on);
    returns ms per step, the per-step wall times, mean stage ms, counts."""
    import torch
    from paper_2409_13418_amd import odc
    for _ in range(warmup):
        ctx.extract(df, params)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    step_ms = []
    stages = {k: 0.0 for k in odc.STAGES}
    counts = None
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        ctx.extract_async(df, params, cap_hint=(ctx.cap_v, ctx.cap_t))
        counts = ctx.sync()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        for k, v in ctx.stage_times().items():
            stages[k] += v
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    ctx.set_timing(False)
    return total_s * 1e3 / steps, step_ms, {k: v / steps for k, v in stages.items()}, counts


def _roofline(odc, field, grid, counts, stages, prec):
    """The dominant stage's kernel against its matrix-core peak, and every
    query stage: algorithmic FLOP = queries the method needs x the network's
    FLOP per query (corners: every corner query made, all of them unless the
    evaluation is coarse to fine, plus the fp32 re-evaluation of the guard
    band; 1D: k per crossing edge; 2D: the per-pair count with early exits).  bf16-guarded and fp32 searches run on the fp32 matrix peak;
    split-bf16 searches on the bf16 peak, executing six bf16 products per
    binary32-accurate one (reported as the executed fraction)."""
    per_query = MLP_FLOP_PER_QUERY(field)
    x3 = prec == odc.PREC_BF16_X3
    search_peak = PEAK_BF16_MFMA if x3 else PEAK_FP32_MFMA
    corner_peak = PEAK_FP32_MFMA if prec == odc.PREC_FP32 else PEAK_BF16_MFMA
    flop = {"labels": counts["n_corner_queries"] * per_query,
            "bisect": counts["n_active_edges"] * grid.iters_1d * per_query,
            "search2d": counts["n_search2d_needed"] * per_query}
    guard = counts["n_guard_corners"] * per_query
    at_peak = {"labels": flop["labels"] / corner_peak + guard / PEAK_FP32_MFMA,
               "bisect": flop["bisect"] / search_peak,
               "search2d": flop["search2d"] / search_peak}
    stages_out = {k: {"ms": stages[k], "ms_at_peak": v * 1e3, "frac": v * 1e3 / stages[k]}
                  for k, v in at_peak.items()}
    stages_out["extraction"] = {
        "ms": sum(stages.values()), "ms_at_peak": sum(at_peak.values()) * 1e3,
        "frac": sum(at_peak.values()) * 1e3 / sum(stages.values())}
    dom = max(("bisect", "search2d", "labels"), key=lambda k: stages[k])
    peak = corner_peak if dom == "labels" else search_peak
    kern = {"labels": "k_labels_mlp", "bisect": "k_bisect_x3" if x3 else "k_bisect_mlp",
            "search2d": "k_search2d_x3" if x3 else "k_search2d_mlp"}[dom]
    achieved = flop[dom] / (stages[dom] / 1e3)
    rl = {"bound": "mfma", "kernel": kern, "achieved": achieved / 1e12, "peak": peak / 1e12,
          "unit": "TFLOP/s", "frac": achieved / peak,
          "traffic": measured_traffic(kern)}
    if x3 and dom != "labels":
        rl["bf16_products_per_flop"] = 6
        rl["executed_frac"] = 6 * achieved / peak
    return rl, stages_out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=("single", "batch", "serve", "copy", "ablation", "csg"),
                    default="single")
    ap.add_argument("--ablation-samples", type=int, default=1000000)
    ap.add_argument("--ablation-field", choices=("occupancy", "sdf"), default="occupancy")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-requests", type=int, default=1200)
    ap.add_argument("--serve-warmup-s", type=float, default=10.0)
    ap.add_argument("--serve-lanes", type=int, default=2)
    ap.add_argument("--serve-budget-gib", type=float, default=24.0)
    ap.add_argument("--serve-policy", choices=("fifo", "shortest", "banded"), default="banded")
    ap.add_argument("--serve-band", type=float, default=8.0)
    ap.add_argument("--serve-age-ms", type=float, default=1000.0)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=("bf16", "fp32", "x3"), default="bf16")
    ap.add_argument("--res", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-seconds-1core", type=float, default=10.0)
    ap.add_argument("--fp32-steps", type=int, default=4,
                    help="timed steps of the plain fp32 path after the guarded path's")
    ap.add_argument("--x3-steps", type=int, default=6,
                    help="timed steps with split-bf16 searches after the guarded path's")
    ap.add_argument("--adaptive-steps", type=int, default=4,
                    help="timed steps with coarse-to-fine corner evaluation after the guarded path's")
    ap.add_argument("--serve-requests-default", type=int, default=300,
                    help="requests of the Poisson trace served after the timed steps (0: none)")
    ap.add_argument("--serve-warmup-default-s", type=float, default=3.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--jsonl", default=None,
                    help="also append the result (and per-step records) to this JSONL file")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library meshes on one GPU only; run with --gpus 1"}))
        sys.exit(2)

    if args.mode == "batch":
        return _batch_mode(args)
    if args.mode == "serve":
        return _serve_mode(args)
    if args.mode == "copy":
        return _copy_mode(args)
    if args.mode == "csg":
        return _csg_mode(args)
    if args.mode == "ablation":
        return _ablation_mode(args)

    import torch
    from paper_2409_13418_amd import odc

    field = I.mlp_field(3)
    grid = I.unit_grid(args.res, 15)
    prec = _prec(odc, args.precision)
    ctx = odc.Context(0)
    df = odc.DeviceField(field)
    params = odc.default_params(grid, prec)
    ms_per_step, step_ms, stages, counts = _timed(ctx, df, params, args.steps, args.warmup)
    value = counts["n_active_cells"] / (ms_per_step / 1e3)
    roofline, roofline_stages = _roofline(odc, field, grid, counts, stages, prec)
    out = {
        "metric": "active cells meshed/sec at 256^3 MLP occupancy",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"mlp{args.res}_{args.precision}", "res": args.res,
                   "field": "sigmoid(-20 sdf + 0.3 MLP): 32 spheres, 6 bands, 4x256 ReLU, seed 3",
                   "iters_1d": grid.iters_1d, "precision": args.precision},
        "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "counts": {k: counts[k] for k in COUNT_KEYS},
        "stages_ms": stages,
        "roofline": roofline,
        "roofline_stages": roofline_stages,
    }
    # the other precisions on the same grid, outside the timed region above:
    # the plain fp32 path (every query on fp32 matrix cores; its mesh must be
    # the guarded path's bit for bit) and split-bf16 searches (same corner
    # signs, hence the same topology)
    if prec == odc.PREC_BF16_GUARDED:
        ref = ctx.extract(df, params, want_local=True)
        ref_tris = ref["triangles"].cpu().numpy().copy()
        ref_labels = ctx.intermediate("labels").copy()
        ref_cells = ctx.intermediate("cell_ids").copy()
        for name, steps in (("fp32", args.fp32_steps), ("x3", args.x3_steps),
                            ("adaptive", args.adaptive_steps)):
            if steps <= 0:
                continue
            p2 = odc.default_params(grid, _prec(odc, "bf16" if name == "adaptive" else name))
            if name == "adaptive":
                # coarse-to-fine corners: 4-cell coarse grid, logit band 1.5 x the
                # exactness condition for a logit slope of 20 (the sdf gain)
                p2.coarse_step = ADAPTIVE_STEP
                p2.coarse_band = 1.5 * 20.0 * math.sqrt(3.0) * ADAPTIVE_STEP / grid.res
            ms2, _, st2, c2 = _timed(ctx, df, p2, steps, 1)
            r2 = ctx.extract(df, p2, want_local=True)
            same_topo = bool(np.array_equal(ctx.intermediate("labels"), ref_labels) and
                             np.array_equal(ctx.intermediate("cell_ids"), ref_cells))
            same = bool(np.array_equal(r2["triangles"].cpu().numpy(), ref_tris))
            rl, rs = _roofline(odc, field, grid, c2, st2, p2.precision)
            out[f"{name}_path"] = {
                "value": c2["n_active_cells"] / (ms2 / 1e3), "unit": "cells/s",
                "ms_per_step": ms2, "steps": steps, "stages_ms": st2,
                "counts": {k: c2[k] for k in COUNT_KEYS},
                "same_labels_and_cells_as_bf16": same_topo, "same_mesh_as_bf16": same,
                "roofline": rl, "roofline_stages": rs}
    out["quality"] = mesh_quality(ctx, df, grid, params=params)
    if args.serve_requests_default > 0:
        sv = serve_run(args, args.serve_requests_default, args.serve_warmup_default_s)
        out["serve"] = {k: sv[k] for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "completed",
                                          "failed", "batches", "window_s", "p50_ms_by_res",
                                          "p99_ms_by_res")}
        out["serve"].update({"cells_per_s": sv["value"], "config": sv["config"]})
    if not args.no_cpu_baseline:
        precs = {args.precision: prec}
        if prec == odc.PREC_BF16_GUARDED:
            precs["fp32"] = odc.PREC_FP32
            precs["x3"] = odc.PREC_BF16_X3
        cb = cpu_baseline(field, grid, args.cpu_seconds, chamfer=(ctx, df, precs))
        cham = cb.pop("chamfer_vs_oracle", None)
        one = cpu_baseline(field, grid, args.cpu_seconds_1core, seed=1, threads=1)
        cb["one_core"] = {k: one[k] for k in ("value", "unit", "cores", "sample")}
        out["cpu_baseline"] = cb
        if cham is not None:
            out["chamfer_vs_oracle"] = cham
    emit(out, args, [{"step": i, "ms": t, "workload": out["config"]["workload"]}
                     for i, t in enumerate(step_ms)])


if __name__ == "__main__":
    main()
