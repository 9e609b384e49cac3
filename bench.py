#!/usr/bin/env python3
"""Benchmark of the fused implicit mover + ten-moment gathering on one GPU.

Workload: Harris-sheet box of 128x64x32 cells, 64 particles per cell x 4
species (67,108,864 particles), dt = 0.25, three mover iterations, fixed
analytic fields.  One step = the fused mover + moment pass over every
species (plus the cell sort at its cadence).  The headline `value` is the
FP32-particle / FP64-moment path; the FP64 path is reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2008_04397_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s (mover+moments) FP32 vs FP64; % HBM peak; p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n_particles: int, nodes: int, s_p: int, s_f: int) -> float:
    """Bytes one fused launch over one species must move: read x,y,z,u,v,w,q
    (7 s_p), write x,y,z,u,v,w (6 s_p) per particle; read the six field
    arrays and write the ten FP64 moment arrays once."""
    return n_particles * 13 * s_p + 6 * nodes * s_f + 10 * nodes * 8


def run_gpu(h, dtype_name: str, steps: int, warmup: int, sort_every: int, path: int):
    import torch
    from paper_2008_04397_amd import spic

    dt = torch.float32 if dtype_name == "f32" else torch.float64
    g = h.grid
    ctx = spic.Context(0)
    if path:
        ctx.set_option("path", path)
    log("[bench] generating %s inputs (%d particles)" % (dtype_name, h.n_total))
    t0 = time.time()
    f = spic.to_device(W.make_fields(h), dt)
    species = []
    for s in range(4):
        sp = W.make_species(h, s, dtype=np.float32 if dtype_name == "f32" else np.float64, with_id=False)
        species.append(spic.to_device(sp, dt))
        del sp
    moms = spic.moment_buffers(g, 4, torch.float64)
    log("[bench] inputs resident in HBM after %.1f s" % (time.time() - t0))
    stream = torch.cuda.current_stream()

    def step(k, ev=None):
        prm = spic.make_params(h.dt, h.c, h.niter, sort_every, k)
        if ev is None:
            spic.spic_mover(ctx, g, prm, f, species, h.qoms, moms, stream=stream)
            return
        # one call per species so each fused launch is bracketed by events
        for s in range(4):
            ev[s][0].record(stream)
            spic.spic_mover(ctx, g, prm, f, [species[s]], [h.qoms[s]], [moms[s]], stream=stream)
            ev[s][1].record(stream)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(4)]
           for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(steps):
        step(warmup + k, evs[k])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    launch_ms = np.array([[evs[k][s][0].elapsed_time(evs[k][s][1]) for s in range(4)] for k in range(steps)])
    ctx.close()
    del species, f, moms
    torch.cuda.empty_cache()
    n = h.n_total
    s_p = 4 if dtype_name == "f32" else 8
    per_launch_bytes = algorithmic_bytes(h.n_per_species, g.nodes, s_p, s_p)
    avg_launch_s = float(launch_ms.mean()) / 1e3
    achieved = per_launch_bytes / avg_launch_s / 1e9
    step_ms = total_ms / steps
    per_step = launch_ms.sum(axis=1)
    return {
        "value": n * steps / (total_ms / 1e3),
        "ms_per_step": step_ms,
        "ms_per_step_mean": float(per_step.mean()),
        "ms_per_step_std": float(per_step.std()),
        "ms_per_step_median": float(np.median(per_step)),
        "wall_s": wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": per_launch_bytes, "avg_launch_ms": avg_launch_s * 1e3},
    }


def cpu_baseline(h, target_s: float = 12.0):
    """The FP64 oracle on a bounded sample: a seeded 1/64 subsample of every
    species of the same workload (full grid), stepped until ~target_s."""
    from oracle import oracle as O
    f = W.make_fields(h)
    subs = []
    for s in range(4):
        sp = W.make_species(h, s)
        m = W.subsample_mask(sp["id"], 64, seed=7)
        subs.append({k: v[m] for k, v in sp.items()})
        del sp
    n = sum(s["x"].size for s in subs)
    steps = 0
    t0 = time.perf_counter()
    states = subs
    while True:
        states = [O.step(h.grid, h.dt, h.c, h.niter, h.qoms[s], f, states[s])[0] for s in range(4)]
        steps += 1
        el = time.perf_counter() - t0
        if el >= target_s or steps >= 40:
            break
    return {"value": n * steps / el, "unit": "particle-steps/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": "seeded 1/64 subsample by particle-id hash of all 4 species (%d particles) on the full "
                      "128x64x32 grid, %d fused steps (mover + FP64 deposit), %.1f s" % (n, steps, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--path", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the particle decomposition across GPUs is described, not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2008_04397_amd import spic
    spic.lib()  # fail loudly if the HIP library is missing

    h = W.harris_128x64x32()
    r32 = run_gpu(h, "f32", args.steps, args.warmup, args.sort_every, args.path)
    log("[bench] f32: %.3e particle-steps/s, %.3f ms/step, %.1f%% HBM" %
        (r32["value"], r32["ms_per_step"], 100 * r32["roofline"]["frac"]))
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(h, "f64", args.steps, args.warmup, args.sort_every, args.path)
        log("[bench] f64: %.3e particle-steps/s, %.3f ms/step, %.1f%% HBM" %
            (r64["value"], r64["ms_per_step"], 100 * r64["roofline"]["frac"]))
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(h)
        log("[bench] cpu oracle: %.3e particle-steps/s on %d threads" % (cpu["value"], cpu["cores"]))
    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "harris_128x64x32_ppc64_4species", "cells": [128, 64, 32],
                   "particles": h.n_total, "species": 4, "ppc": 64, "niter_mover": h.niter, "dt": h.dt,
                   "precision": "f32 particles and mover, f64 moment accumulation",
                   "sort_every": args.sort_every, "path": args.path or "auto"},
        "roofline": r32["roofline"],
        "cpu_baseline": cpu,
        "ms_per_step_stats": {k: r32[k] for k in ("ms_per_step_mean", "ms_per_step_std", "ms_per_step_median")},
    }
    if r64 is not None:
        out["fp64"] = {"value": r64["value"], "unit": "particle-steps/s", "dtype": "f64",
                       "ms_per_step": r64["ms_per_step"], "roofline": r64["roofline"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
