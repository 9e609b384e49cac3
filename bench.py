#!/usr/bin/env python3
"""Benchmark of the fused implicit mover + ten-moment gathering on one GPU.

Workload: Harris-sheet box of 128x64x32 cells, 64 particles per cell x 4
species (67,108,864 particles), dt = 0.25, three mover iterations, fixed
analytic fields.  One step = the fused mover + moment pass over every
species (plus the cell sort at its cadence).  The headline `value` is the
FP32-particle / FP64-moment path; the FP64 path is reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu] [--tune]
Prints one JSON line.

Other measured configurations (one JSON line each):
  --mode ensemble   64 independent Harris boxes of uneven size (16x8x4 ..
                    128x64x8 cells, ppc 8/27/64, B0 in [0.01, 0.03], mass
                    ratio 25/64/100), FP32, 50 steps each, one batch
                    submission (persistent work-list launch per step, hipGraph
                    replay)
  --mode streamed   512x256x32 cells x 125 ppc x 4 species (2.1e9 FP32
                    particles in pinned host memory) streamed through a 16 GB
                    HBM budget in batches of 2^26, sort every 4 steps, 5 steps
                    (--fraction f keeps the first f of the x-slabs)
  --mode cadence    the 128x64x32 box for --steps steps (e.g. 500) with a sort
                    only at step 0 and every 1, 4 and 10 steps: throughput
                    per window of steps (how fast locality decays)
  --mode serving    Poisson arrivals (20/s) of Harris-box runs (16x8x4 ..
                    256x128x8 cells, ppc 8..64, 10..200 steps), continuous
                    batching vs one-at-a-time on the same GPU, p50/p99 latency
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2008_04397_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# what each path computes in which precision (the default launch)
PRECISION = {
    "f32": "f32 particles and mover; deposit weights in f64, the ten terms in f32 and summed in f32 over the "
           "particles one lane holds in one cell (~16 at 64 per cell), every further sum in f64",
    "f64": "f64 particles, mover and moment accumulation",
}
METRIC = "particle-steps/s (mover+moments) FP32 vs FP64; % HBM peak; p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "traffic_harris_128x64x32_{}.md")
KERNEL_SOURCES = ("paper_2008_04397_amd/csrc/spic_tiled.hip", "paper_2008_04397_amd/csrc/spic_device.h",
                  "paper_2008_04397_amd/csrc/spic_impl.h")


SQ_PROFILE = os.path.join(HERE, "profiles", "sq_counters_harris_128x64x32_{}.md")


def _profile_fields(path: str, launch) -> Optional[dict]:
    """The `key: value` lines of a committed profile summary, or None when
    the kernel sources changed since it was taken or the launch settings
    differ from the profiled ones."""
    try:
        txt = open(path).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(\w+): (.*)$", txt, re.M))
    h = hashlib.sha256(b"".join(open(os.path.join(HERE, p), "rb").read() for p in KERNEL_SOURCES)).hexdigest()
    if fields.get("kernel_source_sha256", "").strip() != h:
        return None
    profiled = {k: int(v) for k, v in re.findall(r"(\w+) (\d+)", fields.get("config", ""))}
    if any(launch.get(k) != profiled.get(k) for k in ("tile_variant", "tile_block", "bank_align", "sort_every")):
        return None
    return fields


def valu_ceiling(launch, dtype_name: str, bytes_per_pass: float) -> Optional[dict]:
    """The VALU-issue ceiling of the species pass from the committed SQ
    counters: VALU wave-instructions per particle-wave, the time they take
    at one wave-instruction per CU clock (256 CUs x 2.4 GHz), and the HBM
    fraction the pass could reach if it took only that long."""
    fields = _profile_fields(SQ_PROFILE.format(dtype_name), launch)
    if not fields or "valu_issue_us_per_pass" not in fields:
        return None
    us = float(fields["valu_issue_us_per_pass"])
    return {"valu_per_particle_wave": float(fields["valu_per_particle_wave"]), "valu_issue_ms_per_pass": us / 1e3,
            "hbm_frac_at_valu_issue": bytes_per_pass / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}


def measured_traffic(launch, dtype_name: str) -> Optional[float]:
    """HBM bytes per species pass (the fused kernel, or the mover and
    deposit kernels of the split variant) from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary of that particle dtype, or None when the
    kernel sources changed since the counters were taken or the launch
    configuration differs."""
    fields = _profile_fields(TRAFFIC_PROFILE.format(dtype_name), launch)
    return float(fields["traffic_bytes_per_launch"]) if fields else None


def algorithmic_bytes(n_particles: int, nodes: int, s_p: int, s_f: int) -> float:
    """Bytes one fused launch over one species must move: read x,y,z,u,v,w,q
    (7 s_p), write x,y,z,u,v,w (6 s_p) per particle; read the six field
    arrays and write the ten FP64 moment arrays once."""
    return n_particles * 13 * s_p + 6 * nodes * s_f + 10 * nodes * 8


# library options given on the command line (--option KEY=VALUE), applied to
# every context the bench creates
EXTRA_OPTS = {}


def _new_ctx(spic, *a):
    ctx = spic.Context(*a)
    for k, v in EXTRA_OPTS.items():
        ctx.set_option(k, v)
    return ctx


def _warm_device(seconds: float = 0.3):
    """Keep the GPU busy with plain fills for `seconds` before any timed
    work, so the first timed steps of a fresh process do not run at idle
    clocks (the particle state is not touched)."""
    import torch
    buf = torch.empty(1 << 27, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            buf.fill_(1.0)
        torch.cuda.synchronize()
    del buf


def run_gpu(h, dtype_name: str, steps: int, warmup: int, sort_every: int, path: int, tune: bool = True,
            variant: int = -1, tol: float = 0.0, niter: int = 3):
    import torch
    from paper_2008_04397_amd import autotune, spic

    dt = torch.float32 if dtype_name == "f32" else torch.float64
    g = h.grid
    ctx = _new_ctx(spic, 0)
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
    tuned = None
    if tune and not path:
        key = autotune.workload_class(dtype_name, g, h.ppc)
        tuned = autotune.load(key)
        if tuned is None:
            tuned = autotune.tune(h, f, species, h.qoms, moms, steps=16, log=log, dtype_name=dtype_name)
            autotune.store(key, tuned)
        autotune.apply(ctx, tuned)
        if sort_every < 0:
            sort_every = tuned["sort_every"]
        log("[bench] tuned %s: %s" % (key, tuned))
    if sort_every < 0:
        sort_every = 4
    if variant >= 0:
        ctx.set_option("tile_variant", variant)
    launch = spic.resolved_launch(ctx, "f32" if dtype_name == "f32" else "f64")
    launch["sort_every"] = sort_every

    def step(k, ev=None):
        prm = spic.make_params(h.dt, h.c, niter, sort_every, k, tol=tol)
        if ev is None:
            spic.spic_mover(ctx, g, prm, f, species, h.qoms, moms, stream=stream)
            return
        # one call per species so each fused launch is bracketed by events
        for s in range(4):
            ev[s][0].record(stream)
            spic.spic_mover(ctx, g, prm, f, [species[s]], [h.qoms[s]], [moms[s]], stream=stream)
            ev[s][1].record(stream)

    _warm_device()
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
    # the fused pass's own launches: calls on steps without a sort launch only
    # the moment zeroing (~6 us) and the fused kernel (or, split, the mover
    # and deposit kernels)
    sort_step = np.array([sort_every > 0 and (warmup + k) % sort_every == 0 for k in range(steps)])
    fused_ms = launch_ms[~sort_step] if (~sort_step).any() else launch_ms
    avg_launch_s = float(fused_ms.mean()) / 1e3
    achieved = per_launch_bytes / avg_launch_s / 1e9
    # measured HBM bytes of the same launches (rocprofv3 counters, profiles/)
    traffic_bytes = measured_traffic(launch, dtype_name) if not path else None
    traffic = traffic_bytes / avg_launch_s / 1e9 if traffic_bytes else None
    step_ms = total_ms / steps
    per_step = launch_ms.sum(axis=1)
    sort_ms = float(launch_ms[sort_step].mean() - fused_ms.mean()) if sort_step.any() else 0.0
    return {
        "tuned": tuned, "sort_every": sort_every, "launch": launch,
        "value": n * steps / (total_ms / 1e3),
        "ms_per_step": step_ms,
        "ms_per_step_mean": float(per_step.mean()),
        "ms_per_step_std": float(per_step.std()),
        "ms_per_step_median": float(np.median(per_step)),
        "wall_s": wall,
        "sort_ms_per_species": sort_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("k_fused_tiled (mover) + k_deposit_tiled (sorted register deposit), one pair per "
                                "species" if launch.get("tile_variant") == 2 else "k_fused_tiled (one launch per species)"),
                     "bytes_per_launch": per_launch_bytes, "avg_launch_ms": avg_launch_s * 1e3,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "alu_ceiling": valu_ceiling(launch, dtype_name, per_launch_bytes) if not path else None},
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(h, reps: int = 5):
    """The FP64 oracle (C, OpenMP; never tuned for this) timed on this host:
    the 32x16x4 box in full (4 species x 27 ppc, 10 fused steps) and a
    seeded 1/64 subsample (by particle-id hash) of every species of the
    128x64x32 box on its full grid (one fused step), each on all host cores
    and on one core, the median of `reps` runs.  `value` is the subsample on
    all cores, in particle-steps/s (a fused step: mover + FP64 deposit)."""
    from oracle import oracle as O
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)

    def timed(hh, f, species, nsteps, threads):
        used = O.set_threads(threads)
        n = sum(sp["x"].size for sp in species)
        ts = []
        for _ in range(reps):
            states = species
            t0 = time.perf_counter()
            for _ in range(nsteps):
                states = [O.step(hh.grid, hh.dt, hh.c, hh.niter, hh.qoms[s], f, states[s])[0]
                          for s in range(len(states))]
            ts.append(time.perf_counter() - t0)
        med = float(np.median(ts))
        return {"value": n * nsteps / med, "threads": used, "median_s": med, "particles": n, "steps": nsteps}

    h1 = W.harris_32x16x4()
    f1, sp1 = W.make_fields(h1), W.make_all_species(h1)
    f2 = W.make_fields(h)
    subs = []
    for s in range(4):
        sp = W.make_species(h, s)
        m = W.subsample_mask(sp["id"], 64, seed=7)
        subs.append({k: v[m] for k, v in sp.items()})
        del sp
    runs = {}
    for name, args in (("harris_32x16x4_full_10_steps", (h1, f1, sp1, 10)),
                       ("harris_128x64x32_subsample_1_64_one_step", (h, f2, subs, 1))):
        runs[name] = {"all_cores": timed(*args, nproc), "one_core": timed(*args, 1)}
    O.set_threads(nproc)
    head = runs["harris_128x64x32_subsample_1_64_one_step"]["all_cores"]
    return {"value": head["value"], "unit": "particle-steps/s", "cores": head["threads"], "kind": "oracle",
            "sample": "seeded 1/64 subsample by particle-id hash of all 4 species of the 128x64x32 box (%d "
                      "particles) on its full grid, one fused step (mover + FP64 deposit), median of %d runs on "
                      "all %d host cores" % (head["particles"], reps, head["threads"]),
            "nproc": nproc, "cpu_model": _cpu_model(), "runs": runs}


def _engine_ctx(budget=0, tuned_key=None, variant=-1):
    from paper_2008_04397_amd import autotune, spic
    ctx = _new_ctx(spic, 0, budget)
    cfg = autotune.load(tuned_key) if tuned_key else None
    if cfg:
        autotune.apply(ctx, cfg)
    if variant >= 0:
        ctx.set_option("tile_variant", variant)
    return ctx


def bench_ensemble(args):
    """64 independent boxes, one batch submission, 50 steps each.  With
    --tune the engine's block size, the runs' sort cadence and the work-list
    batch length are first tuned on the same boxes (8-step trials; cached
    per workload)."""
    import torch
    from paper_2008_04397_amd import autotune, spic
    boxes = W.ensemble_boxes(64)
    nsteps = 50
    log("[bench] generating 64 boxes")
    data, total, gbytes = [], 0, 0.0
    for b, h in enumerate(boxes):
        f = W.fields_tensors(h, dtype=torch.float32)
        sps = [W.species_tensors(h, s, dtype=torch.float32) for s in range(4)]
        moms = spic.moment_buffers(h.grid, 4, torch.float64)
        data.append((h, f, sps, moms))
        total += h.n_total
        gbytes += algorithmic_bytes(h.n_total, h.grid.nodes, 4, 4) + 3 * (6 * h.grid.nodes * 4 + 10 * h.grid.nodes * 8)
    torch.cuda.synchronize()

    def make_runs(se, k):
        return [spic.Run(h.grid, spic.make_params(h.dt, h.c, h.niter, se, 0), f, sps, h.qoms, moms, k)
                for h, f, sps, moms in data]

    key = "engine/f32/ensemble64"
    tuned = autotune.load(key) if args.tune else None
    if args.tune and tuned is None:
        log("[bench] tuning the engine on the ensemble")
        snap = [autotune.snapshot(sps) for _, _, sps, _ in data]

        def reset():
            for (_, _, sps, _), sn in zip(data, snap):
                autotune.restore(sps, sn)

        tuned = autotune.tune_runs(lambda: _engine_ctx(variant=args.variant), make_runs,
                                   autotune.engine_candidates(quick=True), steps=8, log=log, reset=reset)
        reset()
        del snap
        autotune.store(key, tuned)
    ctx = _engine_ctx(variant=args.variant)
    se = 4
    if tuned:
        autotune.apply(ctx, tuned)
        se = tuned["sort_every"]
        log("[bench] tuned %s: %s" % (key, tuned))
    log("[bench] %d particles in %d boxes; submitting" % (total, len(boxes)))
    # warm-up: one step of every box (not timed)
    for t in spic.spic_batch_submit(ctx, make_runs(se, 1)):
        spic.spic_wait(ctx, t)
    t0 = time.perf_counter()
    tickets = spic.spic_batch_submit(ctx, make_runs(se, nsteps))
    dev = [spic.spic_wait(ctx, t) for t in tickets]
    wall = time.perf_counter() - t0
    ctx.close()
    ps = total * nsteps
    achieved = gbytes * nsteps / wall / 1e9
    return {"metric": METRIC, "mode": "ensemble", "value": ps / wall, "unit": "particle-steps/s", "n_gpus": 1,
            "steps": nsteps, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "ensemble_64_harris_boxes", "boxes": len(boxes), "particles": total,
                       "precision": PRECISION["f32"], "sort_every": se, "tuned": tuned,
                       "tick_items": (tuned or {}).get("tick_items", 4096)},
            "wall_s": wall, "max_run_device_s": max(dev),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None}}


def bench_streamed(args):
    """The 2.1e9-particle box streamed through a 16 GiB budget (with
    --tune, the batch length and cadence are tuned first)."""
    import torch
    from paper_2008_04397_amd import autotune, spic
    h = W.harris_512x256x32()
    g = h.grid
    nx_used = max(1, int(round(g.nx * args.fraction)))
    n_all = 4 * nx_used * g.ny * g.nz * h.ppc
    # 16 GiB; a reduced box (--fraction) whose particles would fit twice
    # over gets a quarter of its particle bytes instead, so that every step
    # still streams every batch over the link
    budget = 16 * (1 << 30)
    if n_all * 28 < 2 * budget:
        budget = n_all * 28 // 4
    tuned, batch, se = None, 1 << 26, 4
    f = W.fields_tensors(h, dtype=torch.float32)
    species, total = [], 0
    log("[bench] generating %d x-slabs of 512 into pinned host memory" % nx_used)
    t0 = time.time()
    for s in range(4):
        n = nx_used * g.ny * g.nz * h.ppc
        host = {k: torch.empty(n, dtype=torch.float32, pin_memory=True) for k in ("x", "y", "z", "u", "v", "w", "q")}
        step_slabs = 8
        for i0 in range(0, nx_used, step_slabs):
            i1 = min(nx_used, i0 + step_slabs)
            t = W.species_tensors(h, s, i0, i1, dtype=torch.float32)
            a = i0 * g.ny * g.nz * h.ppc
            for k in host:
                host[k][a:a + t[k].numel()].copy_(t[k])
            del t
        species.append(host)
        total += n
        log("[bench] species %d ready (%.1f s)" % (s, time.time() - t0))
    moms = spic.moment_buffers(g, 4, torch.float64)
    nsteps = 5

    def make_runs(se_, k):
        return [spic.Run(g, spic.make_params(h.dt, h.c, h.niter, se_, 0), f, species, h.qoms, moms, k)]

    if args.tune:
        key = "stream/f32/%dx%dx%d/n%d/budget%d" % (nx_used, g.ny, g.nz, total, budget)
        tuned = autotune.load(key)
        if tuned is None:
            log("[bench] tuning the streamed batch length")
            tuned = autotune.tune_runs(lambda: _new_ctx(spic, 0, budget), make_runs,
                                       autotune.stream_candidates(quick=True), steps=4, log=log)
            autotune.store(key, tuned)
        batch, se = tuned["batch_particles"], tuned["sort_every"]
    ctx = _new_ctx(spic, 0, budget)
    ctx.set_option("batch_particles", batch)
    run = make_runs(se, nsteps)[0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dev = spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [run])[0])
    wall = time.perf_counter() - t1
    ctx.close()
    # every step uploads and downloads the 7 FP32 arrays of every batch
    link = total * nsteps * (28 + 28) / wall / 1e9
    return {"metric": METRIC, "mode": "streamed", "value": total * nsteps / wall, "unit": "particle-steps/s",
            "n_gpus": 1, "steps": nsteps, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "harris_512x256x32_ppc125_4species_streamed", "particles": total,
                       "fraction_of_x_slabs": nx_used / g.nx, "hbm_budget_bytes": budget, "batch": batch,
                       "sort_every": se, "tuned": tuned},
            "wall_s": wall, "device_s": dev,
            "roofline": {"bound": "pcie", "achieved": link, "peak": 2 * 64.0, "unit": "GB/s",
                         "frac": link / 128.0, "traffic": None,
                         "note": "host<->device bytes (7 arrays up, 7 back, FP32) per second vs PCIe Gen5 x16 "
                                 "nominal 64 GB/s per direction"}}


def bench_cadence(args):
    """Long-run sort-cadence study on the 128x64x32 box (FP32): throughput
    per window of steps for a sort only at step 0, for sorts every 1, 4 and
    10 steps, for the autotuned cadence (tuned on a separate copy of the
    initial state) and for an adaptive cadence that sorts once the time the
    passes lost since the last sort (each step's time minus the first
    step's after that sort) reaches the sort's own cost (Sec. VI: locality
    decays without re-sorting).  For L2 counters per window, a tiny int32
    fill kernel marks the start of every window and an int64 fill the start
    of every arm, so counter rows can be split by dispatch order."""
    import torch
    from paper_2008_04397_amd import autotune, spic
    h = W.harris_128x64x32()
    g = h.grid
    nsteps, window = args.steps, max(1, args.steps // 10)
    f = spic.to_device(W.make_fields(h), torch.float32)
    moms = spic.moment_buffers(g, 4, torch.float64)
    stream = torch.cuda.current_stream()
    mark_window = torch.zeros(1, dtype=torch.int32, device="cuda")
    mark_arm = torch.zeros(1, dtype=torch.int64, device="cuda")

    def fresh():
        return [spic.to_device(W.make_species(h, s, dtype=np.float32, with_id=False), torch.float32)
                for s in range(4)]

    out, sorts, extra = {}, {}, {}
    for cad in ("once", 1, 4, 10, "tuned", "adaptive"):
        mark_arm.fill_(1)
        ctx = _new_ctx(spic, 0)
        if cad == "tuned":
            trial = fresh()
            cfg = autotune.tune(h, f, trial, h.qoms, moms, steps=16, log=log, dtype_name="f32")
            del trial
            autotune.apply(ctx, cfg)
            extra["tuned"] = cfg
            log("[cadence tuned] %s" % cfg)
        species = fresh()
        torch.cuda.synchronize()
        if cad == "once":
            spic.spic_sort(ctx, g, species, stream=stream)
        fixed = {"once": 0, "tuned": extra.get("tuned", {}).get("sort_every", 4), "adaptive": None}.get(cad, cad)
        rates, nsort = [], 0
        # adaptive state: the sort's cost, the first pass time after it and
        # the time lost since
        sort_cost, t0, lost, want = 0.0, None, 0.0, True
        for w0 in range(0, nsteps, window):
            mark_window.fill_(w0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for k in range(w0, min(nsteps, w0 + window)):
                if fixed is not None:
                    nsort += int(fixed > 0 and k % fixed == 0)
                    spic.spic_mover(ctx, g, spic.make_params(h.dt, h.c, h.niter, fixed, k), f, species, h.qoms,
                                    moms, stream=stream)
                    continue
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                spic.spic_mover(ctx, g, spic.make_params(h.dt, h.c, h.niter, 1 if want else 0, k), f, species,
                                h.qoms, moms, stream=stream)
                e1.record(stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1)
                if want:
                    sort_step_ms, want, t0, lost, nsort = ms, False, None, 0.0, nsort + 1
                elif t0 is None:
                    t0 = ms
                    sort_cost = max(0.0, sort_step_ms - t0)
                else:
                    lost += ms - t0
                    want = lost >= sort_cost
            b.record(stream)
            torch.cuda.synchronize()
            n = min(nsteps, w0 + window) - w0
            rates.append(h.n_total * n / (a.elapsed_time(b) / 1e3))
            log("[cadence %s] steps %d-%d: %.3e particle-steps/s" % (cad, w0, w0 + n - 1, rates[-1]))
        out[str(cad)] = rates
        sorts[str(cad)] = nsort
        ctx.close()
        del species
        torch.cuda.empty_cache()
    mark_arm.fill_(1)
    torch.cuda.synchronize()
    sustained = {k: float(np.mean(v[len(v) * 4 // 5:])) for k, v in out.items()}
    return {"metric": METRIC, "mode": "cadence", "value": float(np.mean(out["4"])), "unit": "particle-steps/s",
            "n_gpus": 1, "steps": nsteps, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "harris_128x64x32_ppc64_4species", "window_steps": window,
                       "cadences": ["sort at step 0 only", 1, 4, 10, "autotuned", "adaptive"],
                       "tuned": extra.get("tuned")},
            "rates_per_window": out, "sorts": sorts,
            "mean_rate": {k: float(np.mean(v)) for k, v in out.items()},
            "sustained_rate_last_fifth": sustained}


def bench_field(args):
    """The implicit field cycle (clean with CG, GMRes solve, update) on the
    128x64x32 box, FP64, with the moments of one mover step of its four
    species (FP32 particles, FP64 fields and moments).  Reports cycles per
    second, the iterations, and the roofline of the field-operator kernel:
    its algorithmic bytes per application are x (24 B), the susceptibility
    (72 B) and y (24 B) per node, timed with HIP events over repeated
    spic_field_apply calls."""
    import torch
    from paper_2008_04397_amd import spic
    h = W.harris_128x64x32()
    g = h.grid
    N = g.nodes
    f64 = spic.to_device(W.make_fields(h), torch.float64)
    moms = spic.moment_buffers(g, 4, torch.float64)
    ctx = _new_ctx(spic, 0)
    species = [spic.to_device(W.make_species(h, s, dtype=np.float32, with_id=False), torch.float32)
               for s in range(4)]
    spic.spic_mover(ctx, g, spic.make_params(h.dt, h.c, h.niter, 1, 0), f64, species, h.qoms, moms)
    torch.cuda.synchronize()
    del species
    torch.cuda.empty_cache()
    fp = spic.make_field_params(h.dt, h.c, theta=1.0, tol=args.field_tol, max_iter=400, restart=30)
    stream = torch.cuda.current_stream()
    # the field operator alone (the residual's product)
    x = torch.randn(3, N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        spic.spic_field_apply(ctx, g, fp, f64, moms, h.qoms, x, y, stream=stream)
    reps = 50
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        spic.spic_field_apply(ctx, g, fp, f64, moms, h.qoms, x, y, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    call_ms = a.elapsed_time(b) / reps
    # whole cycles, fields advanced in place
    stats = [spic.spic_field_cycle(ctx, g, fp, f64, moms, h.qoms, stream=stream)]  # warm-up
    cycles = max(1, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(cycles):
        stats.append(spic.spic_field_cycle(ctx, g, fp, f64, moms, h.qoms, stream=stream))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    timed = stats[1:]
    iters = sum(s.solve_iters for s in timed)
    bytes_apply = 120.0 * N
    return {"metric": "field cycles/s (CG cleaning + GMRes implicit field solve + update)", "mode": "field",
            "value": cycles / wall, "unit": "cycles/s", "n_gpus": 1, "steps": cycles, "higher_is_better": True,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "harris_128x64x32_field_cycle", "nodes": N, "theta": 1.0, "tol": args.field_tol,
                       "restart": 30, "moments": "one mover step of the 4 species"},
            "ms_per_cycle": wall / cycles * 1e3,
            "gmres_iters_per_cycle": iters / cycles, "cg_iters_per_cycle": sum(s.clean_iters for s in timed) / cycles,
            "ms_per_gmres_iter": wall / max(1, iters) * 1e3,
            "final_resid": [s.solve_resid for s in timed],
            "roofline": {"bound": "hbm", "kernel": "k_apply (field operator)",
                         "achieved": bytes_apply / (call_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": bytes_apply / (call_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "bytes_per_launch": bytes_apply,
                         "avg_call_ms": call_ms,
                         "note": "spic_field_apply calls timed with events: the susceptibility kernel (recomputed "
                                 "each call) and the operator kernel; the kernel alone is in the rocprofv3 "
                                 "summary"}}


def bench_serving(args):
    """Poisson request stream: continuous batching vs one at a time."""
    import torch
    from paper_2008_04397_amd import serving, spic
    reqs = W.serving_stream(args.requests, rate=args.rate)
    res = {}
    for mode in ("continuous", "serial"):
        ctx = _engine_ctx(budget=64 * (1 << 30), variant=args.variant)
        if args.srpt_aging >= 0:
            ctx.set_option("srpt_aging", args.srpt_aging)
        # warm the engine and the kernels once
        warm = serving.make_request_run(reqs[0])
        warm.nsteps = 1
        spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [warm])[0])
        log("[bench] serving %d requests (%s)" % (len(reqs), mode))
        done = serving.serve(ctx, reqs, mode=mode, log=log)
        ctx.close()
        res[mode] = serving.summarize(done)
        log("[bench] %s: %s" % (mode, res[mode]))
    c = res["continuous"]
    return {"metric": METRIC, "mode": "serving", "value": c["throughput"], "unit": "particle-steps/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "poisson_%g_per_s_harris_runs" % args.rate, "requests": len(reqs),
                       "precision": "f32 particles, f64 moments", "hbm_budget_bytes": 64 * (1 << 30),
                       "srpt_aging_M_per_s": args.srpt_aging if args.srpt_aging >= 0 else 10000},
            "p50_s": c["p50_s"], "p99_s": c["p99_s"], "continuous": c, "serial": res["serial"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sort-every", type=int, default=-1, help="-1: the autotuned cadence")
    ap.add_argument("--mode", default="main", choices=("main", "ensemble", "streamed", "serving", "cadence", "field"))
    ap.add_argument("--field-tol", type=float, default=1e-8, help="field mode: relative residual target")
    ap.add_argument("--fraction", type=float, default=1.0)
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--rate", type=float, default=20.0, help="serving: mean request arrivals per second")
    ap.add_argument("--srpt-aging", type=int, default=-1,
                    help="serving: engine aging credit in M particle-steps/s (-1: library default)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune block size, variant, layout and cadence first (cached per workload class); "
                         "the default uses the library defaults, which are the measured best on MI355X")
    ap.add_argument("--no-tune", action="store_true", help="(default) use the library defaults")
    ap.add_argument("--variant", type=int, default=-1, help="tiled kernel variant (-1: the library default for the precision)")
    ap.add_argument("--path", type=int, default=0)
    ap.add_argument("--option", action="append", default=[], metavar="KEY=VALUE",
                    help="set a library option on every context (repeatable), e.g. mover_cache=0")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-f32", action="store_true",
                    help="time the FP64 path only (its line then carries the FP64 value and roofline)")
    ap.add_argument("--mover-tol", type=float, default=0.0,
                    help="tolerance-terminated mover iterations (niter_mover is then the cap)")
    ap.add_argument("--niter", type=int, default=3, help="mover iterations (the cap with --mover-tol)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a plain 1 GiB device-to-device copy (reference for HBM counters)")
    args = ap.parse_args()
    for kv in args.option:
        k, v = kv.split("=", 1)
        EXTRA_OPTS[k] = int(v)
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
    if args.mode != "main":
        out = {"ensemble": bench_ensemble, "streamed": bench_streamed, "serving": bench_serving,
               "cadence": bench_cadence, "field": bench_field}[args.mode](args)
        print(json.dumps(out), flush=True)
        return

    h = W.harris_128x64x32()
    tune = args.tune and not args.no_tune
    kw = dict(tune=tune, variant=args.variant, tol=args.mover_tol, niter=args.niter)
    r32 = None
    if not args.no_f32:
        r32 = run_gpu(h, "f32", args.steps, args.warmup, args.sort_every, args.path, **kw)
        log("[bench] f32: %.3e particle-steps/s, %.3f ms/step, %.1f%% HBM" %
            (r32["value"], r32["ms_per_step"], 100 * r32["roofline"]["frac"]))
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(h, "f64", args.steps, args.warmup, args.sort_every, args.path, **kw)
        log("[bench] f64: %.3e particle-steps/s, %.3f ms/step, %.1f%% HBM" %
            (r64["value"], r64["ms_per_step"], 100 * r64["roofline"]["frac"]))
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(h)
        log("[bench] cpu oracle: %.3e particle-steps/s on %d threads" % (cpu["value"], cpu["cores"]))
    head = r32 if r32 is not None else r64
    hname = "f32" if r32 is not None else "f64"
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hname,
        "data": "synthetic",
        "config": {"workload": "harris_128x64x32_ppc64_4species", "cells": [128, 64, 32],
                   "particles": h.n_total, "species": 4, "ppc": 64, "niter_mover": args.niter, "dt": h.dt,
                   "mover_tol": args.mover_tol,
                   "precision": PRECISION[hname],
                   "sort_every": head["sort_every"], "path": args.path or "auto", "launch": head["launch"],
                   "tuned": head["tuned"]},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "ms_per_step_stats": {k: head[k] for k in ("ms_per_step_mean", "ms_per_step_std", "ms_per_step_median",
                                                    "sort_ms_per_species")},
    }
    if r32 is not None and r64 is not None:
        out["fp64"] = {"value": r64["value"], "unit": "particle-steps/s", "dtype": "f64",
                       "precision": PRECISION["f64"],
                       "ms_per_step": r64["ms_per_step"], "roofline": r64["roofline"], "launch": r64["launch"],
                       "tuned": r64["tuned"], "sort_every": r64["sort_every"],
                       "ms_per_step_stats": {k: r64[k] for k in ("ms_per_step_mean", "ms_per_step_std",
                                                                  "ms_per_step_median", "sort_ms_per_species")}}
    if args.copy_calibration:
        # 2^28 FP32 = 1 GiB read + 1 GiB written by one copy kernel
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
