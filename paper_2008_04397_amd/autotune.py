"""Autotuner: picks launch settings and the sort cadence by timing short
runs of the actual workload, and caches the choice per workload class in a
JSON file next to this module.

Three spaces, one per way the library runs a workload:

* one resident box (spic_mover): threads per workgroup, the tiled kernel
  variant (the dtype's candidates), the bank-preserving layout and the sort
  cadence;
* many boxes in one engine submission (spic_batch_submit, an ensemble):
  threads per workgroup, the sort cadence of the runs and the work-list
  batch length (tick_items: (run, tile) items stepped per tick);
* a streamed box (larger than its HBM budget): the batch length
  (batch_particles per streamed batch) and the sort cadence.

The sort costs a pass over the particles but keeps the tiles compact; how
often it pays depends on how fast particles cross cells (Sec. VI: sorting
every few cycles keeps the rate up over long runs), so it is measured, not
assumed.  Batch length trades launch count against the work one tick holds
(Sec. III-B: particles are processed in batches; Sec. V-C sweeps the batch
count per species and the threads per block).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

DEFAULT = {"tile_block": 256, "tile_variant": 2, "halo": 1, "tile_x": 4, "tile_y": 4, "tile_z": 4,
           "bank_align": 1, "sort_ordered": 1, "sort_every": 4}

# keys that are not library options: the cadence goes into each step's
# spic_params.sort_every
RUN_KEYS = ("sort_every",)


def workload_class(dtype_name: str, grid, ppc: int) -> str:
    cells = grid.nx * grid.ny * grid.nz
    return "%s/cells%d/ppc%d" % (dtype_name, 1 << max(0, (cells - 1).bit_length()), ppc)


def load(key: str) -> Optional[Dict[str, int]]:
    try:
        with open(CACHE) as fh:
            return json.load(fh).get(key)
    except (OSError, ValueError):
        return None


def store(key: str, cfg: Dict[str, int]):
    data = {}
    try:
        with open(CACHE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        pass
    data[key] = cfg
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def apply(ctx, cfg: Dict[str, int]):
    """Set every library option of `cfg` on `ctx` (the cadence is not one)."""
    for k, v in cfg.items():
        if k not in RUN_KEYS:
            ctx.set_option(k, v)


def _lcm(values: Iterable[int]) -> int:
    out = 1
    for v in values:
        out = out * v // math.gcd(out, v)
    return out


# ---------------------------------------------------------------- one box

def candidates(quick: bool = True, dtype_name: str = "f32") -> Iterable[Dict[str, int]]:
    """One resident box.  FP32 particles: the split variant (2) and, unless
    quick, the one-kernel variants 0, 1 and 3; FP64 particles: the
    one-kernel variants (their LDS-atomic deposit is exact in FP64).  Blocks
    and cadences as listed; the bank-preserving layout on and off."""
    blocks = (256, 512)
    if dtype_name == "f64":
        variants = (0,) if quick else (0, 1)
    else:
        variants = (2,) if quick else (0, 1, 2, 3)
    cadences = (2, 4, 8) if quick else (1, 2, 4, 8, 16)
    aligns = (1, 0)
    for blk, var, se, al in itertools.product(blocks, variants, cadences, aligns):
        c = dict(DEFAULT)
        c.update(tile_block=blk, tile_variant=var, sort_every=se, bank_align=al)
        yield c


def snapshot(species) -> List[Dict]:
    """Device copies of every species tensor (the state a trial starts from)."""
    return [{k: v.clone() for k, v in sp.items()} for sp in species]


def restore(species, snap) -> None:
    for sp, sn in zip(species, snap):
        for k, v in sp.items():
            v.copy_(sn[k])


def tune(h, fields, species, qoms, moments, steps: int = 16, quick: bool = True, log=None,
         dtype_name: str = "f32") -> Dict[str, int]:
    """Time `steps` fused steps (after a first sort) for every candidate on
    the given device-resident inputs; returns the fastest configuration.
    Every trial starts from the same state (the inputs as given, restored
    from a device copy), so no candidate meets particles that earlier trials
    have spread, and the inputs are restored once more at the end.  `steps`
    is rounded up to a multiple of every candidate cadence, so each trial
    pays its own sorts in full."""
    import torch
    from . import spic
    best, best_ms = None, float("inf")
    cands = list(candidates(quick, dtype_name))
    period = _lcm(c["sort_every"] for c in cands)
    steps = -(-steps // period) * period
    snap = snapshot(species)
    for cfg in cands:
        restore(species, snap)
        ctx = spic.Context(0)
        apply(ctx, cfg)
        se = cfg["sort_every"]
        spic.spic_mover(ctx, h.grid, spic.make_params(h.dt, h.c, h.niter, se, 0), fields, species, qoms, moments)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, steps + 1):
            spic.spic_mover(ctx, h.grid, spic.make_params(h.dt, h.c, h.niter, se, k), fields, species, qoms, moments)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ctx.close()
        if log:
            log("[tune] %s -> %.3f ms/step" % (cfg, ms))
        if ms < best_ms:
            best, best_ms = cfg, ms
    restore(species, snap)
    return best


# ------------------------------------------------ engine runs (ensemble, streamed)

def engine_candidates(quick: bool = True) -> List[Dict[str, int]]:
    """Many boxes per submission: threads per workgroup x sort cadence x
    (run, tile) items per tick (0: every run steps at every tick)."""
    blocks = (256, 512)
    cadences = (2, 4, 8) if quick else (1, 2, 4, 8)
    ticks = (2048, 8192, 0) if quick else (1024, 2048, 4096, 8192, 32768, 0)
    return [{"tile_block": b, "sort_every": se, "tick_items": t} for b, se, t in itertools.product(blocks, cadences,
                                                                                                   ticks)]


def stream_candidates(quick: bool = True) -> List[Dict[str, int]]:
    """A streamed box: particles per streamed batch x sort cadence."""
    batches = (1 << 25, 1 << 26) if quick else (1 << 24, 1 << 25, 1 << 26, 1 << 27)
    cadences = (4,) if quick else (2, 4, 8)
    return [{"batch_particles": b, "sort_every": se} for b, se in itertools.product(batches, cadences)]


def tune_runs(make_ctx: Callable[[], object], make_runs: Callable[[int, int], Sequence], cands: Sequence[Dict],
              steps: int = 8, log=None, reset: Optional[Callable[[], None]] = None) -> Dict[str, int]:
    """Engine tuner.  For every candidate: reset() (when given: put the
    runs' inputs back to the state every trial starts from), a fresh context
    from make_ctx() with the candidate's options, one untimed submission of
    1 step (kernel and engine warm-up), then `steps` steps of
    make_runs(sort_every, steps) submitted together, timed from submission
    to the last spic_wait.  `steps` is rounded up to a multiple of every
    candidate cadence.  Returns the fastest candidate."""
    from . import spic
    period = _lcm(c.get("sort_every", 1) for c in cands)
    steps = -(-steps // period) * period
    best, best_s = None, float("inf")
    for cfg in cands:
        if reset is not None:
            reset()
        ctx = make_ctx()
        try:
            apply(ctx, cfg)
            se = cfg.get("sort_every", 4)
            for t in spic.spic_batch_submit(ctx, make_runs(se, 1)):
                spic.spic_wait(ctx, t)
            t0 = time.perf_counter()
            for t in spic.spic_batch_submit(ctx, make_runs(se, steps)):
                spic.spic_wait(ctx, t)
            secs = time.perf_counter() - t0
        finally:
            ctx.close()
        if log:
            log("[tune] %s -> %.3f s for %d steps" % (cfg, secs, steps))
        if secs < best_s:
            best, best_s = dict(cfg), secs
    return best
