"""Autotuner for the fused tiled path: picks the threads per workgroup, the
kernel variant (LDS atomics; + field corners in registers; home-cell
register accumulation with a queue of drifted particles; bank-balanced
LDS deposit), the halo and the sort
cadence by timing short runs of the actual workload, and caches the choice
per (dtype, workload class) in a JSON file next to this module.

Sorting costs a pass over the particles but keeps the tiles compact; the
best cadence depends on how fast particles cross cells (Sec. VI: sorting
every few cycles keeps the rate high over long runs), so it is measured, not
assumed.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Dict, Iterable, Optional, Sequence

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

DEFAULT = {"tile_block": 256, "tile_variant": 2, "halo": 1, "tile_x": 4, "tile_y": 4, "tile_z": 4,
           "bank_align": 1, "sort_ordered": 1, "sort_every": 4}


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
    for k, v in cfg.items():
        if k != "sort_every":
            ctx.set_option(k, v)


def candidates(quick: bool = True) -> Iterable[Dict[str, int]]:
    """quick: the variants that have won on MI355X (plain LDS atomics and the
    lane-cell register deposit, in one launch and split); otherwise every
    variant, cadence and halo."""
    blocks = (256, 512)
    variants = (2,) if quick else (0, 1, 2)
    cadences = (2, 4, 8) if quick else (1, 2, 4, 8, 16)
    halos = (1,) if quick else (1, 2)
    aligns = (1, 0)
    for blk, var, se, halo, al in itertools.product(blocks, variants, cadences, halos, aligns):
        c = dict(DEFAULT)
        c.update(tile_block=blk, tile_variant=var, sort_every=se, halo=halo, bank_align=al)
        yield c


def tune(h, fields, species, qoms, moments, steps: int = 16, quick: bool = True, log=None) -> Dict[str, int]:
    """Time `steps` fused steps (after the first sort) for every candidate on
    the given device-resident inputs; returns the fastest configuration.  The
    inputs are advanced in time by the trials (a real run's state).  `steps`
    is rounded up to a multiple of every candidate cadence, so each trial
    pays its own sorts in full."""
    import torch
    from . import spic
    best, best_ms = None, float("inf")
    cands = list(candidates(quick))
    period = 1
    for c in cands:
        period = period * c["sort_every"] // math.gcd(period, c["sort_every"])
    steps = -(-steps // period) * period
    for cfg in cands:
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
    return best
