"""Serving loop: a stream of whole multi-step Harris-box runs (requests)
submitted to the batch engine as they arrive.

Continuous mode: every request is handed to spic_batch_submit at its arrival
time, whatever is running; the engine admits it at the next tick once its
HBM footprint fits the budget, steps it together with the other resident
requests (one work-list launch per tick) and retires it when done.

Serial mode (the baseline): the same trace, one request at a time -- a
request is submitted only after the previous one has completed.

Latency of a request = completion time (results back in host memory) -
arrival time in the trace, so time spent queued behind earlier requests
(and any delay of the client itself) counts in both modes.  The client
prepares each request's inputs (fields on the device, particles in pinned
host memory) just before waiting for its arrival time.  Pinned host memory
is finite: while the requests in flight hold more than `max_pinned_bytes`,
the client waits for completions before preparing the next one (that wait
counts in the latency of the requests it delays).
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import spic
from . import workloads as W


@dataclasses.dataclass
class Done:
    rid: int
    arrival: float
    submit: float
    complete: float
    particles: int
    steps: int
    device_s: float

    @property
    def latency(self) -> float:
        return self.complete - self.arrival


def make_request_run(req: W.Request, dtype=None, sort_every: int = 4, device="cuda", with_id: bool = False):
    """Inputs of one request: fields on the device, 4 species in pinned host
    memory (with int64 particle ids when with_id), FP64 moment outputs on the
    device."""
    import torch
    dtype = dtype or torch.float32
    h = req.box
    f = W.fields_tensors(h, device=device, dtype=dtype)
    species = []
    for s in range(4):
        t = W.species_tensors(h, s, device=device, dtype=dtype, seed_offset=req.rid, with_id=with_id)
        species.append({k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True).copy_(v) for k, v in t.items()})
    moms = spic.moment_buffers(h.grid, 4, torch.float64, device)
    prm = spic.make_params(h.dt, h.c, h.niter, sort_every, 0)
    return spic.Run(h.grid, prm, f, species, h.qoms, moms, req.steps)


def pinned_bytes(req: W.Request, dtype=None) -> int:
    """Pinned host bytes of one request's particles (7 arrays + int64 ids)."""
    import torch
    elem = 8 if dtype == torch.float64 else 4
    return int(req.box.n_total) * (7 * elem + 8)


def serve(ctx: "spic.Context", requests: Sequence[W.Request], mode: str = "continuous",
          dtype=None, sort_every: int = 4, time_scale: float = 1.0, log=None, keep=None,
          max_pinned_bytes: int = 16 << 30, with_id: bool = False) -> List[Done]:
    """Replay the arrival trace (arrival times multiplied by time_scale).
    When `keep` is a dict, keep[rid] receives each request's finished run
    (its species and moments hold the results)."""
    import torch
    assert mode in ("continuous", "serial")
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    inflight: Dict[int, tuple] = {}
    done: List[Done] = []

    def poll_all(block: bool = False):
        for tk in list(inflight):
            if block or spic.spic_poll(ctx, tk):
                secs = spic.spic_wait(ctx, tk)
                req, arr, sub, _ = inflight.pop(tk)
                done.append(Done(req.rid, arr, sub, now(), req.box.n_total, req.steps, secs))
                if block:
                    return

    for k, req in enumerate(order):
        need = pinned_bytes(req, dtype)
        while inflight and sum(v[3] for v in inflight.values()) + need > max_pinned_bytes:
            poll_all()
            time.sleep(0.0005)
        run = make_request_run(req, dtype, sort_every, with_id=with_id)
        torch.cuda.current_stream().synchronize()
        arrival = req.arrival * time_scale
        while now() < arrival:
            poll_all()
            time.sleep(0.0005)
        if mode == "serial":
            while inflight:
                poll_all(block=True)
        tk = spic.spic_batch_submit(ctx, [run])[0]
        inflight[tk] = (req, arrival, now(), need)
        if keep is not None:
            keep[req.rid] = run
        if log and k % 20 == 0:
            log("[serve %s] request %d/%d submitted at %.2f s, %d in flight" % (mode, k, len(order), now(),
                                                                              len(inflight)))
    while inflight:  # drain, recording each completion when it happens
        poll_all()
        time.sleep(0.0005)
    return done


def summarize(done: Sequence[Done]) -> Dict[str, float]:
    lat = np.array([d.latency for d in done])
    work = sum(d.particles * d.steps for d in done)
    span = max(d.complete for d in done) - min(d.arrival for d in done)
    return {"requests": len(done), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "particle_steps": int(work),
            "makespan_s": float(span), "throughput": float(work / span)}
