"""Serving: a Poisson stream of small Harris-box runs through the batch
engine with continuous batching; every request's result must equal the
same request run alone: particles bitwise, matched by particle id (the
engine sorts them, so their order differs), and moments within 1e-12
where every deposit term is FP64 (only the order of FP64 additions
differs) or within the FP32 moment tolerance (rel 1e-6) where FP32
partial sums over the particles one thread holds are formed (their
grouping depends on the order inside a cell after a sort)."""
import sys

import numpy as np
import pytest

from paper_2008_04397_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _stream():
    return W.serving_stream(8, rate=40.0, seed=9, max_nx=32, steps_range=(3, 9))


@pytest.mark.parametrize("variant,tol", [(-1, 1e-6), (0, 1e-12)])
def test_each_request_alone_equals_continuous_mix(variant, tol):
    from paper_2008_04397_amd import serving, spic
    reqs = _stream()
    ctx = spic.Context(0, hbm_budget_bytes=256 << 20)
    ctx.set_option("tile_variant", variant)
    mixed = {}
    _say("case serving continuous 8 requests, tile_variant %d" % variant)
    done = serving.serve(ctx, reqs, mode="continuous", keep=mixed, with_id=True)
    assert len(done) == len(reqs)
    s = serving.summarize(done)
    assert s["p99_s"] >= s["p50_s"] > 0
    for req in reqs:
        alone = serving.make_request_run(req, with_id=True)
        spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [alone])[0])
        mix = mixed[req.rid]
        for sa, sb in zip(alone.species, mix.species):
            a = P.by_id({k: v.numpy() for k, v in sa.items()})
            b = P.by_id({k: v.numpy() for k, v in sb.items()})
            assert np.array_equal(a["id"], b["id"]) and np.array_equal(a["id"], np.arange(a["id"].size))
            for k in ("x", "y", "z", "u", "v", "w", "q"):
                assert np.array_equal(a[k], b[k]), (req.rid, k)
        for ma, mb in zip(alone.moments, mix.moments):
            a, b = ma.cpu().numpy(), mb.cpu().numpy()
            for c in range(10):
                nb = np.linalg.norm(a[c])
                assert np.linalg.norm(a[c] - b[c]) <= tol * max(nb, 1e-300)
    ctx.close()


def test_serial_baseline_runs_one_at_a_time():
    from paper_2008_04397_amd import serving, spic
    reqs = _stream()[:4]
    ctx = spic.Context(0)
    done = serving.serve(ctx, reqs, mode="serial")
    ctx.close()
    done.sort(key=lambda d: d.submit)
    for a, b in zip(done, done[1:]):
        assert b.submit >= a.complete - 1e-3
