"""The allocation-free fused step, spic_mover_noalloc, through the C ABI:
each call equals spic_mover with a sort every step on the same inputs
(particles bitwise by id -- the tiled mover's result does not depend on the
order; moments to the FP64 / FP32 moment tolerances, as the summation order
differs), on two calls in a row, the second with a smaller input (the fixed
scratch keeps the first call's contents)."""
import sys

import numpy as np
import pytest

from paper_2008_04397_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _step(spic, ctx, h, fields, species, dtype, noalloc, step=0):
    dev_f = spic.to_device(fields, dtype)
    dev = [spic.to_device(s, dtype) for s in species]
    moms = spic.moment_buffers(h.grid, len(species), torch.float64)
    prm = spic.make_params(h.dt, h.c, h.niter, 1, step)
    fn = spic.spic_mover_noalloc if noalloc else spic.spic_mover
    fn(ctx, h.grid, prm, dev_f, dev, h.qoms, moms)
    torch.cuda.synchronize()
    return [spic.to_host(d) for d in dev], [m.cpu().numpy() for m in moms]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_step_equals_the_allocating_step_on_two_calls(dtype):
    from paper_2008_04397_amd import spic
    spic.lib()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    mtol = P.MOM64 if dtype == "f64" else P.MOM32
    ctx = spic.Context(0)
    ref_ctx = spic.Context(0)
    try:
        boxes = [W.harris_32x16x4(), W.Harris(W.Grid(16, 8, 4), ppc=8)]
        assert boxes[1].n_total < boxes[0].n_total
        for call, h in enumerate(boxes):
            f = W.make_fields(h)
            sps = W.make_all_species(h)
            if dtype == "f32":
                f = {k: v.astype(np.float32) for k, v in f.items()}
                sps = [W.round_state(s, np.float32) for s in sps]
            _say("case noalloc %s call %d: %d particles" % (dtype, call, h.n_total))
            got, gm = _step(spic, ctx, h, f, sps, tdt, True, step=call)
            ref, rm = _step(spic, ref_ctx, h, f, sps, tdt, False, step=call)
            for s in range(4):
                a, b = P.by_id(got[s]), P.by_id(ref[s])
                for k in ("id", "x", "y", "z", "u", "v", "w", "q"):
                    assert np.array_equal(a[k], b[k]), (call, s, k)
                P.assert_moments(gm[s], rm[s], mtol)
    finally:
        ctx.close()
        ref_ctx.close()
