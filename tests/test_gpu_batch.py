"""GPU tests of spic_batch_submit: many runs stepped together by the
persistent work-list kernel, continuous admission under an HBM budget,
host-resident runs, streamed runs (particle batching through two device
slots), hipGraph replay -- each result against the oracle or against the
same run executed alone."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04397_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def spic():
    from paper_2008_04397_amd import spic as S
    S.lib()
    return S


def _boxes():
    """Three small boxes of different shape, ppc and mass ratio."""
    return [W.Harris(W.Grid(16, 8, 4), ppc=8, qom_e=-25.0, B0=0.02, seed=11),
            W.Harris(W.Grid(12, 6, 8), ppc=27, qom_e=-64.0, B0=0.015, seed=12),
            W.Harris(W.Grid(8, 8, 4), ppc=10, qom_e=-100.0, B0=0.03, seed=13)]


def _run_of(spic, h, nsteps, dtype=torch.float64, host=False, sort_every=2):
    f = spic.to_device(W.make_fields(h), dtype)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sps = [W.make_species(h, s, dtype=npdt) for s in range(4)]
    if host:
        dev = [spic.pinned_like(s, dtype) for s in sps]
    else:
        dev = [spic.to_device(s, dtype) for s in sps]
    moms = spic.moment_buffers(h.grid, 4)
    prm = spic.make_params(h.dt, h.c, h.niter, sort_every, 0)
    return spic.Run(h.grid, prm, f, dev, h.qoms, moms, nsteps), sps


def _oracle(h, sps, nsteps):
    f = W.make_fields(h)
    return O.run(h, f, [W.upcast(s) for s in sps], nsteps)


def _host(run):
    return [spic_to_host(s) for s in run.species]


def spic_to_host(s):
    return {k: v.detach().cpu().numpy() for k, v in s.items()}


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_resident_runs_together_match_oracle(spic, variant):
    ctx = spic.Context(0)
    ctx.set_option("tile_variant", variant)
    boxes = _boxes()
    runs, inputs = zip(*[_run_of(spic, h, 4) for h in boxes])
    _say("case batch resident 3 boxes x 4 steps, variant %d" % variant)
    tickets = spic.spic_batch_submit(ctx, runs)
    for t in tickets:
        assert spic.spic_wait(ctx, t) >= 0.0
    for h, run, sps in zip(boxes, runs, inputs):
        st, ms = _oracle(h, sps, 4)
        got = _host(run)
        for s in range(4):
            P.assert_state(got[s], st[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(run.moments[s].cpu().numpy(), ms[s], P.MOM64)
    ctx.close()


def test_each_run_alone_equals_the_mix(spic):
    """Continuous batching must not change results: every run submitted
    alone gives the same particles (bitwise, by id) and moments as in the
    mix, where runs of different lengths overlap."""
    boxes = _boxes()
    steps = [3, 6, 2]
    ctx = spic.Context(0)
    alone = []
    for h, n in zip(boxes, steps):
        run, _ = _run_of(spic, h, n)
        spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [run])[0])
        alone.append(run)
    mixed = [_run_of(spic, h, n)[0] for h, n in zip(boxes, steps)]
    tickets = spic.spic_batch_submit(ctx, mixed[:1])
    tickets += spic.spic_batch_submit(ctx, mixed[1:])   # arrives while the first runs
    for t in tickets:
        spic.spic_wait(ctx, t)
    for a, b, h in zip(alone, mixed, boxes):
        for s in range(4):
            x, y = P.by_id(spic_to_host(a.species[s])), P.by_id(spic_to_host(b.species[s]))
            for k in ("x", "y", "z", "u", "v", "w"):
                assert np.array_equal(x[k], y[k])
            P.assert_moments(b.moments[s].cpu().numpy(), a.moments[s].cpu().numpy(), 1e-14)
    ctx.close()


def test_admission_under_a_small_budget(spic):
    """Host-resident runs whose total footprint exceeds the budget are
    admitted a few at a time as others retire; all complete correctly."""
    boxes = _boxes() * 2
    one = max(sum(W.make_species(h, s)["x"].size for s in range(4)) * (7 * 8 + 8) for h in boxes)
    ctx = spic.Context(0, hbm_budget_bytes=int(2.5 * one) + (1 << 20))
    made = [_run_of(spic, h, 3, host=True) for h in boxes]
    runs = [m[0] for m in made]
    _say("case batch admission budget %d bytes" % int(2.5 * one))
    tickets = spic.spic_batch_submit(ctx, runs)
    for t in tickets:
        spic.spic_wait(ctx, t)
    for (run, sps), h in zip(made, boxes):
        st, ms = _oracle(h, sps, 3)
        got = _host(run)
        for s in range(4):
            P.assert_state(got[s], st[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(run.moments[s].cpu().numpy(), ms[s], P.MOM64)
    ctx.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_streamed_run_equals_resident_run(spic, dtype):
    """A budget of a few MB forces the 32x16x4 box through batches of a few
    thousand particles; the result equals the resident run's."""
    h = W.harris_32x16x4()
    ctx_r = spic.Context(0)
    res, _ = _run_of(spic, h, 3, dtype=dtype, sort_every=2)
    spic.spic_wait(ctx_r, spic.spic_batch_submit(ctx_r, [res])[0])
    ctx_s = spic.Context(0, hbm_budget_bytes=3 << 20)
    ctx_s.set_option("batch_particles", 8192)
    stm, _ = _run_of(spic, h, 3, dtype=dtype, host=True, sort_every=2)
    _say("case streamed %s budget 3 MiB" % dtype)
    secs = spic.spic_wait(ctx_s, spic.spic_batch_submit(ctx_s, [stm])[0])
    assert secs > 0
    for s in range(4):
        a, b = P.by_id(spic_to_host(res.species[s])), P.by_id(spic_to_host(stm.species[s]))
        for k in ("x", "y", "z", "u", "v", "w"):
            assert np.array_equal(a[k], b[k]), k
        # FP32 particles: the lane-cell deposit forms FP32 partial sums over
        # the particles one thread holds, and a streamed batch is sorted and
        # tiled on its own, so the grouping differs: FP32 rounding (the
        # oracle bound for FP32 moments), not the FP64 accumulation order
        tol = 1e-13 if dtype == torch.float64 else P.MOM32
        P.assert_moments(stm.moments[s].cpu().numpy(), res.moments[s].cpu().numpy(), tol)
    ctx_r.close()
    ctx_s.close()


def test_graph_replay_matches_plain_launches(spic):
    boxes = _boxes()
    out = []
    for graph in (1, 0):
        ctx = spic.Context(0)
        ctx.set_option("graph", graph)
        runs = [_run_of(spic, h, 5, sort_every=3)[0] for h in boxes]
        for t in spic.spic_batch_submit(ctx, runs):
            spic.spic_wait(ctx, t)
        out.append(runs)
        ctx.close()
    for a, b in zip(*out):
        for s in range(4):
            x, y = P.by_id(spic_to_host(a.species[s])), P.by_id(spic_to_host(b.species[s]))
            for k in ("x", "y", "z", "u", "v", "w"):
                assert np.array_equal(x[k], y[k])
            P.assert_moments(a.moments[s].cpu().numpy(), b.moments[s].cpu().numpy(), 1e-14)


def test_zero_step_run_and_errors(spic):
    ctx = spic.Context(0)
    h = _boxes()[0]
    run, sps = _run_of(spic, h, 0, host=True)
    spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [run])[0])
    got = _host(run)
    for s in range(4):
        for k in ("x", "u"):
            np.testing.assert_array_equal(got[s][k], sps[s][k])
    assert spic.lib().spic_poll(ctx.handle, 987654, (spic.C.c_int32 * 1)()) == spic.SPIC_E_STATE
    ctx.close()
    tiny = spic.Context(0, hbm_budget_bytes=4096)
    run, _ = _run_of(spic, h, 1, host=True)
    assert spic.spic_batch_submit(tiny, [run], raw=True) == spic.SPIC_E_BUDGET
    tiny.close()


def test_ticks_step_the_shortest_runs_first(spic):
    """With tick_items = 1 every tick steps only the run with the least
    remaining work: short runs submitted with a long one finish while the
    long one has barely started, and all results still match the oracle."""
    ctx = spic.Context(0)
    ctx.set_option("tick_items", 1)
    big = W.Harris(W.Grid(32, 16, 8), ppc=27, seed=21)
    small = _boxes()[:2]
    long_run, long_in = _run_of(spic, big, 60, dtype=torch.float32)
    shorts = [_run_of(spic, h, 3) for h in small]
    _say("case batch SRPT order: 1 long run (60 steps) + 2 short runs (3 steps), tick_items 1")
    tickets = spic.spic_batch_submit(ctx, [long_run] + [r for r, _ in shorts])
    for t in tickets[1:]:
        spic.spic_wait(ctx, t)
    assert not spic.spic_poll(ctx, tickets[0]), "the long run finished before the short ones"
    spic.spic_wait(ctx, tickets[0])
    for h, (run, sps) in zip(small, shorts):
        st, ms = _oracle(h, sps, 3)
        got = _host(run)
        for s in range(4):
            P.assert_state(got[s], st[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(run.moments[s].cpu().numpy(), ms[s], P.MOM64)
    ctx.close()



def _completion_order(spic, ctx, tickets, limit_s=120.0):
    import time
    order, t0 = [], time.monotonic()
    while len(order) < len(tickets) and time.monotonic() - t0 < limit_s:
        for t in tickets:
            if t not in order and spic.spic_poll(ctx, t):
                order.append(t)
    for t in tickets:
        spic.spic_wait(ctx, t)
    return order


@pytest.mark.parametrize("aging", [0, 1 << 40])
def test_aging_credit_bounds_how_long_a_run_waits(spic, aging):
    """A long run is already stepping when short runs arrive.  Without aging
    credit (pure least-remaining-work) the newcomers overtake it; with a very
    large credit rate the run that has waited longer keeps the GPU and
    finishes first.  Results match the oracle either way."""
    import time
    ctx = spic.Context(0)
    ctx.set_option("tick_items", 1)
    ctx.set_option("srpt_aging", aging)
    big = W.Harris(W.Grid(32, 16, 8), ppc=27, seed=21)
    small = _boxes()[:2]
    long_run, _ = _run_of(spic, big, 200, dtype=torch.float32)
    shorts = [_run_of(spic, h, 10) for h in small]
    _say("case batch aging %d: 1 long run (200 steps) then 2 short runs (10 steps), tick_items 1" % aging)
    first = spic.spic_batch_submit(ctx, [long_run])
    time.sleep(0.005)
    later = spic.spic_batch_submit(ctx, [r for r, _ in shorts])
    order = _completion_order(spic, ctx, first + later)
    assert len(order) == 3
    if aging:
        assert order[0] == first[0], "the waiting long run was overtaken"
    else:
        assert order[-1] == first[0], "the short newcomers did not overtake the long run"
    for h, (run, sps) in zip(small, shorts):
        st, ms = _oracle(h, sps, 10)
        got = _host(run)
        for s in range(4):
            P.assert_state(got[s], st[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(run.moments[s].cpu().numpy(), ms[s], P.MOM64)
    ctx.close()

def _fp32_one_step_check(h, run, sps):
    """One FP32 step from the FP32-rounded input against the oracle's step
    of the same state (upcast): positions <= 1e-5 L_d, velocities <= 1e-5
    max(|v|, vth); moments against the oracle's FP64 deposit of the GPU's
    own final FP32 state, rel-L2 <= 1e-6 (Sec. II moment sum of the state
    the mover produced)."""
    f = W.make_fields(h)
    f32 = {k: v.astype(np.float32).astype(np.float64) for k, v in f.items()}
    got = _host(run)
    worst = [0.0, 0.0, 0.0]
    for s in range(4):
        ora = O.mover(h.grid, h.dt, h.c, h.niter, h.qoms[s], f32, W.upcast(sps[s]))
        pe, ve = P.assert_state(got[s], ora, h.grid, P.POS32, P.VEL32, vscale=max(P.vmax(ora), h.vths[s]))
        ref = O.deposit(h.grid, W.upcast(got[s]))
        me = P.assert_moments(run.moments[s].cpu().numpy(), ref, P.MOM32)
        worst = [max(worst[0], pe), max(worst[1], ve), max(worst[2], me)]
    return worst


@pytest.mark.parametrize("variant", [-1, 3])
def test_fp32_work_list_run_matches_oracle(spic, variant):
    """The batch engine's FP32-particle path (work-list launches, FP64
    moments) on three boxes of different shape: one step each against the
    oracle (variant 3 runs the split lists there)."""
    ctx = spic.Context(0)
    ctx.set_option("tile_variant", variant)
    boxes = _boxes()
    made = [_run_of(spic, h, 1, dtype=torch.float32) for h in boxes]
    _say("case batch fp32 work list: 3 boxes x 1 step, variant %d" % variant)
    for t in spic.spic_batch_submit(ctx, [m[0] for m in made]):
        spic.spic_wait(ctx, t)
    for h, (run, sps) in zip(boxes, made):
        _say("fp32 work list %s: pos/L %.2e vel %.2e mom %.2e" % ((h.grid,) + tuple(_fp32_one_step_check(h, run, sps))))
    ctx.close()


def test_streamed_fp64_run_matches_oracle(spic):
    """Streamed through a 3 MiB budget in batches of 8192 particles (sorted
    at step 0 and every 2 steps, per batch), FP64: 3 steps against the
    oracle at the FP64 tolerances."""
    h = W.harris_32x16x4()
    ctx = spic.Context(0, hbm_budget_bytes=3 << 20)
    ctx.set_option("batch_particles", 8192)
    run, sps = _run_of(spic, h, 3, dtype=torch.float64, host=True, sort_every=2)
    _say("case streamed fp64 vs oracle, budget 3 MiB, batches of 8192")
    spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [run])[0])
    st, ms = _oracle(h, sps, 3)
    got = _host(run)
    for s in range(4):
        P.assert_state(got[s], st[s], h.grid, P.POS64, P.VEL64)
        P.assert_moments(run.moments[s].cpu().numpy(), ms[s], P.MOM64)
    ctx.close()


@pytest.mark.parametrize("variant", [-1, 3])
def test_streamed_fp32_step_matches_oracle(spic, variant):
    """The same box streamed with FP32 particles (FP64 moments): one step
    against the oracle at the FP32 tolerances (variant 3: the one-launch
    kernel per streamed batch)."""
    h = W.harris_32x16x4()
    ctx = spic.Context(0, hbm_budget_bytes=3 << 20)
    ctx.set_option("batch_particles", 8192)
    ctx.set_option("tile_variant", variant)
    run, sps = _run_of(spic, h, 1, dtype=torch.float32, host=True)
    _say("case streamed fp32 vs oracle, budget 3 MiB, batches of 8192, variant %d" % variant)
    spic.spic_wait(ctx, spic.spic_batch_submit(ctx, [run])[0])
    _say("streamed fp32: pos/L %.2e vel %.2e mom %.2e" % tuple(_fp32_one_step_check(h, run, sps)))
    ctx.close()
