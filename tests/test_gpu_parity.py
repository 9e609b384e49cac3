"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Inputs are the seeded Harris-sheet workloads (paper Sec. IV setup: four
species, charge-to-mass ratio 64, omega_pi dt = 0.25, three iterations) at
sizes the oracle finishes in seconds, plus ragged and degenerate cases.
Tolerances are those stated in tests/parity.py.
"""
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


@pytest.fixture
def ctx(spic):
    c = spic.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _run_gpu(spic, ctx, h, fields, species, nsteps, dtype, acc=torch.float64, sort_every=0, every_step=None,
             qoms=None):
    qoms = list(qoms if qoms is not None else h.qoms)
    dev_f = spic.to_device(fields, dtype)
    dev_sp = [spic.to_device(s, dtype) for s in species]
    moms = spic.moment_buffers(h.grid, len(species), acc)
    for step in range(nsteps):
        prm = spic.make_params(h.dt, h.c, h.niter, sort_every, step)
        spic.spic_mover(ctx, h.grid, prm, dev_f, dev_sp, qoms, moms)
        if every_step is not None:
            torch.cuda.synchronize()
            every_step(step, [spic.to_host(s) for s in dev_sp], [m.cpu().numpy() for m in moms])
    torch.cuda.synchronize()
    return [spic.to_host(s) for s in dev_sp], [m.cpu().numpy() for m in moms]


# ------------------------------------------------------------------ FP64

def test_fp64_small_box_every_step_matches_oracle(spic, ctx):
    """32x16x4 cells, 27 ppc x 4 species, 10 steps, FP64 end to end."""
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sps = W.make_all_species(h)
    ora = [dict(s) for s in sps]
    worst = [0.0, 0.0, 0.0]

    def check(step, gpu_states, gpu_moms):
        for s in range(4):
            ora[s], m = O.step(h.grid, h.dt, h.c, h.niter, h.qoms[s], f, ora[s])
            pe, ve = P.assert_state(gpu_states[s], ora[s], h.grid, P.POS64, P.VEL64)
            me = P.assert_moments(gpu_moms[s], m, P.MOM64)
            worst[0], worst[1], worst[2] = max(worst[0], pe), max(worst[1], ve), max(worst[2], me)

    _say("case fp64 harris_32x16x4 10 steps")
    _run_gpu(spic, ctx, h, f, sps, 10, torch.float64, every_step=check)
    _say("fp64 worst: pos/L %.2e vel/vmax %.2e mom rel-L2 %.2e" % tuple(worst))


def test_fp64_ragged_counts_and_degenerate_species(spic, ctx):
    """Counts that are not multiples of any block size, a single particle and
    an empty species, in one call."""
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    g = h.grid
    sps = [W.random_particles(g, 10007, 0.05, seed=1), W.random_particles(g, 1, 0.05, seed=2),
           W.random_particles(g, 0, 0.05, seed=3), W.random_particles(g, 333, 0.3, seed=4)]
    qoms = [-64.0, 1.0, -25.0, 3.0]
    _say("case fp64 ragged 10007/1/0/333")
    gpu_st, gpu_m = _run_gpu(spic, ctx, h, f, sps, 2, torch.float64, qoms=qoms)
    for s in range(4):
        st = sps[s]
        for _ in range(2):
            st, m = O.step(g, h.dt, h.c, h.niter, qoms[s], f, st)
        P.assert_state(gpu_st[s], st, g, P.POS64, P.VEL64)
        if st["x"].size:
            P.assert_moments(gpu_m[s], m, P.MOM64)
        else:
            assert np.all(gpu_m[s] == 0)


def test_fp64_particles_far_outside_the_box_are_wrapped(spic, ctx):
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    g = h.grid
    sp = W.random_particles(g, 2000, 0.05, seed=5)
    r = np.random.default_rng(5)
    for k, L in zip(("x", "y", "z"), g.L):
        sp[k] = sp[k] + L * r.integers(-3, 4, sp[k].size)
    _say("case fp64 positions outside the box")
    gpu_st, gpu_m = _run_gpu(spic, ctx, h, f, [sp], 1, torch.float64, qoms=[-64.0])
    st, m = O.step(g, h.dt, h.c, h.niter, -64.0, f, sp)
    P.assert_state(gpu_st[0], st, g, P.POS64, P.VEL64)
    P.assert_moments(gpu_m[0], m, P.MOM64)
    for k, L in zip(("x", "y", "z"), g.L):
        assert np.all((gpu_st[0][k] >= 0) & (gpu_st[0][k] < L))


# ------------------------------------------------------------------ FP32

def _fp32_inputs(h):
    f32 = {k: v.astype(np.float32) for k, v in W.make_fields(h).items()}
    sps32 = [W.round_state(s, np.float32) for s in W.make_all_species(h)]
    return f32, sps32


def test_fp32_one_step_from_identical_state(spic, ctx):
    h = W.harris_32x16x4()
    f32, sps32 = _fp32_inputs(h)
    _say("case fp32 harris_32x16x4 one step")
    gpu_st, gpu_m = _run_gpu(spic, ctx, h, f32, sps32, 1, torch.float32)
    f64 = {k: v.astype(np.float64) for k, v in f32.items()}
    for s in range(4):
        ora = O.mover(h.grid, h.dt, h.c, h.niter, h.qoms[s], f64, W.upcast(sps32[s]))
        pe, ve = P.assert_state(gpu_st[s], ora, h.grid, P.POS32, P.VEL32,
                                vscale=max(P.vmax(ora), h.vths[s]))
        # moments: the oracle's FP64 deposit of the very state the GPU produced
        m_ref = O.deposit(h.grid, W.upcast(gpu_st[s]))
        me = P.assert_moments(gpu_m[s], m_ref, P.MOM32)
        _say("fp32 species %d: pos/L %.2e vel %.2e mom rel-L2 %.2e" % (s, pe, ve, me))


def test_fp32_ten_steps_reported_against_fp64(spic, ctx):
    """Multi-step FP32 trajectories diverge from FP64 by rounding; the error is
    reported and only bounded loosely (it is not a tolerance of the method)."""
    h = W.harris_32x16x4()
    f32, sps32 = _fp32_inputs(h)
    gpu_st, gpu_m = _run_gpu(spic, ctx, h, f32, sps32, 10, torch.float32)
    f64 = {k: v.astype(np.float64) for k, v in f32.items()}
    states, moms = O.run(h, f64, [W.upcast(s) for s in sps32], 10)
    for s in range(4):
        pe, ve = P.state_errors(gpu_st[s], states[s], h.grid)
        me = P.rel_l2(gpu_m[s], moms[s]).max()
        _say("fp32 vs fp64 after 10 steps, species %d: pos/L %.2e vel %.2e mom %.2e" % (s, pe, ve, me))
        assert pe < 1e-3 and me < 1e-2


def test_mixed_precision_moments_beat_pure_single(spic, ctx):
    """Sec. V-D: mixed precision is more accurate than pure single precision.
    Analogue here: FP64-accumulated moments of FP32 particles are closer to
    the oracle's deposit of the same state than FP32-accumulated ones."""
    h = W.harris_32x16x4()
    f32, sps32 = _fp32_inputs(h)
    _, m64 = _run_gpu(spic, ctx, h, f32, sps32, 1, torch.float32, acc=torch.float64)
    st32, m32 = _run_gpu(spic, ctx, h, f32, sps32, 1, torch.float32, acc=torch.float32)
    for s in range(4):
        ref = O.deposit(h.grid, W.upcast(st32[s]))
        e64, e32 = P.rel_l2(m64[s], ref).max(), P.rel_l2(m32[s], ref).max()
        _say("species %d: f64-acc %.2e  f32-acc %.2e" % (s, e64, e32))
        assert e64 < e32


# ---------------------------------------------------------- entry points

def test_move_only_and_deposit_only_compose_to_the_fused_step(spic, ctx):
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sp = W.make_species(h, W.SHEET_E)
    dev_f = spic.to_device(f, torch.float64)
    a = spic.to_device(sp, torch.float64)
    b = spic.to_device(sp, torch.float64)
    ma = spic.moment_buffers(h.grid, 1)
    mb = spic.moment_buffers(h.grid, 1)
    prm = spic.make_params(h.dt, h.c, h.niter)
    spic.spic_mover(ctx, h.grid, prm, dev_f, [a], [h.qom_e], ma)
    spic.spic_mover(ctx, h.grid, prm, dev_f, [b], [h.qom_e], None)
    spic.spic_moments(ctx, h.grid, [b], mb)
    torch.cuda.synchronize()
    for k in ("x", "y", "z", "u", "v", "w"):
        assert torch.equal(a[k], b[k])
    P.assert_moments(mb[0].cpu().numpy(), ma[0].cpu().numpy(), 1e-14)
    # accumulate adds on top
    spic.spic_moments(ctx, h.grid, [b], mb, accumulate=True)
    torch.cuda.synchronize()
    P.assert_moments(mb[0].cpu().numpy(), 2 * ma[0].cpu().numpy(), 1e-14)


@pytest.mark.parametrize("block", [64, 128, 512, 1024])
def test_block_size_does_not_change_results(spic, ctx, block):
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sps = W.make_all_species(h)
    ref_st, ref_m = _run_gpu(spic, ctx, h, f, sps, 2, torch.float64)
    ctx.set_option("block", block)
    st, m = _run_gpu(spic, ctx, h, f, sps, 2, torch.float64)
    for s in range(4):
        a, b = P.by_id(st[s]), P.by_id(ref_st[s])
        for k in ("x", "y", "z", "u", "v", "w"):
            assert np.array_equal(a[k], b[k])
        P.assert_moments(m[s], ref_m[s], 1e-14)


def test_invalid_call_enqueues_nothing(spic, ctx):
    h = W.harris_32x16x4()
    sp = spic.to_device(W.make_species(h, 0), torch.float64)
    f = spic.to_device(W.make_fields(h), torch.float64)
    before = sp["x"].clone()
    prm = spic.make_params(h.dt, h.c, 0)   # niter 0 is invalid
    st = spic.spic_mover(ctx, h.grid, prm, f, [sp], [h.qom_e], None, raw=True)
    torch.cuda.synchronize()
    assert st == spic.SPIC_E_ARG
    assert torch.equal(before, sp["x"])


def test_compensated_fp32_moments(spic, ctx):
    """SPIC_F32C (compensated FP32: FP32 terms, high plane by atomics, the
    exact rounding error of each addition in a low plane, no FP64) after one
    fused step of the FP32 state, and from spic_moments: high + low against
    the oracle's FP64 deposit of the same FP32 state within the FP32 moment
    tolerance, and no worse than plain FP32 accumulation of the same terms."""
    h = W.harris_32x16x4()
    f32 = {k: v.astype(np.float32) for k, v in W.make_fields(h).items()}
    sps = [W.round_state(s, np.float32) for s in W.make_all_species(h)]
    dev_f = spic.to_device(f32, torch.float32)
    dev = [spic.to_device(s, torch.float32) for s in sps]
    mc = spic.moment_buffers(h.grid, 4, compensated=True)
    _say("case compensated fp32 moments")
    spic.spic_mover(ctx, h.grid, spic.make_params(h.dt, h.c, h.niter, 0, 0), dev_f, dev, h.qoms, mc)
    torch.cuda.synchronize()
    m32 = spic.moment_buffers(h.grid, 4, torch.float32)
    spic.spic_moments(ctx, h.grid, dev, m32)
    mc2 = spic.moment_buffers(h.grid, 4, compensated=True)
    spic.spic_moments(ctx, h.grid, dev, mc2)
    torch.cuda.synchronize()
    worst = [0.0, 0.0]
    for s in range(4):
        ref = O.deposit(h.grid, W.upcast(spic.to_host(dev[s])))
        for planes in (mc[s], mc2[s]):
            hi_lo = planes.double().sum(dim=0).cpu().numpy()
            ec = P.assert_moments(hi_lo, ref, P.MOM32)
        e32 = float(P.rel_l2(m32[s].cpu().numpy(), ref).max())
        worst = [max(worst[0], ec), max(worst[1], e32)]
        assert ec <= e32, (s, ec, e32)
    _say("compensated fp32 worst rel-L2 %.2e, plain fp32 %.2e" % tuple(worst))
