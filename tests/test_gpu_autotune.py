"""GPU tests of the autotuner: tune() on one resident box and tune_runs() on
a small ensemble through the batch engine each return one of their
candidates, and steps taken with the chosen settings match the oracle."""
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


def _host(sp):
    return {k: v.detach().cpu().numpy() for k, v in sp.items()}


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_tune_single_box_then_step_matches_oracle(dtype_name, tmp_path, monkeypatch):
    from paper_2008_04397_amd import autotune, spic
    spic.lib()
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuned.json"))
    h = W.Harris(W.Grid(16, 8, 8), ppc=8, qom_e=-25.0, B0=0.02, seed=21)
    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    npdt = np.float64 if dtype_name == "f64" else np.float32
    f = spic.to_device(W.make_fields(h), tdt)
    species = [spic.to_device(W.make_species(h, s, dtype=npdt), tdt) for s in range(4)]
    moms = spic.moment_buffers(h.grid, 4)
    _say("[autotune] tune() %s on 16x8x8" % dtype_name)
    initial = [_host(s) for s in species]
    cfg = autotune.tune(h, f, species, h.qoms, moms, steps=4, quick=True, dtype_name=dtype_name)
    cands = list(autotune.candidates(True, dtype_name))
    assert cfg in cands
    # the trials leave the inputs as they found them
    for a, b in zip(initial, [_host(s) for s in species]):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    key = autotune.workload_class(dtype_name, h.grid, h.ppc)
    autotune.store(key, cfg)
    assert autotune.load(key) == cfg
    # one step with the tuned settings
    start = initial
    ctx = spic.Context(0)
    autotune.apply(ctx, cfg)
    assert spic.resolved_launch(ctx, dtype_name)["tile_block"] == cfg["tile_block"]
    spic.spic_mover(ctx, h.grid, spic.make_params(h.dt, h.c, h.niter, 1, 0), f, species, h.qoms, moms)
    torch.cuda.synchronize()
    ctx.close()
    fo = W.make_fields(h)
    pos, vel, mom = (P.POS64, P.VEL64, P.MOM64) if dtype_name == "f64" else (P.POS32, P.VEL32, P.MOM32)
    for s in range(4):
        ora, om = O.step(h.grid, h.dt, h.c, h.niter, h.qoms[s], fo, W.upcast(start[s]))
        gpu = _host(species[s])
        P.assert_state(gpu, ora, h.grid, pos, vel, vscale=max(P.vmax(ora), h.vths[s]))
        if dtype_name == "f64":
            P.assert_moments(moms[s].cpu().numpy(), om, mom)
        else:
            # FP32 particles: the moments against the FP64 deposit of the
            # kernel's own moved state
            P.assert_moments(moms[s].cpu().numpy(), O.deposit(h.grid, W.upcast(gpu)), mom)


def test_tune_runs_on_an_ensemble_then_runs_match_oracle(tmp_path, monkeypatch):
    from paper_2008_04397_amd import autotune, spic
    spic.lib()
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuned.json"))
    boxes = [W.Harris(W.Grid(16, 8, 4), ppc=8, qom_e=-25.0, B0=0.02, seed=31),
             W.Harris(W.Grid(8, 8, 8), ppc=10, qom_e=-64.0, B0=0.015, seed=32)]
    data = []
    for h in boxes:
        f = spic.to_device(W.make_fields(h), torch.float64)
        sps = [W.make_species(h, s) for s in range(4)]
        data.append((h, f, sps, [spic.to_device(s, torch.float64) for s in sps], spic.moment_buffers(h.grid, 4)))

    def make_runs(se, k):
        return [spic.Run(h.grid, spic.make_params(h.dt, h.c, h.niter, se, 0), f, dev, h.qoms, moms, k)
                for h, f, _, dev, moms in data]

    def reset():  # every trial (and the checked run) starts from the initial states
        for h, f, sps, dev, moms in data:
            for d, s in zip(dev, sps):
                for k in d:
                    d[k].copy_(torch.from_numpy(s[k]))

    cands = autotune.engine_candidates(quick=True)
    _say("[autotune] tune_runs() over %d candidates" % len(cands))
    cfg = autotune.tune_runs(lambda: spic.Context(0), make_runs, cands, steps=2, reset=reset)
    assert cfg in cands
    # 3 steps with the tuned settings from the initial states, vs the oracle
    reset()
    ctx = spic.Context(0)
    autotune.apply(ctx, cfg)
    for t in spic.spic_batch_submit(ctx, make_runs(cfg["sort_every"], 3)):
        spic.spic_wait(ctx, t)
    ctx.close()
    for h, f, sps, dev, moms in data:
        ora, om = O.run(h, W.make_fields(h), sps, 3)
        for s in range(4):
            P.assert_state(_host(dev[s]), ora[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(moms[s].cpu().numpy(), om[s], P.MOM64)
