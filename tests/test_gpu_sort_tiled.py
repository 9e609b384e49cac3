"""GPU tests of the cell sort and of the tiled fused path (the path used once
a species has been sorted), against the FP64 oracle and the generic path.

The sort only permutes particles (checked by id, bitwise); the tiled path
must give the oracle's result whatever the particle order, including
particles that left their tile's LDS region, ragged edge tiles and grids
smaller than one region (periodic images aliased inside the region).
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


def _keys_np(g, st, tile):
    tx, ty, tz = tile
    dx, dy, dz = g.d
    i = np.minimum((np.asarray(st["x"], np.float64) / dx).astype(np.int64), g.nx - 1)
    j = np.minimum((np.asarray(st["y"], np.float64) / dy).astype(np.int64), g.ny - 1)
    k = np.minimum((np.asarray(st["z"], np.float64) / dz).astype(np.int64), g.nz - 1)
    nty, ntz = -(-g.ny // ty), -(-g.nz // tz)
    tile_id = ((i // tx) * nty + (j // ty)) * ntz + (k // tz)
    # local cells: slow axis = the one with the finest cells (ties: z, y, x),
    # then the other two in x, y, z order
    d = [dx, dy, dz]
    slow = 2
    if d[1] < d[slow]:
        slow = 1
    if d[0] < d[slow]:
        slow = 0
    mid, fast = [a for a in range(3) if a != slow]
    loc = [i % tx, j % ty, k % tz]
    t = [tx, ty, tz]
    local = (loc[slow] * t[mid] + loc[mid]) * t[fast] + loc[fast]
    return tile_id, local


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sort_permutes_into_full_rows(spic, ctx, dtype):
    """Full rows: a tile of n particles and C cells holds n // C full
    rows in which slot (r, c) is a particle of cell c whenever cell c has
    more than r particles (the others fill the remaining slots).  The
    default of the split variant; set here for both precisions."""
    ctx.set_option("sort_rows", 1)
    h = W.harris_32x16x4()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = h.grid
    sps = [W.random_particles(g, 20011, 1.0, seed=5), W.make_species(h, W.SHEET_E)]
    for sp in sps:
        perm = np.random.default_rng(3).permutation(sp["x"].size)
        sp = {k: v[perm] for k, v in sp.items()}
        dev = spic.to_device(sp, tdt)
        _say("case sort %s full rows, %d particles" % (dtype, sp["x"].size))
        for rep in range(2):  # the second sort runs the ordered key pass and the tiled gather
            spic.spic_sort(ctx, g, [dev])
            torch.cuda.synchronize()
            out = spic.to_host(dev)
            a, b = P.by_id(out), P.by_id(spic.to_host(spic.to_device(sp, tdt)))
            for k in a:
                assert np.array_equal(a[k], b[k]), k
            tile_id, local = _keys_np(g, out, (4, 4, 4))
            assert np.all(np.diff(tile_id) >= 0), "tiles not contiguous"
            for t in np.unique(tile_id)[:60]:
                loc = local[tile_id == t]
                counts = np.bincount(loc, minlength=64)
                R = loc.size // 64
                for r in range(R):
                    row = loc[64 * r:64 * (r + 1)]
                    home = counts > r
                    assert np.array_equal(row[home], np.flatnonzero(home)), (t, r)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sort_permutes_into_tile_rank_major_order(spic, ctx, dtype):
    ctx.set_option("sort_rows", 0)
    h = W.harris_32x16x4()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sp = W.make_species(h, W.SHEET_E)
    # scramble so the sort has work to do
    perm = np.random.default_rng(1).permutation(sp["x"].size)
    sp = {k: v[perm] for k, v in sp.items()}
    dev = spic.to_device(sp, tdt)
    _say("case sort %s harris_32x16x4 sheet_e" % dtype)
    spic.spic_sort(ctx, h.grid, [dev])
    torch.cuda.synchronize()
    out = spic.to_host(dev)
    a, b = P.by_id(out), P.by_id(spic.to_host(spic.to_device(sp, tdt)))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    tile_id, local = _keys_np(h.grid, out, (4, 4, 4))
    assert np.all(np.diff(tile_id) >= 0), "tiles not contiguous"
    # rank-major inside each tile: inside a rank block local cells increase;
    # a new block starts exactly where the local cell does not increase
    for t in np.unique(tile_id)[:50]:
        loc = local[tile_id == t]
        counts = np.bincount(loc, minlength=64)
        starts = np.flatnonzero(np.diff(loc) <= 0) + 1
        blocks = np.split(loc, starts)
        for r, blk in enumerate(blocks):
            assert np.array_equal(blk, np.flatnonzero(counts > r)), (t, r)


def _oracle_steps(h, f, sps, qoms, nsteps):
    st = [dict(s) for s in sps]
    ms = None
    for _ in range(nsteps):
        ms = []
        for s in range(len(st)):
            st[s], m = O.step(h.grid, h.dt, h.c, h.niter, qoms[s], f, st[s])
            ms.append(m)
    return st, ms


def _gpu_steps(spic, ctx, h, f, sps, qoms, nsteps, dtype=torch.float64, sort_every=4, check=None):
    dev_f = spic.to_device(f, dtype)
    dev = [spic.to_device(s, dtype) for s in sps]
    moms = spic.moment_buffers(h.grid, len(sps))
    for step in range(nsteps):
        prm = spic.make_params(h.dt, h.c, h.niter, sort_every, step)
        spic.spic_mover(ctx, h.grid, prm, dev_f, dev, qoms, moms)
        if check:
            torch.cuda.synchronize()
            check(step, [spic.to_host(d) for d in dev], [m.cpu().numpy() for m in moms])
    torch.cuda.synchronize()
    return [spic.to_host(d) for d in dev], [m.cpu().numpy() for m in moms]


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_tiled_fp64_every_step_matches_oracle(spic, ctx, variant):
    """32x16x4 cells, 4 species, 10 steps, sorted every 4 steps: every
    variant (LDS-atomic deposit, with the mover's corner cache, and the
    split launch with the sorted register deposit)."""
    ctx.set_option("tile_variant", variant)
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sps = W.make_all_species(h)
    ora = [dict(s) for s in sps]

    def check(step, states, moms):
        for s in range(4):
            ora[s], m = O.step(h.grid, h.dt, h.c, h.niter, h.qoms[s], f, ora[s])
            P.assert_state(states[s], ora[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(moms[s], m, P.MOM64)

    _say("case tiled fp64 harris_32x16x4 sort_every 4")
    _gpu_steps(spic, ctx, h, f, sps, h.qoms, 10, check=check)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_tiled_fp32_one_step(spic, ctx, variant):
    ctx.set_option("tile_variant", variant)
    h = W.harris_32x16x4()
    f32 = {k: v.astype(np.float32) for k, v in W.make_fields(h).items()}
    sps = [W.round_state(s, np.float32) for s in W.make_all_species(h)]
    _say("case tiled fp32 one step")
    st, ms = _gpu_steps(spic, ctx, h, f32, sps, h.qoms, 1, dtype=torch.float32, sort_every=1)
    f64 = {k: v.astype(np.float64) for k, v in f32.items()}
    for s in range(4):
        ora = O.mover(h.grid, h.dt, h.c, h.niter, h.qoms[s], f64, W.upcast(sps[s]))
        P.assert_state(st[s], ora, h.grid, P.POS32, P.VEL32, vscale=max(P.vmax(ora), h.vths[s]))
        P.assert_moments(ms[s], O.deposit(h.grid, W.upcast(st[s])), P.MOM32)


# FP32 cases for the one-launch variant: (grid, species maker, tile, halo,
# steps, sort cadence)
def _lanecell_case(name):
    h = W.harris_32x16x4()
    g = h.grid
    if name in ("harris", "harris_block512"):
        return h, W.make_all_species(h), h.qoms, (4, 4, 4), 1, 6, 3
    if name == "tiles_2x4x8":
        return h, W.make_all_species(h), h.qoms, (2, 4, 8), 1, 4, 2
    if name == "tiles_3x3x3_halo2":
        return h, W.make_all_species(h), h.qoms, (3, 3, 3), 2, 4, 2
    if name == "fast":  # particles leave their tile and the region
        return h, [W.random_particles(g, 20011, 2.0, seed=7), W.make_species(h, W.SHEET_I)], [-64.0, 1.0], \
            (4, 4, 4), 1, 3, 2
    if name == "crowded":  # one tile: full bins, then an out list past its capacity
        hc = W.Harris(W.Grid(4, 4, 4, 2.0, 2.0, 2.0), ppc=8)
        return hc, [W.random_particles(hc.grid, 40000, 0.5, seed=3), W.random_particles(hc.grid, 30000, 0.1, seed=4)], \
            [-64.0, 1.0], (4, 4, 4), 1, 3, 1
    hs = W.Harris(W.Grid(5, 3, 2, 3.0, 2.0, 1.0), ppc=8)  # tiny: periodic images alias in the region
    return hs, [W.make_species(hs, s) for s in range(4)], hs.qoms, (4, 4, 4), 1, 3, 1


@pytest.mark.parametrize("case", ["harris", "harris_block512", "tiles_2x4x8", "tiles_3x3x3_halo2", "fast", "crowded",
                                  "tiny"])
def test_one_launch_variant_matches_split_fp32(spic, ctx, case):
    """Variant 3 (the mover and the sorted register deposit in one launch)
    against variant 2 on the same FP32 input: the particles are bitwise
    equal by id (the same mover arithmetic), the moments agree to the FP32
    partial sums' rounding, and the moments of the last step match the
    oracle's deposit of the moved state."""
    h, sps, qoms, tile, halo, nsteps, cadence = _lanecell_case(case)
    f32 = {k: v.astype(np.float32) for k, v in W.make_fields(h).items()}
    s32 = [W.round_state(x, np.float32) for x in sps]
    runs = []
    for variant in (2, 3):
        c = spic.Context(0)
        c.set_option("tile_x", tile[0]); c.set_option("tile_y", tile[1]); c.set_option("tile_z", tile[2])
        c.set_option("halo", halo)
        c.set_option("tile_variant", variant)
        if case == "harris_block512":
            c.set_option("tile_block", 512)
        _say("case one-launch fp32 %s variant %d (%d steps, sort every %d)" % (case, variant, nsteps, cadence))
        runs.append(_gpu_steps(spic, c, h, f32, s32, qoms, nsteps, dtype=torch.float32, sort_every=cadence))
        c.close()
    (a_st, a_m), (b_st, b_m) = runs
    for s in range(len(sps)):
        a, b = P.by_id(a_st[s]), P.by_id(b_st[s])
        for k in ("x", "y", "z", "u", "v", "w", "q"):
            assert np.array_equal(a[k], b[k]), (s, k)
        P.assert_moments(b_m[s], a_m[s], P.MOM32)
        P.assert_moments(b_m[s], O.deposit(h.grid, W.upcast(b_st[s])), P.MOM32)


@pytest.mark.parametrize("tile,halo,variant", [((4, 4, 4), 0, 0), ((4, 4, 4), 0, 2), ((2, 4, 8), 1, 1),
                                               ((3, 3, 3), 1, 2), ((2, 2, 2), 2, 2), ((2, 8, 4), 1, 2),
                                               ((4, 4, 2), 1, 1), ((4, 4, 4), 1, 0), ((4, 4, 4), 0, 1),
                                               ((3, 2, 4), 2, 2), ((2, 4, 8), 1, 2), ((3, 3, 3), 2, 0),
                                               ((4, 4, 2), 1, 2), ((3, 3, 3), 2, 1), ((1, 1, 1), 1, 2),
                                               ((8, 8, 1), 1, 2)])
def test_tile_shapes_and_halo_overflow_match_oracle(spic, ctx, tile, halo, variant):
    """Fast particles leave small regions (halo 0) -> global fallbacks; tile
    shapes that do not divide the grid leave ragged edge tiles."""
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    g = h.grid
    sps = [W.random_particles(g, 20011, 2.0, seed=7), W.make_species(h, W.SHEET_I)]
    qoms = [-64.0, 1.0]
    ctx.set_option("tile_x", tile[0]); ctx.set_option("tile_y", tile[1]); ctx.set_option("tile_z", tile[2])
    ctx.set_option("halo", halo)
    ctx.set_option("tile_variant", variant)
    _say("case tiles %s halo %d variant %d" % (tile, halo, variant))
    st, ms = _gpu_steps(spic, ctx, h, f, sps, qoms, 3, sort_every=2)
    ora, oms = _oracle_steps(h, f, sps, qoms, 3)
    for s in range(2):
        P.assert_state(st[s], ora[s], g, P.POS64, P.VEL64)
        P.assert_moments(ms[s], oms[s], P.MOM64)


@pytest.mark.parametrize("cache", [1, 0])
@pytest.mark.parametrize("tile,halo,mover_halo", [((4, 4, 4), 1, 0), ((4, 4, 4), 1, 1), ((4, 4, 4), 1, 2),
                                                    ((4, 4, 4), 1, 3), ((4, 4, 4), 0, -1), ((2, 4, 8), 1, -1),
                                                    ((3, 3, 3), 2, 4)])
def test_split_variant_mover_halo(spic, ctx, tile, halo, mover_halo, cache):
    """Variant 2's mover stages its own field region (by default one
    cell of halo more than the deposit's), with or without the last cell's
    field corners in registers; fast particles leave both regions."""
    ctx.set_option("mover_cache", cache)
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    g = h.grid
    sps = [W.random_particles(g, 20011, 2.0, seed=11), W.make_species(h, W.SHEET_E)]
    qoms = [-64.0, -64.0]
    ctx.set_option("tile_x", tile[0]); ctx.set_option("tile_y", tile[1]); ctx.set_option("tile_z", tile[2])
    ctx.set_option("halo", halo)
    ctx.set_option("mover_halo", mover_halo)
    ctx.set_option("tile_variant", 2)
    _say("case split mover halo: tiles %s halo %d mover_halo %d cache %d" % (tile, halo, mover_halo, cache))
    st, ms = _gpu_steps(spic, ctx, h, f, sps, qoms, 3, sort_every=2)
    ora, oms = _oracle_steps(h, f, sps, qoms, 3)
    for s in range(2):
        P.assert_state(st[s], ora[s], g, P.POS64, P.VEL64)
        P.assert_moments(ms[s], oms[s], P.MOM64)


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("cells", [(5, 3, 2), (2, 2, 2), (9, 7, 5)])
def test_tiny_and_odd_grids(spic, ctx, cells, variant):
    """Grids smaller than one LDS region: periodic images alias inside it."""
    ctx.set_option("tile_variant", variant)
    h = W.Harris(W.Grid(*cells, 3.0, 2.0, 1.0), ppc=8)
    f = W.make_fields(h)
    sps = [W.make_species(h, s) for s in range(4)]
    _say("case tiny grid %s variant %d" % (cells, variant))
    st, ms = _gpu_steps(spic, ctx, h, f, sps, h.qoms, 3, sort_every=1)
    ora, oms = _oracle_steps(h, f, sps, h.qoms, 3)
    for s in range(4):
        P.assert_state(st[s], ora[s], h.grid, P.POS64, P.VEL64)
        P.assert_moments(ms[s], oms[s], P.MOM64)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("L", [(1.0, 4.0, 2.0), (4.0, 1.0, 2.0), (4.0, 2.0, 1.0)])
def test_lane_cell_variant_with_each_slow_axis(spic, ctx, L, variant):
    """The sorted deposit gives lane l of every wave local cell l of its
    tile, whose index depends on which axis is the slow one (the finest
    cells): x, y and z in turn, 3 steps with a sort every step and every 2
    steps (variant 1 with its corner cache for comparison)."""
    ctx.set_option("tile_variant", variant)
    h = W.Harris(W.Grid(8, 8, 8, *L), ppc=8)
    f = W.make_fields(h)
    sps = [W.make_species(h, s) for s in range(4)]
    for cadence in (1, 2):
        _say("case lane cells variant %d L=%s sort_every %d" % (variant, L, cadence))
        st, ms = _gpu_steps(spic, ctx, h, f, sps, h.qoms, 3, sort_every=cadence)
        ora, oms = _oracle_steps(h, f, sps, h.qoms, 3)
        for s in range(4):
            P.assert_state(st[s], ora[s], h.grid, P.POS64, P.VEL64)
            P.assert_moments(ms[s], oms[s], P.MOM64)


def test_resort_of_a_crowded_tile(spic, ctx):
    """A re-sort stages each array's old tile range in LDS up to a fixed
    capacity (8192 FP32 or 4096 FP64 values) and reads the rest of the tile
    from global memory: one 4x4x4 tile holding 40,000 particles, FP64 steps
    sorted every step against the oracle, and FP32 steps sorted every step
    equal (by id, bitwise) to FP32 steps never sorted."""
    h = W.Harris(W.Grid(4, 4, 4, 2.0, 2.0, 2.0), ppc=8)
    g = h.grid
    f = W.make_fields(h)
    sps = [W.random_particles(g, 40000, 0.5, seed=3), W.random_particles(g, 30000, 0.1, seed=4)]
    qoms = [-64.0, 1.0]
    _say("case crowded tile fp64 (40000 + 30000 particles, 1 tile)")
    st, ms = _gpu_steps(spic, ctx, h, f, sps, qoms, 3, sort_every=1)
    ora, oms = _oracle_steps(h, f, sps, qoms, 3)
    for s in range(2):
        P.assert_state(st[s], ora[s], g, P.POS64, P.VEL64)
        P.assert_moments(ms[s], oms[s], P.MOM64)
    _say("case crowded tile fp32 sorted vs unsorted")
    f32 = {k: v.astype(np.float32) for k, v in f.items()}
    s32 = [W.round_state(x, np.float32) for x in sps]
    a_st, _ = _gpu_steps(spic, ctx, h, f32, s32, qoms, 3, dtype=torch.float32, sort_every=1)
    ctx2 = spic.Context(0)
    b_st, _ = _gpu_steps(spic, ctx2, h, f32, s32, qoms, 3, dtype=torch.float32, sort_every=0)
    ctx2.close()
    for s in range(2):
        a, b = P.by_id(a_st[s]), P.by_id(b_st[s])
        for k in ("x", "y", "z", "u", "v", "w", "q"):
            assert np.array_equal(a[k], b[k]), k


def test_sorted_and_unsorted_runs_agree(spic, ctx):
    """Sorting only reorders: the same particles (by id) and the same moments
    up to summation order."""
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sps = W.make_all_species(h)
    a_st, a_m = _gpu_steps(spic, ctx, h, f, sps, h.qoms, 6, sort_every=2)
    ctx2 = spic.Context(0)
    b_st, b_m = _gpu_steps(spic, ctx2, h, f, sps, h.qoms, 6, sort_every=0)
    ctx2.close()
    for s in range(4):
        a, b = P.by_id(a_st[s]), P.by_id(b_st[s])
        for k in ("x", "y", "z", "u", "v", "w"):
            assert np.array_equal(a[k], b[k]), k
        P.assert_moments(a_m[s], b_m[s], 1e-14)


def test_run_to_run_repeatability(spic, ctx):
    """Particles are bitwise repeatable; moments agree to rounding (atomics
    add in a varying order)."""
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sps = W.make_all_species(h)
    r1 = _gpu_steps(spic, ctx, h, f, sps, h.qoms, 3, sort_every=1)
    r2 = _gpu_steps(spic, ctx, h, f, sps, h.qoms, 3, sort_every=1)
    for s in range(4):
        a, b = P.by_id(r1[0][s]), P.by_id(r2[0][s])
        for k in ("x", "y", "z", "u", "v", "w"):
            assert np.array_equal(a[k], b[k])
        P.assert_moments(r1[1][s], r2[1][s], 1e-15)


@pytest.mark.parametrize("variant", [0, 2])
@pytest.mark.parametrize("group", [0, 4, 10])
def test_tile_group_mapping_matches_slabs(spic, ctx, group, variant):
    """Tiles dealt to the XCDs in groups of 2^group (4 is the default; 2^10
    exceeds the 128 tiles here, so most workgroups find no tile) run the
    same tile bodies as the XCD slabs: particles bitwise equal by id,
    moments equal to rounding, and both match the oracle."""
    h = W.harris_32x16x4()
    f = W.make_fields(h)
    sps = W.make_all_species(h)
    ctx.set_option("tile_variant", variant)
    ctx.set_option("tile_group", -1)
    a_st, a_m = _gpu_steps(spic, ctx, h, f, sps, h.qoms, 3, sort_every=2)
    ctx2 = spic.Context(0)
    ctx2.set_option("tile_variant", variant)
    ctx2.set_option("tile_group", group)
    _say("case tile_group %d variant %d" % (group, variant))
    b_st, b_m = _gpu_steps(spic, ctx2, h, f, sps, h.qoms, 3, sort_every=2)
    ctx2.close()
    ora, om = _oracle_steps(h, f, sps, h.qoms, 3)
    for s in range(4):
        a, b = P.by_id(a_st[s]), P.by_id(b_st[s])
        for k in ("x", "y", "z", "u", "v", "w"):
            assert np.array_equal(a[k], b[k]), k
        P.assert_moments(b_m[s], a_m[s], 1e-14)
        P.assert_state(b_st[s], ora[s], h.grid, P.POS64, P.VEL64)
        P.assert_moments(b_m[s], om[s], P.MOM64)
