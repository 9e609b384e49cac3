"""Properties of the seeded input generator (Harris sheet, species, streams)."""
import numpy as np

from paper_2008_04397_amd import workloads as W


def test_small_box_sizes():
    h = W.harris_32x16x4()
    assert h.grid.cells == 2048 and h.n_per_species == 55296 and h.n_total == 221184
    h2 = W.harris_128x64x32()
    assert h2.n_total == 67108864


def test_species_are_cell_sorted_and_inside_their_cells():
    h = W.harris_32x16x4()
    g = h.grid
    dx, dy, dz = g.d
    for s in range(4):
        sp = W.make_species(h, s)
        i = np.floor(sp["x"] / dx).astype(int)
        j = np.floor(sp["y"] / dy).astype(int)
        k = np.floor(sp["z"] / dz).astype(int)
        cell = (i * g.ny + j) * g.nz + k
        assert np.all(np.diff(cell) >= 0)
        assert np.all(np.bincount(cell, minlength=g.cells) == h.ppc)
        assert np.all(np.sign(sp["q"]) == np.sign(h.qoms[s]))
        np.testing.assert_allclose(sp["u"].std(), h.vths[s], rtol=0.05)
        assert np.array_equal(sp["id"], np.arange(h.n_per_species))


def test_slabs_concatenate_to_the_species():
    h = W.harris_32x16x4()
    whole = W.make_species(h, W.BG_E)
    parts = [W.species_slab(h, W.BG_E, a, b) for a, b in ((0, 5), (5, 17), (17, 32))]
    for k in whole:
        assert np.array_equal(whole[k], np.concatenate([p[k] for p in parts]))


def test_fields_are_seeded_and_shaped():
    h = W.harris_32x16x4()
    a, b = W.make_fields(h), W.make_fields(h)
    for k in a:
        assert a[k].shape == (h.grid.nodes,) and np.array_equal(a[k], b[k])
    assert np.abs(a["ex"]).max() <= 0.01 * h.B0
    assert np.abs(a["bx"]).max() <= h.B0 * 1.01


def test_non_cube_ppc_and_subsample():
    h = W.Harris(W.Grid(8, 4, 4), ppc=10)
    sp = W.make_species(h, 0)
    assert sp["x"].size == 8 * 4 * 4 * 10
    m = W.subsample_mask(np.arange(1 << 16), 64)
    assert 0.8 / 64 < m.mean() < 1.2 / 64


def test_ensemble_and_serving_streams():
    boxes = W.ensemble_boxes(64)
    assert len(boxes) == 64 and len({b.grid for b in boxes}) > 4
    assert all(b.ppc in (8, 27, 64) for b in boxes)
    reqs = W.serving_stream(200)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0) and 5.0 < t[-1] < 15.0
