"""Seeded synthetic inputs: determinism, porosity, percolation, structure."""
import numpy as np

from paper_1704_03126_amd import geometry as G


def test_porous_deterministic_and_porosity():
    a = G.porous_discs(96, 0.6, 1003)
    b = G.porous_discs(96, 0.6, 1003)
    assert np.array_equal(a.mask, b.mask) and a.seed == b.seed
    assert a.mask.dtype == np.uint8 and a.mask.shape == (96, 96)
    assert 0.5 < a.porosity <= 0.6 + 1e-12
    labels, perc = G.component_labels(a.mask, periodic_y=True)
    assert perc.size > 0 and perc.all()          # every pore carries flux in x
    c = G.porous_discs(96, 0.6, 1004)
    assert not np.array_equal(a.mask, c.mask)


def test_fill_nonpercolating_hand_drawn():
    m = np.zeros((6, 8), dtype=np.uint8)
    m[1:5, 2] = 1
    m[1:5, 5] = 1
    m[1, 2:6] = 1
    m[4, 2:6] = 1                       # closed box around cells (2..3, 3..4)
    out = G.fill_nonpercolating(m, periodic_y=False)
    assert out[2:4, 3:5].all()          # isolated pore filled
    assert (out[0] == 0).all() and (out[5] == 0).all()
    # a pore that wraps only in y does not percolate along x
    m2 = np.ones((6, 6), dtype=np.uint8)
    m2[:, 2] = 0                         # vertical slot, periodic in y
    m2[3, :] = 0                         # horizontal slot, wraps in x
    labels, perc = G.component_labels(m2, periodic_y=True)
    assert perc.tolist() == [True]
    m3 = np.ones((6, 6), dtype=np.uint8)
    m3[:, 2] = 0
    assert G.fill_nonpercolating(m3, periodic_y=True).all()


def test_rough_channel_structure():
    g = G.cfg_rough_channel()
    assert g.mask.shape == (128, 256) and not g.periodic_y
    assert g.mask[:26, :128].all() and g.mask[-26:, :128].all()
    assert not g.mask[26:-26].any() and not g.mask[:, 128:].any()
    assert np.array_equal(g.mask, g.mask[::-1])          # aligned blocks
    assert g.n_fluid == 256 * 128 - 2 * 26 * 128
    assert g.cells_per_H == 128.0


def test_delta_field_statistics():
    d = G.delta_field((64, 64), 1005)
    lg = np.log(d)
    assert abs(lg.mean()) < 1e-12 and abs(lg.std() - 0.2) < 1e-12
    assert np.array_equal(d, G.delta_field((64, 64), 1005))
    # smoothed over ~8 cells: neighbours are strongly correlated
    corr = np.corrcoef(lg[:, :-1].ravel(), lg[:, 1:].ravel())[0, 1]
    assert corr > 0.95


def test_batch_instances_uneven_and_seeded():
    b1 = G.batch_instances(6, seed=1004)
    b2 = G.batch_instances(6, seed=1004)
    for x, y in zip(b1, b2):
        assert np.array_equal(x.mask, y.mask) and x.meta["delta"] == y.meta["delta"]
    assert b1[0].periodic_y and not b1[1].periodic_y
    sizes = {x.mask.shape for x in b1}
    assert len(sizes) > 1
    for x in b1:
        assert 64 <= x.nx <= 384 and 0.01 <= x.meta["delta"] <= 100


def test_fractal_couette_channel():
    from paper_1704_03126_amd.geometry import fractal_couette_channel, wm_profile
    g = fractal_couette_channel(32, eps=0.02)
    r = g.meta["profile"]
    assert g.nx == 160 and not g.periodic_y
    assert abs(np.sqrt(np.mean(r ** 2)) - 0.02) <= 1e-14           # sigma / H
    # the profile is Eq. (WM) with the stored amplitude, cut at gamma^n <= 16
    xc = (np.arange(160) + 0.5) / 32
    assert g.meta["n_max"] == 6
    assert np.allclose(r, wm_profile(xc, g.meta["A"], 1.5, 1.5, -4, 6), rtol=0, atol=1e-15)
    # solid below the surface, fluid above, H = 32 rows above the mean line
    nb = g.meta["rows_below"]
    assert g.ny == nb + 32
    yc = (np.arange(g.ny) - nb + 0.5) / 32
    assert np.array_equal(g.mask, (yc[:, None] < r[None, :]).astype(np.uint8))
    assert np.all(g.mask[nb + 8:] == 0)
    # every column is solid from the bottom up to its surface only
    assert np.all(np.diff(g.mask.astype(int), axis=0) <= 0)
