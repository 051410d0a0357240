"""Pins of the oracle's inference occupancy grid (Sec. 3.3): the lattice,
the dilation, and the composition with the deform / density oracle."""
import numpy as np

import oracle as orc
from paper_2212_10550_amd import synth


def test_lattice_points_are_cell_centres():
    p = orc.lattice_points(2, (0, 0, 0, 1, 1, 1))
    assert p.dtype == np.float32 and p.shape == (8, 3)
    # point n = x + 2 (y + 2 z)
    np.testing.assert_array_equal(p[0], [0.25, 0.25, 0.25])
    np.testing.assert_array_equal(p[1], [0.75, 0.25, 0.25])
    np.testing.assert_array_equal(p[2], [0.25, 0.75, 0.25])
    np.testing.assert_array_equal(p[4], [0.25, 0.25, 0.75])
    q = orc.lattice_points(5, (-1, 0, 2, 1, 4, 3))
    # every point is inside its own cell, cells tile the box in order
    for a, (lo, hi) in enumerate([(-1, 1), (0, 4), (2, 3)]):
        v = np.unique(q[:, a])
        assert len(v) == 5 and np.all(np.diff(v) > 0)
        cell = np.floor((v - lo) / (hi - lo) * 5).astype(int)
        np.testing.assert_array_equal(cell, np.arange(5))


def test_dilation_closed_forms():
    G = 9
    occ = np.zeros((G, G, G), bool)
    occ[4, 4, 4] = True
    np.testing.assert_array_equal(orc.dilate(occ, 0), occ)
    d1 = orc.dilate(occ, 1)
    assert d1.sum() == 27 and d1[3:6, 3:6, 3:6].all()
    d2 = orc.dilate(occ, 2)
    assert d2.sum() == 125 and d2[2:7, 2:7, 2:7].all()
    # a corner cell is clipped by the grid: 2 x 2 x 2 for r = 1
    c = np.zeros((G, G, G), bool)
    c[0, 0, G - 1] = True
    dc = orc.dilate(c, 1)
    assert dc.sum() == 8 and dc[:2, :2, G - 2:].all()
    # asymmetric sizes per axis are handled independently
    e = np.zeros((3, 4, 5), bool)
    e[1, 0, 4] = True
    de = orc.dilate(e, 1)
    assert de.sum() == 3 * 2 * 2 and de[0:3, 0:2, 3:5].all()
    # dilation is monotone and idempotent in r: d(d(x, 1), 1) = d(x, 2)
    rng = np.random.default_rng(0)
    x = rng.random((G, G, G)) < 0.02
    np.testing.assert_array_equal(orc.dilate(orc.dilate(x, 1), 1), orc.dilate(x, 2))
    assert (orc.dilate(x, 1) >= x).all()


def test_occgrid_composition():
    """Against the stages it composes: the roots of the lattice points are
    the deform oracle's, the densities the encode+MLP oracle's, and every
    cell with a density above the threshold is occupied after dilation.
    Rest pose (identity bones): the roots are the lattice points themselves."""
    w = synth.tiny_forward()
    nb = w.B.shape[0]
    B = np.tile(np.eye(3, 4), (nb, 1, 1))
    G = 6
    res = orc.resolutions(w.L, w.base_res, w.growth)
    params = synth.make_mlp(seed=3)
    table = synth.make_hash_table(w.L, w.table.shape[1], 2, seed=5, scale=0.3)
    pts = orc.lattice_points(G, (0, 0, 0, 1, 1, 1))
    d = orc.deform(pts, B, w.W, w.skin_aabb, w.hash_aabb)
    assert (d["bone"] >= 0).all()
    np.testing.assert_allclose(d["xc"], pts, atol=1e-9)
    feat = orc.hash_encode(d["xc"], table, res, w.hash_aabb)
    sigma, _ = orc.mlp_fwd(feat, params, w.widths)
    thresh = float(np.median(sigma))
    out = orc.occgrid_build(G, (0, 0, 0, 1, 1, 1), B, w.W, w.skin_aabb, w.hash_aabb, table, res, params,
                            w.widths, thresh, 1)
    np.testing.assert_array_equal(out["points"], pts)
    np.testing.assert_array_equal(out["sigma"], sigma)
    occ = (sigma > thresh).reshape(G, G, G)
    assert 0 < occ.sum() < occ.size
    np.testing.assert_array_equal(out["occ"], occ)
    assert (out["grid"] >= occ).all()
    np.testing.assert_array_equal(out["grid"], orc.dilate(occ, 1))
    # a point whose multi-init search finds no root has density 0 (empty)
    far = orc.occgrid_build(2, (5, 5, 5, 6, 6, 6), B, w.W, w.skin_aabb, w.hash_aabb, table, res, params,
                            w.widths, -1.0, 0)
    assert (far["deform"]["bone"] < 0).all() and (far["sigma"] == 0).all() and far["grid"].all()


def test_jittered_points_stay_in_their_cells():
    G = 7
    rng = np.random.default_rng(1)
    u = rng.random((3, G ** 3)).astype(np.float32) * np.float32(0.999)
    box = (-0.5, 0.0, 1.0, 1.5, 2.0, 1.25)
    p = orc.jittered_points(G, box, u)
    c = orc.point_cells(p, box, G)
    n = np.arange(G ** 3)
    np.testing.assert_array_equal(c, np.stack([n % G, (n // G) % G, n // (G * G)], 1))
    # u = 1/2 is the lattice of cell centres
    np.testing.assert_array_equal(orc.jittered_points(G, box, np.full((3, G ** 3), 0.5, np.float32)),
                                  orc.lattice_points(G, box))


def test_point_cells_closed_forms():
    box = (0, 0, 0, 1, 1, 1)
    x = np.array([[0.0, 0.0, 0.0], [0.999, 0.5, 0.25], [1.0, -0.1, 2.0], [0.125, 0.375, 0.875]], np.float32)
    np.testing.assert_array_equal(orc.point_cells(x, box, 8), [[0, 0, 0], [7, 4, 2], [7, 0, 7], [1, 3, 7]])


def test_occgrid_update_moving_average():
    """beta = 0 is the inference grid at the jittered points; beta = 1
    keeps the old values; in between, the values are the stated average."""
    w = synth.tiny_forward()
    nb = w.B.shape[0]
    B = np.tile(np.eye(3, 4), (nb, 1, 1))
    G = 4
    res = orc.resolutions(w.L, w.base_res, w.growth)
    params = synth.make_mlp(seed=3)
    table = synth.make_hash_table(w.L, w.table.shape[1], 2, seed=5, scale=0.3)
    u = np.random.default_rng(2).random((3, G ** 3)).astype(np.float32)
    old = np.random.default_rng(3).random(G ** 3) * 2.0
    box = (0, 0, 0, 1, 1, 1)
    a = orc.occgrid_update(old, G, box, u, B, w.W, w.skin_aabb, w.hash_aabb, table, res, params, w.widths, 0.0,
                           0.8, 0)
    d = orc.deform(a["points"], B, w.W, w.skin_aabb, w.hash_aabb)
    feat = orc.hash_encode(d["xc"], table, res, w.hash_aabb, valid=d["bone"])
    sigma, _ = orc.mlp_fwd(feat, params, w.widths, valid=d["bone"])
    np.testing.assert_array_equal(a["values"], sigma)
    np.testing.assert_array_equal(a["grid"], (sigma > 0.8).reshape(G, G, G))
    b = orc.occgrid_update(old, G, box, u, B, w.W, w.skin_aabb, w.hash_aabb, table, res, params, w.widths, 1.0,
                           0.8, 0)
    np.testing.assert_array_equal(b["values"], old)
    c = orc.occgrid_update(old, G, box, u, B, w.W, w.skin_aabb, w.hash_aabb, table, res, params, w.widths, 0.75,
                           0.8, 1)
    np.testing.assert_allclose(c["values"], 0.75 * old + 0.25 * sigma, rtol=1e-15)
    np.testing.assert_array_equal(c["grid"], orc.dilate((c["values"] > 0.8).reshape(G, G, G), 1))


def test_density_reg_closed_form():
    G = 4
    grid = np.zeros((G, G, G), bool)
    grid[1, 2, 3] = True  # z = 1, y = 2, x = 3 occupied
    box = (0, 0, 0, 1, 1, 1)
    x = np.array([[0.875, 0.625, 0.375],    # cell (3, 2, 1): occupied
                  [0.125, 0.125, 0.125],    # empty
                  [0.6, 0.9, 0.1]], np.float32)  # empty
    sigma = np.array([5.0, 2.0, 0.5])
    loss, grad = orc.density_reg(x, sigma, grid, box, 0.1)
    assert abs(loss - 0.1 * (2.0 + 0.5) / 3) < 1e-15
    np.testing.assert_allclose(grad, [0.0, 0.1 / 3, 0.1 / 3], rtol=1e-15)
    # finite differences of the loss in sigma
    eps = 1e-6
    for i in range(3):
        s2 = sigma.copy()
        s2[i] += eps
        l2, _ = orc.density_reg(x, s2, grid, box, 0.1)
        assert abs((l2 - loss) / eps - grad[i]) < 1e-8


def test_occgrid_update_on_a_subset_of_cells():
    """Listed cells get the average, the others keep their values; the
    listed cells' points are those of the full update."""
    w = synth.tiny_forward()
    nb = w.B.shape[0]
    B = np.tile(np.eye(3, 4), (nb, 1, 1))
    G = 4
    res = orc.resolutions(w.L, w.base_res, w.growth)
    params = synth.make_mlp(seed=3)
    table = synth.make_hash_table(w.L, w.table.shape[1], 2, seed=5, scale=0.3)
    rng = np.random.default_rng(4)
    u = rng.random((3, G ** 3)).astype(np.float32)
    old = rng.random(G ** 3) * 2.0
    cells = np.sort(rng.choice(G ** 3, 20, replace=False))
    box = (0, 0, 0, 1, 1, 1)
    full = orc.occgrid_update(old, G, box, u, B, w.W, w.skin_aabb, w.hash_aabb, table, res, params, w.widths, 0.5,
                              0.8, 0)
    sub = orc.occgrid_update(old, G, box, u[:, cells], B, w.W, w.skin_aabb, w.hash_aabb, table, res, params,
                             w.widths, 0.5, 0.8, 0, cells=cells)
    np.testing.assert_array_equal(sub["points"], full["points"][cells])
    np.testing.assert_array_equal(sub["values"][cells], full["values"][cells])
    rest = np.setdiff1d(np.arange(G ** 3), cells)
    np.testing.assert_array_equal(sub["values"][rest], old[rest])
