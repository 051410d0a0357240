"""Pins of the oracle's multi-root aggregation."""
import numpy as np

import oracle as orc
from paper_2212_10550_amd import synth


def test_single_root_points_reduce_to_the_lowest_residual_root():
    """Where every point has one root, aggregation is the paper's path."""
    w = synth.ray_subset(synth.train_step(), np.arange(0, 8192, 64))
    a = orc.forward_max_density(w)
    f = orc.forward(w)
    assert (a["n_roots"] <= 1).all()
    ok = f["deform"]["bone"] >= 0
    np.testing.assert_array_equal(a["n_roots"] == 1, ok)
    np.testing.assert_allclose(a["sigma"][ok], f["sigma"][ok], rtol=1e-12)
    np.testing.assert_allclose(a["color"], f["color"], rtol=1e-12, atol=1e-15)


def test_folded_pose_roots_and_maximum():
    """On a fold, points with two roots: each is a root of the LBS equation
    (the SciPy-pinned blend), distinct, and the chosen density is the larger
    of the two densities computed root by root."""
    w = synth.folded_frame(res=540)
    m = orc.march(w.rays_o[::97], w.rays_d[::97], w.occ, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps)
    a = orc.max_density_roots(m["xs"], w)
    multi = np.nonzero(a["n_roots"] >= 2)[0]
    assert len(multi) > 5
    res = orc.resolutions(w.L, w.base_res, w.growth)
    for n in multi[:20]:
        roots = a["deform"]["roots"][n, :a["n_roots"][n]]
        assert np.linalg.norm(roots[0] - roots[1]) > 1e-3
        for r in roots:
            xp = orc.lbs(w.B, w.W, w.skin_aabb, r[None])[0]
            assert np.abs(xp - m["xs"][n]).max() < 1e-9
        feat = orc.hash_encode(roots, w.table, res, w.hash_aabb)
        s, c = orc.mlp_fwd(feat, w.mlp, w.widths)
        k = int(np.argmax(s))
        assert a["sigma"][n] == s[k] and np.array_equal(a["rgb"][n], c[k])
