"""Pins of the oracle's skinning field, LBS (Eq. 7) and root finding (Sec. 3.1)."""
import numpy as np
import pytest
import scipy.optimize as so

from paper_2212_10550_amd import synth
from tests import indep

BOX = np.array([0, 0, 0, 1, 1, 1], np.float64)


def _rot(axis, deg):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = np.radians(deg)
    return np.eye(3) + np.sin(t) * k + (1 - np.cos(t)) * k @ k


def _bone(R, pivot, trans=(0, 0, 0)):
    B = np.zeros((3, 4))
    B[:, :3] = R
    B[:, 3] = np.asarray(pivot) + np.asarray(trans) - R @ np.asarray(pivot)
    return B


def test_skin_weights_match_scipy(orc):
    w = synth.train_step()
    x = synth.random_points(2000, 11, lo=(-0.1, -0.1, 0.1), hi=(1.1, 1.1, 0.9))
    got = orc.skin_weights(w.W, w.skin_aabb, x)
    ref = indep.grid_interp(w.W, w.skin_aabb)(x)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(got.sum(1), 1.0, atol=2e-6)


def test_skin_gradient_matches_fd_of_scipy(orc):
    w = synth.tiny_forward()
    rng = np.random.default_rng(5)
    # points strictly inside cells (fractional coordinate in [0.1, 0.9])
    cells = rng.integers(0, 31, size=(200, 3))
    x = (cells + rng.uniform(0.1, 0.9, size=(200, 3))) / 31.0
    _, dw = orc.skin_weights(w.W, w.skin_aabb, x, grad=True)
    f = indep.grid_interp(w.W, w.skin_aabb)
    h = 1e-7
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (f(x + e) - f(x - e)) / (2 * h)
        np.testing.assert_allclose(dw[:, :, a], fd, atol=1e-6)


def test_lbs_matches_scipy_blend(orc):
    w = synth.train_step()
    x = synth.random_points(1000, 12)
    np.testing.assert_allclose(orc.lbs(w.B, w.W, w.skin_aabb, x),
                               indep.lbs_scipy(w.B, w.W, w.skin_aabb)(x), atol=1e-13)


def test_identity_pose_returns_point(orc):
    w = synth.tiny_forward()
    xp = synth.random_points(500, 3)
    d = orc.deform(xp, synth.identity_pose(), w.W, w.skin_aabb, w.hash_aabb, details=True)
    assert (d["bone"] == 0).all()
    assert (d["init_it"] == 0).all()
    np.testing.assert_allclose(d["xc"], xp.astype(np.float64), atol=1e-12)


def test_common_rigid_transform_is_one_step(orc):
    """All bones share one rigid B and the weights sum to one exactly: g is
    affine, so the first (Newton) step lands on x* = B^{-1} x'."""
    nb = 4
    rng = np.random.default_rng(1)
    lab = rng.integers(0, nb, size=(6, 6, 6))
    W = np.eye(nb)[lab]  # one-hot per vertex
    Bc = _bone(_rot([1, 2, 3], 25), [0.5, 0.5, 0.5], [0.02, -0.01, 0.03])
    B = np.repeat(Bc[None], nb, 0)
    x_true = synth.random_points(300, 4, lo=(0.1,) * 3, hi=(0.9,) * 3).astype(np.float64)
    xp = x_true @ Bc[:, :3].T + Bc[:, 3]
    d = orc.deform(xp, B, W, BOX, BOX, details=True)
    assert (d["bone"] >= 0).all()
    assert (d["init_it"] <= 1).all()
    np.testing.assert_allclose(d["xc"], x_true, atol=1e-12)
    np.testing.assert_allclose(d["init_x"][:, 0], x_true, atol=1e-12)


def test_piecewise_rigid_regions(orc):
    """One-hot weights: bone 0 on vertices with x < 0.5, bone 1 elsewhere.
    Points whose cells are entirely bone 0 (resp. 1) invert through B_0
    (resp. B_1) only -- pins the bone <-> channel <-> transform indexing."""
    D = 9
    W = np.zeros((D, D, D, 2))
    xs = np.linspace(0, 1, D)
    W[:, :, xs < 0.5, 0] = 1
    W[:, :, xs >= 0.5, 1] = 1
    B0 = _bone(_rot([0, 0, 1], 10), [0.25, 0.5, 0.5], [0.01, 0, 0])
    B1 = _bone(_rot([0, 1, 0], -12), [0.75, 0.5, 0.5], [-0.01, 0.02, 0])
    B = np.stack([B0, B1])
    rng = np.random.default_rng(2)
    x0 = np.c_[rng.uniform(0.1, 0.3, 200), rng.uniform(0.2, 0.8, 200), rng.uniform(0.2, 0.8, 200)]
    x1 = np.c_[rng.uniform(0.65, 0.85, 200), rng.uniform(0.2, 0.8, 200), rng.uniform(0.2, 0.8, 200)]
    for xt, Bk in ((x0, B0), (x1, B1)):
        xp = xt @ Bk[:, :3].T + Bk[:, 3]
        d = orc.deform(xp, B, W, BOX, BOX, details=True)
        assert (d["bone"] >= 0).all()
        assert (d["n_roots"] == 1).all()
        np.testing.assert_allclose(d["xc"], xt, atol=1e-12)


def test_round_trip_and_residual(orc):
    w = synth.train_step()
    rng = np.random.default_rng(9)
    xt = np.c_[rng.uniform(0.15, 0.85, 3000), rng.uniform(0.15, 0.85, 3000), rng.uniform(0.35, 0.65, 3000)]
    f = indep.lbs_scipy(w.B, w.W, w.skin_aabb)
    xp = f(xt)
    d = orc.deform(xp, w.B, w.W, w.skin_aabb, w.hash_aabb, details=True)
    ok = d["bone"] >= 0
    assert ok.mean() > 0.99
    # Broyden from each bone init converges in a few steps on this smooth field
    assert d["init_it"].mean() < 5
    # every accepted root solves Eq. (7) per SciPy's interpolant
    assert np.abs(f(d["xc"][ok]) - xp[ok]).max() < 1e-12
    # where the root is unique it is the point we started from
    one = ok & (d["n_roots"] == 1)
    assert one.mean() > 0.95
    np.testing.assert_allclose(d["xc"][one], xt[one], atol=1e-10)
    # every init's own Broyden residual is what it reports
    r = np.linalg.norm(f(d["init_x"].reshape(-1, 3)) - np.repeat(xp, w.B.shape[0], 0), axis=1)
    fin = np.isfinite(d["init_r"].ravel())
    np.testing.assert_allclose(d["init_r"].ravel()[fin], r[fin], rtol=1e-9, atol=1e-15)


def test_scipy_root_agrees_with_polished_root(orc):
    w = synth.tiny_forward()
    xp = synth.random_points(60, 13, lo=(0.3,) * 3, hi=(0.7,) * 3).astype(np.float64)
    d = orc.deform(xp, w.B, w.W, w.skin_aabb, w.hash_aabb)
    f = indep.lbs_scipy(w.B, w.W, w.skin_aabb)
    for n in np.nonzero(d["bone"] >= 0)[0]:
        sol = so.root(lambda x: f(x)[0] - xp[n], d["xc"][n], method="hybr", options={"xtol": 1e-14})
        assert np.abs(sol.x - d["xc"][n]).max() < 1e-10


def _brute_force_roots(f, xp, n=81):
    g = np.linspace(0, 1, n)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X, Y, Z], -1).reshape(-1, 3)
    r = np.linalg.norm(f(P) - xp, axis=1).reshape(n, n, n)
    pad = np.pad(r, 1, constant_values=np.inf)
    c = pad[1:-1, 1:-1, 1:-1]
    locmin = np.ones_like(c, bool)
    for ax in range(3):
        for s in (-1, 1):
            locmin &= c <= np.roll(pad, s, ax)[1:-1, 1:-1, 1:-1]
    cand = np.argwhere(locmin & (c < 0.05))
    roots = []
    for kz, ky, kx in cand:
        sol = so.root(lambda x: f(x)[0] - xp, np.array([g[kx], g[ky], g[kz]]), method="hybr",
                      options={"xtol": 1e-14})
        x = sol.x
        if np.linalg.norm(f(x)[0] - xp) < 1e-10 and (x >= 0).all() and (x <= 1).all():
            if not any(np.linalg.norm(x - y) < 1e-6 for y in roots):
                roots.append(x)
    return roots


@pytest.mark.slow
def test_brute_force_root_set_tiny_grid(orc):
    """4^3 x 3 bones with large rotations, so some posed points have several
    preimages.  Every distinct root the oracle reports is in the brute-force
    root set of a lattice scan refined by SciPy's root finder."""
    rng = np.random.default_rng(21)
    W = rng.dirichlet(np.ones(3) * 0.5, size=(4, 4, 4))
    B = np.stack([_bone(_rot([0, 0, 1], 70), [0.3, 0.3, 0.5]),
                  _bone(_rot([0, 0, 1], -70), [0.7, 0.7, 0.5]),
                  _bone(_rot([1, 0, 0], 40), [0.5, 0.5, 0.5], [0.05, 0, 0])])
    f = indep.lbs_scipy(B, W, BOX)
    xt = rng.uniform(0.2, 0.8, size=(12, 3))
    xp = f(xt)
    d = orc.deform(xp, B, W, BOX, BOX, max_iter=30, tol_stop=1e-10, tol_valid=1e-9, details=True)
    found = missed = multi = 0
    for n in range(len(xp)):
        bf = _brute_force_roots(f, xp[n])
        assert any(np.linalg.norm(xt[n] - y) < 1e-6 for y in bf)
        for k in range(d["n_roots"][n]):
            assert any(np.linalg.norm(d["roots"][n, k] - y) < 1e-6 for y in bf)
            found += 1
        missed += len(bf) - d["n_roots"][n]
        multi += len(bf) > 1
    assert found >= len(xp)
    assert multi >= 1  # the case really has several preimages somewhere
    print(f"oracle roots found {found}, brute-force roots missed by all inits {missed}, multi-root points {multi}")
