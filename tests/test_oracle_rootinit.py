"""Pins of the oracle's learned root initialiser and guided root finding."""
import numpy as np
import torch

from paper_2212_10550_amd import synth
from tests import indep


def _torch_init(xp, pose, params, B, hidden=64):
    nb = B.shape[0]
    widths = (3 + 6 * nb, hidden, hidden, nb + 3)
    x = torch.tensor(np.concatenate([xp, np.repeat(pose.reshape(1, -1), len(xp), 0)], 1), dtype=torch.float64)
    p = torch.tensor(params, dtype=torch.float64)
    o = 0
    for l in range(3):
        fi, fo = widths[l], widths[l + 1]
        Wl = p[o:o + fi * fo].view(fo, fi)
        o += fi * fo
        x = x @ Wl.T + p[o:o + fo]
        o += fo
        if l < 2:
            x = torch.relu(x)
    x = x.numpy()
    k = x[:, :nb].argmax(1)
    Bk = B[k]
    x0 = np.einsum("nij,nj->ni", np.linalg.inv(Bk[:, :, :3]), xp - Bk[:, :, 3]) + x[:, nb:]
    return k, x0


def test_rootinit_matches_torch(orc):
    w = synth.train_step()
    params = synth.make_rootinit_params(seed=4).astype(np.float32).astype(np.float64)
    params[-27:-3] += np.linspace(0, 0.5, 24)  # spread the logits' biases
    xp = synth.sample_posed_points(synth.make_skeleton(0), w.B.astype(np.float64), 500, 3).astype(np.float64)
    pose = w.pose_params.astype(np.float64)
    B = w.B.astype(np.float64)
    k, x0 = orc.rootinit_fwd(xp, pose, params, B)
    rk, rx0 = _torch_init(xp, pose, params, B)
    np.testing.assert_array_equal(k, rk)
    np.testing.assert_allclose(x0, rx0, atol=1e-12)


def test_guided_from_exact_root_takes_no_step(orc):
    w = synth.train_step()
    rng = np.random.default_rng(5)
    xt = np.c_[rng.uniform(0.15, 0.85, 400), rng.uniform(0.15, 0.85, 400), rng.uniform(0.35, 0.65, 400)]
    xp = indep.lbs_scipy(w.B, w.W, w.skin_aabb)(xt)
    d = orc.deform(xp, w.B, w.W, w.skin_aabb, w.hash_aabb)
    ok = d["bone"] >= 0
    guide = np.full(len(xp), 7, np.int32)
    g = orc.deform_guided(xp[ok], d["xc"][ok], guide[ok], w.B, w.W, w.skin_aabb, w.hash_aabb)
    assert (g["steps"] == 0).all() and (g["fallback"] == 0).all() and (g["bone"] == 7).all()
    np.testing.assert_allclose(g["xc"], d["xc"][ok], atol=1e-12)


def test_guided_fallback_equals_multi_init(orc):
    """Accepted guided roots solve Eq. 7 (SciPy residual < 1e-5, inside the
    box); rejected ones fall back to exactly the multi-init result."""
    w = synth.train_step()
    skel = synth.make_skeleton(0)
    xp = synth.sample_posed_points(skel, w.B.astype(np.float64), 600, 8).astype(np.float64)
    # two Broyden steps: far starts cannot converge, near ones can
    ref = orc.deform(xp, w.B, w.W, w.skin_aabb, w.hash_aabb, max_iter=2)
    rng = np.random.default_rng(6)
    x0 = ref["xc"] + rng.normal(0, 0.01, ref["xc"].shape)
    x0[::3] = [4.0, -3.0, 5.0]  # hopeless starts: far outside the skinning box
    guide = rng.integers(0, 24, len(xp)).astype(np.int32)
    g = orc.deform_guided(xp, x0, guide, w.B, w.W, w.skin_aabb, w.hash_aabb, max_iter=2)
    fb = g["fallback"] == 1
    assert fb.any() and (~fb).any()
    np.testing.assert_array_equal(g["bone"][fb], ref["bone"][fb])
    np.testing.assert_array_equal(g["xc"][fb], ref["xc"][fb])
    acc = ~fb
    np.testing.assert_array_equal(g["bone"][acc], guide[acc])
    f = indep.lbs_scipy(w.B, w.W, w.skin_aabb)
    assert np.abs(f(g["xc"][acc]) - xp[acc]).max() < 1e-10
    assert ((g["xc"][acc] >= 0) & (g["xc"][acc] <= 1)).all()
    print(f"fallback rate {fb.mean():.3f}")
