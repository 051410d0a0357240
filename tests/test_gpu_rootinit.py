"""GPU parity of the learned root initialiser and the guided root finding
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests import indep
from tests.gpu_util import assert_mixed, dev, host, soa, up

pytestmark = pytest.mark.gpu


def _K():
    from paper_2212_10550_amd import lib as K
    return K


def _params():
    p = synth.make_rootinit_params(seed=4).astype(np.float32)
    p[-27:-3] += np.linspace(0, 0.5, 24, dtype=np.float32)
    return p


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_rootinit_fwd(orc, dtype):
    K = _K()
    w = synth.train_step()
    skel = synth.make_skeleton(0)
    S = 3000
    xp = synth.sample_posed_points(skel, w.B.astype(np.float64), S, 3)
    params = _params()
    bone = torch.empty(S, dtype=torch.int16, device=dev())
    x0 = torch.empty(3, S + 7, device=dev())
    K.rootinit_fwd(soa(xp, S + 7), S, S + 7, up(w.pose_params.reshape(-1)), up(params), up(w.B),
                   K.F32 if dtype == "f32" else K.BF16, bone, x0)
    torch.cuda.synchronize()
    rb, rx0 = orc.rootinit_fwd(xp, w.pose_params, params, w.B)
    gb = host(bone).astype(int)
    agree = gb == rb
    gx = host(x0[:, :S]).T
    print(f"rootinit {dtype}: bone agreement {agree.mean():.4f}, x0 max err {np.abs(gx - rx0)[agree].max():.2e}")
    if dtype == "f32":
        assert agree.mean() > 0.999
        assert_mixed(gx[agree], rx0[agree], 1e-5, "x0")
    else:
        assert agree.mean() > 0.95
        assert np.abs(gx - rx0)[agree].mean() < 1e-2


def test_rootinit_bf16_unaligned_params():
    """BF16 initialiser with its parameter block at an address that is not a
    multiple of 16 bytes (the fragments are then gathered one value at a
    time instead of two 16-byte loads): outputs bit-equal to the aligned
    call's."""
    K = _K()
    w = synth.train_step()
    skel = synth.make_skeleton(0)
    S = 2001
    xp = synth.sample_posed_points(skel, w.B.astype(np.float64), S, 5)
    params = _params()
    pa = up(params)
    buf = torch.zeros(params.size + 1, device=dev())
    buf[1:] = pa
    pu = buf[1:]  # 4 bytes past a 16-byte boundary
    assert pu.data_ptr() % 16 != 0
    outs = []
    for p in (pa, pu):
        bone = torch.empty(S, dtype=torch.int16, device=dev())
        x0 = torch.empty(3, S, device=dev())
        K.rootinit_fwd(soa(xp), S, S, up(w.pose_params.reshape(-1)), p, up(w.B), K.BF16, bone, x0)
        torch.cuda.synchronize()
        outs.append((host(bone), host(x0)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1].view(np.uint32), outs[1][1].view(np.uint32))


def test_deform_guided(orc):
    K = _K()
    w = synth.train_step()
    skel = synth.make_skeleton(0)
    S = 4000
    xp = synth.sample_posed_points(skel, w.B.astype(np.float64), S, 9)
    ref = orc.deform(xp, w.B, w.W, w.skin_aabb, w.hash_aabb, max_iter=2, details=True)
    rng = np.random.default_rng(6)
    x0 = (ref["xc"] + rng.normal(0, 0.01, ref["xc"].shape)).astype(np.float32)
    x0[::3] = [4.0, -3.0, 5.0]
    guide = rng.integers(0, 24, S).astype(np.int16)
    g = orc.deform_guided(xp, x0, guide, w.B, w.W, w.skin_aabb, w.hash_aabb, max_iter=2)
    Dz, Dy, Dx, nb = w.W.shape
    xc = torch.empty(3, S, device=dev())
    bone = torch.empty(S, dtype=torch.int16, device=dev())
    steps = torch.empty(S, dtype=torch.int16, device=dev())
    nfb = torch.zeros(1, dtype=torch.int32, device=dev())
    ws = torch.empty(K.deform_guided_workspace_size(S, Dx, Dy, Dz), dtype=torch.uint8, device=dev())
    K.snarf_deform_guided(soa(xp), S, S, soa(x0), up(guide), up(w.B), up(w.W), w.skin_aabb, w.hash_aabb, 2, 1e-6,
                          1e-5, xc, bone, None, steps, nfb, ws)
    torch.cuda.synchronize()
    gb = host(bone).astype(int)
    gx = host(xc).T
    gfb = gb != guide  # accepted guided samples keep the guide's bone
    ofb = g["fallback"] == 1
    flips = (gfb != ofb) & ~((gb == guide) & ofb)  # a fallback may pick the guide's bone by chance
    assert flips.mean() < 0.01, flips.mean()
    assert int(nfb.item()) >= ofb.sum() * 0.9
    valid = gb >= 0
    f = indep.lbs_scipy(w.B, w.W, w.skin_aabb)
    assert (np.linalg.norm(f(gx[valid]) - xp[valid], axis=1) < 1e-5).all()
    # every GPU root is one of the distinct roots the full multi-init solve finds
    full = orc.deform(xp, w.B, w.W, w.skin_aabb, w.hash_aabb, details=True)
    both = valid & (full["n_roots"] > 0)
    assert both.mean() > 0.9
    dist = np.linalg.norm(full["roots"][both] - gx[both][:, None, :], axis=2)
    dist = np.where(np.arange(nb)[None, :] < full["n_roots"][both][:, None], dist, np.inf)
    k = dist.argmin(1)
    assert_mixed(gx[both], full["roots"][both][np.arange(both.sum()), k], 1e-5, "guided roots")
    print(f"guided: fallback gpu {int(nfb.item())} oracle {ofb.sum()} of {S}")


def test_learned_init_end_to_end():
    """Fit a small initialiser on solver roots of 16 poses, then guided
    solves on held-out poses: every accepted root is a valid root, and most
    samples need no fallback."""
    from paper_2212_10550_amd import rootinit
    data = rootinit.make_dataset(range(1000, 1016), 2048, device="cuda:0")
    params = rootinit.fit(data, epochs=8)
    test = rootinit.make_dataset(range(2000, 2004), 2048, device="cuda:0")
    K = _K()
    w = synth.train_step()
    fallbacks, n = 0, 0
    for p in range(4):
        sel = test["pose_index"] == p
        xp = test["xp"][sel].T.contiguous()
        S = xp.shape[1]
        gd = rootinit.GuidedDeform(params, w, S, device="cuda:0")
        xc = torch.empty(3, S, device=dev())
        bone = torch.empty(S, dtype=torch.int16, device=dev())
        W_t = up(w.W)
        gd.run(xp, S, S, test["pose"][p].contiguous(), test["B"][p].contiguous(), W_t, xc, bone, None, None)
        torch.cuda.synchronize()
        gx = host(xc).T
        B = host(test["B"][p])
        f = indep.lbs_scipy(B, w.W, w.skin_aabb)
        ok = host(bone) >= 0
        assert ok.mean() > 0.99
        assert (np.linalg.norm(f(gx[ok]) - host(xp).T[ok], axis=1) < 1e-5).all()
        fallbacks += int(gd.n_fallback.item())
        n += S
    print(f"learned init: fallback rate {fallbacks / n:.4f}")
    assert fallbacks / n < 0.5
