"""GPU parity of the backward stages and of a whole training step against the
FP64 oracle, through the C ABI.

Bar for gradients: |gpu - oracle| <= 1e-4 * max(|oracle|, 1e-3 * max|oracle|)
(summation order and atomics make per-element bits order dependent; the
floor keeps near-zero entries of a large gradient from dominating).
"""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests import bounds
from tests.gpu_util import feat_dev, feat_host, assert_mixed, dev, host, soa, up

pytestmark = pytest.mark.gpu

GTOL = 1e-4


def _K():
    from paper_2212_10550_amd import lib as K
    return K


def gclose(got, ref, what):
    ref = np.asarray(ref, np.float64)
    scale = 1e-3 * (np.abs(ref).max() if ref.size else 1.0)
    return assert_mixed(got, ref, GTOL, what, scale=max(scale, 1e-30))


def gclose_rows(got, ref, what):
    """Per-sample gradient vectors: |gpu - oracle| <= 1e-4 * ||oracle row||
    (a component that cancels to near zero inherits the row's rounding)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    rn = np.linalg.norm(ref, axis=1, keepdims=True)
    floor = 1e-3 * rn.max() if rn.size else 1.0
    err = np.abs(got - ref) / np.maximum(np.maximum(rn, floor), 1e-30)
    assert (err <= GTOL).all(), f"{what}: max row-relative error {err.max():.3e} ({(err > GTOL).sum()} elements)"
    return float(err.max())


def normclose(got, ref, tol, what):
    """Norm-wise: ||gpu - oracle||_2 <= tol * ||oracle||_2, for arrays whose
    entries are sums of per-sample terms that may cancel."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    e = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert e <= tol, f"{what}: norm-wise relative error {e:.3e} > {tol:.1e}"
    return float(e)


@pytest.mark.parametrize("thr", [0.0, 0.2])
def test_volrender_bwd(orc, thr):
    K = _K()
    rng = np.random.default_rng(1)
    cnt = rng.integers(0, 70, 999)
    cnt[:3] = [0, 1, 128]
    off = np.r_[0, np.cumsum(cnt)].astype(np.int64)
    S, R = int(off[-1]), len(cnt)
    sig = rng.uniform(0, 40, S).astype(np.float32)
    rgb = rng.uniform(0, 1, (S, 3)).astype(np.float32)
    dt = rng.uniform(0.005, 0.02, R).astype(np.float32)
    gC = rng.normal(size=(R, 3)).astype(np.float32)
    gA = rng.normal(size=R).astype(np.float32)
    color, opac = torch.empty(R, 3, device=dev()), torch.empty(R, device=dev())
    n_used, Tf = torch.empty(R, dtype=torch.int32, device=dev()), torch.empty(R, device=dev())
    sig_t, rgb_t, off_t, dt_t = up(sig), soa(rgb), up(off), up(dt)
    K.volrender_fwd(sig_t, rgb_t, S, off_t, dt_t, R, thr, color, opac, n_used, Tf)
    gs, gr = torch.full((S,), 7.0, device=dev()), torch.full((3, S), 7.0, device=dev())
    K.volrender_bwd(up(gC), up(gA), sig_t, rgb_t, S, off_t, dt_t, n_used, color, Tf, R, gs, gr)
    torch.cuda.synchronize()
    fwd = orc.composite_fwd(sig, rgb, off, dt, thr)
    assert (host(n_used) == fwd["n_used"]).all()
    rs, rr = orc.composite_bwd(gC, sig, rgb, off, dt, fwd["n_used"], grad_opacity=gA)
    # per-ray scale: the gradient of a ray is bounded by |g| (delta + ...)
    assert_mixed(host(gs), rs, GTOL, "grad_sigma", scale=1e-3)
    assert_mixed(host(gr).T, rr, GTOL, "grad_rgb", scale=1e-3)


def test_l2_loss(orc):
    K = _K()
    rng = np.random.default_rng(2)
    C, T = rng.uniform(size=(8192, 3)).astype(np.float32), rng.uniform(size=(8192, 3)).astype(np.float32)
    loss, g = torch.empty(1, device=dev()), torch.empty(8192, 3, device=dev())
    K.l2_loss(up(C), up(T), loss, g)
    torch.cuda.synchronize()
    Lr, gr = orc.l2_loss(C, T)
    assert_mixed(host(loss), [Lr], 1e-5, "loss")
    assert_mixed(host(g), gr, 1e-5, "grad_color", scale=1e-6)


@pytest.mark.parametrize("S", [7, 16, 4099, 40000])
def test_mlp_bwd_f32(orc, S):
    K = _K()
    rng = np.random.default_rng(S)
    feat = rng.normal(0, 0.5, (S, 32)).astype(np.float32)
    params = synth.make_mlp(seed=3, sigma_bias=0.3).astype(np.float32)
    bone = np.where(rng.uniform(size=S) < 0.1, -1, 1).astype(np.int16)
    gsig = rng.normal(size=S).astype(np.float32)
    grgb = rng.normal(size=(S, 3)).astype(np.float32)
    ld = S + 3
    ft = feat_dev(feat, ld)
    gp = torch.full((6532,), 0.25, device=dev())  # accumulated into
    gf = torch.empty(16 * ld * 2, device=dev())
    ws = torch.empty(K.mlp_bwd_workspace_size(S), dtype=torch.uint8, device=dev())
    K.mlp_bwd(up(gsig), soa(grgb, ld), ft, up(bone), S, ld, up(params), K.F32, gp, gf, ws)
    torch.cuda.synchronize()
    rp, rf = orc.mlp_bwd(gsig, grgb, feat, params, valid=bone)
    # each weight gradient sums S random-sign per-sample terms (heavy
    # cancellation at large S): every element within 1e-4 of the sum of its
    # terms' magnitudes (the bound of any summation order), and every
    # parameter block norm-wise at 1e-4
    got = host(gp) - 0.25
    offs = [0, 2048, 2112, 6208, 6272, 6528, 6532]
    for a, b in zip(offs[:-1], offs[1:]):
        normclose(got[a:b], rp[a:b], GTOL, f"grad_params[{a}:{b}]")
    mag, _ = bounds.mlp_grad_magnitude(feat, params, gsig, grgb, bone)
    bounds.check_scaled(got, rp, mag, GTOL, "grad_params")
    gclose_rows(feat_host(gf, S, ld), rf, "grad_feat")


@pytest.mark.parametrize("log2T,tdt,overwrite,pad", [
    (14, np.float32, True, 0), (19, np.float32, False, 5), (19, np.float16, True, 0), (21, np.float16, False, 0),
    (19, np.float32, True, 3)])
def test_hash_bwd(orc, log2T, tdt, overwrite, pad):
    """Table and position gradients against the oracle.  overwrite: the table
    starts as garbage and must be replaced; otherwise it starts at 0.25 and
    the gradient is added to it.  S = 6007 leaves a ragged last block; the
    coarse levels (run aggregation) and the hashed levels (16 lanes per
    item) are both exercised; pad > 0 gives ld > S."""
    K = _K()
    S = 6007
    ld = S + pad
    x = synth.random_points(S, 41)
    table = synth.make_hash_table(16, 1 << log2T, 2, seed=6, scale=0.3).astype(tdt)
    rng = np.random.default_rng(7)
    gfeat = rng.normal(size=(S, 32)).astype(np.float32)
    bone = np.where(np.arange(S) % 11 == 5, -1, 0).astype(np.int16)
    gt = torch.full((16, 1 << log2T, 2), 7.0 if overwrite else 0.25, device=dev())
    gx = torch.full((3, ld), 3.0, device=dev())
    ws = torch.empty(K.hashgrid_encode_bwd_workspace_size(S, 16), dtype=torch.uint8, device=dev())
    K.hashgrid_encode_bwd(feat_dev(gfeat, ld), soa(x, ld), up(bone), S, ld,
                          up(table), 16.0, 1.38, (0, 0, 0, 1, 1, 1), gt, gx, K.OVERWRITE if overwrite else 0, ws=ws)
    torch.cuda.synchronize()
    rt, rx = orc.hash_encode_bwd(gfeat, x, table, orc.resolutions(16), np.array([0, 0, 0, 1, 1, 1.0]), valid=bone)
    gclose(host(gt) - (0.0 if overwrite else 0.25), rt, "grad_table")
    # the position gradient scales with N_l |theta|; FP32 weights carry ~1e-7 relative error
    gclose_rows(host(gx[:, :S]).T, rx, "grad_x")
    assert (host(gx[:, :S]).T[bone < 0] == 0).all()
    assert (host(gx[:, S:]) == 3.0).all()


@pytest.mark.parametrize("L", [6, 12])
def test_hash_bwd_level_counts(orc, L):
    """Table and position gradients for level counts other than 16 (one level
    per lane with L <= 8; XCDs 4-7 with a single level at L = 12)."""
    K = _K()
    S = 3001
    x = synth.random_points(S, 43)
    table = synth.make_hash_table(L, 1 << 16, 2, seed=9, scale=0.3).astype(np.float32)
    rng = np.random.default_rng(8)
    gfeat = rng.normal(size=(S, 2 * L)).astype(np.float32)
    bone = np.where(np.arange(S) % 9 == 4, -1, 0).astype(np.int16)
    gt = torch.full((L, 1 << 16, 2), 7.0, device=dev())
    gx = torch.full((3, S), 3.0, device=dev())
    ws = torch.empty(K.hashgrid_encode_bwd_workspace_size(S, L), dtype=torch.uint8, device=dev())
    gf = up(gfeat.reshape(S, L, 2).transpose(1, 0, 2).reshape(-1))
    K.hashgrid_encode_bwd(gf, soa(x), up(bone), S, S, up(table), 16.0, 1.38, (0, 0, 0, 1, 1, 1), gt, gx,
                          K.OVERWRITE, ws=ws)
    torch.cuda.synchronize()
    rt, rx = orc.hash_encode_bwd(gfeat, x, table, orc.resolutions(L), np.array([0, 0, 0, 1, 1, 1.0]), valid=bone)
    gclose(host(gt), rt, f"grad_table L={L}")
    gclose_rows(host(gx).T, rx, f"grad_x L={L}")
    assert (host(gx).T[bone < 0] == 0).all()


@pytest.mark.parametrize("overwrite", [False, True])
def test_hash_bwd_level_groups(orc, overwrite):
    """The coarse and the fine level groups, called separately (as two
    streams do), give the oracle's table gradient; each call leaves the other
    group's slice as it was."""
    K = _K()
    S, log2T = 5003, 19
    x = synth.random_points(S, 43)
    table = synth.make_hash_table(16, 1 << log2T, 2, seed=6, scale=0.3).astype(np.float32)
    gfeat = np.random.default_rng(9).normal(size=(S, 32)).astype(np.float32)
    res = orc.resolutions(16)
    ncoarse = int(np.sum((np.asarray(res) <= 32) & ((np.asarray(res, dtype=np.int64) + 1) ** 3 <= (1 << log2T))))
    assert 0 < ncoarse < 16
    start = 7.0 if overwrite else 0.25
    gt = torch.full((16, 1 << log2T, 2), start, device=dev())
    args = (feat_dev(gfeat, S), soa(x, S), None, S, S, up(table), 16.0, 1.38, (0, 0, 0, 1, 1, 1), gt, None)
    ow = K.OVERWRITE if overwrite else 0
    K.hashgrid_encode_bwd(*args, ow | K.TABLE_COARSE)
    torch.cuda.synchronize()
    assert (host(gt[ncoarse:]) == start).all()
    K.hashgrid_encode_bwd(*args, ow | K.TABLE_FINE)
    torch.cuda.synchronize()
    rt, _ = orc.hash_encode_bwd(gfeat, x, table, res, np.array([0, 0, 0, 1, 1, 1.0]))
    gclose(host(gt) - (0.0 if overwrite else 0.25), rt, "grad_table (two groups)")


def test_deform_bwd(orc):
    K = _K()
    w = synth.train_step()
    rng = np.random.default_rng(8)
    S = 3001
    xc = np.c_[rng.uniform(0.05, 0.95, S), rng.uniform(0.05, 0.95, S), rng.uniform(0.3, 0.7, S)].astype(np.float32)
    xc[:2] = [[0.5, 0.5, 0.2], [0.5, 0.5, 0.8]]  # outside the skinning box along z (clamped)
    u = rng.normal(size=(S, 3)).astype(np.float32)
    bone = np.where(np.arange(S) % 13 == 4, -1, 2).astype(np.int16)
    ld = S + 1
    gxp = torch.full((3, ld), 5.0, device=dev())
    gB = torch.full(w.B.shape, 0.5, device=dev())
    gW = torch.zeros(w.W.shape, device=dev())
    Dz, Dy, Dx, nb = w.W.shape
    ws = torch.empty(K.deform_bwd_workspace_size(S, Dx, Dy, Dz, nb), dtype=torch.uint8, device=dev())
    K.snarf_deform_bwd(soa(u, ld), soa(xc, ld), up(bone), S, ld, up(w.B), up(w.W), w.skin_aabb, gxp, gB, gW, ws)
    torch.cuda.synchronize()
    rxp, rB, rW = orc.deform_bwd(u, xc, bone, w.B, w.W, w.skin_aabb)
    e1 = gclose_rows(host(gxp[:, :S]).T, rxp, "grad_xp")
    e2 = gclose(host(gB) - 0.5, rB, "grad_B")
    # grad_W entries sum tri_c(x*) v . (B_b x_h) over samples and cancel when
    # v is nearly orthogonal to B_b x_h: every entry within 1e-4 of the sum
    # of its terms' magnitudes (|v| |B_b x_h| per term); the two clamped
    # samples (rows 0 and 1) and the bone and vertex indexing are covered
    mag_B, mag_W, cnt_W = bounds.deform_grad_magnitude(rxp, xc, bone, w.B, w.W, w.skin_aabb)
    # plus the absolute error of the FP32 cell fractions, which reaches a
    # corner weight whatever its size
    ef = bounds.cell_fraction_error((Dx, Dy, Dz))
    e3 = bounds.check_bound(host(gW), rW, GTOL * mag_W + ef * cnt_W + 1e-10 * GTOL * mag_W.max(), "grad_W")
    e4 = bounds.check_scaled(host(gB) - 0.5, rB, mag_B, GTOL, "grad_B (of its magnitude sum)")
    e5 = normclose(host(gW), rW, GTOL, "grad_W")
    print(f"deform bwd: grad_xp row err {e1:.2e}, grad_B err {e2:.2e} ({e4:.2e} of magnitude), "
          f"grad_W {e3:.2e} of its bound, norm-wise {e5:.2e}")


def test_train_step_subset(orc):
    """A whole training step (forward, L2 loss, every backward) on 1/8 of the
    training rays: loss, colours and every gradient against the oracle.

    The GPU root x* differs from the oracle's polished root by dx (<= 1e-5
    by the deform bar, ~2e-7 in practice); the finest hash level turns that
    into a corner-weight change of N_max dx.  Gradients that pass through the
    encoding (table, x*, x', B, W) are therefore compared norm-wise against
    1e-4 + 32 N_max dx; the stage tests and the step from the oracle's roots
    check every gradient element by element on identical inputs."""
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.ray_subset(synth.train_step(), np.arange(0, 8192, 8))
    p = Pipeline(w)
    S = p.train_step()
    torch.cuda.synchronize()
    ref = orc.train_step(w)
    assert S == ref["march"]["xs"].shape[0]
    gb = host(p.bone[:S]).astype(int)
    assert ((gb >= 0) == (ref["deform"]["bone"] >= 0)).all(), "validity differs: gradients not comparable"
    ok = gb >= 0
    dx = np.abs(p.soa(p.xc)[ok] - ref["deform"]["xc"][ok]).max()
    assert dx <= 1e-5
    # a root shift dx moves each fraction by N dx; every component of a
    # corner-weight gradient has two fraction factors, over eight corners
    # (16 N dx of the terms), and the corner sum of random-valued table
    # entries can be up to about twice smaller than the sum of its terms'
    # magnitudes: 32 N dx.  (The element-wise check of every gradient is
    # the step from the oracle's roots, test_gpu_step_parity.py.)
    tol = GTOL + 32 * orc.resolutions(16).max() * dx
    assert_mixed(host(p.color), ref["color"], 1e-5, "colour")
    assert_mixed(host(p.loss), [ref["loss"]], 1e-5, "loss")
    gclose(host(p.grad_sigma[:S]), ref["grad_sigma"], "grad_sigma")
    gclose(host(p.grad_params), ref["grad_params"], "grad_params")
    errs = {k: normclose(got, ref[k], tol, k) for k, got in [
        ("grad_table", host(p.grad_table)), ("grad_xc", p.soa(p.grad_xc)), ("grad_xp", p.soa(p.grad_xp)),
        ("grad_B", host(p.grad_B)), ("grad_W", host(p.grad_W))]}
    print(f"train subset: S={S} loss={float(p.loss.item()):.6f} root err {dx:.2e} tol {tol:.2e} "
          + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))


def test_mlp_bwd_bf16(orc):
    """BF16 MLP backward (BF16 MFMA, FP32 accumulate) against the oracle's
    BF16 storage form on the same BF16 features and FP32 master weights: the
    kernel stores the weights, hidden activations and backpropagated deltas
    as bfloat16 and takes the ReLU decisions on its FP32 pre-activations, as
    that form does, so the two differ by FP32 accumulation only, which can
    move a stored value by one bfloat16 step where it sits on a rounding
    boundary.  Bars: every element within 2^-8 of the sum of its terms'
    magnitudes (any such steps), and 1e-3 in norm per parameter block (a
    step changes one sample's term by 2^-8 of it).
    The error against the FP64 form on the rounded weights (the parameter
    rounding alone) is reported."""
    K = _K()
    S = 4099
    rng = np.random.default_rng(12)
    feat = rng.normal(0, 0.5, (S, 32)).astype(np.float32)
    params = synth.make_mlp(seed=3, sigma_bias=0.3).astype(np.float32)
    gsig = rng.normal(size=S).astype(np.float32)
    grgb = rng.normal(size=(S, 3)).astype(np.float32)
    fb = up(feat.reshape(S, 16, 2).transpose(1, 0, 2).reshape(-1), torch.bfloat16)
    gp = torch.empty(6532, device=dev())
    gf = torch.empty(16 * S * 2, device=dev())
    ws = torch.empty(K.mlp_bwd_workspace_size(S), dtype=torch.uint8, device=dev())
    K.mlp_bwd(up(gsig), soa(grgb), fb, None, S, S, up(params), K.BF16, gp, gf, ws, flags=K.OVERWRITE)
    torch.cuda.synchronize()
    feat_b = host(fb).reshape(16, S, 2).transpose(1, 0, 2).reshape(S, 32)
    got = host(gp)
    gfh = host(gf).reshape(16, S, 2).transpose(1, 0, 2).reshape(S, 32)
    rq, rfq = orc.mlp_bwd(gsig, grgb, feat_b, params, bf16=True)
    mag, mag_f = bounds.mlp_grad_magnitude(feat_b, params, gsig, grgb)
    ep = bounds.check_scaled(got, rq, mag, 2.0 ** -8, "bf16 grad_params (storage form)")
    ef = bounds.check_scaled(gfh, rfq, mag_f, 2.0 ** -8, "bf16 grad_feat (storage form)")
    offs = [0, 2048, 2112, 6208, 6272, 6528, 6532]
    errs = [normclose(got[a:b], rq[a:b], 1e-3, f"bf16 grad_params[{a}:{b}] (storage form)")
            for a, b in zip(offs[:-1], offs[1:])]
    nf = normclose(gfh, rfq, 1e-3, "bf16 grad_feat (storage form)")
    # reported: the FP64 form on the rounded weights
    params_b = host(up(params).bfloat16())
    rp, rf = orc.mlp_bwd(gsig, grgb, feat_b, params_b)
    e64 = [float(np.linalg.norm(got[a:b] - rp[a:b]) / np.linalg.norm(rp[a:b])) for a, b in zip(offs[:-1], offs[1:])]
    print(f"bf16 mlp bwd vs storage form: element max {ep:.2e} (params) {ef:.2e} (grad_feat) of the magnitude; "
          f"block norm errors {', '.join(f'{e:.1e}' for e in errs)}, grad_feat {nf:.1e}; vs FP64 on rounded "
          f"weights (norm per block): {', '.join(f'{e:.1e}' for e in e64)}")
