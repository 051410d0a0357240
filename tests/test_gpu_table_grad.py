"""GPU parity of the binned (atomic-free) hash-table gradient against the FP64
oracle and against the atomic path, through the C ABI.

Bar: the table-gradient bar of the other backward tests,
|gpu - oracle| <= 1e-4 * max(|oracle|, 1e-3 * max|oracle|); with T = 4
entries per level (thousands of terms of either sign per entry) the error
is bounded by 1e-6 of the sum of the terms' magnitudes instead.
"""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests.gpu_util import feat_dev, dev, host, soa, up
from tests.test_gpu_backward import gclose

pytestmark = pytest.mark.gpu

AABB = (0, 0, 0, 1, 1, 1)
AABB_NP = np.array([0, 0, 0, 1, 1, 1.0])


def _K():
    from paper_2212_10550_amd import lib as K
    return K


def _inputs(S, seed, log2T):
    x = synth.random_points(S, seed)
    gfeat = np.random.default_rng(seed + 1).normal(size=(S, 32)).astype(np.float32)
    bone = np.where(np.arange(S) % 11 == 5, -1, 0).astype(np.int16)
    table = np.zeros((16, 1 << log2T, 2), np.float32)  # the table gradient does not read it
    return x, gfeat, bone, table


@pytest.mark.parametrize("log2T,overwrite,pad,device_count", [
    (14, True, 0, False), (19, False, 5, False), (19, True, 0, True), (21, False, 0, True), (12, True, 3, False),
    (2, True, 0, False)])
def test_table_grad_binned(orc, log2T, overwrite, pad, device_count):
    """S = 6007 puts 48k records of level 0 in one tile (split over twelve
    accumulation workgroups that add with atomics) and leaves ragged blocks;
    T = 2^12 and 2^2 give a single tile per level; pad > 0 gives ld > S; with
    a device count the capacity exceeds the count."""
    K = _K()
    S = 6007
    x, gfeat, bone, table = _inputs(S, 51, log2T)
    cap = S + 200 if device_count else S
    ld = cap + pad
    xp = np.concatenate([x, np.full((cap - S, 3), 0.5, np.float32)])
    gp = np.concatenate([gfeat, np.ones((cap - S, 32), np.float32)])
    bp = np.concatenate([bone, np.zeros(cap - S, np.int16)])
    start = 7.0 if overwrite else 0.25
    gt = torch.full((16, 1 << log2T, 2), start, device=dev())
    ws = torch.empty(K.hashgrid_table_grad_workspace_size(cap, 16, 1 << log2T), dtype=torch.uint8, device=dev())
    Sd = torch.tensor([S], dtype=torch.int64, device=dev()) if device_count else None
    K.hashgrid_table_grad(feat_dev(gp, ld), soa(xp, ld), up(bp), cap, ld, 16.0, 1.38, AABB, gt, ws,
                          K.OVERWRITE if overwrite else 0, S_dev=Sd)
    torch.cuda.synchronize()
    rt, _ = orc.hash_encode_bwd(gfeat, x, table, orc.resolutions(16), AABB_NP, valid=bone)
    got = host(gt) - (0.0 if overwrite else start)
    if log2T > 4:
        gclose(got, rt, "grad_table (binned)")
    else:
        # ~12k terms of either sign per entry: FP32 summation error scales
        # with the sum of the terms' magnitudes (the oracle's gradient of
        # |dL/dfeat|, the weights being nonnegative), not with the result
        absum, _ = orc.hash_encode_bwd(np.abs(gfeat), x, table, orc.resolutions(16), AABB_NP, valid=bone)
        err = np.abs(got - rt) / absum
        assert err.max() <= 1e-6, f"grad_table (binned, T=4): error {err.max():.2e} of the terms' magnitude sum"


@pytest.mark.parametrize("overwrite", [False, True])
def test_table_grad_binned_level_groups(orc, overwrite):
    """Coarse and fine groups called separately (separate workspaces, as two
    streams need); each leaves the other group's slice as it was."""
    K = _K()
    S, log2T = 5003, 19
    x, gfeat, _, table = _inputs(S, 43, log2T)
    res = orc.resolutions(16)
    ncoarse = int(np.sum((np.asarray(res) <= 32) & ((np.asarray(res, dtype=np.int64) + 1) ** 3 <= (1 << log2T))))
    assert 0 < ncoarse < 16
    start = 7.0 if overwrite else 0.25
    gt = torch.full((16, 1 << log2T, 2), start, device=dev())
    nbytes = K.hashgrid_table_grad_workspace_size(S, 16, 1 << log2T)
    ws1 = torch.empty(nbytes, dtype=torch.uint8, device=dev())
    ws2 = torch.empty(nbytes, dtype=torch.uint8, device=dev())
    args = (feat_dev(gfeat, S), soa(x, S), None, S, S, 16.0, 1.38, AABB, gt)
    ow = K.OVERWRITE if overwrite else 0
    K.hashgrid_table_grad(*args, ws1, ow | K.TABLE_COARSE)
    torch.cuda.synchronize()
    assert (host(gt[ncoarse:]) == start).all()
    K.hashgrid_table_grad(*args, ws2, ow | K.TABLE_FINE)
    torch.cuda.synchronize()
    rt, _ = orc.hash_encode_bwd(gfeat, x, table, res, AABB_NP)
    gclose(host(gt) - (0.0 if overwrite else start), rt, "grad_table (binned, two groups)")


def test_table_grad_binned_vs_atomic_train_size():
    """The training step's size (8192 rays of the synthetic frame, ~36.5k
    posed samples, T = 2^19) on the pipeline's inputs: the binned and the
    atomic table gradients agree to FP32 summation-order rounding."""
    K = _K()
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.train_step()
    p = Pipeline(w, device="cuda:0")
    S = p.forward()
    p.backward()
    torch.cuda.synchronize()
    ref = torch.empty_like(p.grad_table)
    K.hashgrid_encode_bwd(p.grad_feat, p.xc, p.bone, S, p.cap, p.table, w.base_res, w.growth, w.hash_aabb, ref, None,
                          K.OVERWRITE)
    got = torch.full_like(p.grad_table, 9.0)
    L, T, _ = got.shape
    ws = torch.empty(K.hashgrid_table_grad_workspace_size(p.cap, L, T), dtype=torch.uint8, device=dev())
    K.hashgrid_table_grad(p.grad_feat, p.xc, p.bone, S, p.cap, w.base_res, w.growth, w.hash_aabb, got, ws,
                          K.OVERWRITE)
    torch.cuda.synchronize()
    r = host(ref).astype(np.float64)
    gclose(host(got), r, "grad_table binned vs atomic")
    assert ((host(got) == 0) == (r == 0)).mean() > 0.999


def test_table_grad_binned_empty():
    """No samples: an overwrite clears the slice; an add leaves it; a device
    count of 0 with a capacity behaves the same."""
    K = _K()
    log2T = 14
    gt = torch.full((16, 1 << log2T, 2), 3.0, device=dev())
    cap = 1000
    ws = torch.empty(K.hashgrid_table_grad_workspace_size(cap, 16, 1 << log2T), dtype=torch.uint8, device=dev())
    x = soa(synth.random_points(cap, 3), cap)
    gf = torch.ones(16 * cap * 2, device=dev())
    zero = torch.zeros(1, dtype=torch.int64, device=dev())
    K.hashgrid_table_grad(gf, x, None, cap, cap, 16.0, 1.38, AABB, gt, ws, 0, S_dev=zero)
    torch.cuda.synchronize()
    assert (host(gt) == 3.0).all()
    K.hashgrid_table_grad(gf, x, None, cap, cap, 16.0, 1.38, AABB, gt, ws, K.OVERWRITE | K.TABLE_FINE, S_dev=zero)
    torch.cuda.synchronize()
    g = host(gt)
    fine0 = int(np.argmax(np.any(g == 0, axis=(1, 2))))
    assert fine0 > 0 and (g[fine0:] == 0).all() and (g[:fine0] == 3.0).all()
    K.hashgrid_table_grad(gf, x, None, 0, 0, 16.0, 1.38, AABB, gt, ws, K.OVERWRITE)
    torch.cuda.synchronize()
    assert (host(gt) == 0).all()


def test_table_grad_binned_errors():
    K = _K()
    gt = torch.zeros((16, 1 << 14, 2), device=dev())
    S = 100
    x = soa(synth.random_points(S, 3), S)
    gf = torch.ones(16 * S * 2, device=dev())
    small = torch.empty(K.hashgrid_table_grad_workspace_size(S, 16, 1 << 14) - 256, dtype=torch.uint8, device=dev())
    with pytest.raises(RuntimeError):
        K.hashgrid_table_grad(gf, x, None, S, S, 16.0, 1.38, AABB, gt, small, K.OVERWRITE)
    assert K.hashgrid_table_grad_workspace_size(S, 16, 1 << 23) == 0  # more than 16384 tiles


def test_table_grad_binned_two_phase(orc):
    """A plan made from the positions alone (no gradient given), then the
    rest on that plan, gives the one-call result; a plan call writes nothing
    to the table gradient."""
    K = _K()
    S, log2T = 6007, 19
    x, gfeat, bone, table = _inputs(S, 61, log2T)
    cap = S + 100
    xp = np.concatenate([x, np.full((cap - S, 3), 0.5, np.float32)])
    gp = np.concatenate([gfeat, np.ones((cap - S, 32), np.float32)])
    bp = np.concatenate([bone, np.zeros(cap - S, np.int16)])
    Sd = torch.tensor([S], dtype=torch.int64, device=dev())
    ws = torch.empty(K.hashgrid_table_grad_workspace_size(cap, 16, 1 << log2T), dtype=torch.uint8, device=dev())
    xs, bs, gf = soa(xp, cap), up(bp), feat_dev(gp, cap)
    gt = torch.full((16, 1 << log2T, 2), 5.0, device=dev())
    K.hashgrid_table_grad(None, xs, bs, cap, cap, 16.0, 1.38, AABB, gt, ws, K.TABLE_PLAN, S_dev=Sd)
    torch.cuda.synchronize()
    assert (host(gt) == 5.0).all()
    K.hashgrid_table_grad(gf, xs, bs, cap, cap, 16.0, 1.38, AABB, gt, ws, K.OVERWRITE | K.TABLE_REUSE_PLAN, S_dev=Sd)
    one = torch.full_like(gt, 5.0)
    ws2 = torch.empty_like(ws)
    K.hashgrid_table_grad(gf, xs, bs, cap, cap, 16.0, 1.38, AABB, one, ws2, K.OVERWRITE, S_dev=Sd)
    torch.cuda.synchronize()
    rt, _ = orc.hash_encode_bwd(gfeat, x, table, orc.resolutions(16), AABB_NP, valid=bone)
    gclose(host(gt), rt, "grad_table (two-phase)")
    gclose(host(gt), host(one).astype(np.float64), "two-phase vs one call")
    with pytest.raises(RuntimeError):
        K.hashgrid_table_grad(gf, xs, bs, cap, cap, 16.0, 1.38, AABB, gt, ws, K.TABLE_PLAN | K.TABLE_REUSE_PLAN)


def test_pipeline_binned_and_atomic_steps_agree():
    """The captured training step with the binned table gradient (default)
    and with the atomic one (three-stream schedule) give the same gradients
    to summation-order rounding."""
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.train_step()
    out = {}
    for mode in ("binned", "atomic"):
        p = Pipeline(w, device="cuda:0", device_count=True, table_grad=mode)
        p.capture_train_step()
        for _ in range(2):
            p.replay()
        torch.cuda.synchronize()
        out[mode] = (host(p.grad_table).astype(np.float64), host(p.grad_params).astype(np.float64),
                     host(p.grad_B).astype(np.float64), float(p.loss.item()))
        del p
    b, a = out["binned"], out["atomic"]
    assert b[3] == a[3]  # the forward does not depend on the mode
    gclose(b[0], a[0], "grad_table binned vs atomic (step)")
    gclose(b[1], a[1], "grad_params binned vs atomic (step)")
    gclose(b[2], a[2], "grad_B binned vs atomic (step)")


def test_table_grad_binned_nonfinite(orc):
    """A NaN and an infinite feature gradient reach exactly the entries of
    their samples' corners (as FP32 adds would); every other entry matches
    the oracle at the gradient bar."""
    K = _K()
    S, log2T = 3001, 14
    x, gfeat, bone, table = _inputs(S, 71, log2T)
    gfeat[100, 2 * 9] = np.nan      # sample 100, level 9, feature 0
    gfeat[2000, 2 * 12 + 1] = np.inf  # sample 2000, level 12, feature 1
    bone[[100, 2000]] = 0
    gt = torch.full((16, 1 << log2T, 2), 7.0, device=dev())
    ws = torch.empty(K.hashgrid_table_grad_workspace_size(S, 16, 1 << log2T), dtype=torch.uint8, device=dev())
    K.hashgrid_table_grad(feat_dev(gfeat, S), soa(x, S), up(bone), S, S, 16.0, 1.38, AABB, gt, ws, K.OVERWRITE)
    torch.cuda.synchronize()
    got = host(gt).astype(np.float64)
    with np.errstate(invalid="ignore"):
        rt, _ = orc.hash_encode_bwd(gfeat, x, table, orc.resolutions(16), AABB_NP, valid=bone)
    assert np.array_equal(np.isnan(got), np.isnan(rt))
    assert np.array_equal(np.isposinf(got), np.isposinf(rt)) and np.isposinf(got).any()
    fin = np.isfinite(rt)
    clean = np.asarray(gfeat, np.float64).copy()
    clean[~np.isfinite(clean)] = 0.0
    rc, _ = orc.hash_encode_bwd(clean, x, table, orc.resolutions(16), AABB_NP, valid=bone)
    gclose(np.where(fin, got, 0.0), np.where(fin, rc, 0.0), "grad_table (finite entries)")


@pytest.mark.parametrize("small", [1e-12, 1e-17])
def test_table_grad_binned_mixed_magnitudes(orc, small):
    """One tile mixes a value near 1 and values near `small`.  The binned
    sum's own error is absolute, relative to the chunk's largest |value| m
    (here m <= 1 < 2^1): (records into the entry) * 2^-47 plus one FP32
    rounding.  Checked against the oracle on the dense levels 0-1 (where the
    FP32 corner weights are accurate to about 6 N 2^-24, N <= 22), adding
    that weight error per record, and against the FP32-atomic path on every
    level (same records; its FP32 sums round at 2^-24 per add).  With
    small = 1e-12 the small entries keep about eight significant bits; with
    1e-17 (below m 2^-48) they come out zero, where FP32 adds keep them."""
    K = _K()
    log2T = 14
    # sample 0: gradient 1 on every feature; samples 1..3: `small`; all four
    # in the coarse dense levels' first tile
    x = np.array([[0.11, 0.12, 0.13], [0.31, 0.12, 0.13], [0.11, 0.33, 0.13], [0.14, 0.15, 0.35]], np.float32)
    S = x.shape[0]
    gfeat = np.full((S, 32), small, np.float32)
    gfeat[0] = 1.0
    bone = np.zeros(S, np.int16)
    table = np.zeros((16, 1 << log2T, 2), np.float32)
    ws = torch.empty(K.hashgrid_table_grad_workspace_size(S, 16, 1 << log2T), dtype=torch.uint8, device=dev())
    gt = torch.full((16, 1 << log2T, 2), 7.0, device=dev())
    K.hashgrid_table_grad(feat_dev(gfeat, S), soa(x, S), up(bone), S, S, 16.0, 1.38, AABB, gt, ws, K.OVERWRITE)
    ga = torch.zeros((16, 1 << log2T, 2), device=dev())
    K.hashgrid_encode_bwd(feat_dev(gfeat, S), soa(x, S), up(bone), S, S, torch.zeros_like(ga), 16.0, 1.38, AABB,
                          ga, None)
    torch.cuda.synchronize()
    got = host(gt).astype(np.float64)
    atom = host(ga).astype(np.float64)
    res = orc.resolutions(16)
    ref, _ = orc.hash_encode_bwd(gfeat, x, table, res, AABB_NP, valid=bone)
    n_rec = 8 * S  # records into one entry, at most
    fixed = n_rec * 2.0 ** -47
    # against the FP32-atomic path, every level
    b_at = fixed + 2.0 ** -24 * np.abs(got) + n_rec * 2.0 ** -24 * np.abs(atom)
    e_at = np.abs(got - atom)
    i = np.unravel_index(np.argmax(e_at / b_at), e_at.shape)
    assert (e_at <= b_at).all(), f"binned vs atomic at {i}: {got[i]!r} vs {atom[i]!r}, bound {b_at[i]:.3e}"
    # against the oracle, dense levels 0-1: per record, |g| times the corner
    # weight's error (6 N 2^-24 over the three axes, plus its own rounding)
    ew = np.array([6 * 2.0 ** -24 * n + 2.0 ** -23 for n in res[:2]])[:, None, None]
    w0, _ = orc.hash_encode_bwd(np.r_[np.ones((1, 32)), np.zeros((S - 1, 32))], x, table, res, AABB_NP, valid=bone)
    g_rec = np.where(w0[:2] > 0, 8 * 1.0 + 8 * (S - 1) * small, 8 * (S - 1) * small)  # sum of |g| over its records
    b_or = g_rec * ew + fixed + 2.0 ** -24 * np.abs(ref[:2])
    e_or = np.abs(got[:2] - ref[:2])
    i = np.unravel_index(np.argmax(e_or / b_or), e_or.shape)
    assert (e_or <= b_or).all(), f"binned vs oracle at {i}: {got[:2][i]!r} vs {ref[:2][i]!r}, bound {b_or[i]:.3e}"
    # entries reached only by the small samples, in tiles that sample 0 also
    # reaches (on the dense levels each entry holds at most one corner of a
    # sample, so sample 0's largest weight in a tile is that tile's largest
    # record m, a lower bound of the chunk's)
    only_small = (w0 == 0) & (ref != 0)
    tile_of = np.arange(1 << log2T) >> 12
    m_tile = np.zeros((16, 4))
    for l in range(16):
        np.maximum.at(m_tile[l], tile_of, w0[l].max(axis=1))
    m_ent = m_tile[:, tile_of][:, :, None] * np.ones((1, 1, 2))
    shared = only_small & (m_ent > 0)
    assert shared.any()
    rel = np.abs(got[shared] - ref[shared]) / np.abs(ref[shared])
    print(f"small={small:g}: {shared.sum()} small-only entries in tiles holding values near 1, relative error "
          f"max {rel.max():.2e}, zero results {(got[shared] == 0).sum()}, atomic path zero results "
          f"{(atom[shared] == 0).sum()}")
    dense = np.zeros_like(shared)
    dense[:2] = True
    below = shared & dense & (small < m_ent * 2.0 ** -48)  # every record of the entry is below m 2^-48
    if small < 1e-15:
        assert below.any() and (got[below] == 0).all() and (atom[below] != 0).all()
