"""Error scales for element-wise gradient checks.

A gradient entry that sums per-sample terms (a weight gradient, a table or
skinning-grid entry) can cancel to far below the size of its terms, and the
rounding error of any implementation of it is bounded by the sum of the
terms' magnitudes, not by the result.  These helpers compute that sum of
magnitudes from the oracle's per-sample values, so that a test can hold each
entry to |gpu - oracle| <= tol * magnitude.  They produce tolerance scales
only, never expected values.
"""
from __future__ import annotations

import numpy as np

_MLP_OFFS = (0, 2048, 2112, 6208, 6272, 6528, 6532)  # W1 b1 W2 b2 W3 b3 (32 -> 64 -> 64 -> 4)


def _unflat(params):
    p = np.asarray(params, np.float64)
    W1 = p[0:2048].reshape(64, 32)
    b1 = p[2048:2112]
    W2 = p[2112:6208].reshape(64, 64)
    b2 = p[6208:6272]
    W3 = p[6272:6528].reshape(4, 64)
    b3 = p[6528:6532]
    return W1, b1, W2, b2, W3, b3


def mlp_grad_magnitude(feat, params, grad_sigma, grad_rgb, valid=None):
    """Sum over samples of |per-sample term| for every MLP parameter gradient
    (flat, the parameter layout), with the backpropagated deltas themselves
    replaced by magnitude bounds (|W|^T |delta|), so that cancellation inside
    a delta is covered too.  Also returns the per-sample magnitude of the
    feature gradient [S, 32]."""
    W1, b1, W2, b2, W3, b3 = _unflat(params)
    f = np.asarray(feat, np.float64)
    z1 = f @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    o = h2 @ W3.T + b3
    sig = np.exp(np.minimum(o[:, 0], 80.0))
    c = 1.0 / (1.0 + np.exp(-o[:, 1:]))
    gs = np.asarray(grad_sigma, np.float64).reshape(-1)
    gr = np.asarray(grad_rgb, np.float64).reshape(-1, 3)
    dO = np.abs(np.c_[gs * sig, gr * c * (1.0 - c)])
    if valid is not None:
        dO[np.asarray(valid) < 0] = 0.0
    d2 = (dO @ np.abs(W3)) * (z2 > 0)
    d1 = (d2 @ np.abs(W2)) * (z1 > 0)
    mag = np.concatenate([(d1.T @ np.abs(f)).ravel(), d1.sum(0), (d2.T @ h1).ravel(), d2.sum(0),
                          (dO.T @ h2).ravel(), dO.sum(0)])
    return mag, d1 @ np.abs(W1)


def _cell(x, lo, hi, D):
    """Align-corners cell of points x in a box with D vertices per axis
    (clamped): base vertex [n,3] and fractions [n,3]."""
    p = (np.clip(x, lo, hi) - lo) / (hi - lo) * (D - 1)
    i = np.clip(np.floor(p).astype(np.int64), 0, D - 2)
    return i, p - i


def deform_grad_magnitude(v, xc, bone, B, W, skin_aabb):
    """Magnitude sums for the implicit-function-theorem parameter gradients:
    grad_B[b] sums w_b(x*) v x_h^T and grad_W[c, b] sums tri_c(x*) v . (B_b x_h)
    over samples.  Each term is bounded with |v| the norm of the sample's v
    (so the error of v, relative to its norm, is covered).  Returns
    (mag_B [nb,3,4], mag_W [Dz,Dy,Dx,nb], cnt_W [Dz,Dy,Dx,nb]); cnt_W is the
    same sum with every corner weight replaced by 1: an error in a cell
    fraction is absolute (FP32 positions, about D 2^-24 of a cell), so the
    error it leaves in a corner weight is bounded by cnt_W times it, not by
    the weight."""
    W = np.asarray(W, np.float64)
    B = np.asarray(B, np.float64)
    Dz, Dy, Dx, nb = W.shape
    ok = np.asarray(bone) >= 0
    x = np.asarray(xc, np.float64).reshape(-1, 3)[ok]
    vn = np.linalg.norm(np.asarray(v, np.float64).reshape(-1, 3)[ok], axis=1)
    lo, hi = np.asarray(skin_aabb[:3], np.float64), np.asarray(skin_aabb[3:], np.float64)
    D = np.array([Dx, Dy, Dz])
    i0, f = _cell(x, lo, hi, D)
    xh = np.c_[x, np.ones(len(x))]
    Bx = np.abs(np.einsum("bij,nj->nbi", B, xh))  # [n, nb, 3]
    Bxn = np.linalg.norm(Bx, axis=2)  # [n, nb]
    mag_W = np.zeros((Dz, Dy, Dx, nb))
    cnt_W = np.zeros((Dz, Dy, Dx, nb))
    wsum = np.zeros((len(x), nb))
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                t = ((f[:, 0] if cx else 1 - f[:, 0]) * (f[:, 1] if cy else 1 - f[:, 1])
                     * (f[:, 2] if cz else 1 - f[:, 2]))
                iz, iy, ix = i0[:, 2] + cz, i0[:, 1] + cy, i0[:, 0] + cx
                np.add.at(mag_W, (iz, iy, ix), (t * vn)[:, None] * Bxn)
                np.add.at(cnt_W, (iz, iy, ix), vn[:, None] * Bxn)
                wsum += t[:, None] * W[iz, iy, ix]
    mag_B = np.einsum("nb,n,nj->bj", np.abs(wsum), vn, np.abs(xh))[:, None, :].repeat(3, axis=1)
    return mag_B, mag_W, cnt_W


def cell_fraction_error(dims):
    """Bound on the sum over the three axes of the absolute error of an FP32
    cell fraction p = (x - lo) (D - 1) / (hi - lo): three roundings of
    relative size 2^-24 on a value up to D - 1."""
    return float(sum(3 * 2.0 ** -24 * (d - 1) for d in dims))


def table_grad_magnitude(orc, feat_grad_mag, xc, table, res, aabb, valid=None):
    """Sum over samples of w_c * |feature gradient| at every table entry,
    given a non-negative per-sample magnitude of the feature gradient
    [S, L*F]: the oracle's table gradient of those values (the corner weights
    are non-negative, so nothing cancels)."""
    mag = np.asarray(feat_grad_mag, np.float64)
    assert (mag >= 0).all()
    return orc.hash_encode_bwd(mag, xc, table, res, aabb, valid=valid)[0]


def mlp_fwd_magnitude(feat_mag, params):
    """|W3| relu-magnitude(|W2| (|W1| |f| + |b1|) + |b2|) + |b3| per sample
    [S, 4]: a bound on the size of every product summed into the outputs."""
    W1, b1, W2, b2, W3, b3 = _unflat(params)
    m1 = np.asarray(feat_mag, np.float64) @ np.abs(W1).T + np.abs(b1)
    m2 = m1 @ np.abs(W2).T + np.abs(b2)
    return m2 @ np.abs(W3).T + np.abs(b3)


def feature_magnitude(orc, xc, table, res, aabb, valid=None):
    """sum_c w_c |theta_c| per feature: the encoding of the table's absolute
    values (weights are non-negative)."""
    return orc.hash_encode(xc, np.abs(np.asarray(table, np.float64)), res, aabb, valid=valid)


def check_scaled(got, ref, mag, tol, what, floor_frac=1e-6):
    """|got - ref| <= tol * max(mag, floor_frac * max(mag)) element-wise."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    mag = np.asarray(mag, np.float64)
    assert got.shape == ref.shape == mag.shape, (what, got.shape, ref.shape, mag.shape)
    floor = floor_frac * (mag.max() if mag.size else 0.0)
    scale = np.maximum(mag, max(floor, 1e-300))
    err = np.abs(got - ref) / scale
    if err.size and not (err <= tol).all():
        i = np.unravel_index(np.argmax(err), err.shape)
        raise AssertionError(f"{what}: max error {err.max():.3e} of the magnitude sum > {tol:.1e} at {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} magnitude {mag[i]!r} "
                             f"({(err > tol).sum()} of {err.size} elements)")
    return float(err.max()) if err.size else 0.0


def check_bound(got, ref, bound, what):
    """|got - ref| <= bound element-wise (bound: absolute, same shape)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    bound = np.asarray(bound, np.float64)
    assert got.shape == ref.shape == bound.shape, (what, got.shape, ref.shape, bound.shape)
    err = np.abs(got - ref) / np.maximum(bound, 1e-300)
    if err.size and not (err <= 1.0).all():
        i = np.unravel_index(np.argmax(err), err.shape)
        raise AssertionError(f"{what}: error {err.max():.3e} of its bound at {i}: got {got[i]!r} ref {ref[i]!r} "
                             f"bound {bound[i]!r} ({(err > 1).sum()} of {err.size} elements)")
    return float(err.max()) if err.size else 0.0


def error_stats(got, ref):
    """mean, p99.9 and max of |got - ref|, and max |ref| (the output's scale)."""
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64)).ravel()
    r = np.abs(np.asarray(ref, np.float64)).ravel()
    if d.size == 0:
        return dict(mean=0.0, p999=0.0, max=0.0, ref_max=0.0)
    return dict(mean=float(d.mean()), p999=float(np.quantile(d, 0.999)), max=float(d.max()),
                ref_max=float(r.max()))
