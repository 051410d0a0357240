"""ctypes wrapper of the FP64 oracle (``oracle.c``).  Test infrastructure only.

Each wrapper takes numpy arrays (any float dtype; they are promoted to
float64, which is exact for the float32/float16 storage values) and returns
float64 numpy arrays.  ``forward`` and ``train_step`` chain the stages in the
order of Fig. 2 of the paper: march -> deform -> encode -> MLP -> composite.
"""
from __future__ import annotations

import ctypes
import functools

import numpy as np

from .build import ensure_built

_d = ctypes.POINTER(ctypes.c_double)
_f = ctypes.POINTER(ctypes.c_float)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double


@functools.lru_cache(maxsize=None)
def lib():
    L = ctypes.CDLL(ensure_built())
    L.oracle_num_threads.restype = _I32
    L.oracle_num_threads.argtypes = []
    L.oracle_set_num_threads.restype = None
    L.oracle_set_num_threads.argtypes = [_I32]
    L.oracle_march.restype = _I64
    L.oracle_march.argtypes = [_f, _f, _I64, _u8, _I32, _f, ctypes.c_float, _I32, _I32,
                               _d, _d, _i64, _I64, _i64, _i32, _d]
    L.oracle_skin_weights.restype = None
    L.oracle_skin_weights.argtypes = [_d, _I32, _I32, _I32, _I32, _d, _d, _I64, _d, _d]
    L.oracle_lbs.restype = None
    L.oracle_lbs.argtypes = [_d, _I32, _d, _I32, _I32, _I32, _d, _d, _I64, _d]
    L.oracle_deform.restype = None
    L.oracle_deform.argtypes = [_d, _I64, _d, _I32, _d, _I32, _I32, _I32, _d, _d, _I32, _D, _D,
                                _d, _i32, _d, _d, _d, _i32, _i32, _d]
    L.oracle_deform_bwd.restype = None
    L.oracle_deform_bwd.argtypes = [_d, _d, _i32, _I64, _d, _I32, _d, _I32, _I32, _I32, _d, _d, _d, _d]
    L.oracle_hash_resolutions.restype = None
    L.oracle_hash_resolutions.argtypes = [_I32, _D, _D, _i32]
    L.oracle_hash_encode.restype = None
    L.oracle_hash_encode.argtypes = [_d, _i32, _I64, _d, _I32, _I32, _I64, _i32, _d, _d]
    L.oracle_hash_encode_bwd.restype = None
    L.oracle_hash_encode_bwd.argtypes = [_d, _d, _i32, _I64, _d, _I32, _I32, _I64, _i32, _d, _d, _d]
    L.oracle_mlp_fwd.restype = None
    L.oracle_mlp_fwd.argtypes = [_d, _i32, _I64, _d, _i32, _I32, _I32, _d, _d]
    L.oracle_mlp_bwd.restype = None
    L.oracle_mlp_bwd.argtypes = [_d, _d, _d, _i32, _I64, _d, _i32, _I32, _I32, _d, _d]
    L.oracle_composite_fwd.restype = None
    L.oracle_composite_fwd.argtypes = [_d, _d, _i64, _d, _I64, _D, _d, _d, _i32, _d]
    L.oracle_composite_bwd.restype = None
    L.oracle_composite_bwd.argtypes = [_d, _d, _d, _d, _i64, _d, _i32, _I64, _d, _d]
    L.oracle_rootinit_fwd.restype = None
    L.oracle_rootinit_fwd.argtypes = [_d, _I64, _d, _I32, _d, _I32, _d, _i32, _d]
    L.oracle_deform_guided.restype = None
    L.oracle_deform_guided.argtypes = [_d, _I64, _d, _i32, _d, _I32, _d, _I32, _I32, _I32, _d, _d, _I32, _D, _D,
                                       _d, _i32, _i32, _i32]
    L.oracle_l2_loss.restype = _D
    L.oracle_l2_loss.argtypes = [_d, _d, _I64, _d]
    return L


def num_threads():
    return int(lib().oracle_num_threads())


def set_num_threads(n):
    lib().oracle_set_num_threads(int(n))


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _c(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


# ---------------------------------------------------------------- march
def march(rays_o, rays_d, occ, aabb, dt=0.0, n_per_ray=0, max_steps=128):
    """Sec. 3.2-3.3: uniform midpoint samples along each ray inside the
    occupancy box, keeping those in occupied cells (FP32 decisions)."""
    ro = _c(rays_o, np.float32)
    rd = _c(rays_d, np.float32)
    R = ro.shape[0]
    occ_p = None
    G = 0
    if occ is not None:
        occ = _c(occ, np.uint8)
        G = occ.shape[0]
        occ_p = _p(occ, _u8)
    box = _c(aabb, np.float32)
    ray_off = np.zeros(R + 1, np.int64)
    ray_cnt = np.zeros(R, np.int32)
    ray_dt = np.zeros(R, np.float64)
    z = np.zeros(1)
    zi = np.zeros(1, np.int64)
    total = lib().oracle_march(_p(ro, _f), _p(rd, _f), R, occ_p, G, _p(box, _f), float(dt), n_per_ray,
                               max_steps, _p(z, _d), _p(z, _d), _p(zi, _i64), 0,
                               _p(ray_off, _i64), _p(ray_cnt, _i32), _p(ray_dt, _d))
    xs = np.zeros((total, 3))
    ts = np.zeros(total)
    rid = np.zeros(total, np.int64)
    lib().oracle_march(_p(ro, _f), _p(rd, _f), R, occ_p, G, _p(box, _f), float(dt), n_per_ray,
                       max_steps, _p(xs, _d), _p(ts, _d), _p(rid, _i64), total,
                       _p(ray_off, _i64), _p(ray_cnt, _i32), _p(ray_dt, _d))
    return dict(xs=xs, ts=ts, ray_id=rid, ray_off=ray_off, ray_cnt=ray_cnt, ray_dt=ray_dt)


# ------------------------------------------------------- skinning / LBS
def skin_weights(W, skin_aabb, x, grad=False):
    W = _f64(W)
    Dz, Dy, Dx, nb = W.shape
    x = _f64(x).reshape(-1, 3)
    n = x.shape[0]
    w = np.zeros((n, nb))
    dw = np.zeros((n, nb, 3)) if grad else None
    box = _f64(skin_aabb)
    lib().oracle_skin_weights(_p(W, _d), Dx, Dy, Dz, nb, _p(box, _d), _p(x, _d), n, _p(w, _d), _p(dw, _d))
    return (w, dw) if grad else w


def lbs(B, W, skin_aabb, x):
    """Eq. (7): posed position of canonical points x."""
    W = _f64(W)
    Dz, Dy, Dx, nb = W.shape
    B = _f64(B)
    x = _f64(x).reshape(-1, 3)
    out = np.zeros_like(x)
    lib().oracle_lbs(_p(B, _d), nb, _p(W, _d), Dx, Dy, Dz, _p(_f64(skin_aabb), _d), _p(x, _d), x.shape[0],
                     _p(out, _d))
    return out


def deform(xp, B, W, skin_aabb, hash_aabb, max_iter=10, tol_stop=1e-6, tol_valid=1e-5, details=False):
    """Sec. 3.1: canonical correspondences x* of posed points by multi-init
    Broyden root finding.  Returns dict(xc, bone, resid[, init_x, init_r,
    init_it, n_roots, roots])."""
    W = _f64(W)
    Dz, Dy, Dx, nb = W.shape
    B = _f64(B)
    xp = _f64(xp).reshape(-1, 3)
    S = xp.shape[0]
    out = dict(xc=np.zeros((S, 3)), bone=np.zeros(S, np.int32), resid=np.zeros(S))
    if details:
        out.update(init_x=np.zeros((S, nb, 3)), init_r=np.zeros((S, nb)), init_it=np.zeros((S, nb), np.int32),
                   n_roots=np.zeros(S, np.int32), roots=np.zeros((S, nb, 3)))
    g = out.get
    lib().oracle_deform(_p(xp, _d), S, _p(B, _d), nb, _p(W, _d), Dx, Dy, Dz, _p(_f64(skin_aabb), _d),
                        _p(_f64(hash_aabb), _d), max_iter, tol_stop, tol_valid,
                        _p(out["xc"], _d), _p(out["bone"], _i32), _p(out["resid"], _d),
                        _p(g("init_x"), _d), _p(g("init_r"), _d), _p(g("init_it"), _i32),
                        _p(g("n_roots"), _i32), _p(g("roots"), _d))
    return out


def deform_bwd(grad_xc, xc, bone, B, W, skin_aabb):
    """Implicit-function-theorem backward through the root finder."""
    W = _f64(W)
    Dz, Dy, Dx, nb = W.shape
    B = _f64(B)
    xc = _f64(xc).reshape(-1, 3)
    S = xc.shape[0]
    gxp = np.zeros((S, 3))
    gB = np.zeros(B.shape)
    gW = np.zeros(W.shape)
    lib().oracle_deform_bwd(_p(_f64(grad_xc), _d), _p(xc, _d), _p(_c(bone, np.int32), _i32), S, _p(B, _d), nb,
                            _p(W, _d), Dx, Dy, Dz, _p(_f64(skin_aabb), _d), _p(gxp, _d), _p(gB, _d), _p(gW, _d))
    return gxp, gB, gW


# ----------------------------------------------------------- hash grid
def resolutions(L, base=16.0, growth=1.38):
    res = np.zeros(L, np.int32)
    lib().oracle_hash_resolutions(L, base, growth, _p(res, _i32))
    return res


def hash_encode(x, table, res, aabb, valid=None):
    table = _f64(table)
    L, T, F = table.shape
    x = _f64(x).reshape(-1, 3)
    S = x.shape[0]
    feat = np.zeros((S, L * F))
    v = None if valid is None else _c(valid, np.int32)
    lib().oracle_hash_encode(_p(x, _d), _p(v, _i32), S, _p(table, _d), L, F, T, _p(_c(res, np.int32), _i32),
                             _p(_f64(aabb), _d), _p(feat, _d))
    return feat


def hash_encode_bwd(grad_feat, x, table, res, aabb, valid=None):
    table = _f64(table)
    L, T, F = table.shape
    x = _f64(x).reshape(-1, 3)
    S = x.shape[0]
    gt = np.zeros(table.shape)
    gx = np.zeros((S, 3))
    v = None if valid is None else _c(valid, np.int32)
    lib().oracle_hash_encode_bwd(_p(_f64(grad_feat), _d), _p(x, _d), _p(v, _i32), S, _p(table, _d), L, F, T,
                                 _p(_c(res, np.int32), _i32), _p(_f64(aabb), _d), _p(gt, _d), _p(gx, _d))
    return gt, gx


# ----------------------------------------------------------------- MLP
def mlp_fwd(feat, params, widths=(32, 64, 64, 4), valid=None, bf16=False):
    """Eq. 1-2 decoder.  bf16: the BF16 storage form (features, hidden
    activations and weight matrices rounded to bfloat16, FP64 sums; the ReLU
    decisions taken on those values)."""
    feat = _f64(feat)
    S = feat.shape[0]
    sigma = np.zeros(S)
    rgb = np.zeros((S, 3))
    v = None if valid is None else _c(valid, np.int32)
    w = np.asarray(widths, np.int32)
    lib().oracle_mlp_fwd(_p(feat, _d), _p(v, _i32), S, _p(_f64(params), _d), _p(w, _i32), len(widths) - 1,
                         int(bool(bf16)), _p(sigma, _d), _p(rgb, _d))
    return sigma, rgb


def mlp_bwd(grad_sigma, grad_rgb, feat, params, widths=(32, 64, 64, 4), valid=None, bf16=False):
    """Backward of mlp_fwd (same bf16 form; the deltas are also stored as
    bfloat16 where they multiply, the bias gradients sum them unrounded)."""
    feat = _f64(feat)
    S = feat.shape[0]
    params = _f64(params)
    gp = np.zeros(params.shape)
    gf = np.zeros(feat.shape)
    v = None if valid is None else _c(valid, np.int32)
    w = np.asarray(widths, np.int32)
    lib().oracle_mlp_bwd(_p(_f64(grad_sigma), _d), _p(_f64(grad_rgb), _d), _p(feat, _d), _p(v, _i32), S,
                         _p(params, _d), _p(w, _i32), len(widths) - 1, int(bool(bf16)), _p(gp, _d), _p(gf, _d))
    return gp, gf


# ----------------------------------------------------------- composite
def composite_fwd(sigma, rgb, ray_off, ray_dt, T_thresh=0.0):
    ray_off = _c(ray_off, np.int64)
    R = ray_off.shape[0] - 1
    color = np.zeros((R, 3))
    opac = np.zeros(R)
    n_used = np.zeros(R, np.int32)
    Tf = np.zeros(R)
    lib().oracle_composite_fwd(_p(_f64(sigma), _d), _p(_f64(rgb), _d), _p(ray_off, _i64), _p(_f64(ray_dt), _d),
                               R, float(T_thresh), _p(color, _d), _p(opac, _d), _p(n_used, _i32), _p(Tf, _d))
    return dict(color=color, opacity=opac, n_used=n_used, T_final=Tf)


def composite_bwd(grad_color, sigma, rgb, ray_off, ray_dt, n_used, grad_opacity=None):
    ray_off = _c(ray_off, np.int64)
    R = ray_off.shape[0] - 1
    S = int(ray_off[-1])
    gs = np.zeros(S)
    gr = np.zeros((S, 3))
    go = None if grad_opacity is None else _f64(grad_opacity)
    lib().oracle_composite_bwd(_p(_f64(grad_color), _d), _p(go, _d), _p(_f64(sigma), _d), _p(_f64(rgb), _d),
                               _p(ray_off, _i64), _p(_f64(ray_dt), _d), _p(_c(n_used, np.int32), _i32), R,
                               _p(gs, _d), _p(gr, _d))
    return gs, gr


def l2_loss(color, target):
    color = _f64(color)
    g = np.zeros(color.shape)
    Lv = lib().oracle_l2_loss(_p(color, _d), _p(_f64(target), _d), color.shape[0], _p(g, _d))
    return Lv, g


# ------------------------------------------------ learned root initialiser
def rootinit_fwd(xp, pose, params, B, hidden=64):
    """Predicted bone and start point x0 = B_k^{-1} x' + offset per posed point."""
    xp = _f64(xp).reshape(-1, 3)
    pose = _f64(pose).reshape(-1)
    B = _f64(B)
    nb = B.shape[0]
    S = xp.shape[0]
    bone = np.zeros(S, np.int32)
    x0 = np.zeros((S, 3))
    lib().oracle_rootinit_fwd(_p(xp, _d), S, _p(pose, _d), nb, _p(_f64(params), _d), hidden, _p(B, _d),
                              _p(bone, _i32), _p(x0, _d))
    return bone, x0


def deform_guided(xp, x0, guide_bone, B, W, skin_aabb, hash_aabb, max_iter=10, tol_stop=1e-6, tol_valid=1e-5):
    """One Broyden solve from x0, falling back to the multi-init solve."""
    W = _f64(W)
    Dz, Dy, Dx, nb = W.shape
    B = _f64(B)
    xp = _f64(xp).reshape(-1, 3)
    S = xp.shape[0]
    out = dict(xc=np.zeros((S, 3)), bone=np.zeros(S, np.int32), steps=np.zeros(S, np.int32),
               fallback=np.zeros(S, np.int32))
    lib().oracle_deform_guided(_p(xp, _d), S, _p(_f64(x0), _d), _p(_c(guide_bone, np.int32), _i32), _p(B, _d), nb,
                               _p(W, _d), Dx, Dy, Dz, _p(_f64(skin_aabb), _d), _p(_f64(hash_aabb), _d), max_iter,
                               tol_stop, tol_valid, _p(out["xc"], _d), _p(out["bone"], _i32), _p(out["steps"], _i32),
                               _p(out["fallback"], _i32))
    return out


# ------------------------------------------------------- whole chain
def forward(w, details=False, table=None, params=None, roots=None, mlp_bf16=False):
    """Fig. 2 order on a synth.Workload: march, deform, encode, MLP, composite.
    ``table`` / ``params`` override the workload's (e.g. FP16/BF16-rounded copies).
    ``roots`` = (xc [S,3], bone [S]) replaces the deform stage's output (the
    root finding of Sec. 3.1 is skipped and every later stage starts from
    these canonical points), so that a checked implementation and this
    chain can be run from one set of points.  ``mlp_bf16``: the decoder in
    its BF16 storage form (``mlp_fwd(bf16=True)``)."""
    m = march(w.rays_o, w.rays_d, w.occ, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps)
    if roots is None:
        d = deform(m["xs"], w.B, w.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop, w.tol_valid, details=details)
    else:
        xc, bone = _f64(roots[0]).reshape(-1, 3), np.asarray(roots[1]).astype(np.int32)
        if xc.shape[0] != m["xs"].shape[0] or bone.shape != (xc.shape[0],):
            raise ValueError("roots must hold one point and one bone per marched sample")
        d = dict(xc=xc, bone=bone)
    res = resolutions(w.L, w.base_res, w.growth)
    tab = w.table if table is None else table
    prm = w.mlp if params is None else params
    feat = hash_encode(d["xc"], tab, res, w.hash_aabb, valid=d["bone"])
    sigma, rgb = mlp_fwd(feat, prm, w.widths, valid=d["bone"], bf16=mlp_bf16)
    c = composite_fwd(sigma, rgb, m["ray_off"], m["ray_dt"], w.T_thresh)
    return dict(march=m, deform=d, res=res, feat=feat, sigma=sigma, rgb=rgb, **c)


def train_step(w, table=None, params=None, roots=None, mlp_bf16=False):
    """Forward, L2 loss against w.target, and every backward pass:
    composite -> MLP -> hash encode (table and x*) -> deform (x', B, W).
    ``table``, ``params``, ``roots`` and ``mlp_bf16`` as in ``forward``; the
    backward uses the same table and MLP values and form as the forward."""
    f = forward(w, table=table, params=params, roots=roots, mlp_bf16=mlp_bf16)
    tab = w.table if table is None else table
    prm = w.mlp if params is None else params
    loss, gC = l2_loss(f["color"], w.target)
    gs, gr = composite_bwd(gC, f["sigma"], f["rgb"], f["march"]["ray_off"], f["march"]["ray_dt"], f["n_used"])
    gp, gfeat = mlp_bwd(gs, gr, f["feat"], prm, w.widths, valid=f["deform"]["bone"], bf16=mlp_bf16)
    gt, gx = hash_encode_bwd(gfeat, f["deform"]["xc"], tab, f["res"], w.hash_aabb, valid=f["deform"]["bone"])
    gxp, gB, gW = deform_bwd(gx, f["deform"]["xc"], f["deform"]["bone"], w.B, w.W, w.skin_aabb)
    f.update(loss=loss, grad_color=gC, grad_sigma=gs, grad_rgb=gr, grad_params=gp, grad_feat=gfeat,
             grad_table=gt, grad_xc=gx, grad_xp=gxp, grad_B=gB, grad_W=gW)
    return f


# ------------------------------------------- inference occupancy grid
def lattice_points(G, aabb):
    """Sample points of the posed-space occupancy grid (Sec. 3.3, inference):
    the centres of the G^3 cells of ``aabb``, point n = x + G (y + G z) at
    lo + ((i + 1/2) / G) * (hi - lo) per axis, every operation rounded to
    IEEE single (the grid decides integers, so both sides use one precision).
    Returns [G^3, 3] float32."""
    lo = np.asarray(aabb[:3], np.float32)
    ext = np.asarray(aabb[3:], np.float32) - lo
    u = ((np.arange(G, dtype=np.float32) + np.float32(0.5)) / np.float32(G)).astype(np.float32)
    ax = [(lo[a] + u * ext[a]).astype(np.float32) for a in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float32)


def dilate(occ, r):
    """Occupied cells grown by r cells in every direction (a (2r+1)^3 box,
    clipped at the grid boundary): out[c] = any occ[c'] with
    max_a |c_a - c'_a| <= r.  occ: bool [G][G][G]."""
    occ = np.asarray(occ, bool)
    out = np.zeros_like(occ)
    G = occ.shape
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                src = occ[max(dz, 0):G[0] + min(dz, 0), max(dy, 0):G[1] + min(dy, 0), max(dx, 0):G[2] + min(dx, 0)]
                out[max(-dz, 0):G[0] + min(-dz, 0), max(-dy, 0):G[1] + min(-dy, 0), max(-dx, 0):G[2] + min(-dx, 0)] |= src
    return out


def occgrid_build(G, aabb, B, W, skin_aabb, hash_aabb, table, res, params, widths, sigma_thresh, r, max_iter=10,
                  tol_stop=1e-6, tol_valid=1e-5):
    """Per-pose occupancy grid for rendering (Sec. 3.3, inference): the
    lattice points are mapped to canonical space (the multi-init root of
    Sec. 3.1, no root -> density 0), their density is queried (hash encoding
    and MLP, Eq. 1-2), thresholded (sigma > sigma_thresh) and the occupied
    region is dilated by r cells.  Returns points, deform, sigma [G^3], occ
    and the dilated grid, both bool [G][G][G] (z, y, x)."""
    pts = lattice_points(G, aabb)
    d = deform(pts, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid)
    feat = hash_encode(d["xc"], table, res, hash_aabb, valid=d["bone"])
    sigma, _ = mlp_fwd(feat, params, widths, valid=d["bone"])
    occ = (sigma > sigma_thresh).reshape(G, G, G)
    return dict(points=pts, deform=d, sigma=sigma, occ=occ, grid=dilate(occ, r))


# ------------------------------------------- training occupancy grid
def jittered_points(G, aabb, u, cells=None):
    """One point per cell of the G^3 grid of ``aabb`` at a random position
    inside it (Sec. 3.3, training stage: the densities are taken at random
    points): for cell c = x + G (y + G z), lo + ((i + u) / G) * (hi - lo) per
    axis with u [3][M] in [0, 1) supplied by the caller, every operation in
    IEEE single.  ``cells`` [M] lists the cells (default: all G^3 in order).
    Returns [M, 3] float32."""
    lo = np.asarray(aabb[:3], np.float32)
    ext = np.asarray(aabb[3:], np.float32) - lo
    c = np.arange(G ** 3) if cells is None else np.asarray(cells, np.int64)
    M = len(c)
    u = np.asarray(u, np.float32).reshape(3, M)
    idx = [c % G, (c // G) % G, c // (G * G)]
    out = np.empty((M, 3), np.float32)
    g = np.float32(G)
    for a in range(3):
        out[:, a] = lo[a] + ((idx[a].astype(np.float32) + u[a]) / g) * ext[a]
    return out


def occgrid_update(values, G, aabb, u, B, W, skin_aabb, hash_aabb, table, res, params, widths, beta, sigma_thresh,
                   r, max_iter=10, tol_stop=1e-6, tol_valid=1e-5, cells=None):
    """One update of the shared training occupancy grid (Sec. 3.3, training
    stage): densities of one random point in each listed cell (default all;
    distinct cells) in the posed space of the given frame (no root -> 0), a
    moving average with those cells' current values, v <- beta v +
    (1 - beta) sigma (other cells keep theirs), then the threshold and
    dilation of the inference grid.  values: [G^3] float64 (new array
    returned)."""
    pts = jittered_points(G, aabb, u, cells)
    d = deform(pts, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid)
    feat = hash_encode(d["xc"], table, res, hash_aabb, valid=d["bone"])
    sigma, _ = mlp_fwd(feat, params, widths, valid=d["bone"])
    v = np.array(values, np.float64)
    c = np.arange(G ** 3) if cells is None else np.asarray(cells, np.int64)
    v[c] = beta * v[c] + (1.0 - beta) * sigma
    occ = (v > sigma_thresh).reshape(G, G, G)
    return dict(points=pts, deform=d, sigma=sigma, values=v, grid=dilate(occ, r))


def point_cells(x, aabb, G):
    """Cell (x, y, z) of each point of [n, 3] in the G^3 grid of ``aabb``:
    floor((x - lo) / (hi - lo) * G) clamped to [0, G - 1], every operation in
    IEEE single (the march's keep test)."""
    x = np.asarray(x, np.float32)
    lo = np.asarray(aabb[:3], np.float32)
    ext = np.asarray(aabb[3:], np.float32) - lo
    u = ((x - lo) / ext).astype(np.float32) * np.float32(G)
    return np.clip(np.floor(u).astype(np.int64), 0, G - 1)


def density_reg(x, sigma, grid, aabb, lam):
    """Occupancy-based density regulariser (Sec. 3.4, L_density): the mean
    over the n points of lam * |sigma| for points in empty cells of the
    occupancy grid (bool [G][G][G], z-major), 0 elsewhere.  Returns the
    loss and dL/dsigma."""
    sigma = np.asarray(sigma, np.float64)
    n = len(sigma)
    G = grid.shape[0]
    c = point_cells(x, aabb, G)
    empty = ~grid[c[:, 2], c[:, 1], c[:, 0]]
    loss = lam * np.sum(np.abs(sigma) * empty) / n
    grad = lam * np.sign(sigma) * empty / n
    return loss, grad


# ------------------------------------------------------ full loss set
def huber(r, delta):
    """Huber function rho of a non-negative residual norm."""
    r = np.asarray(r, np.float64)
    return np.where(r <= delta, 0.5 * r * r, delta * (r - 0.5 * delta))


def hard_surface(a):
    """Hard-surface term of Sec. 3.4: -log(exp(-|a|) + exp(-|a - 1|)) plus
    the constant log(1 + exp(-1)) that makes its minimum (at a = 0 and a = 1)
    zero."""
    a = np.asarray(a, np.float64)
    return -np.log(np.exp(-np.abs(a)) + np.exp(-np.abs(a - 1.0))) + np.log(1.0 + np.exp(-1.0))


def loss_full(color, opacity, target, alpha_gt, delta, lam_alpha, lam_hard):
    """Training loss of Sec. 3.4 averaged over the R rays: Huber of the colour
    error norm (L_rgb), lam_alpha |A - A_gt| (L_alpha) and lam_hard times the
    hard-surface term of A (L_hard).  Returns (loss, dL/dcolor [R][3],
    dL/dopacity [R]); at the kinks (A = A_gt, A = 0, A = 1) the gradient
    formula takes sign(0) = 0."""
    C = np.asarray(color, np.float64).reshape(-1, 3)
    T = np.asarray(target, np.float64).reshape(-1, 3)
    A = np.asarray(opacity, np.float64)
    Ag = np.asarray(alpha_gt, np.float64)
    R = len(A)
    e = C - T
    r = np.linalg.norm(e, axis=1)
    loss = (huber(r, delta).sum() + lam_alpha * np.abs(A - Ag).sum() + lam_hard * hard_surface(A).sum()) / R
    scale = np.where(r <= delta, 1.0, delta / np.where(r > 0, r, 1.0))
    gC = e * scale[:, None] / R
    ea, eb = np.exp(-np.abs(A)), np.exp(-np.abs(A - 1.0))
    gh = (ea * np.sign(A) + eb * np.sign(A - 1.0)) / (ea + eb)
    gA = (lam_alpha * np.sign(A - Ag) + lam_hard * gh) / R
    return loss, gC, gA


def adam_step(p, g, m, v, t, lr, beta1, beta2, eps):
    """One Adam step (Kingma and Ba), bias-corrected, step t >= 1.  Returns
    new (p, m, v) in float64."""
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------ multi-root aggregation
def max_density_roots(xs, w, table=None, params=None):
    """Multi-root aggregation (an alternative to keeping the lowest-residual
    root, Sec. 3.1): the density and colour of every distinct valid root of
    each posed point; the point takes the root with the largest density
    (first in init order among equals) and that root's colour.  A point
    without a root has density and colour 0.  Returns dict(sigma [S],
    rgb [S,3], xc [S,3] (chosen root), n_roots [S], deform)."""
    tab = w.table if table is None else table
    prm = w.mlp if params is None else params
    d = deform(xs, w.B, w.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop, w.tol_valid, details=True)
    nr = d["n_roots"]
    S = len(nr)
    own = np.repeat(np.arange(S), nr)
    flat = np.concatenate([d["roots"][n, :nr[n]] for n in range(S)]) if nr.sum() else np.zeros((0, 3))
    res = resolutions(w.L, w.base_res, w.growth)
    feat = hash_encode(flat, tab, res, w.hash_aabb)
    sig, rgb = mlp_fwd(feat, prm, w.widths)
    sigma = np.zeros(S)
    col = np.zeros((S, 3))
    xc = np.zeros((S, 3))
    start = np.concatenate([[0], np.cumsum(nr)])
    for n in range(S):
        if nr[n] == 0:
            continue
        k = start[n] + int(np.argmax(sig[start[n]:start[n + 1]]))
        sigma[n], col[n], xc[n] = sig[k], rgb[k], flat[k]
    return dict(sigma=sigma, rgb=col, xc=xc, n_roots=nr, deform=d, own=own, all_sigma=sig)


def forward_max_density(w):
    """Fig. 2 order with multi-root aggregation: march, every root, the
    largest density per sample, composite."""
    m = march(w.rays_o, w.rays_d, w.occ, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps)
    a = max_density_roots(m["xs"], w)
    c = composite_fwd(a["sigma"], a["rgb"], m["ray_off"], m["ray_dt"], w.T_thresh)
    return dict(march=m, **a, **c)
