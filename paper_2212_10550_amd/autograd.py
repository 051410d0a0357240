"""PyTorch autograd front end of the deform-and-query path.

Each differentiable stage is a ``torch.autograd.Function`` whose forward
and backward are the library's HIP kernels; PyTorch only allocates the
outputs and carries the gradients between stages.

* ``snarf_deform``: canonical roots x* of the posed points (Sec. 3.1,
  Eq. 5-7, multi-init Broyden, lowest residual kept).  Its backward is the
  implicit-function-theorem gradient at the root: with J the Jacobian of
  x -> sum_i w_i(x) B_i x at x*, dL/dx' = J^{-T} dL/dx*, and the gradients
  of the bones and the skinning grid follow from the same vector; the
  Broyden iterations are not unrolled.
* ``hash_encode`` (Sec. 3.2, multiresolution hash encoding) and ``mlp``
  (Eq. 1-2): per stage, FP32 features.
* ``canonical_field``: encode and MLP fused into one Function, for the
  FP16-table / BF16-MLP form: the features stay inside, so their gradient
  stays FP32 (autograd casts a gradient to its input's dtype).  The FP32
  master table gets the gradient; the FP16 copy is only read.
* ``volume_render`` (Eq. 8, with early termination) and ``l2_loss``.
* ``march`` (Sec. 3.2-3.3): not differentiable; returns the kept samples.

Shapes follow the C interface: points [3][S] (structure of arrays), bones
[nb][3][4], skinning grid [Dz][Dy][Dx][nb], table [L][T][F], features
[L][S][F], rgb [3][S], colours [R][3].
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import lib as K

__all__ = ["DeformConfig", "HashConfig", "march", "snarf_deform", "hash_encode", "mlp", "canonical_field",
           "volume_render", "l2_loss"]


@dataclass(frozen=True)
class DeformConfig:
    skin_aabb: tuple
    hash_aabb: tuple
    max_iter: int = 10
    tol_stop: float = 1e-5
    tol_valid: float = 1e-5


@dataclass(frozen=True)
class HashConfig:
    base_res: float
    growth: float
    aabb: tuple


def _empty(*shape, dtype=torch.float32, like):
    return torch.empty(*shape, dtype=dtype, device=like.device)


def march(rays_o, rays_d, occ_bits, G, aabb, dt, n_per_ray, max_steps):
    """Kept samples of rays [R][3] through a packed occupancy grid (a host
    count: one synchronisation).  Returns xs [3][S], ray_off [R+1], ray_dt [R]."""
    R = rays_o.shape[0]
    cnt = _empty(R, dtype=torch.int32, like=rays_o)
    ray_off = _empty(R + 1, dtype=torch.int64, like=rays_o)
    ray_dt = _empty(R, like=rays_o)
    n = _empty(1, dtype=torch.int64, like=rays_o)
    ws = _empty(K.march_workspace_size(R, max_steps), dtype=torch.uint8, like=rays_o)
    K.occgrid_march(rays_o, rays_d, occ_bits, G, aabb, dt, n_per_ray, max_steps, None, None, None, 0, ray_off, cnt,
                    ray_dt, n, ws)
    S = int(n.item())
    xs = _empty(3, max(S, 1), like=rays_o)
    ts = _empty(max(S, 1), like=rays_o)
    rid = _empty(max(S, 1), dtype=torch.int32, like=rays_o)
    K.occgrid_march(rays_o, rays_d, occ_bits, G, aabb, dt, n_per_ray, max_steps, xs, ts, rid, max(S, 1), ray_off,
                    cnt, ray_dt, n, ws)
    return xs[:, :S], ray_off, ray_dt


class _Deform(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xp, B, W, cfg):
        S = xp.shape[1]
        Dz, Dy, Dx, nb = W.shape
        xc = _empty(3, S, like=xp)
        bone = _empty(S, dtype=torch.int16, like=xp)
        ws = _empty(K.deform_workspace_size(Dx, Dy, Dz), dtype=torch.uint8, like=xp)
        K.snarf_deform(xp, S, S, B, W, cfg.skin_aabb, cfg.hash_aabb, cfg.max_iter, cfg.tol_stop, cfg.tol_valid, xc,
                       bone, None, None, ws)
        ctx.save_for_backward(xc, bone, B, W)
        ctx.cfg = cfg
        ctx.mark_non_differentiable(bone)
        return xc, bone

    @staticmethod
    def backward(ctx, grad_xc, _grad_bone):
        xc, bone, B, W = ctx.saved_tensors
        S = xc.shape[1]
        Dz, Dy, Dx, nb = W.shape
        need_xp, need_B, need_W = ctx.needs_input_grad[:3]
        grad_xp = _empty(3, S, like=xc) if need_xp else None
        grad_B = _empty(*B.shape, like=B) if need_B else None
        grad_W = _empty(*W.shape, like=W) if need_W else None
        ws = _empty(K.deform_bwd_workspace_size(S, Dx, Dy, Dz, nb), dtype=torch.uint8, like=xc)
        K.snarf_deform_bwd(grad_xc.contiguous(), xc, bone, S, S, B, W, ctx.cfg.skin_aabb, grad_xp, grad_B, grad_W,
                           ws, flags=K.OVERWRITE)
        return grad_xp, grad_B, grad_W, None


def snarf_deform(xp, B, W, cfg: DeformConfig):
    """Canonical roots of posed points xp [3][S]: (x* [3][S], bone int16 [S],
    -1 where no init converged).  Differentiable in xp, B and W."""
    return _Deform.apply(xp.contiguous(), B.contiguous(), W.contiguous(), cfg)


class _Encode(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xc, bone, table, cfg):
        S = xc.shape[1]
        L, T, F = table.shape
        feat = _empty(L, S, F, like=xc)
        K.hashgrid_encode(xc, bone, S, S, table, cfg.base_res, cfg.growth, cfg.aabb, feat)
        ctx.save_for_backward(xc, bone, table)
        ctx.cfg = cfg
        return feat

    @staticmethod
    def backward(ctx, grad_feat):
        xc, bone, table = ctx.saved_tensors
        cfg = ctx.cfg
        S = xc.shape[1]
        grad_xc = _empty(3, S, like=xc) if ctx.needs_input_grad[0] else None
        grad_table = _empty(*table.shape, like=table) if ctx.needs_input_grad[2] else None
        _hash_bwd(grad_feat.contiguous(), xc, bone, S, table, cfg, grad_table, grad_xc)
        return grad_xc, None, grad_table, None


def _hash_bwd(grad_feat, xc, bone, S, table, cfg, grad_table, grad_xc):
    """Position gradient (the table is read) and table gradient: binned
    (ia355_hashgrid_table_grad) when the table's size is within its tile
    limit, FP32 atomics otherwise."""
    L, T = grad_table.shape[:2] if grad_table is not None else (table.shape[0], table.shape[1])
    binned = grad_table is not None and K.hashgrid_table_grad_workspace_size(S, L, T) > 0
    if grad_xc is not None or (grad_table is not None and not binned):
        ws = _empty(K.hashgrid_encode_bwd_workspace_size(S, L), dtype=torch.uint8, like=xc)
        K.hashgrid_encode_bwd(grad_feat, xc, bone, S, S, table, cfg.base_res, cfg.growth, cfg.aabb,
                              None if binned else grad_table, grad_xc, flags=K.OVERWRITE, ws=ws)
    if binned:
        ws = _empty(K.hashgrid_table_grad_workspace_size(S, L, T), dtype=torch.uint8, like=xc)
        K.hashgrid_table_grad(grad_feat, xc, bone, S, S, cfg.base_res, cfg.growth, cfg.aabb, grad_table, ws,
                              K.OVERWRITE)


def hash_encode(xc, bone, table, cfg: HashConfig):
    """Features [L][S][F] FP32 of canonical points xc [3][S] (zero where
    bone < 0) from an FP32 table [L][T][F]; differentiable in xc and table."""
    if table.dtype != torch.float32:
        raise TypeError("hash_encode takes an FP32 table; use canonical_field for the FP16 table")
    return _Encode.apply(xc.contiguous(), bone, table, cfg)


class _MLP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, feat, bone, params, dtype):
        S = feat.shape[1]
        sigma = _empty(S, like=feat)
        rgb = _empty(3, S, like=feat)
        K.mlp_fwd(feat, bone, S, S, params, dtype, sigma, rgb)
        ctx.save_for_backward(feat, bone, params)
        ctx.dtype = dtype
        return sigma, rgb

    @staticmethod
    def backward(ctx, grad_sigma, grad_rgb):
        feat, bone, params = ctx.saved_tensors
        S = feat.shape[1]
        grad_params = _empty(*params.shape, like=params)
        grad_feat = _empty(*feat.shape, like=feat) if ctx.needs_input_grad[0] else None
        ws = _empty(K.mlp_bwd_workspace_size(S), dtype=torch.uint8, like=feat)
        K.mlp_bwd(grad_sigma.contiguous(), grad_rgb.contiguous(), feat, bone, S, S, params, ctx.dtype, grad_params,
                  grad_feat, ws, flags=K.OVERWRITE)
        return grad_feat, None, grad_params if ctx.needs_input_grad[2] else None, None


def mlp(feat, bone, params, dtype=K.F32):
    """Density and colour (Eq. 1-2) of features [L][S][F] FP32: (sigma [S],
    rgb [3][S]); dtype K.F32 or K.BF16 (MFMA, FP32 accumulate)."""
    if feat.dtype != torch.float32:
        raise TypeError("mlp takes FP32 features; use canonical_field for BF16 features")
    return _MLP.apply(feat.contiguous(), bone, params.contiguous(), dtype)


class _Field(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xc, bone, table, params, table_read, hcfg, mlp_dtype, feat_dtype):
        S = xc.shape[1]
        L, T, F = table.shape
        feat = _empty(L, S, F, dtype=feat_dtype, like=xc)
        K.hashgrid_encode(xc, bone, S, S, table_read, hcfg.base_res, hcfg.growth, hcfg.aabb, feat)
        sigma = _empty(S, like=xc)
        rgb = _empty(3, S, like=xc)
        K.mlp_fwd(feat, bone, S, S, params, mlp_dtype, sigma, rgb)
        ctx.save_for_backward(xc, bone, table_read, params, feat)
        ctx.cfg = (hcfg, mlp_dtype, table.shape)
        return sigma, rgb

    @staticmethod
    def backward(ctx, grad_sigma, grad_rgb):
        xc, bone, table_read, params, feat = ctx.saved_tensors
        hcfg, mlp_dtype, tshape = ctx.cfg
        S = xc.shape[1]
        grad_params = _empty(*params.shape, like=params)
        grad_feat = _empty(*feat.shape, like=xc)
        ws = _empty(K.mlp_bwd_workspace_size(S), dtype=torch.uint8, like=xc)
        K.mlp_bwd(grad_sigma.contiguous(), grad_rgb.contiguous(), feat, bone, S, S, params, mlp_dtype, grad_params,
                  grad_feat, ws, flags=K.OVERWRITE)
        grad_xc = _empty(3, S, like=xc) if ctx.needs_input_grad[0] else None
        grad_table = _empty(*tshape, like=xc) if ctx.needs_input_grad[2] else None
        _hash_bwd(grad_feat, xc, bone, S, table_read, hcfg, grad_table, grad_xc)
        return (grad_xc, None, grad_table, grad_params if ctx.needs_input_grad[3] else None, None, None, None,
                None)


def canonical_field(xc, bone, table, params, cfg: HashConfig, table_f16=None, mlp_dtype=K.F32,
                    feat_dtype=torch.float32):
    """Encode + MLP in one Function: (sigma [S], rgb [3][S]).  ``table`` is
    the FP32 master [L][T][F] and gets the gradient; ``table_f16``, if
    given, is the FP16 copy the forward and the position gradient read.
    feat_dtype float32 or bfloat16 (the features are internal)."""
    read = table if table_f16 is None else table_f16
    return _Field.apply(xc.contiguous(), bone, table, params.contiguous(), read, cfg, mlp_dtype, feat_dtype)


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, rgb, ray_off, ray_dt, T_thresh):
        R = ray_dt.shape[0]
        S = sigma.shape[0]
        color = _empty(R, 3, like=sigma)
        opacity = _empty(R, like=sigma)
        n_used = _empty(R, dtype=torch.int32, like=sigma)
        T_final = _empty(R, like=sigma)
        K.volrender_fwd(sigma, rgb, S, ray_off, ray_dt, R, T_thresh, color, opacity, n_used, T_final)
        ctx.save_for_backward(sigma, rgb, ray_off, ray_dt, n_used, color, T_final)
        ctx.mark_non_differentiable(n_used)
        return color, opacity, n_used

    @staticmethod
    def backward(ctx, grad_color, grad_opacity, _grad_n):
        sigma, rgb, ray_off, ray_dt, n_used, color, T_final = ctx.saved_tensors
        S, R = sigma.shape[0], ray_dt.shape[0]
        grad_sigma = _empty(S, like=sigma)
        grad_rgb = _empty(3, S, like=sigma)
        K.volrender_bwd(grad_color.contiguous(), None if grad_opacity is None else grad_opacity.contiguous(), sigma,
                        rgb, S, ray_off, ray_dt, n_used, color, T_final, R, grad_sigma, grad_rgb)
        return grad_sigma, grad_rgb, None, None, None


def volume_render(sigma, rgb, ray_off, ray_dt, T_thresh=0.0):
    """Alpha compositing along each ray (Eq. 8), stopping once transmittance
    falls below T_thresh: (color [R][3], opacity [R], n_used [R])."""
    return _Render.apply(sigma.contiguous(), rgb.contiguous(), ray_off, ray_dt, float(T_thresh))


class _L2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, color, target):
        loss = _empty(1, like=color)
        grad = _empty(*color.shape, like=color)
        K.l2_loss(color.contiguous(), target.contiguous(), loss, grad)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_loss):
        (grad,) = ctx.saved_tensors
        return grad * grad_loss, None


def l2_loss(color, target):
    """Mean squared error over the R x 3 colour entries (the photometric
    loss of the training step)."""
    return _L2.apply(color, target)
