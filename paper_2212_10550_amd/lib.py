"""Thin ctypes binding of ``libia355.so`` (the C ABI in ``include/ia355.h``).

Argument marshalling only: every function takes torch tensors that already
live on the GPU, checks dtype/contiguity/device, passes raw pointers and the
current HIP stream, and raises on a non-zero status.  All arithmetic happens
in the library's HIP kernels.  There is no fallback: if the library is
missing or the tensors are not on a GPU, the call fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libia355.so")

F32, F16, BF16 = 0, 1, 2
OVERWRITE = 1  # backward flag: write gradients instead of adding to them
CAPACITY = 6  # IA355_ERR_CAPACITY
MLP_WIDTHS = (32, 64, 64, 4)  # the decoder shape the library implements
TABLE_COARSE = 2  # hash-table gradient: only the coarse dense levels
TABLE_FINE = 4  # hash-table gradient: only the other levels
TABLE_PLAN = 8  # binned table gradient: only the passes that depend on the positions
TABLE_REUSE_PLAN = 16  # binned table gradient: the rest, on a plan made before
_DT = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f = ctypes.c_float
_d = ctypes.c_double
_sz = ctypes.c_size_t
_fp = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes); names are the C entry points without "ia355_"
_SIGS = {
    "version": (_i32, []),
    "error_string": (ctypes.c_char_p, [_i32]),
    "zero": (_i32, [_vp, _sz, _vp]),
    "occ_words": (_sz, [_i32]),
    "occ_pack": (_i32, [_vp, _i32, _vp, _vp]),
    "march_workspace_size": (_sz, [_i64, _i32]),
    "snarf_deform_roots": (_i32, [_vp, _i64, _vp, _i64, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _fp, _i32, _f, _f,
                                  _i32, _f, _vp, _vp, _vp, _vp, _sz, _vp]),
    "select_max_density": (_i32, [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "loss_full": (_i32, [_vp, _vp, _vp, _vp, _i64, _f, _f, _f, _vp, _vp, _vp, _vp]),
    "adam": (_i32, [_vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _i32, _vp, _vp, _vp]),
    "count_step": (_i32, [_vp, _vp]),
    "occgrid_update": (_i32, [_i32, _fp, _vp, _vp, _i64, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _fp, _i32, _f, _f,
                              _vp, _i32,
                              _i32, _i32, _i32, _d, _d, _vp, _i32, _f, _f, _i32, _vp, _vp, _vp, _sz, _vp]),
    "density_reg_workspace_size": (_sz, [_i64]),
    "density_reg": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _i32, _fp, _f, _vp, _vp, _vp, _sz, _vp]),
    "occ_from_density": (_i32, [_vp, _i32, _f, _i32, _vp, _vp]),
    "occgrid_build_workspace_size": (_sz, [_i32, _i32, _i32, _i32, _i32, _i32, _i32]),
    "occgrid_build": (_i32, [_i32, _fp, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _fp, _i32, _f, _f, _vp, _i32, _i32,
                             _i32, _i32, _d, _d, _vp, _i32, _f, _i32, _vp, _vp, _vp, _sz, _vp]),
    "occgrid_march": (_i32, [_vp, _vp, _i64, _vp, _i32, _fp, _f, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp,
                             _vp, ctypes.POINTER(ctypes.c_int64), _vp, _sz, _vp]),
    "deform_workspace_size": (_sz, [_i32, _i32, _i32]),
    "snarf_deform": (_i32, [_vp, _i64, _vp, _i64, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _fp, _i32, _f, _f, _vp, _vp, _vp,
                            _vp, _vp, _sz, _vp]),
    "snarf_deform_noalloc": (_i32, [_vp, _i64, _vp, _i64, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _fp, _i32, _f, _f, _vp,
                                    _vp, _vp, _vp, _vp]),
    "deform_bwd_workspace_size": (_sz, [_i64, _i32, _i32, _i32, _i32]),
    "snarf_deform_bwd": (_i32, [_vp, _vp, _vp, _i64, _vp, _i64, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _vp, _vp, _vp,
                                ctypes.c_uint32, _vp, _sz, _vp]),
    "rootinit_fwd": (_i32, [_vp, _i64, _vp, _i64, _vp, _vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp]),
    "deform_guided_workspace_size": (_sz, [_i64, _i32, _i32, _i32]),
    "snarf_deform_guided": (_i32, [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _i32, _i32, _i32, _fp, _fp, _i32, _f,
                                   _f, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "hashgrid_encode": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _i32, _i32, _i32, _i32, _d, _d, _fp, _vp, _i32, _vp]),
    "hashgrid_encode_bwd_workspace_size": (_sz, [_i64, _i32]),
    "hashgrid_encode_bwd": (_i32, [_vp, _vp, _vp, _i64, _vp, _i64, _vp, _i32, _i32, _i32, _i32, _d, _d, _fp, _vp, _vp,
                                   ctypes.c_uint32, _vp, _sz, _vp]),
    "hashgrid_table_grad_workspace_size": (_sz, [_i64, _i32, _i32]),
    "hashgrid_table_grad": (_i32, [_vp, _vp, _vp, _i64, _vp, _i64, _i32, _i32, _i32, _d, _d, _fp, _vp, ctypes.c_uint32,
                                   _vp, _sz, _vp]),
    "mlp_fwd": (_i32, [_vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp, _i32, _i32, _vp, _vp, _vp]),
    "mlp_bwd_workspace_size": (_sz, [_i64]),
    "mlp_bwd": (_i32, [_vp, _vp, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _vp, _i32, _i32, _vp, _vp, ctypes.c_uint32, _vp,
                       _sz, _vp]),
    "volrender_fwd": (_i32, [_vp, _vp, _i64, _vp, _vp, _i64, _f, _vp, _vp, _vp, _vp, _vp]),
    "volrender_bwd": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "l2_loss": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "batch_workspace_size": (_sz, [_i32, _i32, _i32, _i32, _i32]),
    "batch_lds_bytes": (_sz, [_i32, _i32, _i32]),
    "batch_render": (_i32, [_vp, _sz, _i32, _i32, _i32, _i32, _vp]),
}


class BatchPose(ctypes.Structure):
    """``ia355_batch_pose`` (include/ia355.h)."""
    _fields_ = [("rays_o", _vp), ("rays_d", _vp), ("R", _i64), ("occ_bits", _vp), ("G", _i32),
                ("occ_aabb", _f * 6), ("dt", _f), ("n_per_ray", _i32), ("max_steps", _i32), ("B", _vp),
                ("pose", _vp), ("color", _vp), ("opacity", _vp), ("n_used", _vp), ("T_final", _vp),
                ("n_fallback", _vp), ("n_evaluated", _vp)]


class BatchModel(ctypes.Structure):
    """``ia355_batch_model`` (include/ia355.h)."""
    _fields_ = [("W", _vp), ("Dx", _i32), ("Dy", _i32), ("Dz", _i32), ("nb", _i32), ("skin_aabb", _f * 6),
                ("hash_aabb", _f * 6), ("max_iter", _i32), ("tol_stop", _f), ("tol_valid", _f), ("table", _vp),
                ("L", _i32), ("log2T", _i32), ("base_res", _d), ("growth", _d), ("mlp_params", _vp),
                ("init_params", _vp), ("init_hidden", _i32), ("T_thresh", _f)]


_SIGS["batch_plan"] = (_i32, [ctypes.POINTER(BatchPose), _i32, ctypes.POINTER(BatchModel), _vp, _sz, _vp])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; "
                               "g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, "ia355_" + name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _p(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    return _vp(t.data_ptr())


def _box(b):
    b = [float(v) for v in b]
    if len(b) != 6:
        raise ValueError("box must have 6 values")
    return (ctypes.c_float * 6)(*b)


def _check(status, name):
    if status != 0:
        raise RuntimeError(f"ia355_{name}: {lib().ia355_error_string(status).decode()} (status {status})")


def version():
    return lib().ia355_version()


def zero(t):
    _check(lib().ia355_zero(_p(t), t.numel() * t.element_size(), _stream()), "zero")


def occ_words(G):
    """int32 words of a packed G^3 occupancy grid."""
    return lib().ia355_occ_words(G)


def occ_pack(occ_u8, bits):
    G = occ_u8.shape[0]
    if tuple(occ_u8.shape) != (G, G, G) or bits.numel() < occ_words(G):
        raise ValueError(f"occ_pack: grid {tuple(occ_u8.shape)} / bits {bits.numel()} words "
                         f"(need a cube and {occ_words(G)} words)")
    _check(lib().ia355_occ_pack(_p(occ_u8, torch.uint8, "occ"), G, _p(bits, torch.int32, "bits"), _stream()),
           "occ_pack")


def occ_from_density(sigma, G, sigma_thresh, dilate, bits):
    if sigma.numel() < G ** 3 or bits.numel() < occ_words(G):
        raise ValueError("occ_from_density: sigma needs G^3 values and bits occ_words(G) words")
    _check(lib().ia355_occ_from_density(_p(sigma, torch.float32, "sigma"), G, float(sigma_thresh), dilate,
                                        _p(bits, torch.int32, "bits"), _stream()), "occ_from_density")


def occgrid_build_workspace_size(G, L, F, mlp_dtype, Dx, Dy, Dz):
    return lib().ia355_occgrid_build_workspace_size(G, L, F, mlp_dtype, Dx, Dy, Dz)


def occgrid_build(G, aabb, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, table, base_res, growth,
                  params, mlp_dtype, sigma_thresh, dilate, bits, sigma, ws):
    """Per-pose occupancy grid (Sec. 3.3, inference): see the C header."""
    Dz, Dy, Dx, nb = W.shape
    L, T, F = table.shape
    if bits.numel() < occ_words(G) or (sigma is not None and sigma.numel() < G ** 3):
        raise ValueError("occgrid_build: bits need occ_words(G) words, sigma G^3 values")
    _check(lib().ia355_occgrid_build(
        G, _box(aabb), _p(B, torch.float32, "B"), nb, _p(W, torch.float32, "W"), Dx, Dy, Dz, _box(skin_aabb),
        _box(hash_aabb), max_iter, tol_stop, tol_valid, _p(table, name="table"), _DT[table.dtype], L, F,
        T.bit_length() - 1, base_res, growth, _p(params, torch.float32, "params"), mlp_dtype, float(sigma_thresh),
        dilate, _p(bits, torch.int32, "bits"), _p(sigma, torch.float32, "sigma"), _p(ws, name="ws"),
        ws.numel() * ws.element_size(), _stream()), "occgrid_build")


def occgrid_update(G, aabb, jitter, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, table, base_res,
                   growth, params, mlp_dtype, beta, sigma_thresh, dilate, values, bits, ws, cells=None):
    """One update of the training occupancy grid (Sec. 3.3), of every cell or
    of the listed ones (int32 [M], distinct): see the C header."""
    Dz, Dy, Dx, nb = W.shape
    L, T, F = table.shape
    M = G ** 3 if cells is None else cells.numel()
    if jitter.numel() < 3 * M or values.numel() < G ** 3 or bits.numel() < occ_words(G):
        raise ValueError("occgrid_update: jitter [3][M], values [G^3], bits occ_words(G)")
    _check(lib().ia355_occgrid_update(
        G, _box(aabb), _p(jitter, torch.float32, "jitter"), _p(cells, torch.int32, "cells"), M,
        _p(B, torch.float32, "B"), nb, _p(W, torch.float32, "W"),
        Dx, Dy, Dz, _box(skin_aabb), _box(hash_aabb), max_iter, tol_stop, tol_valid, _p(table, name="table"),
        _DT[table.dtype], L, F, T.bit_length() - 1, base_res, growth, _p(params, torch.float32, "params"), mlp_dtype,
        float(beta), float(sigma_thresh), dilate, _p(values, torch.float32, "values"), _p(bits, torch.int32, "bits"),
        _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()), "occgrid_update")


def density_reg_workspace_size(S):
    return lib().ia355_density_reg_workspace_size(S)


def density_reg(x, sigma, S, ld, bits, G, aabb, lam, loss, grad_sigma, ws, S_dev=None):
    """Occupancy-based density regulariser (Sec. 3.4): see the C header."""
    _check(lib().ia355_density_reg(
        _p(x, torch.float32, "x"), _p(sigma, torch.float32, "sigma"), S, _p(S_dev, torch.int64, "S_dev"), ld,
        _p(bits, torch.int32, "bits"), G, _box(aabb), float(lam), _p(loss, torch.float32, "loss"),
        _p(grad_sigma, torch.float32, "grad_sigma"), _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()),
        "density_reg")


def loss_full(color, opacity, target, alpha_gt, delta, lam_alpha, lam_hard, loss, grad_color, grad_opacity):
    """Training loss of Sec. 3.4 (loss[4] = total, rgb, alpha, hard): see the C header."""
    R = color.shape[0]
    _check(lib().ia355_loss_full(
        _p(color, torch.float32, "color"), _p(opacity, torch.float32, "opacity"), _p(target, torch.float32, "target"),
        _p(alpha_gt, torch.float32, "alpha_gt"), R, float(delta), float(lam_alpha), float(lam_hard),
        _p(loss, torch.float32, "loss"), _p(grad_color, torch.float32, "grad_color"),
        _p(grad_opacity, torch.float32, "grad_opacity"), _stream()), "loss_full")


def adam(param, grad, m, v, lr, beta1=0.9, beta2=0.99, eps=1e-15, step=1, step_dev=None, param_f16=None):
    """One Adam step on flat FP32 arrays: see the C header."""
    n = param.numel()
    if grad.numel() != n or m.numel() != n or v.numel() != n or (param_f16 is not None and param_f16.numel() != n):
        raise ValueError("adam: param, grad, m, v (and param_f16) must have the same size")
    _check(lib().ia355_adam(
        _p(param, torch.float32, "param"), _p(grad, torch.float32, "grad"), _p(m, torch.float32, "m"),
        _p(v, torch.float32, "v"), n, float(lr), float(beta1), float(beta2), float(eps), int(step),
        _p(step_dev, torch.int32, "step_dev"), _p(param_f16, torch.float16, "param_f16"), _stream()), "adam")


def count_step(step_dev):
    _check(lib().ia355_count_step(_p(step_dev, torch.int32, "step_dev"), _stream()), "count_step")


def snarf_deform_roots(xp, S, ld, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, K, dup_tol, roots,
                       root_bone, n_roots, ws, S_dev=None):
    """Every distinct valid root (up to K per sample): see the C header."""
    Dz, Dy, Dx, nb = W.shape
    _check(lib().ia355_snarf_deform_roots(
        _p(xp, torch.float32, "xp"), S, _p(S_dev, torch.int64, "S_dev"), ld, _p(B, torch.float32, "B"), nb,
        _p(W, torch.float32, "W"), Dx, Dy, Dz, _box(skin_aabb), _box(hash_aabb), max_iter, tol_stop, tol_valid, K,
        float(dup_tol), _p(roots, torch.float32, "roots"), _p(root_bone, torch.int16, "root_bone"),
        _p(n_roots, torch.int32, "n_roots"), _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()),
        "snarf_deform_roots")


def select_max_density(K, S, sigma_k, rgb_k, roots, root_bone, n_roots, ld, xc, bone, sigma, rgb):
    _check(lib().ia355_select_max_density(
        K, S, _p(sigma_k, torch.float32, "sigma_k"), _p(rgb_k, torch.float32, "rgb_k"),
        _p(roots, torch.float32, "roots"), _p(root_bone, torch.int16, "root_bone"),
        _p(n_roots, torch.int32, "n_roots"), ld, _p(xc, torch.float32, "xc"), _p(bone, torch.int16, "bone"),
        _p(sigma, torch.float32, "sigma"), _p(rgb, torch.float32, "rgb"), _stream()), "select_max_density")


def march_workspace_size(R, max_steps):
    return lib().ia355_march_workspace_size(R, max_steps)


class CapacityError(RuntimeError):
    """The march kept more samples than the buffers hold (IA355_ERR_CAPACITY)."""

    def __init__(self, n_required, cap):
        super().__init__(f"ia355_occgrid_march: {n_required} samples kept, capacity {cap}")
        self.n_required = n_required
        self.cap = cap


def occgrid_march(rays_o, rays_d, occ_bits, G, aabb, dt, n_per_ray, max_steps, xs, ts, ray_id, cap, ray_off,
                  ray_cnt, ray_dt, n_samples, ws, check=False):
    """check=False: asynchronous (n_samples holds the count on the device).
    check=True: the call waits for the stream and returns the kept count,
    raising CapacityError when it exceeds cap."""
    R = rays_o.shape[0]
    req = ctypes.c_int64(-1) if check else None
    st = lib().ia355_occgrid_march(
        _p(rays_o, torch.float32, "rays_o"), _p(rays_d, torch.float32, "rays_d"), R,
        _p(occ_bits, torch.int32, "occ_bits"), G, _box(aabb), float(dt), n_per_ray, max_steps,
        _p(xs, torch.float32, "xs"), _p(ts, torch.float32, "ts"), _p(ray_id, torch.int32, "ray_id"), cap,
        _p(ray_off, torch.int64, "ray_off"), _p(ray_cnt, torch.int32, "ray_cnt"), _p(ray_dt, torch.float32, "ray_dt"),
        _p(n_samples, torch.int64, "n_samples"), None if req is None else ctypes.byref(req),
        _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream())
    if st == CAPACITY:
        raise CapacityError(req.value, cap)
    _check(st, "occgrid_march")
    return None if req is None else req.value


def deform_workspace_size(Dx, Dy, Dz):
    return lib().ia355_deform_workspace_size(Dx, Dy, Dz)


def snarf_deform(xp, S, ld, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, xc, bone, resid, steps, ws,
                 S_dev=None):
    Dz, Dy, Dx, nb = W.shape
    _check(lib().ia355_snarf_deform(
        _p(xp, torch.float32, "xp"), S, _p(S_dev, torch.int64, "S_dev"), ld, _p(B, torch.float32, "B"), nb,
        _p(W, torch.float32, "W"), Dx, Dy, Dz,
        _box(skin_aabb), _box(hash_aabb), max_iter, tol_stop, tol_valid, _p(xc, torch.float32, "xc"),
        _p(bone, torch.int16, "bone"), _p(resid, torch.float32, "resid"), _p(steps, torch.int16, "steps"),
        _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()), "snarf_deform")


DEFORM_NOALLOC_MAX_VERTS = 1 << 17  # IA355_DEFORM_NOALLOC_MAX_VERTS


def snarf_deform_noalloc(xp, S, ld, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, xc, bone, resid, steps,
                         S_dev=None):
    """ia355_snarf_deform without a workspace (library-owned scratch)."""
    Dz, Dy, Dx, nb = W.shape
    _check(lib().ia355_snarf_deform_noalloc(
        _p(xp, torch.float32, "xp"), S, _p(S_dev, torch.int64, "S_dev"), ld, _p(B, torch.float32, "B"), nb,
        _p(W, torch.float32, "W"), Dx, Dy, Dz,
        _box(skin_aabb), _box(hash_aabb), max_iter, tol_stop, tol_valid, _p(xc, torch.float32, "xc"),
        _p(bone, torch.int16, "bone"), _p(resid, torch.float32, "resid"), _p(steps, torch.int16, "steps"),
        _stream()), "snarf_deform_noalloc")


def deform_bwd_workspace_size(S, Dx, Dy, Dz, nb):
    return lib().ia355_deform_bwd_workspace_size(S, Dx, Dy, Dz, nb)


def snarf_deform_bwd(grad_xc, xc, bone, S, ld, B, W, skin_aabb, grad_xp, grad_B, grad_W, ws, flags=0, S_dev=None):
    Dz, Dy, Dx, nb = W.shape
    _check(lib().ia355_snarf_deform_bwd(
        _p(grad_xc, torch.float32, "grad_xc"), _p(xc, torch.float32, "xc"), _p(bone, torch.int16, "bone"), S,
        _p(S_dev, torch.int64, "S_dev"), ld, _p(B, torch.float32, "B"), nb, _p(W, torch.float32, "W"), Dx, Dy, Dz, _box(skin_aabb),
        _p(grad_xp, torch.float32, "grad_xp"), _p(grad_B, torch.float32, "grad_B"),
        _p(grad_W, torch.float32, "grad_W"), flags, _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()),
        "snarf_deform_bwd")


def rootinit_fwd(xp, S, ld, pose, params, B, dtype, init_bone, x0, hidden=64, S_dev=None):
    nb = B.shape[0]
    _check(lib().ia355_rootinit_fwd(
        _p(xp, torch.float32, "xp"), S, _p(S_dev, torch.int64, "S_dev"), ld, _p(pose, torch.float32, "pose"),
        _p(params, torch.float32, "params"),
        hidden, _p(B, torch.float32, "B"), nb, dtype, _p(init_bone, torch.int16, "init_bone"),
        _p(x0, torch.float32, "x0"), _stream()), "rootinit_fwd")


def deform_guided_workspace_size(S, Dx, Dy, Dz):
    return lib().ia355_deform_guided_workspace_size(S, Dx, Dy, Dz)


def snarf_deform_guided(xp, S, ld, x0, init_bone, B, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, xc,
                        bone, resid, steps, n_fallback, ws, S_dev=None):
    Dz, Dy, Dx, nb = W.shape
    _check(lib().ia355_snarf_deform_guided(
        _p(xp, torch.float32, "xp"), S, _p(S_dev, torch.int64, "S_dev"), ld, _p(x0, torch.float32, "x0"),
        _p(init_bone, torch.int16, "init_bone"),
        _p(B, torch.float32, "B"), nb, _p(W, torch.float32, "W"), Dx, Dy, Dz, _box(skin_aabb), _box(hash_aabb),
        max_iter, tol_stop, tol_valid, _p(xc, torch.float32, "xc"), _p(bone, torch.int16, "bone"),
        _p(resid, torch.float32, "resid"), _p(steps, torch.int16, "steps"), _p(n_fallback, torch.int32, "n_fallback"),
        _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()), "snarf_deform_guided")


def hashgrid_encode(xc, bone, S, ld, table, base_res, growth, aabb, feat, S_dev=None):
    L, T, F = table.shape
    _check(lib().ia355_hashgrid_encode(
        _p(xc, torch.float32, "xc"), _p(bone, torch.int16, "bone"), S, _p(S_dev, torch.int64, "S_dev"), ld,
        _p(table, name="table"), _DT[table.dtype],
        L, F, T.bit_length() - 1, base_res, growth, _box(aabb), _p(feat, name="feat"), _DT[feat.dtype], _stream()),
        "hashgrid_encode")


def hashgrid_encode_bwd_workspace_size(S, L):
    return lib().ia355_hashgrid_encode_bwd_workspace_size(S, L)


def hashgrid_encode_bwd(grad_feat, xc, bone, S, ld, table, base_res, growth, aabb, grad_table, grad_xc, flags=0,
                        S_dev=None, ws=None):
    """ws: hashgrid_encode_bwd_workspace_size(S, L) bytes, needed with grad_xc."""
    L, T, F = table.shape
    _check(lib().ia355_hashgrid_encode_bwd(
        _p(grad_feat, torch.float32, "grad_feat"), _p(xc, torch.float32, "xc"), _p(bone, torch.int16, "bone"), S,
        _p(S_dev, torch.int64, "S_dev"), ld, _p(table, name="table"), _DT[table.dtype], L, F, T.bit_length() - 1,
        base_res, growth, _box(aabb), _p(grad_table, torch.float32, "grad_table"),
        _p(grad_xc, torch.float32, "grad_xc"), flags, _p(ws, name="ws"),
        0 if ws is None else ws.numel() * ws.element_size(), _stream()), "hashgrid_encode_bwd")


def hashgrid_table_grad_workspace_size(S, L, T):
    """Workspace bytes of hashgrid_table_grad for capacity S, L levels of T entries."""
    if T <= 0 or T & (T - 1):
        raise ValueError(f"T must be a power of two, got {T}")
    return lib().ia355_hashgrid_table_grad_workspace_size(S, L, T.bit_length() - 1)


def hashgrid_table_grad(grad_feat, xc, bone, S, ld, base_res, growth, aabb, grad_table, ws, flags=0, S_dev=None):
    """Table gradient without global atomics (binned); grad_table [L, T, 2]
    FP32; ws: hashgrid_table_grad_workspace_size(S, L, T) bytes.  With
    TABLE_PLAN only the position-dependent passes run (grad_feat may be
    None); TABLE_REUSE_PLAN then runs the rest on the same positions."""
    L, T, F = grad_table.shape
    _check(lib().ia355_hashgrid_table_grad(
        _p(grad_feat, torch.float32, "grad_feat"), _p(xc, torch.float32, "xc"), _p(bone, torch.int16, "bone"), S,
        _p(S_dev, torch.int64, "S_dev"), ld, L, F, T.bit_length() - 1, base_res, growth, _box(aabb),
        _p(grad_table, torch.float32, "grad_table"), flags, _p(ws, name="ws"),
        0 if ws is None else ws.numel() * ws.element_size(), _stream()), "hashgrid_table_grad")


def _widths(widths):
    w = [int(v) for v in widths]
    return (ctypes.c_int32 * len(w))(*w), len(w) - 1


def mlp_fwd(feat, bone, S, ld, params, dtype, sigma, rgb, S_dev=None, widths=MLP_WIDTHS):
    wa, nl = _widths(widths)
    _check(lib().ia355_mlp_fwd(
        _p(feat, name="feat"), _DT[feat.dtype], _p(bone, torch.int16, "bone"), S, _p(S_dev, torch.int64, "S_dev"), ld,
        _p(params, torch.float32, "params"), wa, nl, dtype, _p(sigma, torch.float32, "sigma"),
        _p(rgb, torch.float32, "rgb"), _stream()), "mlp_fwd")


def mlp_bwd_workspace_size(S):
    return lib().ia355_mlp_bwd_workspace_size(S)


def mlp_bwd(grad_sigma, grad_rgb, feat, bone, S, ld, params, dtype, grad_params, grad_feat, ws, flags=0, S_dev=None,
            widths=MLP_WIDTHS):
    wa, nl = _widths(widths)
    _check(lib().ia355_mlp_bwd(
        _p(grad_sigma, torch.float32, "grad_sigma"), _p(grad_rgb, torch.float32, "grad_rgb"), _p(feat, name="feat"),
        _DT[feat.dtype], _p(bone, torch.int16, "bone"), S, _p(S_dev, torch.int64, "S_dev"), ld,
        _p(params, torch.float32, "params"), wa, nl, dtype,
        _p(grad_params, torch.float32, "grad_params"), _p(grad_feat, torch.float32, "grad_feat"), flags,
        _p(ws, name="ws"), ws.numel() * ws.element_size(), _stream()), "mlp_bwd")


def volrender_fwd(sigma, rgb, ld, ray_off, ray_dt, R, T_thresh, color, opacity, n_used, T_final):
    _check(lib().ia355_volrender_fwd(
        _p(sigma, torch.float32, "sigma"), _p(rgb, torch.float32, "rgb"), ld, _p(ray_off, torch.int64, "ray_off"),
        _p(ray_dt, torch.float32, "ray_dt"), R, T_thresh, _p(color, torch.float32, "color"),
        _p(opacity, torch.float32, "opacity"), _p(n_used, torch.int32, "n_used"), _p(T_final, torch.float32, "T_final"),
        _stream()), "volrender_fwd")


def volrender_bwd(grad_color, grad_opacity, sigma, rgb, ld, ray_off, ray_dt, n_used, color, T_final, R, grad_sigma,
                  grad_rgb):
    _check(lib().ia355_volrender_bwd(
        _p(grad_color, torch.float32, "grad_color"), _p(grad_opacity, torch.float32, "grad_opacity"),
        _p(sigma, torch.float32, "sigma"), _p(rgb, torch.float32, "rgb"), ld, _p(ray_off, torch.int64, "ray_off"),
        _p(ray_dt, torch.float32, "ray_dt"), _p(n_used, torch.int32, "n_used"), _p(color, torch.float32, "color"),
        _p(T_final, torch.float32, "T_final"), R, _p(grad_sigma, torch.float32, "grad_sigma"),
        _p(grad_rgb, torch.float32, "grad_rgb"), _stream()), "volrender_bwd")


def l2_loss(color, target, loss, grad_color):
    R = color.shape[0]
    _check(lib().ia355_l2_loss(_p(color, torch.float32, "color"), _p(target, torch.float32, "target"), R,
                               _p(loss, torch.float32, "loss"), _p(grad_color, torch.float32, "grad_color"),
                               _stream()), "l2_loss")


BATCH_MAX_POSES = 64


def batch_workspace_size(n_poses, Dx, Dy, Dz, nb):
    return lib().ia355_batch_workspace_size(n_poses, Dx, Dy, Dz, nb)


def batch_lds_bytes(rays_per_tile, samples_per_segment, waves_per_group=4):
    """LDS bytes per workgroup of a render schedule (0: invalid shape)."""
    return lib().ia355_batch_lds_bytes(rays_per_tile, samples_per_segment, waves_per_group)


def batch_pose(rays_o, rays_d, occ_bits, G, occ_aabb, dt, n_per_ray, max_steps, B, pose, color, opacity, n_used,
               T_final, n_fallback=None, n_evaluated=None):
    """One ``ia355_batch_pose`` from GPU tensors (the tensors must outlive
    every render that uses the plan)."""
    R = rays_o.shape[0]
    for t, n in ((rays_d, "rays_d"), (color, "color")):
        if t.shape[0] != R:
            raise ValueError(f"batch_pose: {n} has {t.shape[0]} rows, rays_o {R}")
    for t, n in ((opacity, "opacity"), (n_used, "n_used"), (T_final, "T_final")):
        if t.numel() != R:
            raise ValueError(f"batch_pose: {n} has {t.numel()} values for {R} rays")
    return BatchPose(_p(rays_o, torch.float32, "rays_o"), _p(rays_d, torch.float32, "rays_d"), R,
                     _p(occ_bits, torch.int32, "occ_bits"), G, _box(occ_aabb), float(dt), n_per_ray, max_steps,
                     _p(B, torch.float32, "B"), _p(pose, torch.float32, "pose"), _p(color, torch.float32, "color"),
                     _p(opacity, torch.float32, "opacity"), _p(n_used, torch.int32, "n_used"),
                     _p(T_final, torch.float32, "T_final"), _p(n_fallback, torch.int32, "n_fallback"),
                     _p(n_evaluated, torch.int32, "n_evaluated"))


def batch_plan(poses, W, skin_aabb, hash_aabb, max_iter, tol_stop, tol_valid, table, base_res, growth, mlp_params,
               init_params, T_thresh, ws, init_hidden=64):
    """Validate the poses (a list of ``batch_pose``) and the shared model and
    write the plan into ws (synchronises the stream)."""
    Dz, Dy, Dx, nb = W.shape
    L, T, F = table.shape
    if table.dtype != torch.float16 or F != 2:
        raise TypeError("batch_plan: the table must be FP16 [L][T][2]")
    m = BatchModel(_p(W, torch.float32, "W"), Dx, Dy, Dz, nb, _box(skin_aabb), _box(hash_aabb), max_iter,
                   float(tol_stop), float(tol_valid), _p(table, torch.float16, "table"), L, T.bit_length() - 1,
                   float(base_res), float(growth), _p(mlp_params, torch.float32, "mlp_params"),
                   _p(init_params, torch.float32, "init_params"), init_hidden, float(T_thresh))
    arr = (BatchPose * len(poses))(*poses)
    _check(lib().ia355_batch_plan(arr, len(poses), ctypes.byref(m), _p(ws, name="ws"),
                                  ws.numel() * ws.element_size(), _stream()), "batch_plan")


def batch_render(ws, rays_per_tile, samples_per_segment, waves_per_group, blocks_per_cu):
    """Enqueue the batched render of the plan in ws (capturable)."""
    _check(lib().ia355_batch_render(_p(ws, name="ws"), ws.numel() * ws.element_size(), rays_per_tile,
                                    samples_per_segment, waves_per_group, blocks_per_cu, _stream()),
           "batch_render")
