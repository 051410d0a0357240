"""Device-resident pipeline: one training step or one frame of the
deform-and-query path (Fig. 2 of the paper) as a fixed sequence of C-ABI
calls on preallocated HBM buffers.

    march -> deform -> hash encode -> MLP -> composite           (forward)
    L2 loss -> composite bwd -> MLP bwd -> encode bwd -> deform bwd (IFT)

PyTorch only provides the device allocations and the stream; no torch
operator runs inside ``forward`` / ``backward`` / ``train_step``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lib as K

NPARAM = 6532


class StageTimer:
    """HIP events on the launch stream around each named stage; ``mark(name)``
    closes the open stage and opens ``name`` (None closes only).  Durations
    are summed per stage after a synchronisation."""

    def __init__(self):
        self.events = []  # (name, start, end)
        self._open = None

    def mark(self, name):
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(torch.cuda.current_stream())
        if self._open is not None:
            self.events.append((self._open[0], self._open[1], ev))
        self._open = (name, ev) if name is not None else None

    def totals_ms(self):
        torch.cuda.synchronize()
        out = {}
        for name, a, b in self.events:
            out[name] = out.get(name, 0.0) + a.elapsed_time(b)
        return out

    def counts(self):
        out = {}
        for name, _, _ in self.events:
            out[name] = out.get(name, 0) + 1
        return out


class Pipeline:
    def __init__(self, w, device="cuda", table_dtype=torch.float32, mlp_dtype=K.F32, cap=None,
                 grad_W=True, grad_B=True, rootinit_params=None, rootinit_dtype=K.BF16):
        self.w = w
        self.dev = torch.device(device)
        dev = self.dev
        t = lambda a, dt=None: torch.as_tensor(np.ascontiguousarray(a), device=dev, dtype=dt)
        self.R = w.R
        self.rays_o = t(w.rays_o, torch.float32)
        self.rays_d = t(w.rays_d, torch.float32)
        self.G = 0
        self.occ_bits = None
        if w.occ is not None:
            self.G = w.occ.shape[0]
            occ = t(w.occ, torch.uint8)
            self.occ_bits = torch.empty((self.G ** 3 + 31) // 32, dtype=torch.int32, device=dev)
            K.occ_pack(occ, self.occ_bits)
        self.B = t(w.B, torch.float32)
        self.W = t(w.W, torch.float32)
        self.table32 = t(w.table, torch.float32)
        self.table = self.table32 if table_dtype == torch.float32 else self.table32.to(table_dtype)
        self.params = t(w.mlp, torch.float32)
        self.target = None if w.target is None else t(w.target, torch.float32)
        self.mlp_dtype = mlp_dtype
        self.feat_dtype = torch.float32 if mlp_dtype == K.F32 else torch.bfloat16
        self.cap = int(cap) if cap is not None else self.R * w.max_steps
        cap = self.cap
        L = w.L
        e = lambda *shape, dt=torch.float32: torch.empty(*shape, dtype=dt, device=dev)
        # march outputs
        self.xs = e(3, cap)
        self.ts = e(cap)
        self.ray_id = e(cap, dt=torch.int32)
        self.ray_off = e(self.R + 1, dt=torch.int64)
        self.ray_cnt = e(self.R, dt=torch.int32)
        self.ray_dt = e(self.R)
        self.n_samples = e(1, dt=torch.int64)
        self.ws_march = e(K.march_workspace_size(self.R), dt=torch.uint8)
        # deform
        Dz, Dy, Dx, nb = w.W.shape
        self.ws_deform = e(K.deform_workspace_size(Dx, Dy, Dz), dt=torch.uint8)
        self.xc = e(3, cap)
        self.bone = e(cap, dt=torch.int16)
        self.resid = e(cap)
        self.steps = e(cap, dt=torch.int16)
        # field
        self.feat = e(L * cap * 2, dt=self.feat_dtype)
        self.sigma = e(cap)
        self.rgb = e(3, cap)
        # composite
        self.color = e(self.R, 3)
        self.opacity = e(self.R)
        self.n_used = e(self.R, dt=torch.int32)
        self.T_final = e(self.R)
        # backward
        self.loss = e(1)
        self.grad_color = e(self.R, 3)
        self.grad_sigma = e(cap)
        self.grad_rgb = e(3, cap)
        self.grad_feat = e(L * cap * 2)
        self.grad_params = e(NPARAM)
        self.ws_mlp = e(K.mlp_bwd_workspace_size(cap), dt=torch.uint8)
        self.grad_table = e(*self.table32.shape)
        self.grad_xc = e(3, cap)
        self.grad_xp = e(3, cap)
        self.grad_B = e(*self.B.shape) if grad_B else None
        self.grad_W = e(*self.W.shape) if grad_W else None
        self.ws_ift = e(K.deform_bwd_workspace_size(cap, Dx, Dy, Dz, nb), dt=torch.uint8)
        self.ws_hash = None  # binned table-gradient scratch, sized on first use for the step's S
        self.S = None
        self.timer = None  # optional StageTimer: HIP events around each stage
        # learned root initialiser (guided solve with multi-init fallback)
        self.guided = None
        if rootinit_params is not None:
            from .rootinit import GuidedDeform
            self.pose_t = t(w.pose_params.reshape(-1), torch.float32)
            self.guided = GuidedDeform(rootinit_params, w, cap, device=device, dtype=rootinit_dtype)

    def _mark(self, name):
        if self.timer is not None:
            self.timer.mark(name)

    # ------------------------------------------------------------ forward
    def march(self):
        w = self.w
        K.occgrid_march(self.rays_o, self.rays_d, self.occ_bits, self.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps,
                        self.xs, self.ts, self.ray_id, self.cap, self.ray_off, self.ray_cnt, self.ray_dt,
                        self.n_samples, self.ws_march)

    def read_count(self):
        S = int(self.n_samples.item())
        if S > self.cap:
            raise RuntimeError(f"sample buffer too small: {S} > {self.cap}")
        self.S = S
        return S

    def field(self, S):
        w = self.w
        self._mark("deform")
        if self.guided is not None:
            self.guided.run(self.xs, S, self.cap, self.pose_t, self.B, self.W, self.xc, self.bone, self.resid,
                            self.steps)
        else:
            K.snarf_deform(self.xs, S, self.cap, self.B, self.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop,
                           w.tol_valid, self.xc, self.bone, self.resid, self.steps, self.ws_deform)
        feat = self.feat[: w.L * S * 2]
        self._mark("hash_fwd")
        K.hashgrid_encode(self.xc, self.bone, S, self.cap, self.table, w.base_res, w.growth, w.hash_aabb, feat)
        self._mark("mlp_fwd")
        K.mlp_fwd(feat, self.bone, S, self.cap, self.params, self.mlp_dtype, self.sigma, self.rgb)

    def composite(self):
        self._mark("render_fwd")
        K.volrender_fwd(self.sigma, self.rgb, self.cap, self.ray_off, self.ray_dt, self.R, self.w.T_thresh,
                        self.color, self.opacity, self.n_used, self.T_final)
        self._mark(None)

    def forward(self):
        self._mark("march")
        self.march()
        self._mark(None)
        S = self.read_count()
        self.field(S)
        self.composite()
        return S

    # ----------------------------------------------------------- backward
    def backward(self, S):
        w = self.w
        self._mark("loss+render_bwd")
        K.l2_loss(self.color, self.target, self.loss, self.grad_color)
        K.volrender_bwd(self.grad_color, None, self.sigma, self.rgb, self.cap, self.ray_off, self.ray_dt, self.n_used,
                        self.color, self.T_final, self.R, self.grad_sigma, self.grad_rgb)
        self._mark("mlp_bwd")
        feat = self.feat[: w.L * S * 2]
        gfeat = self.grad_feat[: w.L * S * 2]
        K.mlp_bwd(self.grad_sigma, self.grad_rgb, feat, self.bone, S, self.cap, self.params, self.mlp_dtype,
                  self.grad_params, gfeat, self.ws_mlp, flags=K.OVERWRITE)
        need = K.hashgrid_bwd_workspace_size(S, w.L, self.table.shape[1].bit_length() - 1)
        if need and (self.ws_hash is None or self.ws_hash.numel() < need):
            self.ws_hash = torch.empty(need + need // 4, dtype=torch.uint8, device=self.dev)
        self._mark("hash_bwd")
        K.hashgrid_encode_bwd(gfeat, self.xc, self.bone, S, self.cap, self.table, w.base_res, w.growth, w.hash_aabb,
                              self.grad_table, self.grad_xc, flags=K.OVERWRITE, ws=self.ws_hash if need else None)
        self._mark("deform_bwd")
        K.snarf_deform_bwd(self.grad_xc, self.xc, self.bone, S, self.cap, self.B, self.W, w.skin_aabb, self.grad_xp,
                           self.grad_B, self.grad_W, self.ws_ift, flags=K.OVERWRITE)
        self._mark(None)

    def train_step(self):
        S = self.forward()
        self.backward(S)
        return S

    # ------------------------------------------------------------ readback
    def soa(self, t, S=None):
        S = self.S if S is None else S
        return t[:, :S].T.double().cpu().numpy()

    def feat_samples(self, S=None):
        S = self.S if S is None else S
        return self.feat[: self.w.L * S * 2].float().view(self.w.L, S, 2).permute(1, 0, 2).reshape(S, -1).double().cpu().numpy()
