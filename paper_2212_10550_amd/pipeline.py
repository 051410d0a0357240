"""Device-resident pipeline: one training step or one frame of the
deform-and-query path (Fig. 2 of the paper) as a fixed sequence of C-ABI
calls on preallocated HBM buffers.

    march -> deform -> hash encode -> MLP -> composite           (forward)
    L2 loss -> composite bwd -> MLP bwd -> encode bwd -> deform bwd (IFT)

PyTorch only provides the device allocations and the stream; no torch
operator runs inside ``forward`` / ``backward`` / ``train_step``.

With ``device_count=True`` no stage waits for the host: the march leaves
the sample count in device memory and every later call reads it there (the
capacity sizes the launches).  A whole step is then enqueued at once and
can be captured in a HIP graph (``capture_train_step``).
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
                 grad_W=True, grad_B=True, rootinit_params=None, rootinit_dtype=K.BF16, device_count=False,
                 table_grad="binned"):
        """table_grad: "binned" (records binned by table tile, summed in LDS,
        no global atomics on the hashed levels) or "atomic" (FP32 global
        atomics, coarse and fine level groups on two streams)."""
        if table_grad not in ("binned", "atomic"):
            raise ValueError(f"table_grad must be 'binned' or 'atomic', got {table_grad!r}")
        self.w = w
        self.table_grad_mode = table_grad
        self.device_count = device_count
        self.graph, self.graph_kind = None, None
        # side streams of the backward (default priority): the coarse and the
        # fine levels of the table gradient
        self.side = torch.cuda.Stream(device=torch.device(device))
        self.side2 = torch.cuda.Stream(device=torch.device(device))
        self._table_zeroed = False
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
            self.occ_bits = torch.empty(K.occ_words(self.G), dtype=torch.int32, device=dev)
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
        self.ws_march = e(K.march_workspace_size(self.R, w.max_steps), dt=torch.uint8)
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
        # the full loss of Sec. 3.4 (set_full_loss); otherwise the L2 loss
        self.full_loss = None
        self.loss4 = e(4)
        self.grad_opacity = e(self.R)
        self.grad_sigma = e(cap)
        self.grad_rgb = e(3, cap)
        self.grad_feat = e(L * cap * 2)
        self.grad_params = e(NPARAM)
        self.ws_mlp = e(K.mlp_bwd_workspace_size(cap), dt=torch.uint8)
        self.grad_table = e(*self.table32.shape)
        self.grad_xc = e(3, cap)
        # per-level partial position gradients (training workloads only)
        self.ws_xgrad = None if w.target is None else e(K.hashgrid_encode_bwd_workspace_size(cap, L), dt=torch.uint8)
        self.ws_tgrad = None
        if w.target is not None and table_grad == "binned":
            self.ws_tgrad = e(K.hashgrid_table_grad_workspace_size(cap, L, self.table32.shape[1]), dt=torch.uint8)
        self.grad_xp = e(3, cap)
        self.grad_B = e(*self.B.shape) if grad_B else None
        self.grad_W = e(*self.W.shape) if grad_W else None
        self.ws_ift = e(K.deform_bwd_workspace_size(cap, Dx, Dy, Dz, nb), dt=torch.uint8)
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
        """The sample count of the last march (synchronises)."""
        S = int(self.n_samples.item())
        if S > self.cap:
            raise RuntimeError(f"sample buffer too small: {S} > {self.cap}")
        self.S = S
        return S

    def _counts(self):
        """(S, S_dev) for the stage calls: the host count after a sync, or the
        capacity and the device counter."""
        if self.device_count:
            return self.cap, self.n_samples
        return self.read_count(), None

    # stages: each reads the outputs of the previous ones and overwrites its
    # own outputs, so it can be run (or replayed) on its own
    def _deform(self, S, Sd):
        w = self.w
        if self.guided is not None:
            self.guided.run(self.xs, S, self.cap, self.pose_t, self.B, self.W, self.xc, self.bone, self.resid,
                            self.steps, S_dev=Sd)
        else:
            K.snarf_deform(self.xs, S, self.cap, self.B, self.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop,
                           w.tol_valid, self.xc, self.bone, self.resid, self.steps, self.ws_deform, S_dev=Sd)

    def _encode(self, S, Sd):
        w = self.w
        K.hashgrid_encode(self.xc, self.bone, S, self.cap, self.table, w.base_res, w.growth, w.hash_aabb, self.feat,
                          S_dev=Sd)

    def _mlp(self, S, Sd):
        K.mlp_fwd(self.feat, self.bone, S, self.cap, self.params, self.mlp_dtype, self.sigma, self.rgb, S_dev=Sd)

    def _render(self):
        K.volrender_fwd(self.sigma, self.rgb, self.cap, self.ray_off, self.ray_dt, self.R, self.w.T_thresh,
                        self.color, self.opacity, self.n_used, self.T_final)

    def set_full_loss(self, alpha_gt=None, delta=0.1, lam_alpha=0.1, lam_hard=0.01):
        """Train on the loss of Sec. 3.4 (Huber colour, L1 opacity against
        alpha_gt [R] if given, hard-surface term) instead of the L2 loss;
        self.loss4 holds (total, rgb, alpha, hard)."""
        self.full_loss = (None if alpha_gt is None else torch.as_tensor(alpha_gt, device=self.dev, dtype=torch.float32),
                          float(delta), float(lam_alpha), float(lam_hard))

    def _render_bwd(self):
        if self.full_loss is None:
            K.l2_loss(self.color, self.target, self.loss, self.grad_color)
            g_op = None
        else:
            alpha_gt, delta, lam_alpha, lam_hard = self.full_loss
            K.loss_full(self.color, self.opacity, self.target, alpha_gt, delta, lam_alpha, lam_hard, self.loss4,
                        self.grad_color, self.grad_opacity)
            g_op = self.grad_opacity
        K.volrender_bwd(self.grad_color, g_op, self.sigma, self.rgb, self.cap, self.ray_off, self.ray_dt, self.n_used,
                        self.color, self.T_final, self.R, self.grad_sigma, self.grad_rgb)

    def _mlp_bwd(self, S, Sd):
        K.mlp_bwd(self.grad_sigma, self.grad_rgb, self.feat, self.bone, S, self.cap, self.params, self.mlp_dtype,
                  self.grad_params, self.grad_feat, self.ws_mlp, flags=K.OVERWRITE, S_dev=Sd)

    def _table_grad(self, S, Sd, overwrite=True, group=0, phase=0):
        """Table gradient of the level group (K.TABLE_COARSE, K.TABLE_FINE,
        or 0 for every level).  Binned mode: phase K.TABLE_PLAN runs only the
        position-dependent passes, K.TABLE_REUSE_PLAN the rest."""
        w = self.w
        if self.table_grad_mode == "binned":
            if self.ws_tgrad is None:
                L, T, _ = self.grad_table.shape
                self.ws_tgrad = torch.empty(K.hashgrid_table_grad_workspace_size(self.cap, L, T), dtype=torch.uint8,
                                            device=self.dev)
            K.hashgrid_table_grad(self.grad_feat, self.xc, self.bone, S, self.cap, w.base_res, w.growth, w.hash_aabb,
                                  self.grad_table, self.ws_tgrad,
                                  flags=(K.OVERWRITE if overwrite else 0) | group | phase, S_dev=Sd)
            return
        K.hashgrid_encode_bwd(self.grad_feat, self.xc, self.bone, S, self.cap, self.table, w.base_res, w.growth,
                              w.hash_aabb, self.grad_table, None, flags=(K.OVERWRITE if overwrite else 0) | group,
                              S_dev=Sd)

    def _zero_table_async(self):
        """Clear the table gradient on the side stream (it overlaps the
        forward); the backward's table gradient then adds to it.  The binned
        table gradient writes every entry itself, so it needs no clear."""
        if self.table_grad_mode == "binned":
            return
        self.side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.side):
            K.zero(self.grad_table)
        self._table_zeroed = True

    def _x_grad(self, S, Sd):
        w = self.w
        if self.ws_xgrad is None:
            self.ws_xgrad = torch.empty(K.hashgrid_encode_bwd_workspace_size(self.cap, w.L), dtype=torch.uint8,
                                        device=self.dev)
        K.hashgrid_encode_bwd(self.grad_feat, self.xc, self.bone, S, self.cap, self.table, w.base_res, w.growth,
                              w.hash_aabb, None, self.grad_xc, S_dev=Sd, ws=self.ws_xgrad)

    def _deform_bwd(self, S, Sd):
        w = self.w
        K.snarf_deform_bwd(self.grad_xc, self.xc, self.bone, S, self.cap, self.B, self.W, w.skin_aabb, self.grad_xp,
                           self.grad_B, self.grad_W, self.ws_ift, flags=K.OVERWRITE, S_dev=Sd)

    def stages(self, S, Sd, backward=True):
        """The step as (name, call) pairs after the march."""
        st = [("deform", lambda: self._deform(S, Sd)), ("hash_fwd", lambda: self._encode(S, Sd)),
              ("mlp_fwd", lambda: self._mlp(S, Sd)), ("render_fwd", self._render)]
        if backward:
            st += [("loss+render_bwd", self._render_bwd), ("mlp_bwd", lambda: self._mlp_bwd(S, Sd)),
                   ("hash_bwd_table", lambda: self._table_grad(S, Sd)), ("hash_bwd_x", lambda: self._x_grad(S, Sd)),
                   ("deform_bwd", lambda: self._deform_bwd(S, Sd))]
        return st

    def forward(self, zero_table=False):
        """One forward; returns the sample count (None with device counts:
        read it later with read_count).  zero_table: fork the clear of the
        table gradient to the side stream after the march (it then overlaps
        the root finding)."""
        self._mark("march")
        self.march()
        self._mark(None)
        if zero_table:
            self._zero_table_async()
        S, Sd = self._counts()
        for name, fn in self.stages(S, Sd, backward=False):
            self._mark(name)
            fn()
        self._mark(None)
        self._last = (S, Sd)
        return None if self.device_count else S

    # ----------------------------------------------------------- backward
    def backward(self, S=None, Sd=None):
        """Loss, composite and MLP backward, then independent branches: the
        hash-table gradient on a side stream (binned: every level in one
        call; atomic: the coarse and the fine levels on two side streams,
        disjoint slices of the table, the coarse levels bound by contention
        on few entries and the fine ones by atomic throughput), and the
        position gradient followed by the implicit-function-theorem backward
        on this stream; the side streams join back before returning."""
        if S is None:
            S, Sd = self._last
        st = dict(self.stages(S, Sd))
        for name in ("loss+render_bwd", "mlp_bwd"):
            self._mark(name)
            st[name]()
        if self.timer is not None:  # stage timing: serial, one stage at a time
            main = torch.cuda.current_stream()
            ow = not self._table_zeroed
            if self._table_zeroed:  # the clear was forked to the side stream
                main.wait_stream(self.side)
                self._table_zeroed = False
            self._mark("hash_bwd_table")
            self._table_grad(S, Sd, overwrite=ow)
            for name in ("hash_bwd_x", "deform_bwd"):
                self._mark(name)
                st[name]()
            self._mark(None)
            return
        main = torch.cuda.current_stream()
        self.side.wait_stream(main)
        if self.table_grad_mode == "binned":
            # every level in one binned call beside the position gradient
            # (its position passes could run earlier, TABLE_PLAN, but beside
            # the forward or the MLP backward they slow those more than they
            # save here)
            with torch.cuda.stream(self.side):
                self._table_grad(S, Sd, overwrite=True)
            st["hash_bwd_x"]()
            st["deform_bwd"]()
            main.wait_stream(self.side)
            return
        self.side2.wait_stream(self.side)  # after the table clear (if any) and the MLP backward
        ow = not self._table_zeroed
        with torch.cuda.stream(self.side):
            self._table_grad(S, Sd, overwrite=ow, group=K.TABLE_COARSE)
        with torch.cuda.stream(self.side2):
            self._table_grad(S, Sd, overwrite=ow, group=K.TABLE_FINE)
        self._table_zeroed = False
        st["hash_bwd_x"]()
        st["deform_bwd"]()
        main.wait_stream(self.side)
        main.wait_stream(self.side2)

    def stage_times(self, n=20, backward=True, reps=10):
        """GPU ms per stage (device counts): each stage's calls captured
        `reps` times back to back in a graph of their own, the graph replayed
        n times after a full step has put the inputs in place (every stage
        overwrites its outputs, so repeating it is idempotent).  Repeating
        the calls inside one graph keeps the host's graph-launch gap out of
        the figure for short stages."""
        if not self.device_count:
            raise RuntimeError("stage_times needs device_count=True")
        self.forward()
        if backward:
            self.backward()
        torch.cuda.synchronize()
        out = {}
        for name, fn in [("march", self.march)] + self.stages(self.cap, self.n_samples, backward):
            fn()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(reps):
                    fn()
            g.replay()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(n):
                g.replay()
            b.record()
            torch.cuda.synchronize()
            out[name] = a.elapsed_time(b) / (n * reps)
            del g
        return out

    def train_step(self):
        """Forward and backward; returns the sample count (None with device
        counts)."""
        if self.graph is not None and self.graph_kind == "train":
            self.graph.replay()
            return None
        S = self.forward(zero_table=self.timer is None)
        self.backward()
        return S

    def capture_train_step(self):
        """Capture one training step (device counts) in a HIP graph; later
        train_step calls replay it."""
        self._capture(lambda: (self.forward(zero_table=True), self.backward()), "train")

    def capture_forward(self):
        """Capture one forward (device counts) in a HIP graph; later
        replay() calls run it."""
        self._capture(self.forward, "forward")

    def _capture(self, fn, kind):
        # torch captures on a side stream; replays go to the current stream
        if not self.device_count:
            raise RuntimeError("graph capture needs device_count=True")
        self.graph = None
        fn()  # warm-up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        torch.cuda.synchronize()
        self.graph, self.graph_kind = g, kind

    def replay(self):
        self.graph.replay()

    # ------------------------------------------------------------ readback
    def soa(self, t, S=None):
        S = self.S if S is None else S
        return t[:, :S].T.double().cpu().numpy()

    def feat_samples(self, S=None):
        S = self.S if S is None else S
        f = self.feat.float().view(self.w.L, self.cap, 2)[:, :S]
        return f.permute(1, 0, 2).reshape(S, -1).double().cpu().numpy()
