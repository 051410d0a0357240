"""Batched render of many poses of one avatar.

Each pose runs the inference forward of the path (Fig. 2): march with
empty-space skipping, learned root initialiser, guided Broyden with
multi-init fallback, FP16 hash encode, BF16 MLP, compositing with early
termination.  Two executions of the same arithmetic:

* persistent (``ia355_batch_render``): one preparation kernel (per-pose
  transform grids and initialiser constants) and one persistent kernel
  whose waves take tiles of rays of any pose from a work counter and carry
  each tile through the whole path on chip; the schedule is the tile shape
  (rays per tile, samples per segment) and the workgroups per CU.
* staged: the path's kernels per pose, every call taking its sample count
  from device memory, poses spread over a few streams inside one graph
  (fork from the capture stream, join back); each stream owns one set of
  sample buffers ("slot") sized for its largest pose (exact counts from a
  march prepass at build time).  The schedule is the number of streams.

Both are captured as one HIP graph; ``autotune`` times every candidate
schedule and keeps the fastest.  Both write the same bits for every pose.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lib as K


class _Pose:
    def __init__(self, w, dev):
        t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a), device=dev, dtype=dt)
        self.w = w
        self.R = w.R
        self.rays_o = t(w.rays_o)
        self.rays_d = t(w.rays_d)
        self.G = w.occ.shape[0]
        occ = t(w.occ, torch.uint8)
        self.occ_bits = torch.empty(K.occ_words(self.G), dtype=torch.int32, device=dev)
        K.occ_pack(occ, self.occ_bits)
        self.B = t(w.B)
        self.pose_t = t(w.pose_params.reshape(-1))
        e = lambda *shape, dt=torch.float32: torch.empty(*shape, dtype=dt, device=dev)
        self.ray_off = e(self.R + 1, dt=torch.int64)
        self.ray_cnt = e(self.R, dt=torch.int32)
        self.ray_dt = e(self.R)
        self.color = e(self.R, 3)
        self.opacity = e(self.R)
        self.n_used = e(self.R, dt=torch.int32)
        self.T_final = e(self.R)
        self.n_fallback = e(1, dt=torch.int32)
        self.n_evaluated = torch.zeros(1, dtype=torch.int32, device=dev)  # persistent render only
        self.S = None  # exact sample count (march prepass)


class _Slot:
    """Sample buffers of one stream."""

    def __init__(self, cap, max_R, max_steps, L, Wshape, feat_dtype, dev):
        e = lambda *shape, dt=torch.float32: torch.empty(*shape, dtype=dt, device=dev)
        Dz, Dy, Dx, nb = Wshape
        self.cap = cap
        self.xs = e(3, cap)
        self.ts = e(cap)
        self.ray_id = e(cap, dt=torch.int32)
        self.n_samples = e(1, dt=torch.int64)
        self.ws_march = e(K.march_workspace_size(max_R, max_steps), dt=torch.uint8)
        self.init_bone = e(cap, dt=torch.int16)
        self.x0 = e(3, cap)
        self.ws_guided = e(K.deform_guided_workspace_size(cap, Dx, Dy, Dz), dt=torch.uint8)
        self.xc = e(3, cap)
        self.bone = e(cap, dt=torch.int16)
        self.feat = e(L * cap * 2, dt=feat_dtype)
        self.sigma = e(cap)
        self.rgb = e(3, cap)
        self.stream = torch.cuda.Stream(device=dev)  # default priority


class BatchRenderer:
    def __init__(self, workloads, rootinit_params, n_streams=1, device="cuda", rootinit_dtype=K.BF16):
        dev = torch.device(device)
        self.dev = dev
        w0 = workloads[0]
        self.w0 = w0
        t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a), device=dev, dtype=dt)
        self.table = t(w0.table).to(torch.float16)
        self.params = t(w0.mlp)
        self.W = t(w0.W)
        self.ri_params = t(rootinit_params)
        self.ri_dtype = rootinit_dtype
        self.poses = [_Pose(w, dev) for w in workloads]
        self.slots = None
        self.persistent = None  # (rays per tile, samples per segment, waves per workgroup, workgroups per CU)
        self._ws = None
        self._prepass()
        self.set_streams(n_streams)
        self.graph = None

    def _prepass(self):
        """Exact sample count of every pose (a march with capacity 0 only counts)."""
        n = torch.empty(1, dtype=torch.int64, device=self.dev)
        for p in self.poses:
            w = p.w
            ws = torch.empty(K.march_workspace_size(p.R, w.max_steps), dtype=torch.uint8, device=self.dev)
            K.occgrid_march(p.rays_o, p.rays_d, p.occ_bits, p.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps,
                            None, None, None, 0, p.ray_off, p.ray_cnt, p.ray_dt, n, ws)
            p.S = int(n.item())

    def set_persistent(self, rays_per_tile=32, samples_per_segment=256, waves_per_group=4, blocks_per_cu=2):
        """Render with the persistent kernel and this schedule (the staged
        buffers are released)."""
        if self.ri_dtype != K.BF16:
            raise ValueError("the persistent render runs the BF16 initialiser")
        if K.batch_lds_bytes(rays_per_tile, samples_per_segment, waves_per_group) == 0:
            raise ValueError(f"invalid tile shape {rays_per_tile} rays / {samples_per_segment} samples / "
                             f"{waves_per_group} waves")
        self.graph = None
        self.slots = None
        torch.cuda.empty_cache()
        self._plan()
        self.persistent = (rays_per_tile, samples_per_segment, waves_per_group, blocks_per_cu)

    def _plan(self):
        if self._ws is not None:
            return
        w0 = self.w0
        for p in self.poses:
            w = p.w
            same = (w.max_iter == w0.max_iter and w.tol_stop == w0.tol_stop and w.tol_valid == w0.tol_valid
                    and w.T_thresh == w0.T_thresh and w.base_res == w0.base_res and w.growth == w0.growth
                    and list(w.skin_aabb) == list(w0.skin_aabb) and list(w.hash_aabb) == list(w0.hash_aabb))
            if not same:
                raise ValueError("the persistent render needs one model (solver, encoding, threshold) for all poses")
        Dz, Dy, Dx, nb = self.W.shape
        self._ws = torch.empty(K.batch_workspace_size(len(self.poses), Dx, Dy, Dz, nb), dtype=torch.uint8,
                               device=self.dev)
        descs = [K.batch_pose(p.rays_o, p.rays_d, p.occ_bits, p.G, p.w.occ_aabb, p.w.dt, p.w.n_per_ray,
                              p.w.max_steps, p.B, p.pose_t, p.color, p.opacity, p.n_used, p.T_final, p.n_fallback,
                              p.n_evaluated)
                 for p in self.poses]
        K.batch_plan(descs, self.W, w0.skin_aabb, w0.hash_aabb, w0.max_iter, w0.tol_stop, w0.tol_valid, self.table,
                     w0.base_res, w0.growth, self.params, self.ri_params, w0.T_thresh, self._ws)

    def set_streams(self, n_streams):
        """Render with the staged kernels: assign poses to n_streams streams,
        longest (most samples) first onto the least loaded stream, and size
        each stream's buffers."""
        self.graph = None
        self.slots = None
        self.persistent = None
        torch.cuda.empty_cache()
        order = sorted(range(len(self.poses)), key=lambda i: -self.poses[i].S)
        load = [0] * n_streams
        self.assign = [[] for _ in range(n_streams)]
        for i in order:
            j = int(np.argmin(load))
            self.assign[j].append(i)
            load[j] += self.poses[i].S
        w0 = self.w0
        self.slots = []
        for j in range(n_streams):
            ps = [self.poses[i] for i in self.assign[j]]
            cap = max([p.S for p in ps] + [1])
            max_R = max([p.R for p in ps] + [1])
            max_steps = max([p.w.max_steps for p in ps] + [1])
            self.slots.append(_Slot(cap, max_R, max_steps, w0.L, w0.W.shape, torch.bfloat16, self.dev))
        self.n_streams = n_streams

    def _pose_forward(self, sl, p):
        w = p.w
        cap, Sd = sl.cap, sl.n_samples
        K.occgrid_march(p.rays_o, p.rays_d, p.occ_bits, p.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps, sl.xs,
                        sl.ts, sl.ray_id, cap, p.ray_off, p.ray_cnt, p.ray_dt, Sd, sl.ws_march)
        K.rootinit_fwd(sl.xs, cap, cap, p.pose_t, self.ri_params, p.B, self.ri_dtype, sl.init_bone, sl.x0, S_dev=Sd)
        K.snarf_deform_guided(sl.xs, cap, cap, sl.x0, sl.init_bone, p.B, self.W, w.skin_aabb, w.hash_aabb,
                              w.max_iter, w.tol_stop, w.tol_valid, sl.xc, sl.bone, None, None, p.n_fallback,
                              sl.ws_guided, S_dev=Sd)
        K.hashgrid_encode(sl.xc, sl.bone, cap, cap, self.table, w.base_res, w.growth, w.hash_aabb, sl.feat, S_dev=Sd)
        K.mlp_fwd(sl.feat, sl.bone, cap, cap, self.params, K.BF16, sl.sigma, sl.rgb, S_dev=Sd)
        K.volrender_fwd(sl.sigma, sl.rgb, cap, p.ray_off, p.ray_dt, p.R, w.T_thresh, p.color, p.opacity, p.n_used,
                        p.T_final)

    def render(self):
        """Enqueue every pose (or replay the captured graph)."""
        if self.graph is not None:
            self.graph.replay()
            return
        if self.persistent is not None:
            K.batch_render(self._ws, *self.persistent)
            return
        main = torch.cuda.current_stream()
        for sl in self.slots:
            sl.stream.wait_stream(main)
        for sl, idx in zip(self.slots, self.assign):
            with torch.cuda.stream(sl.stream):
                for i in idx:
                    self._pose_forward(sl, self.poses[i])
        for sl in self.slots:
            main.wait_stream(sl.stream)

    def capture(self):
        self.graph = None
        self.render()  # warm-up
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.render()
        torch.cuda.synchronize()
        self.graph = g

    def time_ms(self, n=5):
        """ms per replay of the captured batch."""
        if self.graph is None:
            self.capture()
        self.render()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            self.render()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    # (rays per tile, samples per segment, waves per workgroup, workgroups per CU)
    PERSISTENT_CANDIDATES = ((16, 256, 4, 3), (12, 256, 4, 3), (8, 256, 4, 3), (32, 256, 4, 2), (16, 256, 4, 4),
                             (16, 256, 8, 1), (16, 256, 8, 2), (32, 256, 8, 2))

    def autotune(self, candidates=(1, 2, 4), n=3, persistent=None):
        """Time the captured batch for each schedule -- every stream count of
        the staged kernels and every (rays per tile, samples per segment,
        workgroups per CU) of the persistent kernel -- and keep the fastest;
        returns {schedule name: ms}."""
        if persistent is None:
            persistent = self.PERSISTENT_CANDIDATES if self.ri_dtype == K.BF16 else ()
        res, setters = {}, {}
        for c in candidates:
            name = f"staged/{c} streams"
            self.set_streams(c)
            res[name] = self.time_ms(n)
            setters[name] = (self.set_streams, (c,))
        for sched in persistent:
            name = "persistent/{} rays x {} samples, {} waves x {} wg per CU".format(*sched)
            self.set_persistent(*sched)
            try:
                res[name] = self.time_ms(n)
            except RuntimeError as e:  # a schedule the device cannot run (LDS per workgroup)
                if "status 3" not in str(e):
                    raise
                continue
            setters[name] = (self.set_persistent, sched)
        best = min(res, key=res.get)
        fn, a = setters[best]
        fn(*a)
        self.capture()
        self.schedule = best
        return res

    @property
    def total_samples(self):
        return sum(p.S for p in self.poses)
