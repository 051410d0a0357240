"""A training loop of the path on one GPU: the step of `Pipeline` (march,
deform, encode, MLP, composite, the loss of Sec. 3.4, every backward) plus
the Adam update of the hash table and the MLP, captured as one HIP graph,
and every k steps an update of the shared training occupancy grid
(Sec. 3.3) at random points of a random subset of its cells, which the next
steps' march reads.

Random numbers the method draws (the jitter of the occupancy update) come
from a seeded pool drawn once on the host and kept in HBM.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lib as K
from .pipeline import Pipeline


class Trainer:
    def __init__(self, w, lr=1e-2, betas=(0.9, 0.99), eps=1e-15, table_dtype=torch.float32, mlp_dtype=K.F32,
                 alpha_gt=None, loss_args=(0.1, 0.1, 0.01), occ_every=16, occ_beta=0.95, occ_thresh=0.01,
                 occ_dilate=1, occ_fraction=0.125, jitter_pool=8, seed=0, device="cuda"):
        self.p = Pipeline(w, device=device, table_dtype=table_dtype, mlp_dtype=mlp_dtype, device_count=True)
        p = self.p
        if alpha_gt is not None or loss_args is not None:
            p.set_full_loss(alpha_gt, *(loss_args or (0.1, 0.1, 0.01)))
        dev = p.dev
        self.lr, self.betas, self.eps = lr, betas, eps
        z = lambda t: torch.zeros_like(t, dtype=torch.float32)
        self.m_t, self.v_t = z(p.table32), z(p.table32)
        self.m_p, self.v_p = z(p.params), z(p.params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.f16 = p.table if p.table.dtype == torch.float16 else None
        # shared occupancy grid: values start at the workload's grid (occupied
        # cells above the threshold), then follow the field's densities
        self.occ_every = occ_every
        self.occ_beta, self.occ_thresh, self.occ_dilate = occ_beta, occ_thresh, occ_dilate
        self.steps_done = 0
        self.G = p.G
        if self.G and occ_every:
            G = self.G
            occ = torch.as_tensor(np.ascontiguousarray(w.occ), device=dev, dtype=torch.float32).reshape(-1)
            self.occ_values = occ * (2.0 * occ_thresh)
            rng = np.random.default_rng(seed)
            # each update refreshes a random subset of the cells (sorted, so
            # neighbouring points stay close), jittered inside each cell
            M = G ** 3 if occ_fraction >= 1.0 else max(1, int(G ** 3 * occ_fraction))
            self.cells = None if M == G ** 3 else torch.as_tensor(
                np.stack([np.sort(rng.choice(G ** 3, M, replace=False)) for _ in range(jitter_pool)]).astype(
                    np.int32), device=dev)
            self.jitter = torch.as_tensor(rng.random((jitter_pool, 3, M), dtype=np.float32) * np.float32(0.999),
                                          device=dev)
            Dz, Dy, Dx, nb = w.W.shape
            self.ws_occ = torch.empty(K.occgrid_build_workspace_size(G, w.L, 2, p.mlp_dtype, Dx, Dy, Dz),
                                      dtype=torch.uint8, device=dev)
        self.graph = None

    def _optimizer(self):
        p = self.p
        b1, b2 = self.betas
        K.count_step(self.step_dev)
        K.adam(p.table32.view(-1), p.grad_table.view(-1), self.m_t.view(-1), self.v_t.view(-1), self.lr, b1, b2,
               self.eps, step_dev=self.step_dev, param_f16=None if self.f16 is None else self.f16.view(-1))
        K.adam(p.params, p.grad_params, self.m_p, self.v_p, self.lr, b1, b2, self.eps, step_dev=self.step_dev)

    def _step(self):
        self.p.forward(zero_table=True)
        self.p.backward()
        self._optimizer()

    def capture(self):
        """Capture the step; the capture's warm-up runs one real step."""
        self.p._capture(self._step, "trainer")
        self.graph = self.p.graph
        self.steps_done += 1

    def occupancy_update(self):
        """One moving-average update of the shared grid (Sec. 3.3) in the
        posed space of this workload's frame, jitter from the pool."""
        p, w = self.p, self.p.w
        i = (self.steps_done // max(self.occ_every, 1)) % self.jitter.shape[0]
        K.occgrid_update(self.G, w.occ_aabb, self.jitter[i], p.B, p.W, w.skin_aabb, w.hash_aabb, w.max_iter,
                         w.tol_stop, w.tol_valid, p.table, w.base_res, w.growth, p.params, p.mlp_dtype,
                         self.occ_beta, self.occ_thresh, self.occ_dilate, self.occ_values, p.occ_bits, self.ws_occ,
                         cells=None if self.cells is None else self.cells[i])

    def step(self):
        """One training step (graph replay once captured); every occ_every
        steps the occupancy grid is updated first."""
        if self.occ_every and self.G and self.steps_done % self.occ_every == 0 and self.steps_done > 0:
            self.occupancy_update()
        if self.graph is not None:
            self.graph.replay()
        else:
            self._step()
        self.steps_done += 1

    def loss_value(self):
        return float((self.p.loss if self.p.full_loss is None else self.p.loss4[0]).item())
