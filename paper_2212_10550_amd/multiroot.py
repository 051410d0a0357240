"""Multi-root aggregation on the GPU: the march of `Pipeline`, every distinct
valid root of each sample (up to K), the density and colour of each root
(one encode + MLP pass over the K slots), the root with the largest density
per sample, then compositing.  The chosen roots, their features, densities
and colours land in the pipeline's buffers, so `Pipeline.backward` gives the
gradients through them (the derivative of a maximum is the chosen root's).

Host sample counts: the K slots of the expanded batch are laid out per
count, so the buffers are sized after the march.
"""
from __future__ import annotations

import torch

from . import lib as K
from .pipeline import Pipeline


class MaxDensityRenderer:
    def __init__(self, w, K_roots=4, dup_tol=1e-4, device="cuda", **kw):
        self.p = Pipeline(w, device=device, device_count=False, **kw)
        self.K = K_roots
        self.dup_tol = dup_tol
        self.S = None
        self._bufs = None

    def _buffers(self, S):
        """Expanded-batch buffers of exactly K S slots (reused while S holds)."""
        if self._bufs is not None and self._bufs[0] == S:
            return self._bufs[1]
        p, n = self.p, max(S, 1) * self.K
        e = lambda *shape, dt=torch.float32: torch.empty(*shape, dtype=dt, device=p.dev)
        b = dict(roots=e(3, n), rbone=e(n, dt=torch.int16), nroots=e(max(S, 1), dt=torch.int32),
                 feat=e(p.w.L * n * 2, dt=p.feat_dtype), sig=e(n), rgb=e(3, n))
        self._bufs = (S, b)
        return b

    def forward(self):
        p, w, Kr = self.p, self.p.w, self.K
        p.march()
        S = p.read_count()
        b = self._buffers(S)
        KS = Kr * max(S, 1)
        K.snarf_deform_roots(p.xs, S, p.cap, p.B, p.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop, w.tol_valid,
                             Kr, self.dup_tol, b["roots"], b["rbone"], b["nroots"], p.ws_deform)
        if S > 0:
            K.hashgrid_encode(b["roots"], b["rbone"], KS, KS, p.table, w.base_res, w.growth, w.hash_aabb, b["feat"])
            K.mlp_fwd(b["feat"], b["rbone"], KS, KS, p.params, p.mlp_dtype, b["sig"], b["rgb"])
        K.select_max_density(Kr, S, b["sig"], b["rgb"], b["roots"], b["rbone"], b["nroots"], p.cap, p.xc, p.bone,
                             p.sigma, p.rgb)
        # features of the chosen roots, for the backward
        K.hashgrid_encode(p.xc, p.bone, S, p.cap, p.table, w.base_res, w.growth, w.hash_aabb, p.feat)
        p._render()
        p._last = (S, None)
        self.S = S
        self._b = b
        return S

    def n_roots(self):
        return self._b["nroots"][:self.S]

    def roots(self):
        """[3][K][S] view of the kept roots."""
        return self._b["roots"].view(3, self.K, -1)[:, :, :self.S]
