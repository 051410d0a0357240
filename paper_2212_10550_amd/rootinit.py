"""Learned root initialiser: data from the library's own multi-init solver,
an offline fit, and the guided solve used at render time.

Data: for each seeded pose, posed points are sampled around the posed
bones and ``ia355_snarf_deform`` (24 inits) finds their canonical roots.
The target bone is the init whose start B_k^{-1} x' lies nearest the root
(so the regressed offset x* - B_k^{-1} x' is the smallest one available);
the target offset is that difference.

Fit: the 15,387-parameter MLP of ``ia355_rootinit_fwd`` is trained offline
with cross-entropy on the bone logits plus a weighted squared error on the
offset, Adam, in FP32 torch ops on the GPU.  This is a one-time preparation
of an input of the path (like the hash table's values), not part of it; the
path itself runs the fitted weights in ``ia355_rootinit_fwd`` (BF16 or FP32
MFMA) and ``ia355_snarf_deform_guided``.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import lib as K
from . import synth

HIDDEN = 64


def _deform_roots(xp_np, B_np, W_t, w, dev):
    S = xp_np.shape[0]
    Dz, Dy, Dx, nb = W_t.shape
    xp = torch.as_tensor(np.ascontiguousarray(xp_np.T), device=dev)
    B = torch.as_tensor(B_np, device=dev)
    xc = torch.empty(3, S, device=dev)
    bone = torch.empty(S, dtype=torch.int16, device=dev)
    ws = torch.empty(K.deform_workspace_size(Dx, Dy, Dz), dtype=torch.uint8, device=dev)
    K.snarf_deform(xp, S, S, B, W_t, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop, w.tol_valid, xc, bone, None,
                   None, ws)
    return xc.T.contiguous(), bone


def make_dataset(pose_seeds, n_per_pose: int, device="cuda", w=None, point_seed: int = 0):
    """(posed point, pose, root) triples for the given pose seeds; returns
    torch tensors on ``device``: xp [N,3], pose [N,nb*6] (index per pose),
    B per pose, root [N,3], target bone [N], target offset [N,3]."""
    dev = torch.device(device)
    w = synth.train_step() if w is None else w
    skel = synth.make_skeleton(0)
    W_t = torch.as_tensor(w.W, device=dev)
    xs, poses, roots, bones, offs, pidx, Bs = [], [], [], [], [], [], []
    for k, seed in enumerate(pose_seeds):
        pose = synth.make_pose(skel, int(seed))
        B32 = pose.B.astype(np.float32)
        xp = synth.sample_posed_points(skel, pose.B, n_per_pose, seed=point_seed * 100003 + int(seed))
        xc, bone = _deform_roots(xp, B32, W_t, w, dev)
        ok = bone >= 0
        xp_t = torch.as_tensor(xp, device=dev)[ok]
        xc = xc[ok]
        Bt = torch.as_tensor(B32, device=dev)
        Minv = torch.linalg.inv(Bt[:, :, :3].double()).float()
        # every bone's start B_b^{-1} x' for every point: [n, nb, 3]
        start = torch.einsum("bij,nbj->nbi", Minv, xp_t[:, None, :] - Bt[None, :, :, 3])
        d = (start - xc[:, None, :]).norm(dim=-1)
        kb = d.argmin(1)
        xs.append(xp_t)
        roots.append(xc)
        bones.append(kb)
        offs.append(xc - start[torch.arange(len(kb), device=dev), kb])
        pidx.append(torch.full((len(kb),), k, device=dev, dtype=torch.long))
        poses.append(torch.as_tensor(pose.params.astype(np.float32).reshape(-1), device=dev))
        Bs.append(Bt)
    return dict(xp=torch.cat(xs), root=torch.cat(roots), bone=torch.cat(bones), off=torch.cat(offs),
                pose_index=torch.cat(pidx), pose=torch.stack(poses), B=torch.stack(Bs))


def _unflat(p, nb, hidden=HIDDEN):
    widths = (3 + 6 * nb, hidden, hidden, nb + 3)
    out, o = [], 0
    for l in range(3):
        fi, fo = widths[l], widths[l + 1]
        out.append((p[o:o + fi * fo].view(fo, fi), p[o + fi * fo:o + fi * fo + fo]))
        o += fi * fo + fo
    return out


def _forward(params, x, nb):
    h = x
    for l, (Wl, bl) in enumerate(_unflat(params, nb)):
        h = h @ Wl.t() + bl
        if l < 2:
            h = torch.relu(h)
    return h[:, :nb], h[:, nb:]


def fit(data, nb: int = synth.NB, epochs: int = 30, batch: int = 8192, lr: float = 2e-3, offset_weight: float = 1e3,
        seed: int = 11, log=None):
    """Fit the initialiser; returns the flat FP32 parameter vector (numpy)."""
    dev = data["xp"].device
    g = torch.Generator(device="cpu").manual_seed(seed)
    params = torch.as_tensor(synth.make_rootinit_params(nb, HIDDEN, seed), device=dev, dtype=torch.float32)
    params.requires_grad_(True)
    opt = torch.optim.Adam([params], lr=lr)
    N = data["xp"].shape[0]
    steps = epochs * math.ceil(N / batch)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(dev)
        tot = 0.0
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch]
            x = torch.cat([data["xp"][idx], data["pose"][data["pose_index"][idx]]], 1)
            logits, off = _forward(params, x, nb)
            loss = torch.nn.functional.cross_entropy(logits, data["bone"][idx]) + \
                offset_weight * ((off - data["off"][idx]) ** 2).sum(1).mean()
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            sched.step()
            tot += float(loss.detach()) * len(idx)
        if log:
            log(f"rootinit epoch {ep}: loss {tot / N:.5f}")
    return params.detach().cpu().numpy().astype(np.float32)


class GuidedDeform:
    """Device buffers for rootinit_fwd + snarf_deform_guided on a pose."""

    def __init__(self, params_np, w, cap, device="cuda", dtype=K.BF16):
        dev = torch.device(device)
        self.w = w
        self.dtype = dtype
        self.params = torch.as_tensor(params_np, device=dev)
        self.cap = cap
        Dz, Dy, Dx, nb = w.W.shape
        self.init_bone = torch.empty(cap, dtype=torch.int16, device=dev)
        self.x0 = torch.empty(3, cap, device=dev)
        self.n_fallback = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = torch.empty(K.deform_guided_workspace_size(cap, Dx, Dy, Dz), dtype=torch.uint8, device=dev)

    def run(self, xp, S, ld, pose_t, B, W, xc, bone, resid, steps, S_dev=None):
        w = self.w
        K.rootinit_fwd(xp, S, ld, pose_t, self.params, B, self.dtype, self.init_bone, self.x0, S_dev=S_dev)
        K.snarf_deform_guided(xp, S, ld, self.x0, self.init_bone, B, W, w.skin_aabb, w.hash_aabb, w.max_iter,
                              w.tol_stop, w.tol_valid, xc, bone, resid, steps, self.n_fallback, self.ws, S_dev=S_dev)
