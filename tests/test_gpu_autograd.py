"""The autograd front end: the training step written as a chain of
torch.autograd.Functions (march, deform with the IFT backward, encode, MLP,
composite, L2 loss) must give the explicit pipeline's results, which are
themselves held to the FP64 oracle by the stage and end-to-end tests.
Deterministic kernels must agree bit for bit; gradients accumulated with
atomics (table, skinning grid, and the bone gradient contracted from the
atomically accumulated grid moments) to summation-order rounding."""
import numpy as np
import pytest
import torch

from paper_2212_10550_amd import synth
from tests.gpu_util import host

pytestmark = pytest.mark.gpu


def _close(a, b, what, rtol=1e-5):
    a, b = host(a), host(b)
    err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
    assert err <= rtol, f"{what}: {err:.2e}"


def _leaf(t):
    return t.detach().clone().requires_grad_(True)


@pytest.mark.parametrize("mixed", [False, True])
def test_autograd_training_step_matches_pipeline(mixed):
    from paper_2212_10550_amd import autograd as A
    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.train_step()
    kw = dict(table_dtype=torch.float16, mlp_dtype=K.BF16) if mixed else {}
    p = Pipeline(w, **kw)
    S = p.train_step()
    torch.cuda.synchronize()

    xs, ray_off, ray_dt = A.march(p.rays_o, p.rays_d, p.occ_bits, p.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps)
    assert xs.shape[1] == S
    assert torch.equal(ray_off, p.ray_off) and torch.equal(xs, p.xs[:, :S])
    xp, B, W, table, params = (_leaf(t) for t in (xs, p.B, p.W, p.table32, p.params))
    dcfg = A.DeformConfig(tuple(w.skin_aabb), tuple(w.hash_aabb), w.max_iter, w.tol_stop, w.tol_valid)
    hcfg = A.HashConfig(w.base_res, w.growth, tuple(w.hash_aabb))
    xc, bone = A.snarf_deform(xp, B, W, dcfg)
    if mixed:
        sigma, rgb = A.canonical_field(xc, bone, table, params, hcfg, table_f16=p.table, mlp_dtype=K.BF16,
                                       feat_dtype=torch.bfloat16)
    else:
        feat = A.hash_encode(xc, bone, table, hcfg)
        sigma, rgb = A.mlp(feat, bone, params)
    color, opacity, n_used = A.volume_render(sigma, rgb, ray_off, ray_dt, w.T_thresh)
    loss = A.l2_loss(color, p.target)
    loss.backward()
    torch.cuda.synchronize()

    assert torch.equal(xc.detach(), p.xc[:, :S]) and torch.equal(bone, p.bone[:S])
    assert torch.equal(sigma.detach(), p.sigma[:S]) and torch.equal(rgb.detach(), p.rgb[:, :S])
    assert torch.equal(color.detach(), p.color) and torch.equal(loss.detach().view(1), p.loss)
    assert torch.equal(xp.grad, p.grad_xp[:, :S])
    assert torch.equal(params.grad, p.grad_params)
    _close(B.grad, p.grad_B, "grad_B")
    _close(table.grad, p.grad_table, "grad_table")
    _close(W.grad, p.grad_W, "grad_W")
    assert table.grad.dtype == torch.float32 and params.grad.dtype == torch.float32


def test_autograd_partial_requirements():
    """Only the inputs that require a gradient get one (the IFT still runs
    for the skinning grid when the points and bones are frozen)."""
    from paper_2212_10550_amd import autograd as A
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.ray_subset(synth.train_step(), np.arange(0, 8192, 8))
    p = Pipeline(w)
    S = p.train_step()
    torch.cuda.synchronize()
    xs, ray_off, ray_dt = A.march(p.rays_o, p.rays_d, p.occ_bits, p.G, w.occ_aabb, w.dt, w.n_per_ray, w.max_steps)
    W = _leaf(p.W)
    dcfg = A.DeformConfig(tuple(w.skin_aabb), tuple(w.hash_aabb), w.max_iter, w.tol_stop, w.tol_valid)
    hcfg = A.HashConfig(w.base_res, w.growth, tuple(w.hash_aabb))
    xc, bone = A.snarf_deform(xs, p.B, W, dcfg)
    sigma, rgb = A.canonical_field(xc, bone, p.table32, p.params, hcfg)
    color, _, _ = A.volume_render(sigma, rgb, ray_off, ray_dt, w.T_thresh)
    A.l2_loss(color, p.target).backward()
    assert S == xs.shape[1]
    _close(W.grad, p.grad_W, "grad_W")
