"""The training loss of Sec. 3.4 and the Adam update against the FP64
oracle (FP32 bar: 1e-5 relative)."""
import numpy as np
import pytest
import torch

import oracle as orc
from tests.gpu_util import dev, host, up

pytestmark = pytest.mark.gpu


def _K():
    from paper_2212_10550_amd import lib as K
    return K


@pytest.mark.parametrize("with_alpha", [True, False])
def test_loss_full_matches_oracle(with_alpha):
    K = _K()
    R = 8197
    rng = np.random.default_rng(1)
    C = rng.random((R, 3)).astype(np.float32)
    T = rng.random((R, 3)).astype(np.float32)
    T[::3] = (C[::3] + 0.01 * rng.standard_normal((len(C[::3]), 3))).astype(np.float32)  # Huber quadratic part
    A = rng.uniform(0.0, 1.0, R).astype(np.float32)
    Ag = (rng.random(R) < 0.5).astype(np.float32)
    loss = torch.full((4,), float("nan"), device=dev())
    gC = torch.full((R, 3), float("nan"), device=dev())
    gA = torch.full((R,), float("nan"), device=dev())
    args = (0.1, 0.3, 0.05)
    K.loss_full(up(C), up(A), up(T), up(Ag) if with_alpha else None, *args, loss, gC, gA)
    torch.cuda.synchronize()
    rl, rC, rA = orc.loss_full(C, A, T, Ag, args[0], args[1] if with_alpha else 0.0, args[2])
    got = host(loss)
    assert abs(got[0] - rl) <= 1e-5 * abs(rl)
    r = np.linalg.norm(C.astype(np.float64) - T, axis=1)
    assert abs(got[1] - orc.huber(r, 0.1).mean()) <= 1e-5 * got[1]
    assert abs(got[3] - 0.05 * orc.hard_surface(A.astype(np.float64)).mean()) <= 1e-5 * got[3]
    if not with_alpha:
        assert got[2] == 0.0
    for g, ref, what in ((host(gC), rC, "dL/dC"), (host(gA), rA, "dL/dA")):
        err = np.abs(g - ref).max() / np.abs(ref).max()
        assert err <= 1e-5, (what, err)


@pytest.mark.parametrize("device_step,n", [(False, 100003), (True, 100003), (False, 100004), (True, 100004)])
def test_adam_matches_oracle(device_step, n):
    """An odd and a multiple-of-4 parameter count."""
    K = _K()
    rng = np.random.default_rng(2)
    p = rng.standard_normal(n).astype(np.float32)
    g = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    g[::7] = 0.0
    m = (rng.standard_normal(n) * 1e-4).astype(np.float32)
    v = (rng.random(n) * 1e-6).astype(np.float32)
    P, M, V = up(p), up(m), up(v)
    p16 = torch.empty(n, dtype=torch.float16, device=dev())
    lr, b1, b2, eps = 1e-2, 0.9, 0.99, 1e-15
    if device_step:
        t = torch.tensor([2], dtype=torch.int32, device=dev())
        K.count_step(t)  # this step is t = 3
        K.adam(P, up(g), M, V, lr, b1, b2, eps, step_dev=t, param_f16=p16)
    else:
        K.adam(P, up(g), M, V, lr, b1, b2, eps, step=3, param_f16=p16)
    torch.cuda.synchronize()
    rp, rm, rv = orc.adam_step(p, g, m, v, 3, lr, b1, b2, eps)
    # FP32 rounding of b1 m + (1 - b1) g is relative to the terms, not to the
    # (possibly cancelled) result: absolute bar at the moments' scale
    np.testing.assert_allclose(host(M), rm, rtol=1e-6, atol=2e-7 * np.abs(rm).max())
    np.testing.assert_allclose(host(V), rv, rtol=1e-6, atol=2e-7 * np.abs(rv).max())
    # the update is of size ~lr: compare the step taken
    step_ref = rp - p
    step_got = host(P) - p.astype(np.float64)
    assert np.abs(step_got - step_ref).max() <= 1e-5 * lr + 1e-6 * np.abs(p).max()
    assert torch.equal(p16, P.half())
    if device_step:
        assert int(t.item()) == 3
