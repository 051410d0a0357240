"""Pins of the oracle's full loss set (Sec. 3.4) and Adam step."""
import numpy as np

import oracle as orc


def test_huber_closed_forms():
    d = 0.1
    np.testing.assert_allclose(orc.huber([0.0, 0.05, 0.1, 0.3], d), [0.0, 0.00125, 0.005, 0.1 * (0.3 - 0.05)])
    # continuous value and slope at the threshold
    e = 1e-9
    assert abs(orc.huber(d + e, d) - orc.huber(d - e, d)) < 1e-9


def test_hard_surface_minima_and_symmetry():
    assert abs(orc.hard_surface(0.0)) < 1e-15 and abs(orc.hard_surface(1.0)) < 1e-15
    a = np.linspace(-0.5, 1.5, 41)
    np.testing.assert_allclose(orc.hard_surface(a), orc.hard_surface(1.0 - a), atol=1e-15)
    assert (orc.hard_surface(np.array([0.25, 0.5, 0.75])) > 0).all()
    # value at 1/2: -log(2 exp(-1/2)) + log(1 + exp(-1))
    assert abs(orc.hard_surface(0.5) - (-np.log(2 * np.exp(-0.5)) + np.log(1 + np.exp(-1)))) < 1e-15


def test_loss_full_gradients_by_finite_differences():
    rng = np.random.default_rng(0)
    R = 12
    C = rng.random((R, 3))
    T = rng.random((R, 3))
    T[:4] = C[:4] + 0.01 * rng.standard_normal((4, 3))  # quadratic Huber region
    A = rng.uniform(0.05, 0.95, R)
    Ag = (rng.random(R) < 0.5).astype(float)
    args = (0.1, 0.3, 0.2)
    loss, gC, gA = orc.loss_full(C, A, T, Ag, *args)
    eps = 1e-6
    for i in range(R):
        for c in range(3):
            Cp, Cm = C.copy(), C.copy()
            Cp[i, c] += eps
            Cm[i, c] -= eps
            fd = (orc.loss_full(Cp, A, T, Ag, *args)[0] - orc.loss_full(Cm, A, T, Ag, *args)[0]) / (2 * eps)
            assert abs(fd - gC[i, c]) < 1e-8
        Ap, Am = A.copy(), A.copy()
        Ap[i] += eps
        Am[i] -= eps
        fd = (orc.loss_full(C, Ap, T, Ag, *args)[0] - orc.loss_full(C, Am, T, Ag, *args)[0]) / (2 * eps)
        assert abs(fd - gA[i]) < 1e-8
    # the pieces add up
    r = np.linalg.norm(C - T, axis=1)
    ref = (orc.huber(r, 0.1).sum() + 0.3 * np.abs(A - Ag).sum() + 0.2 * orc.hard_surface(A).sum()) / R
    assert abs(loss - ref) < 1e-15


def test_adam_closed_forms():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    z = np.zeros(4)
    # first step: m_hat = g, v_hat = g^2, so the update is lr g / (|g| + eps)
    p1, m1, v1 = orc.adam_step(p, g, z, z, 1, 0.01, 0.9, 0.99, 1e-8)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.01 * g * g)
    # second step with the same gradient: moments by hand
    p2, m2, v2 = orc.adam_step(p1, g, m1, v1, 2, 0.01, 0.9, 0.99, 1e-8)
    m_ref = 0.9 * 0.1 * g + 0.1 * g
    v_ref = 0.99 * 0.01 * g * g + 0.01 * g * g
    np.testing.assert_allclose(m2, m_ref)
    np.testing.assert_allclose(v2, v_ref)
    np.testing.assert_allclose(p2, p1 - 0.01 * (m_ref / 0.19) / (np.sqrt(v_ref / (1 - 0.99 ** 2)) + 1e-8), rtol=1e-14)
