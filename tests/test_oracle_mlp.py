"""Pins of the oracle's closure network: its hand-written reverse-mode gradient
against central finite differences, Adam against its closed formula, and the
zero-weight network (the closure then reduces to the plain level-1 step)."""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.NPARAM == 4930


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed) + 0.05 * rng.standard_normal(mlp.NPARAM)
    x = rng.standard_normal((16, mlp.NIN))
    t = rng.standard_normal((16, mlp.NOUT))
    loss, g = mlp.loss_grad(p, x, t)
    idx = rng.choice(mlp.NPARAM, 120, replace=False)
    idx = np.concatenate([idx, [0, 575, 576, 639, 640, 4735, 4736, 4799, 4800, 4927, 4928, 4929]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss_grad(p + e, x, t)[0] - mlp.loss_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, k


def test_loss_value_by_hand():
    p = np.zeros(mlp.NPARAM)
    W1, b1, W2, b2, W3, b3 = [a.copy() for a in mlp.unpack(p)]
    b3[:] = [0.5, -1.0]
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    x = np.ones((4, mlp.NIN))
    t = np.zeros((4, mlp.NOUT))
    loss, g = mlp.loss_grad(p, x, t)
    # y = b3 for every sample; L = 0.25 + 1.0; dL/db3 = 2 b3
    assert loss == pytest.approx(1.25, rel=1e-15)
    np.testing.assert_allclose(mlp.unpack(g)[5], [1.0, -2.0], rtol=1e-15)


def test_adam_closed_form_first_step():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    p1, m1, v1 = mlp.adam(p, g, m, v, 1, 1e-3)
    # first step: m_hat = g, v_hat = g^2, so p1 = p - lr g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_zero_network_outputs_zero():
    y, _ = mlp.forward(np.zeros(mlp.NPARAM), np.random.default_rng(0).standard_normal((7, mlp.NIN)))
    assert np.all(y == 0.0)


def test_features_periodic_differences():
    h = np.array([1.0, 2.0, 4.0])
    q0 = np.array([0.0, 1.0, 0.0])
    q1 = np.array([3.0, 3.0, 5.0])
    f = mlp.features_1d(h, q0, q1)
    np.testing.assert_array_equal(f[0], [1, 0, 3, 1, 1, 0, -3, 0, -2])
    np.testing.assert_array_equal(f[2], [4, 0, 5, -3, 0, -2, 2, -1, 2])
