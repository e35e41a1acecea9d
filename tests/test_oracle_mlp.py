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


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each
    step moves every parameter by lr g / (|g| + eps): pins the corrections'
    powers of t beyond the first step."""
    rng = np.random.default_rng(4)
    p = rng.standard_normal(40)
    g = rng.standard_normal(40)
    m = np.zeros(40)
    v = np.zeros(40)
    lr = 2e-3
    for t in range(1, 6):
        p_next, m, v = mlp.adam(p, g, m, v, t, lr)
        np.testing.assert_allclose(p - p_next, lr * g / (np.abs(g) + 1e-8), rtol=1e-9)
        np.testing.assert_allclose(m, (1.0 - 0.9 ** t) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1.0 - 0.999 ** t) * g * g, rtol=1e-12)
        p = p_next


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


def test_closure_target_turns_level1_step_into_level8():
    """The target is the rate of q_0, q_1 that, added over one step to the
    level-1 step from the level-8 state, gives the level-8 result: level-1
    step + dt * target = level-8 next state (up to rounding), whatever the
    level-8 state before the step."""
    rng = np.random.default_rng(5)
    n, dt = 33, 1e-3
    q8_now = rng.uniform(0.5, 1.5, (10, n))
    q8_next = q8_now + rng.uniform(-0.01, 0.01, (10, n))
    q1_step = q8_now[:4] + rng.uniform(-0.01, 0.01, (4, n))
    t = mlp.closure_target(q8_now, q8_next, q1_step, dt)
    assert t.shape == (n, 2)
    np.testing.assert_allclose(q1_step[1:3] + dt * t.T, q8_next[1:3], rtol=0, atol=1e-14)
