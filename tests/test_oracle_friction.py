"""Pins of the oracle's implicit (backward-Euler) friction step.

The friction ODE of the splitting (Eq. (3d); slip at the bed and Newtonian
bulk friction of the Sec. 3.4 closure) is linear in the momenta at the fixed
depth of the source step, so one backward-Euler step solves a small linear
system per moment block.  Checked against what the mathematics fixes:

* level 0: S = -C q / h, so q^{n+1} = q* h / (h + C dt) (scalar closed form);
* level 1: the 2x2 system (I - dt S) alpha^{n+1} = alpha*, S acting on alpha
  = [[-C, -C], [-3C, -3(C + 4 nu/h)]] / h, solved by Cramer's rule by hand;
* level 2 without slip: K is diagonal on moments 1, 2 (K_11 = 4, K_22 = 12,
  M_k = 1/(2k+1)), so each moment decays by 1 / (1 + dt nu K_kk / (M_k h^2));
* unconditional stability: far beyond the explicit limit (nu dt / h^2 a
  hundred times too large) the energy sum_k M_k alpha_k^2 falls in every step,
  while the explicit step blows up;
* consistency: one implicit and one explicit step differ by O(dt^2);
* with the flux active, the implicit step of the whole scheme equals the
  hyperbolic predictor followed by the cell-local solve.
"""
import numpy as np
import pytest

from oracle import mesh, sme


def uniform_1d(level, h, alpha, C, nu, implicit=1, n=8):
    m = mesh.mesh_1d(n, 0.0, 1.0, ("periodic", "periodic"))
    o = sme.Oracle(level, m, c_slip=C, nu=nu, implicit_friction=implicit)
    Q = np.zeros((level + 2, n))
    Q[0] = h
    Q[1:] = (h * np.asarray(alpha, float))[:, None]
    return o, Q


def test_level0_closed_form():
    C, h, u, dt = 1.0, 1.3, 0.7, 0.05
    o, Q = uniform_1d(0, h, [u], C, 0.1)
    q = h * u
    for _ in range(20):
        Q, _ = o.step(Q, dt)
        q = q * h / (h + C * dt)
    np.testing.assert_allclose(Q[1], q, rtol=1e-14)
    np.testing.assert_array_equal(Q[0], h)


@pytest.mark.parametrize("C,nu", [(1.0, 0.1), (0.0, 0.3), (2.0, 0.0)])
def test_level1_cramer(C, nu):
    h, dt = 0.9, 0.02
    a = np.array([0.5, -0.3])
    o, Q = uniform_1d(1, h, a, C, nu)
    # (I - dt S) a_new = a_old with S = [[s11, s12], [s21, s22]] on alpha
    s11, s12 = -C / h, -C / h
    s21, s22 = -3 * C / h, -3 * (C + 4 * nu / h) / h
    m11, m12, m21, m22 = 1 - dt * s11, -dt * s12, -dt * s21, 1 - dt * s22
    det = m11 * m22 - m12 * m21
    for _ in range(30):
        Q, _ = o.step(Q, dt)
        a = np.array([(a[0] * m22 - m12 * a[1]) / det, (m11 * a[1] - m21 * a[0]) / det])
    np.testing.assert_allclose(Q[1:, 0] / h, a, rtol=1e-13)


def test_level2_no_slip_modes_decay_independently():
    h, nu, dt = 0.6, 0.2, 0.01
    a = np.array([0.4, 0.3, -0.2])
    o, Q = uniform_1d(2, h, a, 0.0, nu)
    Q, _ = o.step(Q, dt)
    want = a / np.array([1.0, 1 + dt * nu * 4 * 3 / h ** 2, 1 + dt * nu * 12 * 5 / h ** 2])
    np.testing.assert_allclose(Q[1:, 0] / h, want, rtol=1e-14)


@pytest.mark.parametrize("level", [1, 3, 8])
def test_unconditional_energy_decay(level):
    """nu dt / h^2 = 1: far above the explicit limit (at level 8 the largest
    rate nu K/(M h^2) reaches thousands per second)."""
    h, nu, C = 0.5, 0.25, 1.0
    dt = 1.0
    rng = np.random.default_rng(level)
    a = rng.uniform(-0.5, 0.5, level + 1)
    M = 1.0 / (2 * np.arange(level + 1) + 1)
    o, Q = uniform_1d(level, h, a, C, nu)
    e = [np.sum(M * (Q[1:, 0] / h) ** 2)]
    for _ in range(10):
        Q, _ = o.step(Q, dt)
        e.append(np.sum(M * (Q[1:, 0] / h) ** 2))
    assert all(e2 < e1 for e1, e2 in zip(e, e[1:]))
    assert np.all(np.isfinite(Q))
    ox, Qx = uniform_1d(level, h, a, C, nu, implicit=0)
    for _ in range(3):
        Qx, _ = ox.step(Qx, dt)
    assert np.sum(M * (Qx[1:, 0] / h) ** 2) > 10 * e[0]


@pytest.mark.parametrize("level", [1, 4])
def test_consistent_with_explicit_step(level):
    """One step from the same state: implicit minus explicit is O(dt^2)."""
    h, nu, C = 1.1, 0.1, 1.0
    rng = np.random.default_rng(7)
    a = rng.uniform(-0.5, 0.5, level + 1)
    diffs = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        oi, Q = uniform_1d(level, h, a, C, nu, implicit=1)
        oe, _ = uniform_1d(level, h, a, C, nu, implicit=0)
        diffs.append(np.max(np.abs(oi.step(Q, dt)[0] - oe.step(Q, dt)[0])))
    r = [diffs[i] / diffs[i + 1] for i in range(2)]
    assert all(3.6 < x < 4.4 for x in r), (diffs, r)


def test_whole_step_is_predictor_then_solve():
    """2D triangles at level 3 with bathymetry: the implicit step of the whole
    scheme equals the hyperbolic predictor followed by the cell-local solve,
    and the depth is left to the predictor."""
    from paper_2601_04826_amd import workloads as W

    vert, tri = W.delaunay_unit_square(200, seed=3)
    m = mesh.mesh_tri(vert, tri)
    N = 3
    Q = W.random_state_2d(N, m.ncells, seed=4)
    b = 0.1 * np.cos(2 * m.centers[:, 1])
    o = sme.Oracle(N, m, b, c_slip=1.0, nu=0.1, implicit_friction=1)
    dt = 1e-3
    full, _ = o.step(Q, dt)
    pred = o.predict(Q, dt)
    for i in (0, 17, m.ncells - 1):
        want = o.friction_step(pred[:, i], dt)
        np.testing.assert_array_equal(full[:, i], want)
    np.testing.assert_array_equal(full[0], pred[0])
