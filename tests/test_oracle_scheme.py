"""Pins of the oracle's face scheme that the step invariants cannot see.

Lake at rest, mass conservation and the Stoker convergence order hold for any
positive Rusanov speed and for any quadrature of the path integral that is
exact at Delta h = 0, so the two choices below get pins of their own
(path-conservative Rusanov scheme, Sec. 2.1.2; the SME of Eq. (1)):

* the Rusanov speed of a face is the larger of the two cells' wave-speed bounds
  (local Lax-Friedrichs): a face between two states with clearly different
  bounds is compared with the textbook flux written out by hand;
* the non-conservative fluctuation is the integral along the straight path
  Q_i -> Q_j, taken with G-point Gauss-Legendre.  At level 1 the q_1 row of
  B(Q) is -alpha_0 = -q_0/h, so the fluctuation is -Delta q_1 times the integral
  of (a + b s)/(c + d s) over s in [0, 1], which has a closed form.  Three Gauss
  points differ from it by about 2.4e-5 relative for a 2:1 depth jump, one
  point (the midpoint) by about 2.5e-2.  With Delta h = 0 the integrand is linear in s
  and one point is already exact.

Every face value is read off the oracle's hyperbolic predictor on a two-cell
grid with extrapolation ends: cell 0 gets |e| (Fhat + NC/2) from its right face
and -F(Q_0) from the left one (the ghost is a copy, so that face carries the
cell's own flux and no fluctuation).
"""
import math

import numpy as np
import pytest

from oracle import mesh, sme

G = 9.81


def two_cells(level, qa, qb, quad_points=3, dx=1.0):
    """Oracle on [cell a | cell b] (1D, extrapolation ends, flat bed, no friction)."""
    m = mesh.mesh_1d(2, 0.0, 2.0 * dx, ("extrap", "extrap"))
    o = sme.Oracle(level, m, np.zeros(2), c_slip=0.0, nu=0.0, quad_points=quad_points)
    Q = np.stack([np.asarray(qa, float), np.asarray(qb, float)], axis=1)
    dt = 1e-3
    P = o.predict(Q, dt)
    acc = (Q - P) * dx / dt          # acc[:, c] = sum over faces of |e| (Fhat + NC/2) . n
    return o, acc


# --- textbook pieces written out by hand (not taken from the oracle) --------
def swe_flux(q):
    h, hu = q
    return np.array([hu, hu * hu / h + 0.5 * G * h * h])


def sme1_flux(q):
    """Level-1 SME flux (Eq. (1) with N = 1): (h u, h u^2 + h a^2/3 + g h^2/2, 2 h u a)."""
    h, q0, q1 = q
    u, a = q0 / h, q1 / h
    return np.array([h * u, h * u * u + h * a * a / 3 + 0.5 * G * h * h, 2 * h * u * a])


def log_integral(a, b, c, d):
    """int_0^1 (a + b s) / (c + d s) ds for c > 0, c + d > 0, d != 0."""
    return b / d + (a - b * c / d) * math.log1p(d / c) / d


def test_level0_face_is_textbook_rusanov():
    qi = np.array([2.0, 2.0 * 0.5])
    qj = np.array([1.0, 1.0 * -0.3])
    li = 0.5 + math.sqrt(G * 2.0)
    lj = 0.3 + math.sqrt(G * 1.0)
    assert li - lj > 1.0                # the two bounds differ clearly
    s = max(li, lj)
    fhat = 0.5 * (swe_flux(qi) + swe_flux(qj)) - 0.5 * s * (qj - qi)
    _, acc = two_cells(0, qi, qj)
    np.testing.assert_allclose(acc[:, 0], fhat - swe_flux(qi), rtol=1e-12, atol=1e-12)
    # and the other cell sees the same face value with the opposite sign
    np.testing.assert_allclose(acc[:, 1], swe_flux(qj) - fhat, rtol=1e-12, atol=1e-12)


def test_level0_face_speed_from_right_cell():
    """Same pin with the faster state on the right (the max must pick it)."""
    qi = np.array([1.0, 0.1])
    qj = np.array([1.6, 1.6 * -1.2])
    li = 0.1 + math.sqrt(G)
    lj = 1.2 + math.sqrt(G * 1.6)
    assert lj - li > 1.0
    fhat = 0.5 * (swe_flux(qi) + swe_flux(qj)) - 0.5 * lj * (qj - qi)
    _, acc = two_cells(0, qi, qj)
    np.testing.assert_allclose(acc[:, 0], fhat - swe_flux(qi), rtol=1e-12, atol=1e-12)


def test_level1_face_mass_and_mean_momentum():
    """Level 1: the h and q_0 rows carry no fluctuation on a flat bed, so they
    are the Rusanov flux of the level-1 system with s = max(lam_i, lam_j),
    lam = |u| + sqrt(g h + alpha_1^2) (exact at level 1)."""
    qi = np.array([2.0, 2.0 * 0.5, 2.0 * 0.2])
    qj = np.array([1.0, 1.0 * -0.3, 1.0 * -0.25])
    li = 0.5 + math.sqrt(G * 2.0 + 0.2 ** 2)
    lj = 0.3 + math.sqrt(G * 1.0 + 0.25 ** 2)
    s = max(li, lj)
    fhat = 0.5 * (sme1_flux(qi) + sme1_flux(qj)) - 0.5 * s * (qj - qi)
    _, acc = two_cells(1, qi, qj)
    np.testing.assert_allclose(acc[:2, 0], (fhat - sme1_flux(qi))[:2], rtol=1e-12, atol=1e-12)


def nc_q1_row(qi, qj, quad_points):
    """Fluctuation of the q_1 row of the face, from the two cells' predictor
    terms: acc_0 + acc_1 = F(Q_1) - F(Q_0) + NC (the Rusanov parts cancel)."""
    _, acc = two_cells(1, qi, qj, quad_points=quad_points)
    return acc[2, 0] + acc[2, 1] - (sme1_flux(qj)[2] - sme1_flux(qi)[2])


@pytest.mark.parametrize("hi,hj,tol3,tol8", [(2.0, 1.0, 1e-4, 1e-11), (1.0, 2.0, 1e-4, 1e-11),
                                           (3.0, 1.0, 5e-4, 1e-9)])
def test_level1_nc_fluctuation_is_the_path_integral(hi, hj, tol3, tol8):
    ui, uj = 0.5, 0.3                  # same sign: the integrand does not cancel
    ai, aj = 0.2, -0.25
    qi = np.array([hi, hi * ui, hi * ai])
    qj = np.array([hj, hj * uj, hj * aj])
    exact = -(qj[2] - qi[2]) * log_integral(qi[1], qj[1] - qi[1], hi, hj - hi)
    rel = {G_: abs(nc_q1_row(qi, qj, G_) - exact) / abs(exact) for G_ in (1, 3, 8)}
    # three Gauss points: the degree-5 rule on a function analytic near [0, 1]
    # (2.4e-5 for 2:1, 2.0e-4 for 3:1), not exact; the midpoint is off by >1e-2
    assert 1e-7 < rel[3] < tol3, rel
    assert rel[1] > 1e-2, rel
    # the error falls as the rule grows (8 points: near round-off)
    assert rel[8] < tol8, rel


def test_level1_nc_flat_depth_exact_for_any_rule():
    """Delta h = 0: alpha_0 is linear along the path, the integrand is linear in
    s and every Gauss rule (one point included) gives the exact average."""
    qi = np.array([1.5, 1.5 * 0.4, 1.5 * 0.3])
    qj = np.array([1.5, 1.5 * -0.6, 1.5 * 0.1])
    exact = -(qj[2] - qi[2]) * 0.5 * (qi[1] + qj[1]) / 1.5
    for G_ in (1, 2, 3, 5):
        assert nc_q1_row(qi, qj, G_) == pytest.approx(exact, rel=1e-12, abs=1e-14)


def test_level2_flat_depth_rules_agree():
    """Level 2, Delta h = 0 on a 2D face: B(Phi(s)) is linear in s, so one and
    three Gauss points give the same predictor to round-off."""
    m = mesh.mesh_2d_struct(3, 2, 0.0, 1.0, 0.0, 1.0, ("extrap",) * 4)
    rng = np.random.default_rng(12)
    Q = np.zeros((7, 6))
    Q[0] = 1.3
    Q[1:] = 1.3 * rng.uniform(-0.4, 0.4, size=(6, 6))
    P = []
    for G_ in (1, 3):
        o = sme.Oracle(2, m, np.zeros(6), c_slip=0.0, nu=0.0, quad_points=G_)
        P.append(o.predict(Q, 1e-3))
    np.testing.assert_allclose(P[0], P[1], rtol=1e-13, atol=1e-15)
