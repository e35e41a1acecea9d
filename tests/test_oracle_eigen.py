"""Pins of the oracle's flux, non-conservative matrix and wave-speed bound.

The quasilinear matrix of the paper (Sec. 2.1.1: A.n = (dF/dQ + N).n) is built
from the oracle's flux (central differences) and its NC matrix.  Its spectrum
is checked against closed forms that do not come from the oracle:

* level 0 is the shallow water system (Sec. 3.1): u.n and u.n +- sqrt(g h);
* level 1 (1D): u, u +- sqrt(g h + alpha_1^2);
* any level at states with alpha_j = 0 for j >= 2: u +- sqrt(g h + alpha_1^2)
  and u + alpha_1 x_m with x_m the roots of P'_{N+1} (known eigenstructure of the
  SME at linear velocity profiles);
* the speed bound used for CFL and Rusanov is exact at levels 0/1 and never
  below the largest |Re lambda| on random states (levels 2..4, 1D and 2D).
"""
import numpy as np
import pytest

from oracle import mesh, sme

G = 9.81


def quasilinear(o, q, nx, ny=0.0):
    nf = o.nf
    J = np.zeros((nf, nf))
    for c in range(nf):
        e = np.zeros(nf)
        hh = 1e-6 * max(1.0, abs(q[c]))
        e[c] = hh
        J[:, c] = (o.flux(q + e, nx, ny) - o.flux(q - e, nx, ny)) / (2 * hh)
    return J + o.ncmat(q, nx, ny)[:, :nf]


def o1d(N):
    return sme.Oracle(N, mesh.mesh_1d(4, 0.0, 1.0))


def o2d(N):
    return sme.Oracle(N, mesh.mesh_2d_struct(2, 2, 0.0, 1.0, 0.0, 1.0))


def test_level0_flux_is_swe_flux():
    o = o2d(0)
    h, u, v = 1.7, 0.3, -0.8
    q = np.array([h, h * u, h * v])
    np.testing.assert_allclose(o.flux(q, 1.0, 0.0), [h * u, h * u * u + 0.5 * G * h * h, h * u * v], rtol=1e-15)
    np.testing.assert_allclose(o.flux(q, 0.0, 1.0), [h * v, h * u * v, h * v * v + 0.5 * G * h * h], rtol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_level0_eigenvalues(seed):
    rng = np.random.default_rng(seed)
    o = o2d(0)
    h = rng.uniform(0.5, 2.0)
    u, v = rng.uniform(-1, 1, 2)
    th = rng.uniform(0, 2 * np.pi)
    nx, ny = np.cos(th), np.sin(th)
    un = u * nx + v * ny
    ev = np.sort(np.linalg.eigvals(quasilinear(o, np.array([h, h * u, h * v]), nx, ny)).real)
    c = np.sqrt(G * h)
    np.testing.assert_allclose(ev, [un - c, un, un + c], atol=1e-7)
    assert o.lam(np.array([h, h * u, h * v]), nx, ny) == pytest.approx(abs(un) + c, rel=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_level1_eigenvalues_1d(seed):
    rng = np.random.default_rng(seed)
    o = o1d(1)
    h = rng.uniform(0.5, 2.0)
    u, a1 = rng.uniform(-1, 1, 2)
    q = np.array([h, h * u, h * a1])
    ev = np.sort(np.linalg.eigvals(quasilinear(o, q, 1.0)).real)
    c = np.sqrt(G * h + a1 * a1)
    np.testing.assert_allclose(ev, [u - c, u, u + c], atol=1e-7)
    assert o.lam(q, 1.0) == pytest.approx(abs(u) + c, rel=1e-14)


@pytest.mark.parametrize("N", range(1, 7))
def test_linear_profile_eigenvalues(N):
    o = o1d(N)
    h, u, a1 = 1.3, 0.4, 0.7
    q = np.zeros(N + 2)
    q[0], q[1], q[2] = h, h * u, h * a1
    ev = np.sort(np.linalg.eigvals(quasilinear(o, q, 1.0)).real)
    roots = np.polynomial.legendre.Legendre.basis(N + 1).deriv().roots()
    c = np.sqrt(G * h + a1 * a1)
    want = np.sort(np.concatenate([[u - c, u + c], u + a1 * roots]))
    np.testing.assert_allclose(ev, want, atol=1e-7)
    # the bound is the exact spectral radius here
    assert o.lam(q, 1.0) == pytest.approx(abs(u) + c, rel=1e-14)


@pytest.mark.parametrize("N", [0, 1])
def test_bound_exact_2d_levels01(N):
    rng = np.random.default_rng(10 + N)
    o = o2d(N)
    for _ in range(20):
        h = rng.uniform(0.5, 2.0)
        q = np.concatenate([[h], h * rng.uniform(-1, 1, o.nf - 1)])
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        ev = np.linalg.eigvals(quasilinear(o, q, nx, ny))
        assert np.max(np.abs(ev.imag)) < 1e-6
        assert o.lam(q, nx, ny) == pytest.approx(np.max(np.abs(ev.real)), rel=1e-7)


@pytest.mark.parametrize("N,dim", [(2, 1), (3, 1), (4, 1), (2, 2), (3, 2), (4, 2)])
def test_bound_dominates_spectrum(N, dim):
    rng = np.random.default_rng(100 * N + dim)
    o = o1d(N) if dim == 1 else o2d(N)
    for _ in range(200):
        h = rng.uniform(0.3, 2.0)
        q = np.zeros(o.nf)
        q[0] = h
        n = N + 1
        q[1] = h * rng.uniform(-1.5, 1.5)
        for k in range(1, n):
            q[1 + k] = h * rng.uniform(-1, 1) / k
        if dim == 2:
            q[1 + n] = h * rng.uniform(-1.5, 1.5)
            for k in range(1, n):
                q[1 + n + k] = h * rng.uniform(-1, 1) / k
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = (np.cos(th), np.sin(th)) if dim == 2 else (1.0, 0.0)
        ev = np.linalg.eigvals(quasilinear(o, q, nx, ny))
        assert o.lam(q, nx, ny) >= np.max(np.abs(ev.real)) * (1 - 1e-7)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_nc_term_matches_depth_integral(N):
    """B(Q) dQ/dx against the vertical-advection integral it comes from:
    row k of the x-momentum equation carries (1/M_k) * (-int_0^1 u (h omega) phi_k' dzeta)
    with h omega = -sum_{j>=1} d(h alpha_j)/dx Phi_j(zeta) (mass balance in
    sigma-coordinates, Eq. (1)), evaluated here by direct quadrature in zeta."""
    rng = np.random.default_rng(N)
    o = o1d(N)
    L = np.polynomial.legendre
    x, w = L.leggauss(30)
    wz = 0.5 * w
    n = N + 1
    eye = np.eye(n)
    phi = np.array([L.legval(x, eye[k]) for k in range(n)])
    dphi = np.array([-2.0 * L.legval(x, L.legder(eye[k])) for k in range(n)])
    Qi = [L.legint(eye[k]) for k in range(n)]
    Phi = np.array([-0.5 * (L.legval(x, Qi[k]) - L.legval(1.0, Qi[k])) for k in range(n)])
    for _ in range(5):
        h = rng.uniform(0.5, 2)
        al = rng.uniform(-1, 1, n)
        q = np.concatenate([[h], h * al])
        dq = rng.uniform(-1, 1, n + 1)          # d/dx of (h, q_0..q_N)
        u = al @ phi
        hw = -(dq[2:] @ Phi[1:])
        want = np.array([-(u * hw * dphi[k]) @ wz * (2 * k + 1) for k in range(n)])
        got = o.ncmat(q, 1.0)[:, : o.nf] @ dq
        np.testing.assert_allclose(got[0], 0.0, atol=1e-14)
        np.testing.assert_allclose(got[1:], want, atol=1e-12)
