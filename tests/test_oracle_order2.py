"""Pins of the oracle's second-order scheme (limited reconstruction, in-cell
path fluctuation, two-stage SSP Runge-Kutta), on 1D and structured grids.

* smooth periodic level-1 flow (non-conservative products active): the error
  against a reference of a *different* scheme (Richardson extrapolation of the
  first-order scheme on 2048 and 4096 cells) falls at second order; dropping
  the in-cell fluctuation or the second stage breaks this;
* where every cell is a local extremum the limiter returns zero slopes and the
  operator is the first-order one exactly (same faces, no in-cell term);
* the lake at rest stays at rest to round-off over any bed (free-surface
  reconstruction); mass is conserved on periodic domains;
* the wet dam break (Stoker) is approximated better than at first order, and
  its depths stay within the initial range (the limiter takes the smaller
  one-sided difference);
* a cell whose reconstruction would give a negative face depth falls back to
  zero slopes;
* 1D equals 2D with one row; the 2D step is invariant under a 90 deg rotation.
"""
import math

import numpy as np
import pytest

from oracle import mesh, sme, stoker
from paper_2601_04826_amd import workloads as W

G = 9.81


def smooth_state(n, level, L=1.0):
    x = (np.arange(n) + 0.5) * (L / n)
    h = 1.0 + 0.1 * np.sin(2 * np.pi * x / L)
    q = np.zeros((level + 2, n))
    q[0] = h
    q[1] = h * (0.3 + 0.05 * np.cos(2 * np.pi * x / L))
    if level >= 1:
        q[2] = h * 0.1 * np.sin(2 * np.pi * x / L + 0.4)
    return q


def run_1d(n, level, order, T, L=1.0, lam=4.0):
    m = mesh.mesh_1d(n, 0.0, L, ("periodic", "periodic"))
    o = sme.Oracle(level, m, np.zeros(n), c_slip=0.0, nu=0.0, order=order)
    dx = L / n
    steps = int(math.ceil(T / (0.4 * dx / lam)))
    Q, t = o.run(smooth_state(n, level, L), steps, dt_fixed=T / steps)
    assert t == pytest.approx(T, rel=1e-12)
    return Q


def coarsen(Q, k):
    return Q.reshape(Q.shape[0], -1, k).mean(axis=2)


def test_second_order_convergence_smooth_level1():
    T = 0.05
    ref = 2 * coarsen(run_1d(4096, 1, 1, T), 2) - run_1d(2048, 1, 1, T)   # Richardson, O(dx^2)
    errs = []
    for n in (32, 64, 128):
        Q = run_1d(n, 1, 2, T)
        R = coarsen(ref, 2048 // n)
        errs.append(np.mean(np.abs(Q - R)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, (errs, rates)
    # the first-order scheme on the same grids converges at about 1
    e1 = [np.mean(np.abs(run_1d(n, 1, 1, T) - coarsen(ref, 2048 // n))) for n in (64, 128)]
    assert math.log2(e1[0] / e1[1]) < 1.3
    assert errs[2] < 0.2 * e1[1]


def test_zero_slopes_reduce_to_first_order():
    n = 40
    m = mesh.mesh_1d(n, 0.0, 4.0, ("periodic", "periodic"))
    rng = np.random.default_rng(0)
    N = 2
    Q = np.zeros((N + 2, n))
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    Q[0] = 1.0 + 0.3 * alt
    Q[1:] = (rng.uniform(0.1, 0.3, (N + 1, 1)) * alt) * Q[0]
    b = 0.05 * (1 - alt)          # eta, q and b all alternate: every cell is an extremum
    o2 = sme.Oracle(N, m, b, order=2)
    o1 = sme.Oracle(N, m, b, order=1)
    dt = 1e-4
    r1 = (o1.predict(Q, dt) - Q) / dt
    np.testing.assert_allclose(o2.rhs2(Q), r1, rtol=1e-9, atol=1e-9 * np.abs(r1).max())


@pytest.mark.parametrize("N", [0, 2])
def test_lake_at_rest_order2(N):
    m = mesh.mesh_1d(120, 0.0, 10.0, ("wall", "wall"))
    xc = m.centers
    b = 0.3 * np.exp(-((xc - 4.0) ** 2) / 0.5) + 0.1 * np.sin(xc)
    o = sme.Oracle(N, m, b, c_slip=1.0, nu=0.1, order=2)
    Q = np.zeros((o.nf, 120))
    Q[0] = 2.0 - b
    Q1, _ = o.run(Q, 300)
    assert np.max(np.abs(Q1[1:])) <= 1e-12
    assert np.max(np.abs(Q1[0] - Q[0])) <= 1e-12
    p = W.struct_2d(n=32, level=N, steps=0)
    o2 = sme.from_problem(p, order=2)
    Q = np.zeros_like(p["q"])
    Q[0] = 1.5 - p["b"]
    Q2, _ = o2.run(Q, 100)
    assert np.max(np.abs(Q2[1:])) <= 1e-12
    assert np.max(np.abs(Q2[0] - Q[0])) <= 1e-12


def test_dam_break_stays_within_initial_depths_order2():
    """The minmod limiter takes the smaller one-sided difference, so no
    reconstructed face value leaves the range of the neighbouring averages:
    the wet dam break (2 m against 1 m) keeps every depth inside [1, 2] (a
    limiter that took the larger difference overshoots by several per cent)."""
    for level in (0, 1):
        p = W.dam_break_1d(n=400, level=level, hl=2.0, hr=1.0)
        o = sme.from_problem(p, order=2, c_slip=0.0, nu=0.0)
        Q, _ = o.run(p["q"], 300)
        assert Q[0].max() <= 2.0 + 1e-12 and Q[0].min() >= 1.0 - 1e-12


def test_negative_face_depth_falls_back_to_first_order():
    """A shallow cell at the foot of a bed step: its free surface is a local
    minimum (zero slope) while the bed rises, so the linear reconstruction
    would put a negative depth (0.05 - 0.3 / 2) on its upper face.  The cell
    keeps zero slopes instead, and the step stays finite with positive
    depths."""
    n = 8
    m = mesh.mesh_1d(n, 0.0, 0.8, ("wall", "wall"))
    b = np.array([0.0, 0.0, 0.0, 0.3, 0.6, 0.6, 0.6, 0.6])
    Q = np.zeros((2, n))
    Q[0] = [0.5, 0.5, 0.5, 0.05, 0.5, 0.5, 0.5, 0.5]
    o = sme.Oracle(0, m, b, order=2)
    Q1, _ = o.step(Q, 1e-3)
    assert np.all(np.isfinite(Q1))
    assert Q1[0].min() > 0.0


def test_mass_conservation_order2():
    p = W.struct_2d(n=48, level=2)
    o = sme.from_problem(p, order=2)
    m0 = math.fsum(p["q"][0])
    Q1, _ = o.run(p["q"], 150)
    assert abs(math.fsum(Q1[0]) - m0) / m0 <= 1e-13


def test_stoker_better_than_first_order():
    T, errs = 0.5, {}
    for order in (1, 2):
        for n in (250, 500):
            dx = 10.0 / n
            steps = int(round(T / (0.4 * dx / 6.0)))
            p = W.dam_break_1d(n=n, level=0, params=dict(c_slip=0.0, nu=0.0))
            o = sme.from_problem(p, order=order)
            Q, _ = o.run(p["q"], steps, dt_fixed=T / steps)
            he, _ = stoker.solution(o.mesh.centers, T, 5.0, 2.0, 1.0, G)
            errs[order, n] = np.sum(np.abs(Q[0] - he)) * dx
    assert errs[2, 250] < 0.7 * errs[1, 250] and errs[2, 500] < 0.7 * errs[1, 500], errs
    assert errs[2, 500] < errs[2, 250]


def test_1d_equals_2d_single_row_order2():
    N = 1
    p1 = W.dam_break_1d(n=100, level=N, bc=("periodic", "periodic"))
    q = p1["q"].copy()
    q[1:] += 0.1 * q[0]
    o1 = sme.Oracle(N, mesh.mesh_1d(100, 0.0, 10.0, ("periodic", "periodic")), order=2, c_slip=1.0, nu=0.1)
    m2 = mesh.mesh_2d_struct(100, 1, 0.0, 10.0, 0.0, 0.1)
    o2 = sme.Oracle(N, m2, np.zeros(100), order=2, c_slip=1.0, nu=0.1)
    Q2 = np.zeros((o2.nf, 100))
    Q2[:N + 2] = q
    A, _ = o1.run(q, 60, dt_fixed=1e-3)
    B, _ = o2.run(Q2, 60, dt_fixed=1e-3)
    np.testing.assert_allclose(B[:N + 2], A, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(B[N + 2:], 0.0, atol=1e-14)


def test_rotation_invariance_order2():
    n, N = 20, 2
    p = W.struct_2d(n=n, level=N, L=10.0)
    o = sme.from_problem(p, order=2)
    rng = np.random.default_rng(3)
    Q = p["q"].copy()
    k = N + 1
    Q[1:] = Q[0] * rng.uniform(-0.3, 0.3, size=(2 * k, n * n))
    A, _ = o.run(Q, 20, dt_fixed=2e-3)

    def rot(Z, b=False):
        g = Z.reshape(-1, n, n)
        r = np.transpose(g, (0, 2, 1))[:, :, ::-1].reshape(Z.shape)
        if b:
            return r
        out = r.copy()
        out[1:1 + k] = -r[1 + k:]
        out[1 + k:] = r[1:1 + k]
        return out

    o_r = sme.Oracle(N, o.mesh, rot(p["b"][None], b=True)[0], order=2, **{k_: v for k_, v in p["params"].items()
                                                                           if k_ != "order"})
    B, _ = o_r.run(rot(Q), 20, dt_fixed=2e-3)
    np.testing.assert_allclose(B, rot(A), rtol=1e-12, atol=1e-12)
