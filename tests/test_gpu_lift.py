"""GPU parity of the 3D lifting (sme_interpolate_3d) against the oracle.

The kernel evaluates the profiles by the Legendre recurrence and Phi_k from
differences of neighbouring Legendre polynomials, and its uniform-grid
gradients as central or one-sided differences; the oracle uses exact
polynomial coefficients and numpy least squares.  Per output variable:
max |gpu - oracle| / max |oracle| <= 1e-10 (a variable that is zero in the
oracle, v in 1D, must be zero).  States are taken after some steps so every
moment and gradient is generic.
"""
import sys

import numpy as np
import pytest

from oracle import lift as olift
from oracle import mesh as omesh
from oracle import sme as orc
from paper_2601_04826_amd import workloads as W

pytestmark = pytest.mark.gpu

ZETA = np.array([0.0, 0.05, 0.25, 0.5, 0.8, 1.0])


@pytest.fixture(scope="module")
def sme():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_04826_amd import sme as m

    return m


def check(sme, p, steps=10, cells=None, rho=1.0):
    print(f"case {p['kind']} level {p['level']} cells {p['ncells']}", flush=True)
    sys.stdout.flush()
    s = sme.Solver(p)
    s.set_state(p["q"])
    if steps:
        s.run(steps)
    Q = s.get_state()
    got = s.interpolate_3d(ZETA, rho=rho)
    s.close()
    m = orc.mesh_of(p)
    want = olift.interpolate_3d(p["level"], m, Q, p["b"], ZETA, rho=rho, g=p["params"]["g"],
                                spacing=olift.spacing_of(p), cells=cells)
    for k in ("z", "u", "v", "w", "p"):
        g = got[k] if cells is None else got[k][:, cells]
        scale = np.max(np.abs(want[k]))
        if scale == 0.0:
            assert np.all(g == 0.0), k
            continue
        err = np.max(np.abs(g - want[k])) / scale
        assert err <= 1e-10, (k, err)


def with_moments(p, seed, amp=0.3):
    p = dict(p)
    q = p["q"].copy()
    q[1:] = q[0] * np.random.default_rng(seed).uniform(-amp, amp, size=q[1:].shape)
    p["q"] = q
    return p


@pytest.mark.parametrize("level", range(0, 9))
def test_lift_1d(sme, level):
    for bc in (("extrap", "wall"), ("periodic", "periodic")):
        p = with_moments(W.dam_break_1d(n=130, level=level, bc=bc), level)
        p["b"] = 0.1 * np.sin(np.linspace(0, 3, 130))
        check(sme, p)


@pytest.mark.parametrize("level", range(0, 9))
def test_lift_2d(sme, level):
    for bc in (("wall", "wall", "periodic", "periodic"), ("periodic", "periodic", "extrap", "wall")):
        p = with_moments(W.struct_2d(n=48, level=level, L=4.8, bc=bc), 40 + level)
        check(sme, p, rho=1000.0)


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (70, 1), (1, 9)])
def test_lift_degenerate_grids(sme, shape):
    nx, ny = shape
    rng = np.random.default_rng(nx * 10 + ny)
    q = W.random_state_2d(2, nx * ny, seed=3)
    for bc in ("periodic", "wall"):
        p = W._problem("2d", 2, nx * ny, q, rng.uniform(0, 0.05, nx * ny), 5, nx=nx, ny=ny, x0=0.0,
                       x1=nx / 10.0, y0=0.0, y1=ny / 10.0, bc=(bc,) * 4)
        check(sme, p, steps=3)


@pytest.mark.parametrize("level", range(0, 9))
def test_lift_triangles(sme, level):
    vert, tri = W.delaunay_unit_square(500, seed=80 + level)
    q = W.random_state_2d(level, len(tri), seed=level)
    c = vert[tri].mean(axis=1)
    b = 0.1 * np.exp(-((c[:, 0] - 0.4) ** 2 + (c[:, 1] - 0.5) ** 2) / 0.05)
    p = dict(kind="tri", level=level, ncells=len(tri), q=q, b=b, steps=5, vert=vert, tri=tri,
             params=dict(W.DEFAULT_PARAMS))
    check(sme, p, steps=5)


def test_lift_full_size_sampled(sme):
    """The 1024^2 level-2 grid: every cell lifted on the GPU, 2000 sampled
    cells (corners and edges included) against the oracle."""
    p = W.struct_2d(n=1024, level=2, steps=0)
    rng = np.random.default_rng(5)
    n = 1024
    cells = np.concatenate([[0, n - 1, n * (n - 1), n * n - 1], rng.choice(n * n, 1996, replace=False)])
    check(sme, p, steps=20, cells=cells)
