"""GPU parity with physical and numerical parameters away from their usual
values: gravity g = 3.7, CFL number 0.3, slip 0.5 and viscosity 0.02.

The other parity tests run at g = 9.81 and CFL 0.45, so a constant written
into a kernel in place of its parameter would pass them.  Each path of the
library (1D, structured and triangle first order, second order, implicit
friction, the ensemble, the VAM channel, the lifting) is checked here
against the oracle given the same parameters, at the usual tolerances.
"""
import sys

import numpy as np
import pytest

from oracle import lift as olift
from oracle import sme as orc
from oracle import vam as ovam
from paper_2601_04826_amd import workloads as W

pytestmark = pytest.mark.gpu

PRM = dict(g=3.7, cfl=0.3, c_slip=0.5, nu=0.02)


@pytest.fixture(scope="module")
def sme():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_04826_amd import sme as m

    return m


def rel_linf(gpu, ref):
    worst = 0.0
    for f in range(ref.shape[0]):
        scale = np.max(np.abs(ref[f]))
        if scale == 0.0:
            assert np.all(gpu[f] == 0.0)
            continue
        worst = max(worst, np.max(np.abs(gpu[f] - ref[f])) / scale)
    return worst


def with_moments(p, seed, amp=0.3):
    p = dict(p)
    q = p["q"].copy()
    q[1:] = q[0] * np.random.default_rng(seed).uniform(-amp, amp, size=q[1:].shape)
    p["q"] = q
    return p


def run_both(sme, p, steps, **over):
    print(f"case {p['kind']} level {p['level']} cells {p['ncells']} {over}", flush=True)
    sys.stdout.flush()
    s = sme.Solver(p, **over)
    s.set_state(p["q"])
    t_gpu, n = s.run(steps)
    q_gpu = s.get_state()
    s.close()
    q_orc, t_orc = orc.from_problem(p, **over).run(p["q"], steps)
    assert n == steps
    return q_gpu, q_orc, t_gpu, t_orc


def problems(level):
    p1 = with_moments(W.dam_break_1d(n=150, level=level, bc=("extrap", "wall")), 60 + level)
    p2 = with_moments(W.struct_2d(n=70, level=level, L=7.0, bc=("wall", "wall", "periodic", "periodic")), 70 + level)
    vert, tri = W.delaunay_unit_square(500, seed=80 + level)
    c = vert[tri].mean(axis=1)
    q = np.zeros((2 * level + 3, len(tri)))
    q[0] = 1.0 + 0.3 * np.exp(-20 * ((c[:, 0] - 0.4) ** 2 + (c[:, 1] - 0.5) ** 2))
    p3 = with_moments(dict(kind="tri", level=level, ncells=len(tri), q=q, b=0.05 * c[:, 0], steps=30, vert=vert,
                           tri=tri, params=dict(W.DEFAULT_PARAMS)), 90 + level)
    return p1, p2, p3


@pytest.mark.parametrize("level", [0, 2, 5, 8])
def test_first_order_parameters(sme, level):
    for p in problems(level):
        q_gpu, q_orc, t_gpu, t_orc = run_both(sme, p, 30, **PRM)
        assert rel_linf(q_gpu, q_orc) <= 1e-10, p["kind"]
        assert abs(t_gpu - t_orc) <= 1e-12 * t_orc


@pytest.mark.parametrize("level", [1, 3, 7])
def test_second_order_and_implicit_parameters(sme, level):
    p1, p2, _ = problems(level)
    for p in (p1, p2):
        q_gpu, q_orc, t_gpu, t_orc = run_both(sme, p, 20, order=2, **PRM)
        assert rel_linf(q_gpu, q_orc) <= 1e-10, p["kind"]
        assert abs(t_gpu - t_orc) <= 1e-12 * t_orc
    q_gpu, q_orc, _, _ = run_both(sme, p2, 20, implicit_friction=1, **dict(PRM, nu=2.0))
    assert rel_linf(q_gpu, q_orc) <= 1e-10


def test_ensemble_parameters(sme):
    probs = W.batch(n_inst=6, seed=900, steps=30, side=(40, 130), levels=(0, 4), params=PRM)
    bt = sme.Batch(probs)
    for i, p in enumerate(probs):
        bt.set_state(i, p["q"])
    bt.run(30)
    for i, p in enumerate(probs):
        r, t_o = orc.from_problem(p).run(p["q"], 30)
        assert rel_linf(bt.get_state(i), r) <= 1e-10, i
        t, n = bt.time(i)
        assert n == 30 and abs(t - t_o) <= 1e-12 * t_o
    bt.close()


def test_vam_parameters(sme):
    p = W.vam_1d(n=1500, L=15.0, params=dict(g=3.7, cfl=0.3))
    v = sme.Vam(p)
    v.set_state(p["q"])
    dt = v.step()
    q_gpu, p_gpu = v.get_state(), v.pressure()
    v.close()
    prm = p["params"]
    o = ovam.Vam1D(p["nx"], p["x0"], p["x1"], b=p["b"], g=prm["g"], cfl=prm["cfl"], quad_points=prm["quad_points"])
    q_orc, P_orc, dt_orc = o.step(p["q"])
    assert abs(dt - dt_orc) <= 1e-12 * dt_orc
    scale = np.maximum(np.abs(q_orc).max(axis=1), np.abs(p["q"]).max(axis=1))
    assert np.max(np.abs(q_gpu - q_orc).max(axis=1) / scale) <= 1e-9
    assert np.max(np.abs(p_gpu - P_orc)) <= 1e-8 * np.max(np.abs(P_orc))


def test_lifting_parameters(sme):
    zeta = np.array([0.0, 0.4, 1.0])
    _, p2, p3 = problems(2)
    for p in (p2, p3):
        s = sme.Solver(p, g=3.7)
        s.set_state(p["q"])
        s.run(5)
        Q = s.get_state()
        got = s.interpolate_3d(zeta, rho=1025.0)
        s.close()
        want = olift.interpolate_3d(2, orc.mesh_of(p), Q, p["b"], zeta, rho=1025.0, g=3.7,
                                    spacing=olift.spacing_of(p))
        for k in ("z", "u", "v", "w", "p"):
            scale = np.max(np.abs(want[k]))
            assert np.max(np.abs(got[k] - want[k])) <= 1e-10 * scale, (p["kind"], k)
