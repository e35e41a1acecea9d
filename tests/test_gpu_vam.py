"""GPU parity of the non-hydrostatic VAM channel (sme_vam_*) against the oracle.

The kernels assemble the corrector's constraint rows as affine forms and
solve the block-tridiagonal system by block cyclic reduction (each level's
even blocks factored once, the factors reused by the Newton step on the
residual); the oracle probes the same affine map numerically and solves with
a sparse direct solver.  Metric as in the other parity tests: per field max |gpu - oracle| /
max |oracle|.  The state after a step agrees to 1e-9 and the pressure to 1e-8
of its largest value (both sides solve a linear system whose condition number
grows like (h / dx)^2); CFL steps agree to 1e-12.
"""
import sys

import numpy as np
import pytest

from oracle import vam
from paper_2601_04826_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sme():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_04826_amd import sme as m

    return m


def rel(gpu, ref, init=None):
    """per field max |gpu - ref| / max |ref|; with `init`, each field is
    measured against the larger of its final and initial maximum (a
    corrected vertical momentum can be round-off-sized where the constraints
    set it to zero)"""
    worst = 0.0
    for f in range(ref.shape[0]):
        scale = np.max(np.abs(ref[f]))
        if init is not None:
            scale = max(scale, np.max(np.abs(init[f])))
        if scale == 0.0:
            assert np.max(np.abs(gpu[f])) <= 1e-300, f
            continue
        worst = max(worst, np.max(np.abs(gpu[f] - ref[f])) / scale)
    return worst


def oracle_of(p):
    prm = p["params"]
    return vam.Vam1D(p["nx"], p["x0"], p["x1"], b=p["b"], g=prm["g"], cfl=prm["cfl"], quad_points=prm["quad_points"])


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 63, 64, 127, 128, 129, 130, 257, 1000, 1021, 1022, 1024, 1025, 2001])
def test_one_step_matches_oracle(sme, n):
    """Sizes around the solver's boundaries: a system of up to 64 blocks is
    solved entirely in LDS by one wave (n <= 128 cells), a larger one first
    reduces level by level; a reduction workgroup takes 256 even and 255 odd
    blocks, so 511, 512 and 513 blocks (n = 1021 .. 1025) put the last odd
    block at the end of a workgroup, alone in a second one, or leave a
    second workgroup with only its even block."""
    print(f"case vam one step n={n}", flush=True)
    p = W.vam_1d(n=n, L=20.0)
    v = sme.Vam(p)
    v.set_state(p["q"])
    dt = v.step()
    q_gpu, p_gpu = v.get_state(), v.pressure()
    v.close()
    o = oracle_of(p)
    q_orc, P_orc, dt_orc = o.step(p["q"])
    assert abs(dt - dt_orc) <= 1e-12 * dt_orc
    assert rel(q_gpu, q_orc, p["q"]) <= 1e-9
    assert rel(p_gpu, P_orc) <= 1e-8


@pytest.mark.parametrize("G", [1, 2, 5])
def test_quadrature_points(sme, G):
    p = W.vam_1d(n=300, L=10.0, params=dict(quad_points=G))
    v = sme.Vam(p)
    v.set_state(p["q"])
    v.run(20)
    q_gpu = v.get_state()
    v.close()
    q_orc, _, _ = oracle_of(p).run(p["q"], 20)
    assert rel(q_gpu, q_orc, p["q"]) <= 1e-9


def test_undular_bore_200_steps(sme):
    p = W.vam_1d(n=800, L=20.0, moments=False)
    print("case vam bore 800 cells 200 steps", flush=True)
    v = sme.Vam(p)
    v.set_state(p["q"])
    t_gpu, n_gpu = v.run(200)
    q_gpu = v.get_state()
    v.close()
    q_orc, _, t_orc = oracle_of(p).run(p["q"], 200)
    assert n_gpu == 200 and abs(t_gpu - t_orc) <= 1e-11 * t_orc
    assert rel(q_gpu, q_orc, p["q"]) <= 1e-8


def test_lake_at_rest_and_fixed_dt(sme):
    n = 500
    p = W.vam_1d(n=n, L=10.0, moments=False)
    q = np.zeros((5, n))
    q[0] = 1.0 - p["b"]
    p["q"] = q
    v = sme.Vam(p)
    v.set_state(q)
    for _ in range(5):
        assert v.step(1e-3) == 1e-3
    assert np.max(np.abs(v.get_state() - q)) <= 1e-13
    assert np.max(np.abs(v.pressure())) <= 1e-10
    v.close()


def test_end_time_and_state_round_trip(sme):
    import torch

    p = W.vam_1d(n=400, L=10.0)
    v = sme.Vam(p)
    v.set_state(torch.from_numpy(p["q"]).cuda())
    assert np.array_equal(v.get_state(), p["q"])
    t, k = v.run(1000, t_end=0.05)
    assert abs(t - 0.05) <= 1e-15 and k < 1000
    q1 = v.get_state()
    t2, k2 = v.run(10, t_end=0.05)  # past the end time: nothing moves
    assert (t2, k2) == (t, k) and np.array_equal(v.get_state(), q1)
    v.close()


def test_layout_workspace_and_errors(sme):
    assert sme.sme_vam_layout(1000) == 1024
    assert sme.sme_vam_workspace_size(1000) > 52 * 500 * 8
    with pytest.raises(sme.SmeError):
        sme.sme_vam_layout(0)
    p = W.vam_1d(n=100, L=5.0)
    q = p["q"].copy()
    q[0, 10] = -1.0
    v = sme.Vam(p)
    with pytest.raises(sme.SmeError) as e:
        v.set_state(q)
    assert e.value.code == sme.SME_ENONPHYS
    v.close()


def test_full_size_against_oracle(sme):
    """The bench channel (2^20 cells, the launch configuration bench.py
    times), one step element by element against the oracle (its sparse direct
    solve takes a few seconds), plus the properties that hold at any size: the
    corrected state meets both constraints to round-off relative to their
    initial violation, h is the predictor's, mass changes only through the
    two end faces."""
    n = 1 << 20
    p = W.vam_1d(n=n, L=1000.0)
    print("case vam full size", flush=True)
    v = sme.Vam(p)
    v.set_state(p["q"])
    dt = v.step()
    q, pg = v.get_state(), v.pressure()
    v.close()
    o = oracle_of(p)
    q_orc, P_orc, dt_orc = o.step(p["q"])
    assert abs(dt - dt_orc) <= 1e-12 * dt_orc
    assert rel(q, q_orc, p["q"]) <= 1e-9
    assert rel(pg, P_orc) <= 1e-8
    Qs = o.predict(p["q"], dt)
    assert np.max(np.abs(q[0] - Qs[0])) <= 1e-12 * np.max(Qs[0])
    R = o.residual(q)
    scale = np.max(np.abs(o.residual(Qs)))
    assert np.max(np.abs(R)) <= 1e-8 * scale
    flux_ends = dt * (p["q"][1, -1] - p["q"][1, 0]) / o.dx
    assert abs(q[0].sum() - p["q"][0].sum() + flux_ends) <= 1e-9 * p["q"][0].sum()
