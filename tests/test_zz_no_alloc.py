"""The entry point that allocates nothing (sme_step_static) against sme_step.

sme_step_static takes one step on the caller's buffers with its scratch (time
slots, error word, Gauss points) in a static device array.  On the same state,
mesh and parameters it must give bitwise the result of sme_step on a context
(same kernels, same arguments), also on a second call in a row with a smaller
grid (the shared scratch keeps the last call's contents, so a call that did
not clear it would read stale CFL words), with the CFL step and a fixed step.
"""
import sys

import numpy as np
import pytest

from paper_2601_04826_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_04826_amd import sme as m

    return torch, m


def device_state(torch, sme, p):
    """(q, q_next, b) as device tensors in the bound-buffer layout of problem p."""
    mesh, _ = sme.make_mesh(p)
    nf, nc, st = sme.sme_layout(p["level"], mesh)
    q = torch.zeros((nf, st), dtype=torch.float64, device="cuda")
    q[:, :nc] = torch.from_numpy(np.ascontiguousarray(p["q"]))
    qn = torch.full((nf, st), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.zeros(st, dtype=torch.float64, device="cuda")
    if p.get("b") is not None:
        b[:nc] = torch.from_numpy(np.ascontiguousarray(p["b"]))
    return mesh, q, qn, b, nc


def step_with_context(sme, p, dt):
    s = sme.Solver(p)
    s.set_state(p["q"])
    used = s.step(dt, sync=True)
    out = s.get_state()
    s.close()
    return out, used


def check(torch, sme, p, dt):
    print(f"case {p['kind']} level {p['level']} cells {p['ncells']} dt {dt}", flush=True)
    sys.stdout.flush()
    mesh, q, qn, b, nc = device_state(torch, sme, p)
    params = sme.make_params(**p["params"])
    used = sme.sme_step_static(p["level"], mesh, params, q, qn, b, dt)
    torch.cuda.synchronize()
    got = qn[:, :nc].cpu().numpy()
    want, used_ctx = step_with_context(sme, p, dt)
    assert used == used_ctx
    if dt > 0:
        assert used == dt
    assert np.array_equal(got, want)
    # the input is left as it was
    assert np.array_equal(q[:, :nc].cpu().numpy(), p["q"])


def rough(p, seed):
    """Moments switched on (random velocities) so every field is exercised."""
    rng = np.random.default_rng(seed)
    p = dict(p)
    q = p["q"].copy()
    q[1:] = q[0] * rng.uniform(-0.3, 0.3, size=q[1:].shape)
    p["q"] = q
    return p


def test_static_step_two_calls_smaller_second(env):
    torch, sme = env
    big = rough(W.struct_2d(n=200, level=3, steps=1), 1)
    small = rough(W.struct_2d(n=70, level=2, steps=1, bc=("wall", "wall", "extrap", "extrap")), 2)
    check(torch, sme, big, 0.0)
    check(torch, sme, small, 0.0)


def test_static_step_fixed_dt_and_1d(env):
    torch, sme = env
    p1 = rough(W.dam_break_1d(n=1000, level=1), 3)
    check(torch, sme, p1, 0.0)
    p8 = rough(W.dam_break_1d(n=300, level=8), 4)
    check(torch, sme, p8, 1e-4)
    p2 = rough(W.struct_2d(n=64, level=4, steps=1), 5)
    check(torch, sme, p2, 2e-4)


def test_static_step_quadrature_and_sequence(env):
    """Five Gauss points (read from the scratch array) and a sequence of static
    steps against sme_run with fixed steps."""
    torch, sme = env
    p = rough(W.struct_2d(n=90, level=2, steps=1, params=dict(quad_points=5)), 6)
    check(torch, sme, p, 0.0)
    mesh, q, qn, b, nc = device_state(torch, sme, p)
    params = sme.make_params(**p["params"])
    for k in range(6):
        sme.sme_step_static(p["level"], mesh, params, q, qn, b, 0.0, )
        q, qn = qn, q
    torch.cuda.synchronize()
    s = sme.Solver(p)
    s.set_state(p["q"])
    for k in range(6):
        s.step(0.0)
    want = s.get_state()
    s.close()
    assert np.array_equal(q[:, :nc].cpu().numpy(), want)


def test_static_step_rejects_bad_arguments(env):
    torch, sme = env
    p = W.struct_2d(n=40, level=1, steps=1)
    mesh, q, qn, b, nc = device_state(torch, sme, p)
    params = sme.make_params(**p["params"])
    with pytest.raises(sme.SmeError) as e:
        sme.sme_step_static(9, mesh, params, q, qn, b)
    assert e.value.code == sme.SME_EINVAL
    with pytest.raises(sme.SmeError):
        sme.sme_step_static(1, mesh, params, q, q, b)          # in place
    with pytest.raises(sme.SmeError):
        sme.sme_step_static(1, mesh, params, q[:, 1:].contiguous(), qn, b)  # stride 255
    vert = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    t, _ = sme.make_mesh(dict(kind="tri", vert=vert, tri=np.array([[0, 1, 2]], dtype=np.int32)))
    with pytest.raises(sme.SmeError):
        sme.sme_step_static(1, t, params, q, qn, b)
