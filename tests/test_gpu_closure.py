"""GPU tests of the learned closure: the FP32 network kernels against the FP64
oracle network (forward, gradient, Adam), the training samples against the
oracle's level-1 step, the level-1 + closure step (FP32 and FP16 matrix-core
rates) against the oracle, the zero network reducing to plain level 1
bitwise, the out-of-range flag, and the gain of a trained closure on held-out
seeds."""
import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import sme as orc
from paper_2601_04826_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_04826_amd import closure, sme

    return torch, sme, closure


def rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return (omlp.init_params(seed) * scale + 0.02 * rng.standard_normal(omlp.NPARAM)).astype(np.float32)


def test_forward_matches_oracle(env):
    torch, sme, _ = env
    p = rand_params(1)
    x = np.random.default_rng(2).standard_normal((1000, 9)).astype(np.float32)
    m = sme.MLP(p)
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = omlp.forward(p.astype(np.float64), x.astype(np.float64))
    np.testing.assert_allclose(y, ref, rtol=0, atol=2e-5 * max(1.0, np.abs(ref).max()))
    m.close()


@pytest.mark.parametrize("B", [64, 300])
def test_gradient_matches_oracle(env, B):
    torch, sme, _ = env
    p = rand_params(3)
    rng = np.random.default_rng(B)
    x = rng.standard_normal((B, 9)).astype(np.float32)
    t = rng.standard_normal((B, 2)).astype(np.float32)
    m = sme.MLP(p)
    loss, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy()
    lref, gref = omlp.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(lref, rel=1e-5)
    assert np.max(np.abs(g - gref)) <= 1e-4 * np.max(np.abs(gref))
    m.close()


def test_adam_step_matches_oracle(env):
    torch, sme, _ = env
    p = rand_params(5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((256, 9)).astype(np.float32)
    t = rng.standard_normal((256, 2)).astype(np.float32)
    m = sme.MLP(p)
    lr = 1e-3
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    m.train_step(xd, td, lr)
    m.train_step(xd, td, lr)
    got = m.get_params().astype(np.float64)
    pp, mm, vv = p.astype(np.float64), np.zeros(omlp.NPARAM), np.zeros(omlp.NPARAM)
    for step in (1, 2):
        _, g = omlp.loss_grad(pp, x.astype(np.float64), t.astype(np.float64))
        pp, mm, vv = omlp.adam(pp, g, mm, vv, step, lr)
    _, g0 = omlp.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    big = np.abs(g0) > 1e-3 * np.abs(g0).max()
    assert np.max(np.abs(got - pp)[big]) <= 2e-2 * lr
    m.close()


def test_fit_scaling_matches_numpy(env):
    torch, sme, _ = env
    rng = np.random.default_rng(11)
    n = 100003  # not a multiple of any block size
    f = (rng.standard_normal((n, 9)) * rng.uniform(0.01, 3.0, 9) + rng.uniform(-2, 2, 9)).astype(np.float32)
    t = (rng.standard_normal((n, 2)) * [1e-3, 0.3]).astype(np.float32)
    m = sme.MLP(np.zeros(omlp.NPARAM, dtype=np.float32))
    sc = m.fit_scaling(torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda(), margin=0.1)
    f64, t64 = f.astype(np.float64), t.astype(np.float64)
    np.testing.assert_allclose(sc["mu"], f64.mean(0).astype(np.float32), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(sc["sigma"], f64.std(0, ddof=1).astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(sc["out_scale"], t64.std(0, ddof=1).astype(np.float32), rtol=1e-6)
    lo, hi = f64.min(0), f64.max(0)
    np.testing.assert_allclose(sc["box_lo"], lo - 0.1 * (hi - lo), rtol=1e-15)
    np.testing.assert_allclose(sc["box_hi"], hi + 0.1 * (hi - lo), rtol=1e-15)
    m.close()


def test_gradient_with_scaling_and_rows(env):
    """Raw samples, a non-trivial scaling and a batch picked by index: the
    kernels normalise in place exactly as the oracle's inputs are prepared."""
    torch, sme, _ = env
    p = rand_params(12)
    m, mu, sig, osc = scaled_mlp(sme, p, seed=3)
    rng = np.random.default_rng(13)
    x = (rng.standard_normal((1000, 9)) * 2.0 + 0.5).astype(np.float32)
    t = rng.standard_normal((1000, 2)).astype(np.float32)
    idx = rng.permutation(1000)[:300].astype(np.int64)
    loss, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), idx=torch.from_numpy(idx).cuda())
    xn = ((x[idx] - mu) * (np.float32(1.0) / sig)).astype(np.float64)
    tn = (t[idx] / osc).astype(np.float64)
    lref, gref = omlp.loss_grad(p.astype(np.float64), xn, tn)
    assert loss == pytest.approx(lref, rel=1e-5)
    assert np.max(np.abs(g.cpu().numpy() - gref)) <= 1e-4 * np.max(np.abs(gref))
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yref, _ = omlp.forward(p.astype(np.float64), ((x - mu) * (np.float32(1.0) / sig)).astype(np.float64))
    np.testing.assert_allclose(y, yref, rtol=0, atol=2e-5 * max(1.0, np.abs(yref).max()))
    m.close()


def test_training_is_deterministic(env):
    torch, sme, closure = env
    feat, targ = closure.generate(range(1000, 1002), n=256, steps=60, every=3, cells_per_snapshot=64)
    out = []
    for _ in range(2):
        mlp, sc, hist = closure.fit(feat, targ, epochs=2, batch=512, seed=5)
        out.append((mlp.get_params(), hist))
        mlp.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_samples_match_oracle(env):
    torch, sme, _ = env
    p8 = W.smooth_1d(n=512, level=8, seed=1001, steps=30)
    s8 = sme.Solver(p8)
    s8.set_state(p8["q"])
    s8.run(30)
    q8 = s8.get_state()
    dt = s8.step(0.0, sync=True)
    q8n = s8.get_state()
    s8.close()
    p1 = dict(p8, level=1, q=q8[:3].copy())
    q1_orc, _ = orc.from_problem(p1).step(q8[:3].copy(), dt)
    cells = torch.arange(512, device="cuda")
    # GPU level-1 step from the same state
    s1 = sme.Solver(p1)
    s1.set_state(q8[:3].copy())
    s1.step(dt)
    q1 = s1.get_state()
    s1.close()
    f, t = sme.closure_samples(torch.from_numpy(q8).cuda(), torch.from_numpy(q8n).cuda(), torch.from_numpy(q1).cuda(),
                               dt, cells)
    torch.cuda.synchronize()
    f, t = f.cpu().numpy(), t.cpu().numpy()
    fo = omlp.features_1d(q8[0], q8[1], q8[2])
    to = omlp.closure_target(q8, q8n, q1_orc, dt)
    np.testing.assert_allclose(f, fo.astype(np.float32), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(t, to, rtol=1e-5, atol=1e-5 * np.abs(to).max())


def scaled_mlp(sme, p, seed=0):
    m = sme.MLP(p)
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-0.1, 0.1, 9).astype(np.float32)
    sig = rng.uniform(0.5, 2.0, 9).astype(np.float32)
    osc = np.array([0.3, 0.7], dtype=np.float32)
    m.set_scaling(mu, sig, osc, np.full(9, -1e3), np.full(9, 1e3))
    return m, mu, sig, osc


def oracle_rate(p, mu, sig, osc, feat):
    x = ((feat.astype(np.float32) - mu) * (np.float32(1.0) / sig)).astype(np.float64)
    y, _ = omlp.forward(p.astype(np.float64), x)
    return y * osc.astype(np.float64)


def test_closure_step_1d_matches_oracle(env):
    torch, sme, _ = env
    p = rand_params(7, scale=0.3)
    m, mu, sig, osc = scaled_mlp(sme, p)
    prob = W.smooth_1d(n=300, level=1, seed=1003)
    s = sme.Solver(prob)
    s.attach_closure(m)
    s.set_state(prob["q"])
    dt = 2e-3
    s.step(dt)
    got = s.get_state()
    s.close()
    ref, _ = orc.from_problem(prob).step(prob["q"], dt)
    q = prob["q"]
    r = oracle_rate(p, mu, sig, osc, omlp.features_1d(q[0], q[1], q[2]))
    ref[1] += dt * r[:, 0]
    ref[2] += dt * r[:, 1]
    np.testing.assert_allclose(got, ref, rtol=0, atol=5e-9 * np.abs(ref).max())
    m.close()


def test_closure_step_2d_matches_oracle(env):
    torch, sme, _ = env
    p = rand_params(8, scale=0.3)
    m, mu, sig, osc = scaled_mlp(sme, p, seed=1)
    n = 70
    prob = W.struct_2d(n=n, level=1, L=7.0)
    rng = np.random.default_rng(4)
    prob["q"][1:] = prob["q"][0] * rng.uniform(-0.3, 0.3, size=prob["q"][1:].shape)
    s = sme.Solver(prob)
    s.attach_closure(m)
    s.set_state(prob["q"])
    dt = 1e-3
    s.step(dt)
    got = s.get_state()
    s.close()
    ref, _ = orc.from_problem(prob).step(prob["q"], dt)
    q = prob["q"].reshape(5, n, n)  # [f, j, i], periodic

    def feats(h, a, b, axis):
        hp, ap, bp = (np.roll(v, -1, axis=axis) for v in (h, a, b))
        hm, am, bm = (np.roll(v, 1, axis=axis) for v in (h, a, b))
        return np.stack([h, a, b, hp - h, ap - a, bp - b, h - hm, a - am, b - bm], axis=-1).reshape(-1, 9)

    rx = oracle_rate(p, mu, sig, osc, feats(q[0], q[1], q[2], axis=1))
    ry = oracle_rate(p, mu, sig, osc, feats(q[0], q[3], q[4], axis=0))
    ref[1] += dt * rx[:, 0]
    ref[2] += dt * rx[:, 1]
    ref[3] += dt * ry[:, 0]
    ref[4] += dt * ry[:, 1]
    np.testing.assert_allclose(got, ref, rtol=0, atol=5e-9 * np.abs(ref).max())
    m.close()


U16 = 2.0 ** -11  # unit roundoff of FP16


def fp16_bound(p, mu, sig, osc, feat, lam=6.0):
    """Probabilistic error bound of the FP16-operand network per sample and
    output.  Every matrix operand (normalised input, weight, activation) is
    rounded once to FP16 (relative error <= u = 2^-11, so <= 2u per product);
    taking these roundings as independent and zero-mean, Hoeffding's inequality
    bounds a sum of n such terms by lam * 2u * sqrt(sum of squared terms) except
    with probability 2 exp(-lam^2 / 2) (3e-8 for lam = 6).  Errors carried in
    from the previous layer add in quadrature too; tanh' = 1 - a^2; the FP32
    exp2 / reciprocal add <= 1e-6 per activation; FP32 accumulation is
    negligible at these sizes."""
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p.astype(np.float64))
    x = ((feat.astype(np.float32) - mu) * (np.float32(1.0) / sig)).astype(np.float64)
    a1 = np.tanh(x @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    e = lam * 2 * U16
    dz1 = e * np.sqrt((x ** 2) @ (W1 ** 2).T)
    da1 = (1 - a1 ** 2) * dz1 + lam * U16 * np.abs(a1) + 1e-6
    dz2 = np.sqrt((da1 ** 2) @ (W2 ** 2).T) + e * np.sqrt((a1 ** 2) @ (W2 ** 2).T)
    da2 = (1 - a2 ** 2) * dz2 + lam * U16 * np.abs(a2) + 1e-6
    dy = np.sqrt((da2 ** 2) @ (W3 ** 2).T) + e * np.sqrt((a2 ** 2) @ (W3 ** 2).T)
    return dy * osc.astype(np.float64)


def fp16_rate_check(got, plain, r, bound, dt, fields):
    """(got - plain step) / dt is the FP16 rate: within the derived bound of the
    FP64 network's rate, and the bound itself well below the rates."""
    assert np.max(bound) < 0.05 * np.abs(r).max()
    for f, rr, bb in zip(fields, r.T, bound.T):
        d = (got[f] - plain[f]) / dt
        excess = np.abs(d - rr) - (bb + 1e-6 * np.abs(rr).max())
        assert np.max(excess) <= 0, (f, np.max(np.abs(d - rr)), np.max(bb))


@pytest.mark.parametrize("n", [300, 4099])
def test_closure_step_1d_fp16(env, n):
    torch, sme, _ = env
    p = rand_params(7, scale=1.0)  # activations of order one: the FP16 bound is a small fraction of the rates
    m, mu, sig, osc = scaled_mlp(sme, p)
    prob = W.smooth_1d(n=n, level=1, seed=1003)
    s = sme.Solver(prob)
    s.attach_closure(m, precision="fp16")
    s.set_state(prob["q"])
    dt = 2e-3
    s.step(dt)
    got = s.get_state()
    s.close()
    plain, _ = orc.from_problem(prob).step(prob["q"], dt)
    q = prob["q"]
    f = omlp.features_1d(q[0], q[1], q[2])
    r = oracle_rate(p, mu, sig, osc, f)
    np.testing.assert_allclose(got[0], plain[0], rtol=1e-13, atol=0)  # depth untouched
    fp16_rate_check(got, plain, r, fp16_bound(p, mu, sig, osc, f), dt, (1, 2))
    m.close()


def test_closure_step_2d_fp16(env):
    torch, sme, _ = env
    p = rand_params(8, scale=1.0)
    m, mu, sig, osc = scaled_mlp(sme, p, seed=1)
    n = 70  # 4900 cells: a ragged last group of 64
    prob = W.struct_2d(n=n, level=1, L=7.0)
    rng = np.random.default_rng(4)
    prob["q"][1:] = prob["q"][0] * rng.uniform(-0.3, 0.3, size=prob["q"][1:].shape)
    s = sme.Solver(prob)
    s.attach_closure(m, precision="fp16")
    s.set_state(prob["q"])
    dt = 1e-3
    s.step(dt)
    got = s.get_state()
    s.close()
    plain, _ = orc.from_problem(prob).step(prob["q"], dt)
    q = prob["q"].reshape(5, n, n)

    def feats(h, a, b, axis):
        hp, ap, bp = (np.roll(v, -1, axis=axis) for v in (h, a, b))
        hm, am, bm = (np.roll(v, 1, axis=axis) for v in (h, a, b))
        return np.stack([h, a, b, hp - h, ap - a, bp - b, h - hm, a - am, b - bm], axis=-1).reshape(-1, 9)

    fx, fy = feats(q[0], q[1], q[2], axis=1), feats(q[0], q[3], q[4], axis=0)
    rx, ry = oracle_rate(p, mu, sig, osc, fx), oracle_rate(p, mu, sig, osc, fy)
    np.testing.assert_allclose(got[0], plain[0], rtol=1e-13, atol=0)
    fp16_rate_check(got, plain, rx, fp16_bound(p, mu, sig, osc, fx), dt, (1, 2))
    fp16_rate_check(got, plain, ry, fp16_bound(p, mu, sig, osc, fy), dt, (3, 4))
    m.close()


@pytest.mark.parametrize("kind", ["1d", "2d"])
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_zero_network_is_plain_level1(env, kind, precision):
    torch, sme, _ = env
    prob = W.smooth_1d(n=500, level=1, seed=1010) if kind == "1d" else W.struct_2d(n=90, level=1)
    out = []
    for attach in (False, True):
        s = sme.Solver(prob)
        if attach:
            m = sme.MLP(np.zeros(omlp.NPARAM, dtype=np.float32))
            s.attach_closure(m, precision=precision)
        s.set_state(prob["q"])
        s.run(40)
        out.append(s.get_state())
        s.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_out_of_range_flag(env, precision):
    torch, sme, _ = env
    m = sme.MLP(np.zeros(omlp.NPARAM, dtype=np.float32))
    prob = W.smooth_1d(n=256, level=1, seed=1011)
    # a box that excludes depths above 1.0 m
    lo = np.full(9, -1e3)
    hi = np.full(9, 1e3)
    hi[0] = 1.0
    m.set_scaling(np.zeros(9), np.ones(9), np.ones(2), lo, hi)
    s = sme.Solver(prob)
    s.attach_closure(m, precision=precision)
    s.set_state(prob["q"])
    s.run(3)
    n_out = s.out_of_range()
    assert n_out > 0
    # a network that is not trusted anywhere leaves plain level 1
    m2 = sme.MLP(rand_params(9))
    m2.set_scaling(np.zeros(9), np.ones(9), np.ones(2), np.full(9, 1e3), np.full(9, 2e3))
    s.attach_closure(m2, precision=precision)
    s.set_state(prob["q"])
    s.run(10)
    off = s.get_state()
    assert s.out_of_range() == 10 * prob["ncells"]
    p = sme.Solver(prob)
    p.set_state(prob["q"])
    p.run(10)
    assert np.array_equal(off, p.get_state())
    p.close()
    m2.close()
    hi[0] = 1e3
    m.set_scaling(np.zeros(9), np.ones(9), np.ones(2), lo, hi)
    s.attach_closure(m, precision=precision)
    s.set_state(prob["q"])
    s.run(3)
    assert s.out_of_range() == 0
    s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_closure_solver_falls_back_to_level8(env, precision):
    """A network trusted nowhere: the first chunk already leaves the training
    box, so the run restarts with plain level 8 from the lifted state."""
    torch, sme, closure = env
    p8 = W.smooth_1d(n=256, level=8, seed=1012)
    m = sme.MLP(rand_params(14))
    m.set_scaling(np.zeros(9), np.ones(9), np.ones(2), np.full(9, 1e3), np.full(9, 2e3))
    cs = closure.ClosureSolver(p8, m, chunk=20, precision=precision)
    cs.set_state(p8["q"])
    out = cs.run_to(0.05)
    assert cs.fell_back_at == 0.0
    cs.close()
    s8 = sme.Solver(p8)
    s8.set_state(closure._lift_state(closure._project_state(p8["q"], p8), p8))
    s8.run(10 ** 6, t_end=0.05)
    assert np.array_equal(out, s8.get_state())
    s8.close()
    m.close()


def test_closure_solver_in_range_runs_level1(env):
    """A zero network trusted everywhere: no fallback, and the chunked run
    (device checkpoints between chunks) is bitwise one uninterrupted level-1 run."""
    torch, sme, closure = env
    p8 = W.smooth_1d(n=256, level=8, seed=1013)
    m = sme.MLP(np.zeros(omlp.NPARAM, dtype=np.float32))
    cs = closure.ClosureSolver(p8, m, chunk=25)
    cs.set_state(p8["q"])
    out = cs.run_to(0.05)
    assert cs.fell_back_at is None
    cs.close()
    p1 = dict(p8, level=1, q=closure._project_state(p8["q"], p8))
    s1 = sme.Solver(p1)
    s1.set_state(p1["q"])
    s1.run(10 ** 6, t_end=0.05)
    ref = closure._lift_state(s1.get_state(), p8)
    s1.close()
    assert np.array_equal(out, ref)
    assert cs.t == pytest.approx(0.05, rel=1e-14)
    m.close()


def test_trained_closure_gain_on_held_out_seeds(env):
    """Train on level-8 runs the solver generates (seeds 1000..1023), then on
    held-out seeds compare level 1 + closure and plain level 1 against level 8
    at the same time: the closure must cut the relative L1 error of (h, hu)."""
    torch, sme, closure = env
    feat, targ = closure.generate(range(1000, 1024), n=1024, steps=600, every=3, cells_per_snapshot=256)
    print("samples", feat.shape[0], flush=True)
    mlp, sc, hist = closure.fit(feat, targ, epochs=12, batch=4096, lr=3e-3, lr_end=1e-4, seed=0)
    assert hist[-1] < hist[0]
    gains = []
    for seed in (1256, 1257, 1258):
        p8 = W.smooth_1d(n=1024, level=8, seed=seed)
        T = 0.5
        s8 = sme.Solver(p8)
        s8.set_state(p8["q"])
        s8.run(10 ** 6, t_end=T)
        ref = s8.get_state()
        s8.close()
        res = {}
        zero = sme.MLP(np.zeros(omlp.NPARAM, dtype=np.float32))
        for name, net, prec in (("plain", zero, "fp32"), ("closure", mlp, "fp32"), ("closure16", mlp, "fp16")):
            p1 = dict(p8, level=1, q=p8["q"][:3].copy())
            s1 = sme.Solver(p1)
            s1.attach_closure(net, precision=prec)
            s1.set_state(p1["q"])
            s1.run(10 ** 6, t_end=T)
            q1 = s1.get_state()
            assert s1.out_of_range() >= 0
            s1.close()
            e = closure.relative_l1(q1, ref[:3], fields=(0, 1))
            res[name] = e
        g = (res["closure"][0] + res["closure"][1]) / (res["plain"][0] + res["plain"][1])
        g16 = (res["closure16"][0] + res["closure16"][1]) / (res["plain"][0] + res["plain"][1])
        print(f"seed {seed}: plain {res['plain']} closure {res['closure']} gain {g:.3f} (fp16 {g16:.3f})", flush=True)
        gains.append((g, g16))
    gains = np.array(gains)
    assert gains[:, 0].mean() < 1.0
    assert gains[:, 1].mean() < 1.0
