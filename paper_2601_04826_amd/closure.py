"""Learned closure: level 1 plus a small network standing in for level 8.

Everything numeric runs in the library: the level-8 and level-1 SME steps
that generate the data, the sample extraction (features and a-priori
targets), the feature statistics behind the scaling and the training box, the
initialisation and the training loop (forward, backward, Adam, learning-rate
schedule, seeded batch permutations: sme_closure_train), the rates pass
before every level-1 step and the chunked run with its level-8 fallback
(sme_closure_run).  This module only marshals: torch holds device buffers, a
seeded numpy generator draws the cells sampled from each snapshot.

Target (a-priori closure): for consecutive level-8 states Q8^n, Q8^{n+1} with
step dt, r = [P(Q8^{n+1}) - Step_L1(P(Q8^n))] / dt on (q_0, q_1), where P keeps
(h, q_0, q_1) (the Legendre basis is orthogonal, so truncation is the
projection).  Level 1 plus closure then advances Q1^{n+1} = Step_L1(Q1^n) + dt r(Q1^n).
Outside the range of its training features the network is not trusted: such a
cell gets no correction in that step, and once more than a small fraction of
cell-steps of a chunk were out of range the level-1 run stops and the plain
level-8 solver continues from the lifted state.
"""
import numpy as np
import torch

from . import sme, workloads

N_IN, N_OUT = 9, 2


def _project(problem8, level=1):
    p = dict(problem8)
    p["level"] = level
    p["q"] = np.ascontiguousarray(problem8["q"][: level + 2])
    return p


def generate(seeds, n=4096, steps=2000, every=10, cells_per_snapshot=256, stream=None, rng_seed=0):
    """Training samples from level-8 runs of the solver itself.

    Returns (features [S, 9], targets [S, 2]) as float32 CUDA tensors."""
    st = stream or torch.cuda.Stream()
    rng = np.random.default_rng(rng_seed)
    snaps = len(range(0, steps, every))
    total = len(seeds) * snaps * cells_per_snapshot
    feat = torch.empty((total, N_IN), dtype=torch.float32, device="cuda")
    targ = torch.empty((total, N_OUT), dtype=torch.float32, device="cuda")
    at = 0
    with torch.cuda.stream(st):
        for seed in seeds:
            p8 = workloads.smooth_1d(n=n, level=8, seed=seed, steps=steps)
            s8 = sme.Solver(p8, stream=st.cuda_stream)
            s8.set_state(p8["q"])
            p1 = _project(p8)
            s1 = sme.Solver(p1, stream=st.cuda_stream)
            q8 = torch.empty((p8["q"].shape[0], n), dtype=torch.float64, device="cuda")
            q8n = torch.empty_like(q8)
            q1 = torch.empty((3, n), dtype=torch.float64, device="cuda")
            for k in range(steps):
                if k % every:
                    s8.step(0.0)
                    continue
                s8.get_state(q8)
                dt = s8.step(0.0, sync=True)
                s8.get_state(q8n)
                s1.set_state(q8[:3])
                s1.step(dt)
                s1.get_state(q1)
                cells = torch.from_numpy(rng.choice(n, size=cells_per_snapshot, replace=False).astype(np.int64)).cuda()
                sme.closure_samples(q8, q8n, q1, dt, cells, stream=st.cuda_stream,
                                    out=(feat[at:at + cells_per_snapshot], targ[at:at + cells_per_snapshot]))
                at += cells_per_snapshot
            s8.close()
            s1.close()
        st.synchronize()
    assert at == total
    return feat, targ


def fit(feat, targ, epochs=20, batch=4096, lr=2e-3, lr_end=1e-4, seed=0, stream=None, log=None, margin=0.1):
    """Train the network with the library (sme_mlp_init, sme_closure_train:
    scaling and training box from the samples, Adam on normalised targets with
    a geometric learning-rate decay, seeded batch permutations).  Returns
    (MLP, scaling dict, loss history)."""
    st = stream or torch.cuda.Stream()
    with torch.cuda.stream(st):
        mlp = sme.MLP(stream=st.cuda_stream)
        mlp.init(seed)
        hist = mlp.train(feat, targ, epochs, batch, lr, lr_end, seed, margin=margin)
        sc = mlp.get_scaling()
    if log:
        for ep, loss in enumerate(hist):
            log(f"epoch {ep + 1}/{epochs} loss {loss:.5f}")
    return mlp, sc, hist


def relative_l1(q, q_ref, fields=(0, 1)):
    """E_x = sum_i |x_i - x_i^ref| / sum_i |x_i^ref| for x = h and hu (equal cells)."""
    return {f: float(np.sum(np.abs(q[f] - q_ref[f])) / np.sum(np.abs(q_ref[f]))) for f in fields}


class ClosureSolver:
    """Level 1 + closure on a 1D or structured grid, with the plain level-8
    solver as fallback once the features leave the training range
    (sme_closure_run: the chunk checkpoints and the fallback stay on the device)."""

    def __init__(self, problem8, mlp, chunk=50, stream=None, max_out_of_range=1e-3, precision="fp32"):
        self.p8 = problem8
        self.mlp = mlp
        self.chunk = chunk
        self.max_oor = max_out_of_range  # tolerated fraction of out-of-range cell-steps
        self.s1 = sme.Solver(_project_any(problem8), stream=stream)
        self.s1.attach_closure(mlp, precision=precision)
        self.s8 = sme.Solver(problem8, stream=stream)
        self.fell_back_at = None

    def set_state(self, q8):
        self.s1.set_state(_project_state(q8, self.p8))

    def run_to(self, t_end, max_steps=10 ** 7, lifted=True):
        """Advance to t_end; returns the final state lifted to the level-8
        layout (lifted=False: no copy back, see final_solver)."""
        t, n, fb = sme.closure_run(self.s1, self.s8, t_end, self.chunk, max_steps, self.max_oor)
        self.fell_back_at = fb
        self.t, self.steps = t, n
        if not lifted:
            return None
        if fb is not None:
            return self.s8.get_state()
        return _lift_state(self.s1.get_state(), self.p8)

    def final_solver(self):
        """The Solver that holds the final state of the last run_to."""
        return self.s8 if self.fell_back_at is not None else self.s1

    def close(self):
        self.s1.close()
        self.s8.close()


def _project_any(problem8):
    p = dict(problem8)
    p["level"] = 1
    p["q"] = _project_state(problem8["q"], problem8)
    return p


def _project_state(q8, problem8):
    """(h, q_0, q_1) of each direction block of a level-8 state (numpy array,
    or torch tensor kept on its device)."""
    n8 = problem8["level"] + 1
    if isinstance(q8, torch.Tensor):
        if problem8["kind"] == "1d":
            return q8[:3].contiguous()
        return torch.cat([q8[:3], q8[1 + n8:1 + n8 + 2]]).contiguous()
    if problem8["kind"] == "1d":
        return np.ascontiguousarray(q8[:3])
    return np.ascontiguousarray(np.concatenate([q8[:3], q8[1 + n8:1 + n8 + 2]]))


def _lift_state(q1, problem8):
    """Level-1 state padded with zero higher moments to the level-8 layout."""
    n8 = problem8["level"] + 1
    if problem8["kind"] == "1d":
        out = np.zeros((n8 + 1, q1.shape[1]))
        out[:3] = q1
        return out
    out = np.zeros((2 * n8 + 1, q1.shape[1]))
    out[:3] = q1[:3]
    out[1 + n8:1 + n8 + 2] = q1[3:5]
    return out
