"""FP64 reference of the learned closure's network and of its training step.

Test infrastructure only (see ``oracle/__init__``).

The closure lets the level-1 SME stand in for level 8: a small MLP maps
per-cell features of the level-1 state to the missing tendency of the two
momentum moments.  The paper has no learned closure; this is the fixed
specification the library's FP32 kernels are checked against.

Network (4,930 parameters, flat FP32 layout shared with the library's C ABI):
    x~ = (x - mu) / sigma                     9 features
    a1 = tanh(W1 x~ + b1)                     W1: 64 x 9   (row-major, W1[j, i])
    a2 = tanh(W2 a1 + b2)                     W2: 64 x 64
    y~ = W3 a2 + b3                           W3: 2 x 64
    y  = y~ * s_out                           correction rates of (q_0, q_1)
flat order: W1, b1, W2, b2, W3, b3.

Loss on normalised targets t~ = t / s_out:  L = (1/B) sum_b sum_o (y~_bo - t~_bo)^2.
Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Features of cell i along a direction with normal momenta (q_0, q_1):
    (h_i, q0_i, q1_i, h_{i+1}-h_i, q0_{i+1}-q0_i, q1_{i+1}-q1_i,
     h_i-h_{i-1}, q0_i-q0_{i-1}, q1_i-q1_{i-1})
Training target (a-priori closure): r = [P(Q8^{n+1}) - Step_L1(P(Q8^n))] / dt
restricted to (q_0, q_1), where P keeps (h, q_0, q_1) of a level-8 state (the
basis is orthogonal, so truncation is the projection) and Step_L1 is one
level-1 step with the same dt.
"""
import numpy as np

NIN, NH, NOUT = 9, 64, 2
NPARAM = NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + NH * NIN].reshape(NH, NIN); o += NH * NIN
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    W3 = p[o:o + NOUT * NH].reshape(NOUT, NH); o += NOUT * NH
    b3 = p[o:o + NOUT]; o += NOUT
    assert o == NPARAM
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def init_params(seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    def g(o, i):
        a = np.sqrt(6.0 / (i + o))
        return rng.uniform(-a, a, size=(o, i))
    return pack(g(NH, NIN), np.zeros(NH), g(NH, NH), np.zeros(NH), g(NOUT, NH), np.zeros(NOUT))


def forward(p, xn):
    """Normalised inputs (B, 9) -> normalised outputs (B, 2) and activations."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    a1 = np.tanh(xn @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    y = a2 @ W3.T + b3
    return y, (xn, a1, a2)


def loss_grad(p, xn, tn):
    """MSE loss on normalised targets and its gradient (reverse mode by hand)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (x, a1, a2) = forward(p, xn)
    B = x.shape[0]
    r = y - tn
    loss = np.sum(r * r) / B
    dy = 2.0 * r / B
    gW3 = dy.T @ a2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (1.0 - a2 * a2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - a1 * a1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features_1d(h, q0, q1):
    """Per-cell features on a periodic 1D row (arrays of length n)."""
    hp, q0p, q1p = np.roll(h, -1), np.roll(q0, -1), np.roll(q1, -1)
    hm, q0m, q1m = np.roll(h, 1), np.roll(q0, 1), np.roll(q1, 1)
    return np.stack([h, q0, q1, hp - h, q0p - q0, q1p - q1, h - hm, q0 - q0m, q1 - q1m], axis=1)


def closure_target(q8_now, q8_next, q1_step, dt):
    """Training target (B, 2) for the momentum moments q_0, q_1."""
    return np.stack([(q8_next[1] - q1_step[1]) / dt, (q8_next[2] - q1_step[2]) / dt], axis=1)
