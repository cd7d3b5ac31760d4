"""Oracle of the skeleton-rank predictor (test infrastructure only).

The paper has no learned component; this is the project's addition: a small MLP
that maps features of a box (known before its ID: level, box side, active DOFs,
near-field DOFs, ID tolerance, dimension) to log2(k + 1), k the numerical rank
the pivoted QR will find (Section 4.2, (e:id)).

Network: x (F) -> W1 x + b1 -> ReLU -> W2 h + b2 -> ReLU -> W3 h + b3 (scalar).
Weights are rounded to bfloat16 (round to nearest, ties to even) before use;
biases, activations and sums are FP32 on the GPU and FP64 here.  Loss: mean
squared error.  The weight gradient is taken with respect to the rounded
weights and applied to the FP32 master weights (straight-through rounding).
Adam (Kingma & Ba, 2015) updates the master weights.

Flat parameter layout (float32): W1 (H x F, row-major), b1 (H), W2 (H x H),
b2 (H), W3 (H), b3 (1).
"""
import numpy as np

F = 6
H = 64


def n_params():
    return H * F + H + H * H + H + H + 1


def split(p):
    p = np.asarray(p)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def bf16_round(w):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    u = np.asarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def init_params(seed=0):
    """He-style initialization with a fixed seed (float32)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, F)) * np.sqrt(2.0 / F)
    W2 = rng.standard_normal((H, H)) * np.sqrt(2.0 / H)
    W3 = rng.standard_normal(H) * np.sqrt(1.0 / H)
    p = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3, np.zeros(1)])
    return p.astype(np.float32)


def forward(p, X, rounded=True):
    """Predictions (n,) and the activations needed by backward."""
    if rounded:
        W1, b1, W2, b2, W3, b3 = split(np.asarray(p, dtype=np.float32))
        W1, W2, W3 = bf16_round(W1), bf16_round(W2), bf16_round(W3)
    else:
        W1, b1, W2, b2, W3, b3 = split(np.asarray(p, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (a.astype(np.float64) for a in (W1, b1, W2, b2, W3, b3))
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3[0]
    return y, (X, z1, h1, z2, h2, W2, W3)


def loss_and_grad(p, X, t, rounded=True):
    """Mean squared error and its gradient (flat, like p)."""
    y, (X, z1, h1, z2, h2, W2, W3) = forward(p, X, rounded)
    t = np.asarray(t, dtype=np.float64)
    n = len(t)
    r = y - t
    loss = np.mean(r * r)
    dy = 2.0 * r / n
    dW3 = dy @ h2
    db3 = np.array([dy.sum()])
    dz2 = np.outer(dy, W3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, db3])
    return loss, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (returns new p, m, v); step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
