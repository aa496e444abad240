"""TEST INFRASTRUCTURE -- FP64 reference of the learned decimation proposer's
network (the project's addition to the paper's method, so no paper passage
defines it; the definitions are the usual ones, written out plainly).

Network: x (17) -> h1 = relu(x W1 + b1) (64) -> h2 = relu(h1 W2 + b2) (64)
-> z = h2 . w3 + b3. Loss: mean binary cross-entropy of the logit z against
the label y in {0, 1}: log(1 + e^z) - y z. Gradient by the chain rule.
Parameter vector: W1 [17][64] (input-major), b1, W2 [64][64], b2, w3, b3.

Only tests call this module.
"""
import numpy as np

IN, H = 17, 64
N_PARAMS = IN * H + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, np.float64)
    i = 0
    W1 = p[i:i + IN * H].reshape(IN, H)
    i += IN * H
    b1 = p[i:i + H]
    i += H
    W2 = p[i:i + H * H].reshape(H, H)
    i += H * H
    b2 = p[i:i + H]
    i += H
    w3 = p[i:i + H]
    i += H
    b3 = p[i]
    return W1, b1, W2, b2, w3, b3


def forward(p, x):
    """Logits z [n] of features x [n][17]."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, np.float64)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ w3 + b3


def loss(p, x, y):
    z = forward(p, x)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def loss_grad(p, x, y):
    """(mean loss, gradient [N_PARAMS]) by backpropagation."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.shape[0]
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    L = float(np.mean(np.logaddexp(0.0, z) - y * z))
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n          # d loss / d z
    dw3 = h2.T @ dz
    db3 = dz.sum()
    dh2 = np.outer(dz, w3) * (a2 > 0)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (a1 > 0)
    dW1 = x.T @ dh1
    db1 = dh1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
    return L, g


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), bias-corrected, t >= 1; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, x):
    """The inference arithmetic: inputs, weights and the first hidden layer
    rounded to bfloat16, everything else exact (float64 stands in for the
    matrix cores' float32 accumulation)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    xb = bf16(np.asarray(x, np.float32))
    h1 = np.maximum(xb @ bf16(W1.astype(np.float32)) + b1, 0.0)
    h1 = bf16(h1.astype(np.float32))
    h2 = np.maximum(h1 @ bf16(W2.astype(np.float32)) + b2, 0.0)
    return h2 @ w3 + b3
