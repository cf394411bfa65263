"""CPU reference of the moduli-count predictor network (FP64).

TEST INFRASTRUCTURE ONLY: the tests compare the library's FP32 training and
inference kernels with this file; nothing in the product path imports it.

The network is not part of the paper.  It is a plain 3-layer perceptron
    h1 = relu(W1 xs + b1),  h2 = relu(W2 h1 + b2),  z = W3 h2 + b3,
    xs = (x - mu) / sd   (per-feature standardisation, fixed before training)
trained with the mean softmax cross-entropy over a batch,
    L = (1 / B) sum_r [ logsumexp(z_r) - z_r[y_r] ],
and Adam (Kingma and Ba, 2015) with bias correction:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameter vector layout (shared with the C-ABI): W1 (H x F, row-major), b1 (H),
W2 (H x H), b2 (H), W3 (C x H), b3 (C), mu (F), sd (F).
"""
from __future__ import annotations

import numpy as np

F, H, C = 20, 64, 20


def sizes(f=F, h=H, c=C):
    return [h * f, h, h * h, h, c * h, c, f, f]


def unpack(p, f=F, h=H, c=C):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for sz in sizes(f, h, c):
        out.append(p[o:o + sz])
        o += sz
    W1, b1, W2, b2, W3, b3, mu, sd = out
    return (W1.reshape(h, f), b1, W2.reshape(h, h), b2, W3.reshape(c, h), b3, mu, sd)


def n_params(f=F, h=H, c=C):
    return sum(sizes(f, h, c))


def forward(p, X, f=F, h=H, c=C):
    """Logits and the intermediate activations for rows X (B x F)."""
    W1, b1, W2, b2, W3, b3, mu, sd = unpack(p, f, h, c)
    xs = (np.asarray(X, np.float64) - mu) / sd
    a1 = xs @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, dict(xs=xs, a1=a1, h1=h1, a2=a2, h2=h2)


def loss(p, X, y, f=F, h=H, c=C):
    z, _ = forward(p, X, f, h, c)
    zmax = z.max(axis=1, keepdims=True)
    lse = zmax[:, 0] + np.log(np.exp(z - zmax).sum(axis=1))
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def grad(p, X, y, f=F, h=H, c=C):
    """Gradient of the mean cross-entropy w.r.t. the trainable parameters (mu, sd: zero)."""
    W1, b1, W2, b2, W3, b3, mu, sd = unpack(p, f, h, c)
    z, a = forward(p, X, f, h, c)
    B = len(y)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    dz = e / e.sum(axis=1, keepdims=True)
    dz[np.arange(B), y] -= 1.0
    dz /= B
    gW3 = dz.T @ a["h2"]
    gb3 = dz.sum(axis=0)
    dh2 = (dz @ W3) * (a["a2"] > 0)
    gW2 = dh2.T @ a["h1"]
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (a["a1"] > 0)
    gW1 = dh1.T @ a["xs"]
    gb1 = dh1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3,
                           np.zeros(f), np.zeros(f)])


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, n_train=None):
    """One Adam step on the first n_train entries (the trainable ones)."""
    p, m, v = p.copy(), m.copy(), v.copy()
    n = len(p) if n_train is None else n_train
    m[:n] = b1 * m[:n] + (1 - b1) * g[:n]
    v[:n] = b2 * v[:n] + (1 - b2) * g[:n] ** 2
    mh = m[:n] / (1 - b1 ** t)
    vh = v[:n] / (1 - b2 ** t)
    p[:n] = p[:n] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def predict(p, X, f=F, h=H, c=C):
    z, _ = forward(p, X, f, h, c)
    return np.argmax(z, axis=1)
