"""ORACLE — test infrastructure only (see oracle/__init__.py).

fp64 reference of the parameter-choice network: 16 -> 64 -> 64 -> 32, ReLU,
loss = mean over the batch and outputs of (y - target)^2, and one Adam step
(Kingma & Ba 2015).  Parameters are one flat vector laid out as
W1[16][64], b1[64], W2[64][64], b2[64], W3[64][32], b3[32] (y = x W + b).
"""
import numpy as np

F, H, G = 16, 64, 32
SHAPES = [(F, H), (H,), (H, H), (H,), (H, G), (G,)]
NUM_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, off = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(p[off:off + k].reshape(s))
        off += k
    return out


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t):
    y, _ = forward(p, x)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def gradient(p, x, t):
    """Analytic gradient of `loss` by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, x)
    B = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / (B * G)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (z2 > 0)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (z1 > 0)
    dW1 = x.T @ dh1
    db1 = dh1.sum(axis=0)
    return np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])


def adam_step(p, g, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    c1, c2 = 1 - beta1 ** step, 1 - beta2 ** step
    return p - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2


def init_params(rng):
    """He-style initialisation (weights ~ N(0, 2/fan_in), biases 0)."""
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / s[0]), size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)
