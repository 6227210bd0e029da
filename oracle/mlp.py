"""FP64 reference of the learned cost model's network -- TEST
INFRASTRUCTURE ONLY (used by tests to check the GPU kernels).

A 3-layer perceptron d_in -> 64 -> 64 -> 1 with ReLU on the hidden layers
and loss L = mean((p - y)^2) / 2.  Parameters are packed as
[W1 (64 x d_in), b1 (64), W2 (64 x 64), b2 (64), W3 (1 x 64), b3 (1)].
The gradient is the chain rule written out layer by layer; the tests pin
it with central finite differences of ``loss``.

Training follows Adam as Kingma and Ba define it (Adam: A Method for
Stochastic Optimization, 2015, Algorithm 1): exponential moving averages of
the gradient and of its square, each divided by its bias correction, and a
step of -lr * m_hat / (sqrt(v_hat) + eps).  The tests pin it with closed
forms: the first step from zero moments moves every parameter by
-lr * g / (|g| + eps), and a constant gradient keeps that step at every
iteration.
"""
import numpy as np

H = 64


def unpack(p, d_in):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * d_in].reshape(H, d_in); o += H * d_in
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H].reshape(1, H); o += H
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def forward(p, X):
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(p, X.shape[1])
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    return (a2 @ W3.T + b3)[:, 0]


def loss(p, X, y):
    d = forward(p, X) - np.asarray(y, dtype=np.float64)
    return 0.5 * float(np.mean(d * d))


def loss_grad(p, X, y):
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    W1, b1, W2, b2, W3, b3 = unpack(p, X.shape[1])
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    out = (a2 @ W3.T + b3)[:, 0]
    d = out - y
    L = 0.5 * float(np.mean(d * d))
    g3 = (d / n)[:, None]                 # dL/dz3
    gW3 = g3.T @ a2
    gb3 = g3.sum(axis=0)
    g2 = (g3 @ W3) * (z2 > 0)             # dL/dz2
    gW2 = g2.T @ a1
    gb2 = g2.sum(axis=0)
    g1 = (g2 @ W2) * (z1 > 0)             # dL/dz1
    gW1 = g1.T @ X
    gb1 = g1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, grad


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7fff + ((u >> 16) & 1)) & 0xffff0000
    return u.astype(np.uint32).view(np.float32)


def forward_bf16(p, X):
    """Forward pass with bf16 weights, inputs and layer outputs and fp32
    sums (the inference kernel's arithmetic, up to summation rounding)."""
    X = np.asarray(X, dtype=np.float32)
    W1, b1, W2, b2, W3, b3 = (bf16(w.astype(np.float32)) for w in unpack(p, X.shape[1]))
    x = bf16(X)
    a1 = bf16(np.maximum(x @ W1.T + b1, 0))
    a2 = bf16(np.maximum(a1 @ W2.T + b2, 0))
    return (a2 @ W3.T + b3)[:, 0].astype(np.float64)


BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def adam_step(p, g, m, v, t, lr, b1=BETA1, b2=BETA2, eps=EPS):
    """One Adam update at step t (1-based): returns (p, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def train_full_batch(p, X, y, steps, lr):
    """`steps` Adam steps on the whole batch (X, y), from zero moments.
    Returns the parameters and the loss before each step."""
    p = np.asarray(p, dtype=np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for t in range(1, steps + 1):
        L, g = loss_grad(p, X, y)
        losses.append(L)
        p, m, v = adam_step(p, g, m, v, t, lr)
    return p, losses
