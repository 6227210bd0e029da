"""Pins for the FP64 reference of the cost model's network (CPU only):
the analytic gradient against central finite differences, and the forward
pass against a hand-built network whose output is known."""
import numpy as np

import synth
from oracle import mlp as ref


def _params(d, seed):
    rng = synth.rng_for(seed)
    n = ref.H * d + ref.H + ref.H * ref.H + ref.H + ref.H + 1
    return rng.normal(0, 0.3, n)


def test_gradient_matches_finite_differences():
    d = 5
    p = _params(d, 1)
    rng = synth.rng_for(2)
    X = rng.normal(0, 1, (13, d))
    y = rng.normal(0, 1, 13)
    _, g = ref.loss_grad(p, X, y)
    idx = rng.choice(len(p), 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        fd = (ref.loss(p + e, X, y) - ref.loss(p - e, X, y)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_of_a_hand_built_network():
    # W1 copies x0 into unit 0 and -x0 into unit 1, W2 passes both through,
    # W3 adds them: output = relu(x0) + relu(-x0) + 0.5 = |x0| + 0.5
    d = 3
    W1 = np.zeros((ref.H, d))
    W1[0, 0], W1[1, 0] = 1.0, -1.0
    W2 = np.zeros((ref.H, ref.H))
    W2[0, 0] = W2[1, 1] = 1.0
    W3 = np.zeros((1, ref.H))
    W3[0, 0] = W3[0, 1] = 1.0
    p = np.concatenate([W1.ravel(), np.zeros(ref.H), W2.ravel(), np.zeros(ref.H), W3.ravel(), [0.5]])
    X = np.array([[2.0, 7.0, -1.0], [-3.0, 0.0, 0.0], [0.0, 1.0, 1.0]])
    assert ref.forward(p, X).tolist() == [2.5, 3.5, 0.5]
    assert ref.loss(p, X, [2.5, 3.5, 0.5]) == 0.0


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -7, 1.0 + 3 * 2.0 ** -8], dtype=np.float32)
    # halfway cases round to even
    assert ref.bf16(x).tolist() == [1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6]


def test_adam_first_step_closed_form():
    # from zero moments the bias corrections cancel: m_hat = g, v_hat = g^2
    rng = synth.rng_for(4)
    g = rng.normal(0, 1, 50) * np.logspace(-6, 3, 50)
    p0 = rng.normal(0, 1, 50)
    lr = 0.01
    p1, m, v = ref.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr)
    assert np.allclose(p1 - p0, -lr * g / (np.abs(g) + ref.EPS), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_keeps_its_step():
    # with g fixed, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so every
    # bias-corrected step is again -lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, -2e4])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    lr = 1e-3
    for t in range(1, 41):
        p, m, v = ref.adam_step(p, g, m, v, t, lr)
    assert np.allclose(p, -40 * lr * g / (np.abs(g) + ref.EPS), rtol=1e-9, atol=0)


def test_adam_descends_a_quadratic():
    # f(p) = |p - c|^2 / 2 has gradient p - c: Adam approaches c
    c = np.array([1.0, -2.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = ref.adam_step(p, p - c, m, v, t, 0.01)
    assert np.abs(p - c).max() < 1e-2


def test_full_batch_training_lowers_the_loss():
    d = 4
    p = _params(d, 5) * 0.5
    rng = synth.rng_for(6)
    X = rng.normal(0, 1, (64, d))
    y = X[:, 0] - 2 * X[:, 1]
    p1, losses = ref.train_full_batch(p, X, y, 200, 1e-3)
    assert ref.loss(p1, X, y) < 0.5 * losses[0]
