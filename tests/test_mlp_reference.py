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
