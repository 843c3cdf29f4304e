"""Pins for the FP64 reference of the dispatcher network: central finite
differences of the loss, a hand-computed tiny case, and the parameter layout."""
import numpy as np

from oracle import mlp


def _data(seed, rows=12):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.N_PARAMS)
    mu = rng.normal(0, 1, mlp.N_IN)
    sd = rng.uniform(0.5, 2.0, mlp.N_IN)
    X = rng.normal(0, 1, (rows, mlp.N_IN))
    T = rng.normal(0, 1, (rows, mlp.N_OUT))
    M = (rng.random((rows, mlp.N_OUT)) < 0.6).astype(np.float64)
    M[0, 0] = 1.0
    return p, mu, sd, X, T, M


def test_parameter_count():
    assert mlp.N_PARAMS == 5508


def test_gradient_matches_central_differences():
    p, mu, sd, X, T, M = _data(1)
    L, g = mlp.loss_grad(p, mu, sd, X, T, M)
    assert abs(L - mlp.loss(p, mu, sd, X, T, M)) < 1e-12
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 150, replace=False), [0, 1023, 1024, 5503, 5507]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num = (mlp.loss(p + e, mu, sd, X, T, M) - mlp.loss(p - e, mu, sd, X, T, M)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-5 * abs(num), (i, num, g[i])


def test_single_active_path_by_hand():
    # one input feature, one unit per layer active: y0 = w3 * relu(w2 * relu(w1 * x))
    p = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = (np.zeros(s) for s in [(64, 16), (64,), (64, 64), (64,), (4, 64), (4,)])
    W1[0, 0], W2[0, 0], W3[0, 0], b3[1] = 2.0, 3.0, 0.5, 7.0
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    X = np.zeros((1, 16))
    X[0, 0] = 1.5
    Y, _ = mlp.forward(p, np.zeros(16), np.ones(16), X)
    assert np.allclose(Y[0], [0.5 * 3.0 * 2.0 * 1.5, 7.0, 0.0, 0.0])
    X[0, 0] = -1.5  # the first ReLU cuts the path
    Y, _ = mlp.forward(p, np.zeros(16), np.ones(16), X)
    assert np.allclose(Y[0], [0.0, 7.0, 0.0, 0.0])
    # masked loss: only output 0 counts
    T = np.array([[1.0, 100.0, 100.0, 100.0]])
    M = np.array([[1.0, 0.0, 0.0, 0.0]])
    assert mlp.loss(p, np.zeros(16), np.ones(16), X, T, M) == 1.0
