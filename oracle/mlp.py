"""FP64 reference of the dispatcher network and its training loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: 16 standardised inputs -> 64 ReLU -> 64 ReLU -> 4 linear outputs.
Parameter vector layout: W1[64][16] b1[64] W2[64][64] b2[64] W3[4][64] b3[4]
(5,508 numbers).  Loss: masked mean-squared error
    L = sum_i sum_a m_ia (y_ia - t_ia)^2 / sum_ia m_ia.
The gradient is written out by the chain rule (reverse mode) and is pinned in
the tests by central finite differences of ``loss`` itself.
"""
from __future__ import annotations

import numpy as np

N_IN, H1, H2, N_OUT = 16, 64, 64, 4
N_PARAMS = H1 * N_IN + H1 + H2 * H1 + H2 + N_OUT * H2 + N_OUT


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0

    def take(n, shape):
        nonlocal o
        a = p[o:o + n].reshape(shape)
        o += n
        return a

    W1 = take(H1 * N_IN, (H1, N_IN))
    b1 = take(H1, (H1,))
    W2 = take(H2 * H1, (H2, H1))
    b2 = take(H2, (H2,))
    W3 = take(N_OUT * H2, (N_OUT, H2))
    b3 = take(N_OUT, (N_OUT,))
    assert o == N_PARAMS
    return W1, b1, W2, b2, W3, b3


def forward(p, mu, sd, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Z = (np.asarray(X, np.float64) - np.asarray(mu, np.float64)) / np.asarray(sd, np.float64)
    A1 = Z @ W1.T + b1
    H1a = np.maximum(A1, 0.0)
    A2 = H1a @ W2.T + b2
    H2a = np.maximum(A2, 0.0)
    Y = H2a @ W3.T + b3
    return Y, (Z, A1, H1a, A2, H2a)


def loss(p, mu, sd, X, T, M):
    Y, _ = forward(p, mu, sd, X)
    M = np.asarray(M, np.float64)
    return float((M * (Y - np.asarray(T, np.float64)) ** 2).sum() / M.sum())


def loss_grad(p, mu, sd, X, T, M):
    """(loss, gradient) by reverse-mode differentiation of the network."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Y, (Z, A1, H1a, A2, H2a) = forward(p, mu, sd, X)
    M = np.asarray(M, np.float64)
    E = Y - np.asarray(T, np.float64)
    msum = M.sum()
    L = float((M * E ** 2).sum() / msum)
    dY = 2.0 * M * E / msum
    gW3 = dY.T @ H2a
    gb3 = dY.sum(0)
    dH2 = (dY @ W3) * (A2 > 0)
    gW2 = dH2.T @ H1a
    gb2 = dH2.sum(0)
    dH1 = (dH2 @ W2) * (A1 > 0)
    gW1 = dH1.T @ Z
    gb1 = dH1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g
