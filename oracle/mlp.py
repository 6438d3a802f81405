"""FP64 reference of the temperature-step perceptron and its features.

TEST INFRASTRUCTURE ONLY.  Plain numpy in double precision; the device
kernels compute in FP32.  The learned part is not in the paper: the network
proposes the next inverse-temperature step from the population's energy
histogram; the histogram-overlap criterion of the self-adaptive schedule
(Sec. "Algorithm") stays the fallback and decides whether a proposal is taken.

Parameters (one flat vector): W1[64][35], b1[64], W2[64][64], b2[64], w3[64], b3.
Network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = w3 . h2 + b3.
Loss: mean squared error (1/n) sum (y_k - t_k)^2.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 35, 64
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    o = 0
    W1 = p[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    w3 = p[o:o + N_H]; o += N_H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    o = 0
    p[o:o + N_H * N_IN] = rng.uniform(-1, 1, N_H * N_IN) / np.sqrt(N_IN); o += N_H * N_IN
    o += N_H
    p[o:o + N_H * N_H] = rng.uniform(-1, 1, N_H * N_H) / np.sqrt(N_H); o += N_H * N_H
    o += N_H
    p[o:o + N_H] = rng.uniform(-1, 1, N_H) / np.sqrt(N_H)
    return p


def forward(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3, h1, h2


def loss(p, X, T):
    y, _, _ = forward(p, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_and_grad(p, X, T):
    """Backpropagation of the mean squared error by the chain rule."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    y, h1, h2 = forward(p, X)
    r = y - T
    g = 2.0 * r / n                      # dL/dy
    gw3 = h2.T @ g
    gb3 = g.sum()
    d2 = np.outer(g, w3) * (1 - h2 ** 2)  # dL/d(pre-activation 2)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1 - h1 ** 2)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return float(np.mean(r ** 2)), grad


def adam_step(p, m, v, grad, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad ** 2
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(E, beta: float, N: int) -> np.ndarray:
    """35 inputs from a population's energies: the histogram of z = (E - <E>) /
    sigma_E on 32 bins over [-4, 4) normalised to sum 1, beta, <E>/N, Var(E)/N
    (population variance).  Mean and variance come from exact integer sums."""
    E = [int(e) for e in E]
    R = len(E)
    S1 = sum(E)
    S2 = sum(e * e for e in E)
    mean = S1 / R
    var = (R * S2 - S1 * S1) / (R * R)
    sd = var ** 0.5
    counts = np.zeros(32, dtype=np.int64)
    for e in E:
        z = (e - mean) / sd if sd > 0 else 0.0
        b = int(np.floor((z + 4.0) * 4.0))
        if 0 <= b < 32:
            counts[b] += 1
    tot = counts.sum()
    out = np.zeros(N_IN)
    out[:32] = counts / tot if tot else 0.0
    out[32] = beta
    out[33] = mean / N
    out[34] = var / N
    return out
