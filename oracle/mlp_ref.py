"""CPU ORACLE for the selector's cost model -- TEST INFRASTRUCTURE ONLY.

Plain float64 numpy implementation of the multilayer perceptron
16 -> 64 -> 64 -> K with ReLU hidden layers and the loss mean((y - t)^2)
over samples and outputs, used to check the GPU forward and gradient
kernels.  Parameter layout (flat): W1[16][64], b1[64], W2[64][64], b2[64],
W3[64][K], b3[K]; W[i][j] multiplies input i into unit j.

Gradients are the chain rule written out layer by layer; fd_grad gives
central finite differences of the loss (the pin of the analytic gradient).
"""
from __future__ import annotations

import numpy as np

NI, H = 16, 64


def n_params(k: int) -> int:
    return NI * H + H + H * H + H + H * k + k


def unpack(p, k: int):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n_params(k)
    o = 0
    W1 = p[o:o + NI * H].reshape(NI, H); o += NI * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H * k].reshape(H, k); o += H * k
    b3 = p[o:o + k]
    return W1, b1, W2, b2, W3, b3


def forward(p, x, k: int):
    W1, b1, W2, b2, W3, b3 = unpack(p, k)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t, k: int) -> float:
    y, _ = forward(p, x, k)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, x, t, k: int) -> np.ndarray:
    W1, b1, W2, b2, W3, b3 = unpack(p, k)
    y, (x, z1, h1, z2, h2) = forward(p, x, k)
    B = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / (B * k)   # d loss / d y
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def fd_grad(p, x, t, k: int, idx, eps: float = 1e-6) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64).copy()
    out = np.zeros(len(idx))
    for n, i in enumerate(idx):
        old = p[i]
        p[i] = old + eps
        lp = loss(p, x, t, k)
        p[i] = old - eps
        lm = loss(p, x, t, k)
        p[i] = old
        out[n] = (lp - lm) / (2 * eps)
    return out
