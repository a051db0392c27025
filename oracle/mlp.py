"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

Plain numpy forward pass and backpropagation of
    y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3,   loss = mean (y - t)^2,
written from the chain rule, on the same flat parameter layout as the
library (W1 [H][Fp], b1 [H], W2 [H][H], b2 [H], w3 [H], b3), and one step of
the Adam optimiser (Kingma & Ba, 2015: first and second moment estimates with
decays b1, b2, each divided by (1 - b^t) to undo its zero start).
"""
from __future__ import annotations

import numpy as np


def unpack(p, H, Fp):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * Fp].reshape(H, Fp); o += H * Fp
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, H, Fp, X):
    W1, b1, W2, b2, w3, b3 = unpack(p, H, Fp)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3, (X, h1, h2)


def loss(p, H, Fp, X, t):
    y, _ = forward(p, H, Fp, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_grad(p, H, Fp, X, t):
    W1, b1, W2, b2, w3, b3 = unpack(p, H, Fp)
    y, (X, h1, h2) = forward(p, H, Fp, X)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    d2 = np.outer(dy, w3) * (1.0 - h2 ** 2)
    g_W2 = d2.T @ h1
    g_b2 = d2.sum(0)
    d1 = (d2 @ W2) * (1.0 - h1 ** 2)
    g_W1 = d1.T @ X
    g_b1 = d1.sum(0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return float(np.mean((y - t) ** 2)), g


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Step t (1-based) of Adam from moments m, v; returns (p, m, v)."""
    p = np.asarray(p, dtype=np.float64); g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
