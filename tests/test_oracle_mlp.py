"""Pins of the FP64 network reference: central differences of its loss."""
import numpy as np

from oracle import mlp


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(0)
    H, Fp, n = 8, 16, 20
    npar = H * Fp + H + H * H + H + H + 1
    p = rng.standard_normal(npar) * 0.3
    X = rng.standard_normal((n, Fp))
    t = rng.standard_normal(n)
    _, g = mlp.loss_grad(p, H, Fp, X, t)
    eps = 1e-6
    for i in rng.choice(npar, size=40, replace=False):
        e = np.zeros(npar); e[i] = eps
        fd = (mlp.loss(p + e, H, Fp, X, t) - mlp.loss(p - e, H, Fp, X, t)) / (2 * eps)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_loss_at_exact_targets():
    rng = np.random.default_rng(1)
    H, Fp = 4, 8
    p = rng.standard_normal(H * Fp + H + H * H + H + H + 1)
    X = rng.standard_normal((5, Fp))
    y, _ = mlp.forward(p, H, Fp, X)
    l, g = mlp.loss_grad(p, H, Fp, X, y)
    assert l == 0.0 and np.all(g == 0.0)
