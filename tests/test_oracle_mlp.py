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


def test_adam_first_step_is_lr_times_sign():
    """From zero moments the bias-corrected first step is -lr g / (|g| + eps),
    i.e. -lr sign(g) for |g| >> eps (Kingma & Ba, Sec. 2)."""
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50) * np.logspace(-3, 3, 50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    assert np.allclose(p1 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    big = np.abs(g) > 1e-2
    assert np.allclose((p1 - p)[big], -0.01 * np.sign(g[big]), rtol=1e-6, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_moves_linearly():
    """With a constant gradient the corrected moments equal g and g^2 at every
    step (the corrections undo the zero start exactly), so k steps move each
    parameter by -k lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(20)
    g = rng.standard_normal(20)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for t in range(1, 8):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-3)
    assert np.allclose(p - p0, -7e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=1e-15)
