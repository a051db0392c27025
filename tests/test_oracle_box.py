"""Pins of the box-code oracle (oracle/box.py, Sec. 3.1 eq. volume_potential):
the leaf fit reproduces cubics, the quadrature of K0 times the leaf
polynomials matches adaptive 2-D quadrature split at the target, and the
scheme converges at fourth order to the closed-form potential of a plane
wave."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import k0

from oracle import box as X


def _cells(grid):
    x0, y0, h, nx, ny = grid
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    return np.stack([x0 + (i.ravel() + 0.5) * h, y0 + (j.ravel() + 0.5) * h], 1)


def _cubic(x, y):
    return 1.0 + 0.5 * x - 2.0 * y * y + 1.5 * x * x * y - 0.7 * y ** 3


def test_leaf_fit_reproduces_cubics_and_not_quartics():
    grid = (-0.3, 0.1, 0.05, 16, 12)
    c = _cells(grid)
    rng = np.random.default_rng(1)
    pts = np.stack([grid[0] + rng.random(200) * 16 * 0.05, grid[1] + rng.random(200) * 12 * 0.05], 1)
    got = X.leaf_eval(_cubic(c[:, 0], c[:, 1]), grid, pts)
    assert np.max(np.abs(got - _cubic(pts[:, 0], pts[:, 1]))) < 1e-12
    q = lambda x, y: x ** 4 + y ** 4
    got4 = X.leaf_eval(q(c[:, 0], c[:, 1]), grid, pts)
    assert np.max(np.abs(got4 - q(pts[:, 0], pts[:, 1]))) > 1e-9


def _ref(f, grid, alpha, t):
    """(1/(2 pi)) int_D K0(|t - y|/alpha) f(y) dy by adaptive quadrature, the
    domain split at the target."""
    x0, y0, h, nx, ny = grid
    x1, y1 = x0 + nx * h, y0 + ny * h
    tx, ty = t
    tot = 0.0
    for a, b in ((x0, tx), (tx, x1)):
        for c, d in ((y0, ty), (ty, y1)):
            tot += integrate.dblquad(lambda y, x: k0(np.hypot(x - tx, y - ty) / alpha) * f(x, y), a, b, c, d,
                                     epsabs=1e-15, epsrel=1e-13)[0]
    return tot / (2 * np.pi)


@pytest.mark.parametrize("density", ["constant", "cubic"])
def test_potential_matches_adaptive_quadrature(density):
    grid = (0.0, 0.0, 1 / 16, 16, 16)
    alpha = 0.1
    f = (lambda x, y: np.ones_like(np.asarray(x, dtype=float))) if density == "constant" else _cubic
    c = _cells(grid)
    vals = f(c[:, 0], c[:, 1])
    # a cell centre inside, one next to a leaf corner, one off the grid's cells
    tg = np.array([[5.5 / 16, 9.5 / 16], [7.9 / 16, 8.02 / 16], [0.91, 0.13]])
    got = X.potential(vals, grid, alpha, tg)
    ref = np.array([_ref(f, grid, alpha, t) for t in tg])
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-10, (got, ref)


def test_plane_wave_fourth_order():
    """B = exp(k.x), |k| alpha = 1/4: far from the boundary of D the potential
    is exp(k.x) alpha^2 / (1 - alpha^2 |k|^2) up to e^{-dist/alpha}; the
    error of the fitted cubics falls at least 16x per halving of h (about 30x
    here: the fit's residual is orthogonal to the constants on each leaf, so
    its leading term integrates nearly to zero against the smooth kernel away
    from the target)."""
    alpha = 0.02
    kv = np.array([0.6, 0.8]) * 0.25 / alpha
    errs = []
    for n in (64, 128):
        grid = (0.0, 0.0, 1.0 / n, n, n)
        c = _cells(grid)
        vals = np.exp(c @ kv)
        tg = np.array([[0.5, 0.5], [0.45, 0.55], [0.53, 0.47]]) + 0.5 / n   # cell centres
        got = X.potential(vals, grid, alpha, tg)
        exact = np.exp(tg @ kv) * alpha ** 2 / (1 - alpha ** 2 * kv @ kv)
        errs.append(np.max(np.abs(got - exact) / exact))
    print("plane wave errors", errs)
    assert errs[1] < 5e-6 and 12 < errs[0] / errs[1] < 70
