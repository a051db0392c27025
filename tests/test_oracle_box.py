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


def test_adaptive_leaves_integrate_a_cubic_like_the_uniform_grid():
    """A global cubic is fitted exactly on every leaf, so any leaf set over the
    square gives the same potential: adaptive leaves (levels 2-6, refined
    towards a point) against the uniform 64 x 64 grid."""
    root = (0.0, 0.0, 1.0)
    lv, ix, iy = X.balanced_leaves(root, (0.3, 0.6), 6)
    c = X.leaf_cells(lv, ix, iy, root)
    t = np.array([[0.31, 0.61], [0.8, 0.2], [0.05, 0.93]])
    va = X.potential_leaves(lv, ix, iy, root, _cubic(c[:, 0], c[:, 1]), 0.05, t)
    g = (0.0, 0.0, 1 / 64, 64, 64)
    cu = _cells(g)
    vu = X.potential(_cubic(cu[:, 0], cu[:, 1]), g, 0.05, t)
    assert np.max(np.abs(va - vu) / np.abs(vu)) < 1e-10


def test_balanced_leaves_tile_the_square_two_to_one():
    root = (0.0, 0.0, 1.0)
    lv, ix, iy = X.balanced_leaves(root, (0.3, 0.6), 7)
    s = 0.5 ** lv.astype(float)
    assert abs(np.sum(s * s) - 1.0) < 1e-12
    x0, y0 = ix * s, iy * s
    for a in range(len(lv)):
        touch = ((x0 <= x0[a] + s[a]) & (x0[a] <= x0 + s) & (y0 <= y0[a] + s[a]) & (y0[a] <= y0 + s))
        assert np.all(np.abs(lv[touch] - lv[a]) <= 1)


def test_refinement_test_is_fourth_order_and_exact_for_cubics():
    root = (0.0, 0.0, 1.0)
    q = lambda x, y: x ** 4 + 0.3 * y ** 4
    errs = []
    for l in (3, 4, 5):
        n = 2 ** l
        ix, iy = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
        lv = np.full(n * n, l)
        c16 = X.leaf_cells(lv, ix.ravel(), iy.ravel(), root)
        c64 = X.leaf_cells(np.full(4 * n * n, l + 1),
                           (2 * ix.ravel()[:, None] + np.array([0, 1, 0, 1])).ravel(),
                           (2 * iy.ravel()[:, None] + np.array([0, 0, 1, 1])).ravel(), root)
        f16, e16 = X.refine_flags(_cubic(c16[:, 0], c16[:, 1]), _cubic(c64[:, 0], c64[:, 1]), 1e-12)
        assert not f16.any() and e16.max() < 1e-12
        _, e = X.refine_flags(q(c16[:, 0], c16[:, 1]), q(c64[:, 0], c64[:, 1]), 0.0)
        errs.append(e.max())
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18, errs
