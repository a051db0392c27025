"""Pins of the oracle's time schemes, grid quadrature, curve interpolation and
near-boundary evaluation against closed forms (not against the oracle
itself): every pin would fail for a dropped term, a wrong sign or a wrong
factor in the function it covers."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def G():
    from oracle import grid
    return grid


@pytest.fixture(scope="module")
def O():
    import oracle
    return oracle


def annulus(n0=256, n1=128):
    return W.make_boundary([W.circle((0.0, 0.0), 0.4, n0), W.circle((0.0, 0.0), 0.1, n1, ccw=False)])


# ---------------------------------------------------------------------------
# Time schemes (Sec. 2, eq. mod_helm_forced, eq. exg) on one eigenmode
# ---------------------------------------------------------------------------
def _mode_run(G, scheme, lam2, F, y0, T, nsteps):
    """u_t = -lam2 u + F on an eigenfunction of Lap (eigenvalue -lam2): the
    step (1 - alpha^2 Lap) u = B is (1 + alpha^2 lam2) u = B."""
    dt = T / nsteps
    a2 = G.alpha2_of(scheme, dt)
    ex = lambda t: F / lam2 + (y0 - F / lam2) * math.exp(-lam2 * t)
    reg = np.array([-1])
    u_prev, u = None, np.array([y0])
    F_arr = np.array([F])
    k0 = 0
    if scheme == G.SCHEME_GEAR:   # start from the exact values at t = 0 and dt
        u_prev, u = np.array([y0]), np.array([ex(dt)])
        k0 = 1
    for _ in range(k0, nsteps):
        B = G.rhs_imex(scheme, G.REACTION_NONE, u, u_prev, F_arr, F_arr, reg, [], dt)
        u_prev, u = u, B / (1.0 + a2 * lam2)
    return abs(u[0] - ex(T))


@pytest.mark.parametrize("scheme,order", [(0, 1), (1, 2)])
def test_scheme_order_on_a_mode(G, scheme, order):
    errs = [_mode_run(G, scheme, 104.94, 50.0, 1.0, 1e-2, n) for n in (10, 20, 40, 80)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    want = 2.0 ** order
    assert all(abs(r - want) < 0.25 * want for r in ratios), (errs, ratios)


def test_rhs_extension_and_reaction(G):
    u = np.array([0.5, -0.25, 0.9, 2.0])
    up = np.array([0.4, -0.2, 0.8, 3.0])
    reg = np.array([-1, -1, 0, 1])
    F = np.array([1.0, 2.0, 3.0, 4.0])
    dt = 0.1
    # Euler with the Allen-Cahn reaction: outside, u is the curve's constant
    B = G.rhs_imex(G.SCHEME_EULER, G.REACTION_ALLEN_CAHN, u, None, F, None, reg, [0.0, 0.5], dt)
    ub = np.array([0.5, -0.25, 0.0, 0.5])
    assert np.allclose(B, ub + dt * (F + ub * (1 - ub ** 2)), rtol=0, atol=1e-15)
    # Gear without reaction: weights 4/3, -1/3 on u and 4/3, -2/3 on F
    B = G.rhs_imex(G.SCHEME_GEAR, G.REACTION_NONE, u, up, F, 2 * F, reg, [0.0, 0.5], dt)
    ubp = np.array([0.4, -0.2, 0.0, 0.5])
    assert np.allclose(B, 4 / 3 * ub - 1 / 3 * ubp + dt * (4 / 3 * F - 2 / 3 * 2 * F), rtol=0, atol=1e-15)
    # a constant state is reproduced by Gear's u weights (4/3 - 1/3 = 1)
    c = G.rhs_imex(G.SCHEME_GEAR, G.REACTION_NONE, np.ones(4), np.ones(4), None, None, np.full(4, -1), [], dt)
    assert np.allclose(c, 1.0, atol=1e-15)
    assert G.alpha2_of(G.SCHEME_GEAR, 0.3, 2.0) == pytest.approx(0.4)


# ---------------------------------------------------------------------------
# Grid quadrature of the volume potential
# ---------------------------------------------------------------------------
def _plane_wave_up(O, h, a2, corr):
    """U^p(0) for B = cos(k.y + 0.3), |k| = 20, on a grid with a node at the
    target; the exact value is cos(0.3) / (1 + a2 |k|^2)."""
    from oracle import grid
    a = math.sqrt(a2)
    n = int(30 * a / h) + 1
    j = np.arange(-n, n + 1) * h
    X, Y = np.meshgrid(j, j, indexing="ij")
    r = np.hypot(X, Y).ravel()
    kx = ky = 20.0 / math.sqrt(2.0)
    B = np.cos(kx * X + ky * Y + 0.3).ravel()
    nz = r > 0
    G = O.k0(r[nz] / a) / (2 * math.pi * a2)
    w = grid.self_weight(h, a) if corr else O.self_cell(h, a)
    s = np.sum(G * B[nz]) * h * h + math.cos(0.3) * w / a2
    return s - math.cos(0.3) / (1 + a2 * 400.0)


def test_self_weight_lattice_correction(O):
    """The plain rule (cell integral only) is second order in h / alpha; the
    constant-exact lattice weight is about fourth order and far more accurate
    (the window of 30 alpha around the target leaves a floor near 1e-13)."""
    a2 = 1e-3
    e_plain = [_plane_wave_up(O, h, a2, False) for h in (1 / 256, 1 / 512)]
    e_corr = [_plane_wave_up(O, h, a2, True) for h in (1 / 256, 1 / 512, 1 / 1024)]
    assert abs(e_plain[0] / e_plain[1] - 4.0) < 0.5, e_plain
    assert e_corr[0] / e_corr[1] > 10 and e_corr[1] / e_corr[2] > 10, e_corr
    assert abs(e_corr[1]) < 0.01 * abs(e_plain[1])
    # the weight's small-h expansion: the cell integral plus kappa h^2, kappa
    # from the Epstein zeta function (not the naive Euler-Maclaurin 1/24)
    from oracle import grid
    for eps in (0.006, 0.02):
        w = grid.self_weight(eps, 1.0)
        series = O.self_cell(eps, 1.0) + grid.LATTICE_SELF * eps * eps
        naive = O.self_cell(eps, 1.0) + eps * eps / 24
        assert abs(series - w) < 0.06 * eps ** 2 * w
        assert abs(series - w) < 0.02 * abs(naive - w)
    # for cells much larger than alpha the weight tends to alpha^2 (U^p = B)
    assert abs(grid.self_weight(20.0, 1.0) - 1.0) < 1e-6


def test_bicubic_is_exact_on_cubics(G):
    rng = np.random.default_rng(3)
    x0, y0, h, nx, ny = -0.3, -0.2, 0.05, 14, 12
    pts = G.grid_points(x0, y0, h, nx, ny)
    C = rng.standard_normal((4, 4))
    f = lambda x, y: sum(C[a, b] * x ** a * y ** b for a in range(4) for b in range(4))
    q = np.stack([rng.uniform(x0 + 2 * h, x0 + (nx - 2) * h, 200),
                  rng.uniform(y0 + 2 * h, y0 + (ny - 2) * h, 200)], axis=1)
    got = G.bicubic(f(pts[:, 0], pts[:, 1]), x0, y0, h, nx, ny, q)
    assert np.max(np.abs(got - f(q[:, 0], q[:, 1]))) < 1e-12
    # a quartic is not reproduced: the error is O(h^4)
    g4 = lambda x, y: x ** 4
    err = np.max(np.abs(G.bicubic(g4(pts[:, 0], pts[:, 1]), x0, y0, h, nx, ny, q) - g4(q[:, 0], q[:, 1])))
    assert 1e-8 < err < 2 * h ** 4
    with pytest.raises(ValueError):
        G.bicubic(f(pts[:, 0], pts[:, 1]), x0, y0, h, nx, ny, np.array([[x0 + 0.5 * h, 0.0]]))


# ---------------------------------------------------------------------------
# Curve interpolation and projection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [16, 17])
def test_fourier_interpolant_exact_on_trig_polynomials(G, N):
    th = 2 * np.pi * np.arange(N) / N
    last = N // 2 if N % 2 == 0 else None   # the Nyquist mode of an even N is a cosine
    f = lambda t: 0.3 + np.cos(3 * t) - 0.5 * np.sin(7 * t) + (0.25 * np.cos(last * t) if last else 0.0)
    f1 = lambda t: -3 * np.sin(3 * t) - 3.5 * np.cos(7 * t) - (0.25 * last * np.sin(last * t) if last else 0.0)
    f2 = lambda t: -9 * np.cos(3 * t) + 24.5 * np.sin(7 * t) - (0.25 * last ** 2 * np.cos(last * t) if last else 0.0)
    s = G.CurveSeries(f(th))
    t = np.random.default_rng(0).random(64) * 2 * np.pi
    assert np.max(np.abs(s(t) - f(t))) < 1e-13
    assert np.max(np.abs(s(t, 1) - f1(t))) < 1e-12
    assert np.max(np.abs(s(t, 2) - f2(t))) < 1e-10


def test_projection_onto_a_circle(G):
    cv = W.circle((0.1, -0.2), 0.3, 64, ccw=False)
    g = G.CurveGeom(cv.xy, cv.normal)
    rng = np.random.default_rng(7)
    ang = rng.random(50) * 2 * np.pi
    rad = 0.3 + (rng.random(50) - 0.5) * 0.02
    p = np.stack([0.1 + rad * np.cos(ang), -0.2 + rad * np.sin(ang)], axis=1)
    # start from the nearest node
    d2 = ((p[:, None, :] - cv.xy[None]) ** 2).sum(-1)
    j = np.argmin(d2, axis=1)
    # a clockwise circle: theta runs against the polar angle
    th = g.project(p, 2 * np.pi * j / 64)
    y = g.point(th)
    assert np.max(np.abs(np.hypot(*(y - np.array([0.1, -0.2])).T) - 0.3)) < 1e-14
    assert np.max(np.abs(np.arctan2(y[:, 1] + 0.2, y[:, 0] - 0.1) - np.arctan2(p[:, 1] + 0.2, p[:, 0] - 0.1))) < 1e-12
    assert np.allclose(g.spacing(th), 0.3 * 2 * np.pi / 64, rtol=1e-13)
    # the interpolated normal is the given outward one (pointing to the centre of a hole)
    nv = g.normal(th)
    assert np.allclose(nv, -(y - np.array([0.1, -0.2])) / 0.3, atol=1e-13)


# ---------------------------------------------------------------------------
# The corrected trapezoid rule of the integral equation and the near-boundary
# evaluation, against u = exp(k.x), |k| = 1/alpha, which solves u - alpha^2 Lap u = 0
# ---------------------------------------------------------------------------
def _exp_case(O, n0, n1, alpha, diag_shift=0.0):
    b = annulus(n0, n1)
    w = b.weights()
    k = np.array([math.cos(0.7), math.sin(0.7)]) / alpha
    u = lambda p: np.exp(p @ k)
    A = O.dl_matrix(b.xy, b.normal, w, b.curvature, alpha)
    A[np.diag_indices_from(A)] += diag_shift * b.curvature * w ** 3
    import scipy.linalg as sla
    sig = sla.solve(A, -2 * alpha ** 2 * u(b.xy))
    return b, w, u, sig


def test_corrected_diagonal_makes_the_rule_fifth_order(O):
    alpha = 0.05
    far = np.array([[0.25, 0.0], [0.0, -0.2], [0.3, 0.1]])
    errs, plain = [], []
    # the correction is zeta(3) kappa w^3 / (16 pi^3 alpha^2) in the DL matrix,
    # i.e. -2 times that in A; undoing it gives the plain trapezoid rule
    undo = 2 * 1.2020569031595942 / (16 * math.pi ** 3 * alpha ** 2)
    for n0, n1 in ((256, 128), (512, 256)):
        for shift, out in ((0.0, errs), (undo, plain)):
            b, w, u, sig = _exp_case(O, n0, n1, alpha, shift)
            out.append(np.max(np.abs(O.dl_sum(b.xy, b.normal, w * sig, alpha, far) / alpha ** 2 - u(far)) / u(far)))
    assert errs[0] / errs[1] > 20, errs          # fifth order (32)
    assert 6 < plain[0] / plain[1] < 10, plain    # third order without it
    assert errs[1] < 1e-9


def test_near_boundary_evaluation_on_exp_solution(O, G):
    alpha = 0.05
    b, w, u, sig = _exp_case(O, 512, 256, alpha)
    f = u(b.xy)
    rng = np.random.default_rng(1)
    th = rng.random(400) * 2 * np.pi
    ds_in, ds_out = 2 * np.pi * 0.1 / 256, 2 * np.pi * 0.4 / 512
    frac = np.concatenate([[0.0, 0.01, 0.2, 0.5, 0.8, 3.9], rng.random(194) * 4])
    frac = np.concatenate([frac, frac])
    r = np.concatenate([0.1 + frac[:200] * ds_in, 0.4 - frac[200:] * ds_out])
    pts = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    nt = G.near_targets(b.xy, b.normal, b.speed, b.offset, pts)
    # every point is within 4 spacings on the domain side: all are near
    assert np.array_equal(nt[0], np.arange(400))
    assert np.allclose(nt[3], frac * np.concatenate([np.full(200, ds_in), np.full(200, ds_out)]), atol=1e-13)
    plain = O.dl_sum(b.xy, b.normal, w * sig, alpha, pts) / alpha ** 2
    near = G.near_values(b.xy, b.normal, b.offset, sig, f, alpha, pts, nt)
    ex = u(pts)
    scale = np.max(np.abs(ex))
    assert np.max(np.abs(near - ex)) / scale < 1e-8
    assert np.max(np.abs(plain - ex)) / scale > 1e-2   # what the plain rule gives there
    # points outside the domain and beyond the band are not near targets
    out = np.array([[0.0, 0.1 - 0.5 * ds_in], [0.4 + 0.5 * ds_out, 0.0], [0.2, 0.05]])
    assert G.near_targets(b.xy, b.normal, b.speed, b.offset, out)[0].size == 0


def test_grid_step_closed_form(O, G):
    """u = sin(3x) sin(2y) + 1 satisfies (1 - a2 Lap) u = (1 + 13 a2) u - 13 a2;
    with B that smooth field everywhere and f = u on the curves, one grid step
    returns u: up to the grid's O(h^2) at every point inside, the near ones
    included; without the near-boundary evaluation they are far off."""
    b = annulus(512, 256)
    a2 = 2.5e-3
    x0, h, m = -0.5, 1.0 / 64, 64
    pts = G.grid_points(x0, x0, h, m, m)
    uf = lambda p: np.sin(3 * p[:, 0]) * np.sin(2 * p[:, 1]) + 1.0
    B = (1 + 13 * a2) * uf(pts) - 13 * a2
    res = {}
    for near in (True, False):
        u, sig, upb, Up, nt = G.heat_step_grid(b.xy, b.normal, b.weights(), b.curvature, b.speed, b.offset,
                                               (x0, x0, h, m, m), B, uf(b.xy), a2, near=near)
        inside = b.region(pts) < 0
        res[near] = np.abs(u - uf(pts))[inside]
        if near:
            near_idx = nt[0]
    assert near_idx.size > 0
    assert res[True].max() < 2e-4, res[True].max()
    assert res[False].max() > 10 * res[True].max()


# ---------------------------------------------------------------------------
# Integral of the kernel over a square cell at an arbitrary target
# ---------------------------------------------------------------------------
def test_cell_integral_against_quadrature(O, G):
    """The triangle/asinh rule against scipy's adaptive dblquad (the square
    split at the target so the singularity sits on sub-cell corners), at the
    centre against the self-cell integral, and additivity over a 2 x 2 split."""
    from scipy import integrate
    a, h, cx, cy = 0.05, 0.03, 0.1, 0.2
    assert G.cell_k0_integral(cx, cy, cx, cy, h, a)[0] == pytest.approx(O.self_cell(h, a), rel=1e-13)
    for px, py in ((0.101, 0.203), (cx + 0.5 * h, cy), (cx + 0.6 * h, cy + 0.1 * h), (0.2, 0.3)):
        f = lambda y, x: O.k0(math.hypot(x - px, y - py) / a)[0] / (2 * math.pi)
        xs = sorted({cx - h / 2, min(max(px, cx - h / 2), cx + h / 2), cx + h / 2})
        ys = sorted({cy - h / 2, min(max(py, cy - h / 2), cy + h / 2), cy + h / 2})
        ref = sum(integrate.dblquad(f, xs[i], xs[i + 1], ys[j], ys[j + 1], epsabs=1e-16, epsrel=1e-12)[0]
                  for i in range(len(xs) - 1) for j in range(len(ys) - 1))
        assert G.cell_k0_integral(px, py, cx, cy, h, a)[0] == pytest.approx(ref, rel=1e-11)
    p = (0.107, 0.196)
    whole = G.cell_k0_integral(p[0], p[1], cx, cy, h, a)[0]
    parts = sum(G.cell_k0_integral(p[0], p[1], cx + sx * h / 4, cy + sy * h / 4, h / 2, a)[0]
                for sx in (-1, 1) for sy in (-1, 1))
    assert whole == pytest.approx(parts, rel=1e-13)


def test_node_cell_correction_fixes_off_grid_volume_potential(O, G):
    """U^p of B = 1 at points off the grid: the kernel integrates to 1 over the
    plane, so V / alpha^2 -> 1 away from the grid's edge.  Point sums err by
    O(1) for cells larger than alpha and by a log where a point nears a
    centre; with the cells within two sides entering by their integral, what
    is left is the midpoint rule's (h^2 / 24 alpha^2) x K1(x), x = 2 h / alpha."""
    rng = np.random.default_rng(5)
    for h, a, tol in ((0.02, 0.01, 1.5e-2), (0.01, 0.04, 3e-3)):
        grid, pts = W.grid_box(-0.5, 0.5, int(round(1.0 / h)))
        w = np.full(pts.shape[0], h * h)
        tg = rng.uniform(-0.1, 0.1, size=(40, 2))
        tg[0] = pts[np.argmin(np.hypot(pts[:, 0], pts[:, 1]))] + [1e-7, 0.0]   # right next to a centre
        V = O.volume_sum(pts, w, a, tgt_xy=tg)
        plain = V / a ** 2
        fixed = (V + G.node_cell_correction(tg, pts, w, np.ones(pts.shape[0]), a)) / a ** 2
        assert np.max(np.abs(fixed - 1.0)) < tol, (h, a, np.max(np.abs(fixed - 1.0)))
        assert np.max(np.abs(plain - 1.0)) > 10 * np.max(np.abs(fixed - 1.0))
