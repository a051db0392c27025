"""Pins for the CPU oracle, against facts fixed by the paper and by mathematics.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a missing Jacobian, a wrong diagonal, a transposed operand) makes
it fail.  None of them re-types the oracle's own formulas.
"""
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Special functions: independent library routines, arbitrary precision, and a
# closed-form invariant.
# ---------------------------------------------------------------------------
def test_k0_k1_against_scipy(oracle_lib):
    sp = pytest.importorskip("scipy.special")
    z = np.concatenate([np.logspace(-8, math.log10(600.0), 3000), [1.999999, 2.0, 2.000001]])
    for mine, ref in ((oracle_lib.k0, sp.k0), (oracle_lib.k1, sp.k1)):
        a, b = mine(z), ref(z)
        ok = b > 0
        rel = np.abs(a[ok] - b[ok]) / b[ok]
        # conditioning of K_nu at z is ~z (through exp(-z)), so allow z * eps
        tol = 2e-15 * np.maximum(8.0, z[ok])
        assert np.all(rel <= tol), float(np.max(rel / tol))


def test_k0_k1_against_mpmath(oracle_lib):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for z in (1e-7, 3e-3, 0.1, 0.5, 1.0, 1.9999, 2.0001, 3.7, 11.0, 40.0, 150.0):
        for nu, f in ((0, oracle_lib.k0), (1, oracle_lib.k1)):
            exact = float(mp.besselk(nu, z))
            got = float(f(z)[0])
            assert abs(got - exact) <= 4e-15 * max(1.0, z / 4) * abs(exact), (nu, z, got, exact)


def test_wronskian(oracle_lib):
    # I0(z) K1(z) + I1(z) K0(z) = 1/z  (A&S 9.6.15)
    z = np.logspace(-6, math.log10(25.0), 400)
    lhs = oracle_lib.i0(z) * oracle_lib.k1(z) + oracle_lib.i1(z) * oracle_lib.k0(z)
    assert np.max(np.abs(lhs * z - 1.0)) < 1e-13


# ---------------------------------------------------------------------------
# Double-layer kernel: the paper's on-curve limit (golden fixture)
# ---------------------------------------------------------------------------
def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def test_dl_kernel_on_curve_limit(oracle_lib):
    for radius, ccw, alpha, expected in _golden_rows("dl_diagonal_limit.txt"):
        cv = W.circle((0.1, -0.2), radius, 64, ccw=bool(ccw))
        x = cv.xy[0]
        errs = []
        for eps in (1e-2, 1e-3, 1e-4, 1e-5):
            # node y at parameter eps from x along the same curve
            t = eps if ccw else -eps
            y = np.array([0.1 + radius * math.cos(t), -0.2 + radius * math.sin(t)])
            n = (y - np.array([0.1, -0.2])) / radius * (1.0 if ccw else -1.0)
            errs.append(abs(oracle_lib.dl_kernel(x, y, n, alpha) - expected))
        # the deviation is O(z^2 log z) with z = |x - y|/alpha, until the
        # cancellation in (x - y).n_y at tiny separations takes over
        assert min(errs) < 1e-5 * abs(expected), errs
        assert errs[0] > errs[1]
        # the curvature carried by the geometry agrees with the fixture
        assert abs(-0.5 * cv.curvature[0] - expected) < 1e-12


# ---------------------------------------------------------------------------
# Green's representation (pins the DL sign, its 1/alpha, the normals and the
# trapezoid weights): for u with u - alpha^2 Lap u = 0,
#   u(x) = alpha^2 int_Gamma (G du/dnu - u dG/dnu_y) ds   (x in Omega), 0 outside,
# i.e. u = V[w du/dnu] - DL[w u] in the library normalisation.
# ---------------------------------------------------------------------------
def test_green_representation(oracle_lib):
    alpha = 0.1
    cfg = W.config_c0(n_nodes=256, m=8)
    b = cfg["bnd"]
    w = b.weights()
    k = np.array([math.cos(0.7), math.sin(0.7)]) / alpha
    u = lambda p: np.exp(p @ k)
    dudn = (b.normal @ k) * u(b.xy)
    inside = np.array([[0.0, 0.6], [-0.5, -0.3], [0.1, -0.75]])
    outside = np.array([[0.2, 0.0], [0.25, 0.1], [1.6, 0.3]])
    pts = np.concatenate([inside, outside])
    rep = oracle_lib.volume_sum(b.xy, w * dudn, alpha, tgt_xy=pts) - \
        oracle_lib.dl_sum(b.xy, b.normal, w * u(b.xy), alpha, pts)
    exact = np.concatenate([u(inside), np.zeros(3)])
    scale = np.max(np.abs(u(b.xy)))
    assert np.max(np.abs(rep - exact)) < 1e-12 * scale


# ---------------------------------------------------------------------------
# Second-kind equation with a manufactured solution: u = K0(|x - c|/alpha),
# c inside the hole, solves the homogeneous equation in Omega.  The trapezoid
# rule with the diagonal limit converges at O(h^3) for this kernel.
# ---------------------------------------------------------------------------
def _bie_error(oracle_lib, n_nodes, alpha=0.1, flip=False):
    cfg = W.config_c0(n_nodes=n_nodes, m=8)
    b = cfg["bnd"]
    w = b.weights()
    c = np.array([0.2, 0.0])
    ufun = lambda p: oracle_lib.k0(np.hypot(p[:, 0] - c[0], p[:, 1] - c[1]) / alpha)
    g = ufun(b.xy)
    bie = oracle_lib.DenseBIE(b.xy, b.normal, w, b.curvature, alpha)
    if flip:  # plant the printed-kernel sign mistake, on the CPU
        sig = np.linalg.solve(2.0 * np.eye(b.n) - bie.A, -2.0 * alpha ** 2 * g)
    else:
        sig = bie.solve(g)
    pts = np.array([[0.0, 0.7], [-0.6, 0.0], [0.6, -0.1], [0.0, -0.5]])
    uh = oracle_lib.dl_sum(b.xy, b.normal, w * sig, alpha, pts) / alpha ** 2
    return float(np.max(np.abs(uh - ufun(pts)) / np.abs(ufun(pts))))


def test_bie_manufactured_convergence(oracle_lib):
    e128 = _bie_error(oracle_lib, 128)
    e256 = _bie_error(oracle_lib, 256)
    assert e256 < 2e-6
    assert e128 / e256 > 6.0          # third order in h
    assert _bie_error(oracle_lib, 128, flip=True) > 0.1   # sign mistake is caught


def test_bie_matrix_vs_sum(oracle_lib):
    cfg = W.config_c0(n_nodes=64, m=8)
    b = cfg["bnd"]
    w = b.weights()
    rng = np.random.default_rng(5)
    s = rng.standard_normal(b.n)
    A = oracle_lib.dl_matrix(b.xy, b.normal, w, b.curvature, 0.1)
    got = oracle_lib.apply_bie(b.xy, b.normal, w, b.curvature, s, 0.1)
    assert np.max(np.abs(A @ s - got)) < 1e-13 * np.max(np.abs(got))


# ---------------------------------------------------------------------------
# Volume sum: brute force with an independent K0 on a tiny case, symmetry.
# ---------------------------------------------------------------------------
def test_volume_sum_brute_force(oracle_lib):
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(2)
    s = rng.random((40, 2)); t = rng.random((7, 2)); q = rng.standard_normal(40)
    t[3] = s[5]                       # a coincident pair is skipped
    alpha = 0.07
    got = oracle_lib.volume_sum(s, q, alpha, tgt_xy=t)
    ref = np.zeros(7)
    for i in range(7):
        for j in range(40):
            r = math.hypot(*(t[i] - s[j]))
            if r > 0:
                ref[i] += q[j] * sp.k0(r / alpha) / (2 * math.pi)
    assert np.max(np.abs(got - ref)) < 1e-14 * np.max(np.abs(ref))
    self_ = oracle_lib.volume_sum(s, q, alpha)
    ref2 = np.array([sum(q[j] * sp.k0(math.hypot(*(s[i] - s[j])) / alpha) for j in range(40) if j != i)
                     for i in range(40)]) / (2 * math.pi)
    assert np.max(np.abs(self_ - ref2)) < 1e-14 * np.max(np.abs(ref2))


def test_volume_sum_symmetry(oracle_lib):
    rng = np.random.default_rng(3)
    s = rng.random((300, 2)); a = rng.standard_normal(300); b = rng.standard_normal(300)
    lhs = a @ oracle_lib.volume_sum(s, b, 0.05)
    rhs = b @ oracle_lib.volume_sum(s, a, 0.05)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1.0)


def test_dl_sum_brute_force(oracle_lib):
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(4)
    cv = W.ellipse((0.4, 0.5), 0.2, 0.1, 32, rotation=0.3, ccw=False)
    d = rng.standard_normal(32)
    t = rng.random((5, 2))
    alpha = 0.08
    got = oracle_lib.dl_sum(cv.xy, cv.normal, d, alpha, t)
    ref = np.zeros(5)
    for i in range(5):
        for j in range(32):
            dv = t[i] - cv.xy[j]
            r = math.hypot(*dv)
            # d/dnu_y K0(|x - y|/alpha) = -(1/alpha) K0'(r/alpha)... = K1 (x-y).n / (alpha r)
            ref[i] += d[j] * sp.k1(r / alpha) * (dv @ cv.normal[j]) / (alpha * r)
    ref /= 2 * math.pi
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    # the same kernel by a central finite difference along the normal at the node
    i, j, eps = 1, 3, 1e-6
    K0 = lambda y: sp.k0(math.hypot(*(t[i] - y)) / alpha)
    fd = (K0(cv.xy[j] + eps * cv.normal[j]) - K0(cv.xy[j] - eps * cv.normal[j])) / (2 * eps)
    assert abs(oracle_lib.dl_kernel(t[i], cv.xy[j], cv.normal[j], alpha) - fd) < 1e-6 * abs(fd)


# ---------------------------------------------------------------------------
# Self-cell term against an independent 2-D quadrature of K0 over the cell.
# ---------------------------------------------------------------------------
def test_self_cell_vs_2d_quadrature(oracle_lib):
    sp = pytest.importorskip("scipy.special")
    from scipy import integrate
    for h, alpha in ((1.0 / 32, 0.1), (2.0 ** -10, 0.0316), (0.05, 0.01)):
        f = lambda y, x: sp.k0(math.hypot(x, y) / alpha)
        # one quadrant, singularity at its corner
        val, err = integrate.dblquad(f, 0.0, h / 2, 0.0, h / 2, epsabs=1e-15, epsrel=1e-12)
        ref = 4.0 * val / (2 * math.pi)
        got = oracle_lib.self_cell(h, alpha)
        assert abs(got - ref) < 1e-9 * abs(ref), (h, alpha, got, ref)


# ---------------------------------------------------------------------------
# Rothe step with a closed form: (1 - dt Lap)(c sin x sin y) = c (1 + 2 dt) sin x sin y,
# so with boundary data sin x sin y / (1 + 2 dt) the exact step is that
# function.  The weighted-point volume sum converges at O(h^2/alpha^2) roughly.
# ---------------------------------------------------------------------------
def test_rothe_step_closed_form(oracle_lib):
    errs = []
    dt = 0.01
    for m in (32, 64):
        cfg = W.config_c0(n_nodes=256, m=m, dt=dt)
        b = cfg["bnd"]
        f1 = np.sin(b.xy[:, 0]) * np.sin(b.xy[:, 1]) / (1 + 2 * dt)
        vol = cfg["vol"]
        mask = cfg["region"] < 0
        u, sig, _ = oracle_lib.heat_step(b.xy, b.normal, b.weights(), b.curvature, vol,
                                         cfg["vol_w"], cfg["B"], f1, dt, grid_h=cfg["h"],
                                         tgt_mask=mask, offsets=b.offset)
        ex = np.sin(vol[mask, 0]) * np.sin(vol[mask, 1]) / (1 + 2 * dt)
        far = b.distance_to_boundary(vol[mask]) > 0.12
        errs.append(np.max(np.abs(u - ex)[far]) / np.max(np.abs(ex)))
    assert errs[1] < 5e-3
    # the grid points' own weights are exact for constants and the cells next
    # to a node enter by their integral; what is left at the nodes decays like
    # (h/alpha)^2 x K1(x), x = 2h/alpha: a bit over 2 per halving at these h/alpha
    assert errs[0] / errs[1] > 2.0, errs


def test_rothe_step_without_self_cell_is_worse(oracle_lib):
    # dropping the self-cell term (a plausible slip) is visible at once
    dt = 0.01
    cfg = W.config_c0(n_nodes=256, m=32, dt=dt)
    b = cfg["bnd"]
    f1 = np.sin(b.xy[:, 0]) * np.sin(b.xy[:, 1]) / (1 + 2 * dt)
    mask = cfg["region"] < 0
    vol = cfg["vol"]
    ex = np.sin(vol[mask, 0]) * np.sin(vol[mask, 1]) / (1 + 2 * dt)
    far = b.distance_to_boundary(vol[mask]) > 0.12
    res = []
    for gh in (cfg["h"], None):
        u, _, _ = oracle_lib.heat_step(b.xy, b.normal, b.weights(), b.curvature, vol,
                                       cfg["vol_w"], cfg["B"], f1, dt, grid_h=gh, tgt_mask=mask, offsets=b.offset)
        res.append(np.max(np.abs(u - ex)[far]) / np.max(np.abs(ex)))
    assert res[1] > 3 * res[0], res
