"""Time schemes and the cell-centred grid step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU library.  Plain numpy on
top of the direct sums of the oracle package; every function follows one
passage of Kropinski & Quaife (arXiv 1007.5335) or a stated reading of it:

  * rhs_imex: the right-hand side B of the linearly implicit schemes of Sec. 2
    (eq. mod_helm_forced): backward Euler (alpha^2 = nu dt, B = u + dt F) and
    the extrapolated Gear scheme (eq. exg: alpha^2 = 2 nu dt / 3,
    B = 4/3 u^N - 1/3 u^{N-1} + 4/3 dt F^N - 2/3 dt F^{N-1}); F may hold a
    pointwise reaction (the Allen-Cahn term u (1 - u^2) of Sec. 4, Example 3);
    u is extended by the boundary constants outside the domain (Sec. 3.1),
    F by the caller;
  * self_weight: the weight of a grid point's own cell in the lattice rule of
    the volume potential (eq. vol_potential on a uniform grid): the weight
    that makes the rule exact for constant B (the kernel integrates to 1 over
    the plane), alpha^2 - (h^2 / 2 pi) sum' K0(|j| h / alpha); for
    h / alpha < 0.005 its expansion, the cell integral plus kappa h^2 (the
    lattice correction of the logarithmic singularity);
  * bicubic: U^p at off-grid points (the boundary nodes) by tensor cubic
    Lagrange interpolation of the grid values, the point-grid counterpart of
    evaluating each leaf's cubic polynomial (Sec. 3.1);
  * CurveSeries: the trigonometric interpolant of data given at parameter-
    equispaced nodes (Sec. 3.2, Fourier interpolation of sigma), with the
    Nyquist mode of an even N taken as a cosine;
  * near_targets / near_values: the double layer at points closer to a curve
    than a few node spacings (where the trapezoid rule of Sec. 3.2 fails):
    the target is projected onto the interpolated curve; U^h is evaluated at
    K check points along the inward normal at 1..K local node spacings with
    sigma interpolated to m times as many nodes, its interior limit on the
    curve is g (the boundary condition the integral equation imposes), and
    the target's value is the degree-K polynomial in the normal distance
    through these K + 1 values;
  * heat_step_grid: one step on a cell-centred grid with the above.
"""
from __future__ import annotations

import math

import numpy as np

from . import DenseBIE, _f64, dl_sum, self_cell, volume_sum

SCHEME_EULER, SCHEME_GEAR = 0, 1
REACTION_NONE, REACTION_ALLEN_CAHN = 0, 1


# ---------------------------------------------------------------------------
# Time schemes (Sec. 2, eq. mod_helm_forced and eq. exg)
# ---------------------------------------------------------------------------
def alpha2_of(scheme: int, dt: float, nu: float = 1.0) -> float:
    """alpha^2 of the scheme for u_t - nu Lap u = F: nu dt (Euler), 2 nu dt / 3 (Gear)."""
    return nu * dt if scheme == SCHEME_EULER else 2.0 * nu * dt / 3.0


def reaction(kind: int, u):
    """Pointwise reaction term added to F: Allen-Cahn u (1 - u^2) (Sec. 4, Example 3)."""
    u = _f64(u)
    return u * (1.0 - u * u) if kind == REACTION_ALLEN_CAHN else np.zeros_like(u)


def rhs_imex(scheme, reaction_kind, u, u_prev, F, F_prev, region, consts, dt):
    """B at every point.  Inside the domain (region < 0) u is the caller's; at
    other points u is the constant of the curve that encloses them (region k
    selects consts[k], missing constants are 0).  F (and F_prev) apply at every
    point (None = 0); the reaction is evaluated on the extended u."""
    region = np.asarray(region)
    n = region.shape[0]
    c = np.zeros(max(int(region.max(initial=-1)) + 1, len(consts)))
    c[:len(consts)] = consts

    def ext(v):
        v = _f64(v).copy()
        out = region >= 0
        v[out] = c[region[out]]
        return v

    def forcing(Fv, uv):
        f = np.zeros(n) if Fv is None else _f64(Fv)
        return f + reaction(reaction_kind, uv)

    u0 = ext(u)
    if scheme == SCHEME_EULER:
        return u0 + dt * forcing(F, u0)
    u1 = ext(u_prev)
    return (4.0 / 3.0) * u0 - (1.0 / 3.0) * u1 + dt * ((4.0 / 3.0) * forcing(F, u0) - (2.0 / 3.0) * forcing(F_prev, u1))


# ---------------------------------------------------------------------------
# Uniform cell-centred grid (Sec. 3.1 volume potential on point samples)
# ---------------------------------------------------------------------------
def grid_points(x0, y0, h, nx, ny) -> np.ndarray:
    """Cell centres, point j nx + i at (x0 + (i + 1/2) h, y0 + (j + 1/2) h)."""
    gx = x0 + h * (np.arange(nx) + 0.5)
    gy = y0 + h * (np.arange(ny) + 0.5)
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], axis=1))


# kappa = (c_cell - Z'(0)/2) / (2 pi): c_cell = int over [-1/2, 1/2]^2 of log|u|
# = (pi/2 - 3 - log 2) / 2, and Z(s) = sum over the nonzero points j of Z^2 of
# |j|^(-2s) = 4 zeta(s) beta(s) (Epstein zeta function of the square lattice,
# beta the Dirichlet beta function), Z'(0)/2 = log(4 pi)/2 - 2 log Gamma(1/4).
LATTICE_SELF = ((math.pi / 2 - 3 - math.log(2)) / 2
                - (0.5 * math.log(4 * math.pi) - 2 * math.lgamma(0.25))) / (2 * math.pi)


SELF_WEIGHT_SERIES_BELOW = 0.005


def self_weight(h: float, alpha: float) -> float:
    """The own-cell weight w0 (library normalisation, U^p = (V + B w0) / alpha^2).

    The lattice rule sum_j h^2 G(x_i - x_j) B_j with the self pair weighted by
    w0 / alpha^2 integrates a constant B exactly when
      w0 = alpha^2 - (h^2 / 2 pi) sum_{j != 0} K0(|j| h / alpha)
    (the kernel G = K0 / (2 pi alpha^2) integrates to 1 over the plane).  For
    small eps = h / alpha its expansion is the cell integral plus kappa h^2:
    near the target the kernel is -(1/2pi) log|x| times a smooth factor psi;
    by the generalised Euler-Maclaurin expansion of lattice sums (the
    derivative at s = 0 of h^2 sum' |jh|^(-2s) psi(jh) - int |x|^(-2s) psi =
    h^(2-2s) Z(s) psi(0) + ..., Z(0) = -1) the punctured sum of log|x| psi
    misses h^2 psi(0) (log h + Z'(0)/2), while the cell integral supplies
    h^2 psi(0) (log h + c_cell).  The expansion's relative error is about
    0.04 eps^2 (a U^p error of 0.04 eps^4 B); it is used below eps = 0.005,
    where the lattice sum would need more than 10^7 terms."""
    eps = h / alpha
    if eps < SELF_WEIGHT_SERIES_BELOW:
        return self_cell(h, alpha) + LATTICE_SELF * h * h
    from . import lattice_k0_sum
    return alpha * alpha - h * h / (2.0 * math.pi) * lattice_k0_sum(eps)


def bicubic(values, x0, y0, h, nx, ny, pts) -> np.ndarray:
    """Tensor cubic Lagrange interpolation of cell-centre values [ny * nx] at pts.

    For a coordinate x the stencil is the four centres i0 - 1 .. i0 + 2 with
    i0 = floor((x - x0) / h - 1/2), and the weights are the cubic Lagrange
    basis on the nodes -1, 0, 1, 2 at s = (x - x0) / h - 1/2 - i0."""
    V = _f64(values).reshape(ny, nx)
    pts = _f64(pts).reshape(-1, 2)

    def axis(c, o, n):
        s = (c - o) / h - 0.5
        i0 = np.floor(s).astype(np.int64)
        t = s - i0
        if np.any(i0 - 1 < 0) or np.any(i0 + 2 > n - 1):
            raise ValueError("a point's interpolation stencil leaves the grid")
        w = np.stack([-t * (t - 1.0) * (t - 2.0) / 6.0,
                      (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
                      -(t + 1.0) * t * (t - 2.0) / 2.0,
                      (t + 1.0) * t * (t - 1.0) / 6.0], axis=1)
        return i0, w

    ix, wx = axis(pts[:, 0], x0, nx)
    iy, wy = axis(pts[:, 1], y0, ny)
    out = np.zeros(pts.shape[0])
    for b in range(4):
        for a in range(4):
            out += wy[:, b] * wx[:, a] * V[iy + b - 1, ix + a - 1]
    return out


def cell_k0_integral(px, py, cx, cy, h, alpha, n_gauss=64):
    """(1/2pi) int over the square of side h centred at (cx, cy) of K0(|y - p|/alpha) dA.

    The square is the signed sum of the four triangles with apex p and one
    edge each (sign = orientation of (p, a, b)).  Over a triangle, in polar
    coordinates about p, the radial integral is F(R) = alpha^2 - alpha R K1(R/alpha)
    (d/dr of -alpha r K1(r/alpha) is r K0(r/alpha)); along the edge, at signed
    coordinate t from the foot of the perpendicular (distance q), R = q cosh s
    and dtheta = ds / cosh s with t = q sinh s.  The s-integral is taken by
    Gauss-Legendre on unit panels.  Vectorised over the inputs."""
    from . import k1
    px, py, cx, cy, h = (np.atleast_1d(_f64(v)).astype(np.float64) for v in (px, py, cx, cy, h))
    n = max(px.size, cx.size, h.size)
    px, py, cx, cy, h = (np.broadcast_to(v, (n,)).copy() for v in (px, py, cx, cy, h))
    xg, wg = np.polynomial.legendre.leggauss(n_gauss)
    corners = [(-0.5, -0.5), (0.5, -0.5), (0.5, 0.5), (-0.5, 0.5)]
    total = np.zeros(n)
    for e in range(4):
        ax, ay = cx + corners[e][0] * h, cy + corners[e][1] * h
        bx, by = cx + corners[(e + 1) % 4][0] * h, cy + corners[(e + 1) % 4][1] * h
        ex, ey = (bx - ax) / h, (by - ay) / h               # unit edge direction
        q = (ax - px) * ey - (ay - py) * ex                 # signed distance (outward normal (ey, -ex))
        ta = (ax - px) * ex + (ay - py) * ey
        tb = ta + h
        aq = np.abs(q)
        ok = aq > 1e-300
        sa = np.where(ok, np.arcsinh(ta / np.where(ok, aq, 1.0)), 0.0)
        sb = np.where(ok, np.arcsinh(tb / np.where(ok, aq, 1.0)), 0.0)
        npan = np.maximum(1, np.ceil(sb - sa)).astype(np.int64)
        acc = np.zeros(n)
        for npv in np.unique(npan[ok]):          # pairs with the same panel count together
            sel = np.flatnonzero(ok & (npan == npv))
            for c0 in range(0, sel.size, 4096):
                ii = sel[c0:c0 + 4096]
                frac = np.arange(npv + 1) / npv
                edges = sa[ii, None] + (sb[ii] - sa[ii])[:, None] * frac[None, :]   # [m, npv+1]
                mid = 0.5 * (edges[:, 1:] + edges[:, :-1])
                half = 0.5 * (edges[:, 1:] - edges[:, :-1])
                sv = mid[:, :, None] + half[:, :, None] * xg[None, None, :]
                wv = half[:, :, None] * wg[None, None, :]
                R = aq[ii, None, None] * np.cosh(sv)
                F = alpha * alpha - alpha * R * k1((R / alpha).ravel()).reshape(R.shape)
                acc[ii] = np.sum(wv * F / np.cosh(sv), axis=(1, 2))
        total += np.sign(q) * acc
    return total / (2.0 * math.pi)


def node_cell_pairs(bxy, vol_xy, vol_w, reach=2.0):
    """(node, cell) pairs with the node closer to the cell centre than reach
    cell sides (cells: squares of area vol_w centred at vol_xy)."""
    bxy = _f64(bxy); vol_xy = _f64(vol_xy); hs = np.sqrt(_f64(vol_w))
    ni, ci = [], []
    for s0 in range(0, bxy.shape[0], 256):
        blk = bxy[s0:s0 + 256]
        d2 = ((blk[:, None, :] - vol_xy[None, :, :]) ** 2).sum(-1)
        a, c = np.nonzero(d2 < (reach * hs[None, :]) ** 2)
        ni.append(a + s0); ci.append(c)
    return np.concatenate(ni), np.concatenate(ci)


def node_cell_correction(bxy, vol_xy, vol_w, B, alpha):
    """Change of V[q](node) (q = vol_w B, library normalisation without 1/alpha^2)
    when the cells near each node enter with their integral instead of the
    point value: sum over the pairs of B_j (cell integral - point value)."""
    from . import k0
    ni, ci = node_cell_pairs(bxy, vol_xy, vol_w)
    out = np.zeros(_f64(bxy).shape[0])
    if ni.size == 0:
        return out
    vx, bb, w = _f64(vol_xy), _f64(B), _f64(vol_w)
    hs = np.sqrt(w)
    P = _f64(bxy)[ni]
    integ = cell_k0_integral(P[:, 0], P[:, 1], vx[ci, 0], vx[ci, 1], hs[ci], alpha)
    d = np.hypot(P[:, 0] - vx[ci, 0], P[:, 1] - vx[ci, 1])
    point = np.where(d > 0, w[ci] * k0(np.where(d > 0, d, 1.0) / alpha) / (2.0 * math.pi), 0.0)
    np.add.at(out, ni, bb[ci] * (integ - point))
    return out


# ---------------------------------------------------------------------------
# Trigonometric interpolation on a curve (Sec. 3.2, Fourier interpolation)
# ---------------------------------------------------------------------------
class CurveSeries:
    """Trigonometric interpolant of real data at theta_j = 2 pi j / N."""

    def __init__(self, values):
        v = _f64(values)
        self.n = v.shape[0]
        self.c = np.fft.fft(v, axis=0) / self.n
        k = np.arange(self.n)
        self.k = np.where(k <= self.n // 2, k, k - self.n).astype(np.float64)
        self.nyq = (self.n % 2 == 0)

    def __call__(self, theta, deriv: int = 0):
        th = np.atleast_1d(_f64(theta))
        k = self.k.copy()
        c = self.c.copy()
        if self.nyq:       # Nyquist mode handled separately as c cos(N theta / 2)
            c[self.n // 2] = 0.0
        E = np.exp(1j * np.outer(th, k))
        f = (1j * k) ** deriv
        out = (E @ (c * f)).real
        if self.nyq:
            cn = self.c[self.n // 2].real
            h = self.n / 2.0
            ph = h * th
            d = [np.cos(ph), -h * np.sin(ph), -h * h * np.cos(ph), h ** 3 * np.sin(ph)][deriv]
            out = out + cn * d
        return out


class CurveGeom:
    """One boundary curve as trigonometric interpolants of its node positions."""

    def __init__(self, xy, normal):
        xy = _f64(xy)
        self.n = xy.shape[0]
        self.sx = CurveSeries(xy[:, 0])
        self.sy = CurveSeries(xy[:, 1])
        # orientation of (y', -x') relative to the given outward normals
        th = 2.0 * math.pi * np.arange(self.n) / self.n
        xp, yp = self.sx(th, 1), self.sy(th, 1)
        self.sign = 1.0 if np.sum(_f64(normal)[:, 0] * yp - _f64(normal)[:, 1] * xp) >= 0 else -1.0

    def point(self, th, deriv=0):
        return np.stack([self.sx(th, deriv), self.sy(th, deriv)], axis=1)

    def normal(self, th):
        d = self.point(th, 1)
        s = np.hypot(d[:, 0], d[:, 1])
        return self.sign * np.stack([d[:, 1], -d[:, 0]], axis=1) / s[:, None]

    def spacing(self, th):
        """Local node spacing |y'(theta)| 2 pi / N."""
        d = self.point(th, 1)
        return np.hypot(d[:, 0], d[:, 1]) * (2.0 * math.pi / self.n)

    def project(self, p, th0, iters: int = 40):
        """Newton on (y(theta) - p) . y'(theta) = 0 from th0; theta in [0, 2 pi)."""
        th = _f64(th0).copy()
        p = _f64(p).reshape(-1, 2)
        for _ in range(iters):
            y, y1, y2 = self.point(th), self.point(th, 1), self.point(th, 2)
            r = y - p
            f = np.sum(r * y1, axis=1)
            fp = np.sum(y1 * y1, axis=1) + np.sum(r * y2, axis=1)
            step = f / fp
            th = th - step
            if np.all(np.abs(step) < 1e-15):
                break
        return np.mod(th, 2.0 * math.pi)


# ---------------------------------------------------------------------------
# Near-boundary evaluation of the double layer (Sec. 3.2; reading in the header)
# ---------------------------------------------------------------------------
NEAR_BAND = 4.0      # targets closer than this many local node spacings
NEAR_REACH = 5.0     # candidates: within this many spacings of their nearest node
NEAR_CHECK = 6       # check points at 1 .. K spacings
NEAR_UPSAMPLE = 8    # fine nodes per node for the check points


def curve_geoms(bxy, bnormal, offsets):
    return [CurveGeom(bxy[offsets[k]:offsets[k + 1]], bnormal[offsets[k]:offsets[k + 1]])
            for k in range(len(offsets) - 1)]


def near_targets(bxy, bnormal, bspeed, offsets, pts, band=NEAR_BAND, reach=NEAR_REACH):
    """Points inside the domain within `band` local node spacings of a curve.

    Each point's nearest node j (the lowest index among equally near ones)
    makes it a candidate when the distance is below reach * spacing_j; its
    projection theta* onto the interpolated curve of j follows by Newton from
    theta_j; the point is kept when it lies on the domain side
    ((p - y(theta*)) . n(theta*) <= 0, n outward, or d <= 1e-9 spacing: on
    the curve) and its distance d is below band * spacing(theta*).
    Returns (idx, curve, theta*, d, spacing)."""
    bxy = _f64(bxy); pts = _f64(pts)
    off = np.asarray(offsets, dtype=np.int64)
    ncur = len(off) - 1
    cid = np.repeat(np.arange(ncur), np.diff(off))
    ncj = np.diff(off)[cid]
    w = (2.0 * math.pi / ncj) * _f64(bspeed)
    geoms = curve_geoms(bxy, bnormal, off)
    jn = np.empty(pts.shape[0], dtype=np.int64)
    dn = np.empty(pts.shape[0])
    for s in range(0, pts.shape[0], 2048):
        blk = pts[s:s + 2048]
        d2 = ((blk[:, None, :] - bxy[None, :, :]) ** 2).sum(-1)
        j = np.argmin(d2, axis=1)
        jn[s:s + 2048] = j
        dn[s:s + 2048] = np.sqrt(d2[np.arange(blk.shape[0]), j])
    cand = np.flatnonzero(dn < reach * w[jn])
    idx, cur, th, dd, sp = [], [], [], [], []
    for k in range(ncur):
        sel = cand[cid[jn[cand]] == k]
        if sel.size == 0:
            continue
        g = geoms[k]
        th0 = 2.0 * math.pi * (jn[sel] - off[k]) / g.n
        ts = g.project(pts[sel], th0)
        y = g.point(ts)
        nv = g.normal(ts)
        r = pts[sel] - y
        d = np.hypot(r[:, 0], r[:, 1])
        spc = g.spacing(ts)
        on_side = (np.sum(r * nv, axis=1) <= 0.0) | (d <= 1e-9 * spc)   # points on the curve count as inside
        keep = on_side & (d < band * spc)
        idx.append(sel[keep]); cur.append(np.full(keep.sum(), k)); th.append(ts[keep])
        dd.append(d[keep]); sp.append(spc[keep])
    if not idx:
        z = np.zeros(0)
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), z, z, z
    idx = np.concatenate(idx); order = np.argsort(idx, kind="stable")
    return (idx[order], np.concatenate(cur)[order], np.concatenate(th)[order],
            np.concatenate(dd)[order], np.concatenate(sp)[order])


def fine_nodes(geoms, sigma, offsets, m=NEAR_UPSAMPLE):
    """Nodes, outward normals and weights of the m-times finer trapezoid rule on
    every curve, with sigma interpolated there."""
    xs, ns, ds = [], [], []
    for k, g in enumerate(geoms):
        M = m * g.n
        th = 2.0 * math.pi * np.arange(M) / M
        y = g.point(th)
        y1 = g.point(th, 1)
        wf = np.hypot(y1[:, 0], y1[:, 1]) * (2.0 * math.pi / M)
        sf = CurveSeries(_f64(sigma)[offsets[k]:offsets[k + 1]])(th)
        xs.append(y); ns.append(g.normal(th)); ds.append(wf * sf)
    return np.concatenate(xs), np.concatenate(ns), np.concatenate(ds)


def lagrange_eval(nodes, values, t):
    """Value at t of the polynomial through (nodes[k], values[:, k])."""
    nodes = _f64(nodes)
    out = np.zeros(values.shape[0])
    for k in range(len(nodes)):
        lk = np.ones_like(t)
        for i in range(len(nodes)):
            if i != k:
                lk = lk * (t - nodes[i]) / (nodes[k] - nodes[i])
        out += lk * values[:, k]
    return out


def near_values(bxy, bnormal, offsets, sigma, g, alpha, pts, near, K=NEAR_CHECK, m=NEAR_UPSAMPLE):
    """U^h (with its 1/alpha^2) at the near targets `near` = near_targets(...)."""
    idx, cur, th, d, sp = near
    if idx.size == 0:
        return np.zeros(0)
    off = np.asarray(offsets, dtype=np.int64)
    geoms = curve_geoms(_f64(bxy), _f64(bnormal), off)
    fx, fn, fd = fine_nodes(geoms, sigma, off, m)
    vals = np.zeros((idx.size, K + 1))
    for k, gm in enumerate(geoms):
        sel = np.flatnonzero(cur == k)
        if sel.size == 0:
            continue
        y = gm.point(th[sel])
        nv = gm.normal(th[sel])
        vals[sel, 0] = CurveSeries(_f64(g)[off[k]:off[k + 1]])(th[sel])
        for kk in range(1, K + 1):
            cpt = y - (kk * sp[sel])[:, None] * nv
            vals[sel, kk] = dl_sum(fx, fn, fd, alpha, cpt) / alpha ** 2
    return lagrange_eval(np.arange(K + 1, dtype=np.float64), vals, d / sp)


# ---------------------------------------------------------------------------
# One step on the grid
# ---------------------------------------------------------------------------
def heat_step_grid(bnd_xy, bnd_normal, bnd_w, bnd_kappa, bnd_speed, offsets, grid, B, f_next, alpha2,
                   bie=None, near=True):
    """One step of (1 - alpha^2 Lap) u = B with u = f_next on the curves, on the
    cell-centred grid (x0, y0, h, nx, ny); B at every grid point.

      q    = h^2 B
      U^p  = (V[q] + B self_weight(h, alpha)) / alpha^2       at the grid points
      U^p  at the nodes by bicubic interpolation of the grid values
      g    = f_next - U^p(nodes);  sigma = A^{-1} (-2 alpha^2 g)
      U^h  = DL[w sigma] / alpha^2 at the grid points; near targets by near_values
      u    = U^p + U^h
    Returns (u, sigma, U^p on the nodes, U^p on the grid, near targets)."""
    x0, y0, h, nx, ny = grid
    alpha = math.sqrt(alpha2)
    pts = grid_points(x0, y0, h, nx, ny)
    B = _f64(B)
    V = volume_sum(pts, h * h * B, alpha)
    Up = (V + B * self_weight(h, alpha)) / alpha2
    up_b = bicubic(Up, x0, y0, h, nx, ny, bnd_xy)
    g = _f64(f_next) - up_b
    if bie is None:
        bie = DenseBIE(bnd_xy, bnd_normal, bnd_w, bnd_kappa, alpha)
    sigma = bie.solve(g)
    Uh = dl_sum(bnd_xy, bnd_normal, _f64(bnd_w) * sigma, alpha, pts) / alpha2
    nt = None
    if near:
        nt = near_targets(bnd_xy, bnd_normal, bnd_speed, offsets, pts)
        Uh[nt[0]] = near_values(bnd_xy, bnd_normal, offsets, sigma, g, alpha, pts, nt)
    return Up + Uh, sigma, up_b, Up, nt
