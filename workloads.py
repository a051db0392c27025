"""Seeded synthetic inputs for the Yukawa heat-step path.

This module is shared by the tests, the benchmark and the smoke check.  It
holds geometry and problem data only (node positions, analytic normals and
curvatures, point clouds, manufactured solutions, boundary constants) and none
of the method's arithmetic: no kernel sums, no solves, no K0/K1.  The one
closed form built from Bessel functions is Example 1's exact solution (J0/Y0
from scipy.special), the reference the temporal study is measured against.
Both the CPU oracle and the GPU library receive what it produces as plain
arrays.

Conventions (Kropinski & Quaife, Sec. 3.2 and the kernel-continuity passage
of Sec. 2):
  * curve 0 is the outer boundary, traversed counter-clockwise; every hole is
    traversed clockwise, so the normal n = (y2', -y1')/|y'| points out of the
    domain on every curve;
  * curvature is signed, kappa = (y1' y2'' - y2' y1'') / |y'|^3: +1/R on a
    counter-clockwise circle of radius R, -1/R on a clockwise one;
  * each curve has N_k nodes equispaced in its parameter on [0, 2 pi), and the
    trapezoid weight of node j is w_j = (2 pi / N_k) |y'(theta_j)|.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Curve", "Boundary", "circle", "ellipse", "make_boundary",
    "config_c0", "config_c1", "config_c2", "config_c3", "config_c4",
    "small_fmm_case", "sample_targets", "adaptive_cells", "example1", "example3", "grid_box",
]


# ----------------------------------------------------------------------------
# Curves
# ----------------------------------------------------------------------------
@dataclass
class Curve:
    """One closed curve sampled at N parameter-equispaced nodes."""
    xy: np.ndarray        # [N, 2]
    normal: np.ndarray    # [N, 2], unit, outward from the domain
    speed: np.ndarray     # [N], |y'(theta)|
    curvature: np.ndarray  # [N], signed
    kind: str             # "circle" / "ellipse"
    params: dict          # centre, radii, rotation, orientation

    @property
    def n(self) -> int:
        return self.xy.shape[0]


def _from_derivatives(y, yp, ypp, kind, params) -> Curve:
    sp = np.hypot(yp[:, 0], yp[:, 1])
    nrm = np.stack([yp[:, 1], -yp[:, 0]], axis=1) / sp[:, None]
    kap = (yp[:, 0] * ypp[:, 1] - yp[:, 1] * ypp[:, 0]) / sp**3
    return Curve(np.ascontiguousarray(y), np.ascontiguousarray(nrm),
                 np.ascontiguousarray(sp), np.ascontiguousarray(kap), kind, params)


def ellipse(center, a, b, n, rotation=0.0, ccw=True) -> Curve:
    """Ellipse with semi-axes a, b rotated by `rotation`, analytic derivatives."""
    th = 2.0 * np.pi * np.arange(n) / n
    s = 1.0 if ccw else -1.0
    c, si = math.cos(rotation), math.sin(rotation)
    # local parametrisation (a cos t, s b sin t)
    lx, ly = a * np.cos(th), s * b * np.sin(th)
    lxp, lyp = -a * np.sin(th), s * b * np.cos(th)
    lxpp, lypp = -a * np.cos(th), -s * b * np.sin(th)
    rot = lambda u, v: np.stack([c * u - si * v, si * u + c * v], axis=1)
    y = rot(lx, ly) + np.asarray(center, dtype=np.float64)[None, :]
    yp = rot(lxp, lyp)
    ypp = rot(lxpp, lypp)
    return _from_derivatives(y, yp, ypp, "ellipse",
                             dict(center=tuple(center), a=a, b=b, rotation=rotation, ccw=ccw))


def circle(center, r, n, ccw=True) -> Curve:
    cv = ellipse(center, r, r, n, 0.0, ccw)
    cv.kind = "circle"
    cv.params = dict(center=tuple(center), r=r, ccw=ccw)
    return cv


@dataclass
class Boundary:
    """Multiply connected boundary: curve 0 outer, curves 1.. holes."""
    curves: list
    xy: np.ndarray = field(init=False)
    normal: np.ndarray = field(init=False)
    speed: np.ndarray = field(init=False)
    curvature: np.ndarray = field(init=False)
    offset: np.ndarray = field(init=False)   # int64 [n_curves + 1]

    def __post_init__(self):
        self.xy = np.ascontiguousarray(np.concatenate([c.xy for c in self.curves]))
        self.normal = np.ascontiguousarray(np.concatenate([c.normal for c in self.curves]))
        self.speed = np.ascontiguousarray(np.concatenate([c.speed for c in self.curves]))
        self.curvature = np.ascontiguousarray(np.concatenate([c.curvature for c in self.curves]))
        self.offset = np.zeros(len(self.curves) + 1, dtype=np.int64)
        self.offset[1:] = np.cumsum([c.n for c in self.curves])

    @property
    def n(self) -> int:
        return int(self.offset[-1])

    @property
    def n_curves(self) -> int:
        return len(self.curves)

    def weights(self) -> np.ndarray:
        """Trapezoid weights (2 pi / N_k) |y'| (the arc-length element)."""
        w = np.empty(self.n)
        for k, c in enumerate(self.curves):
            w[self.offset[k]:self.offset[k + 1]] = (2.0 * np.pi / c.n) * c.speed
        return w

    def curve_id(self) -> np.ndarray:
        cid = np.empty(self.n, dtype=np.int32)
        for k in range(self.n_curves):
            cid[self.offset[k]:self.offset[k + 1]] = k
        return cid

    def region(self, pts: np.ndarray) -> np.ndarray:
        """-1 inside the domain, 0 outside the outer curve, k inside hole k."""
        reg = np.full(pts.shape[0], -1, dtype=np.int32)
        for k in range(self.n_curves - 1, -1, -1):
            ins = _inside_curve(self.curves[k], pts)
            if k == 0:
                reg[~ins] = 0
            else:
                reg[ins] = k
        return reg

    def distance_to_boundary(self, pts: np.ndarray) -> np.ndarray:
        """Distance to the nearest boundary node (a proxy used to keep
        accuracy checks away from the layer where the trapezoid rule fails)."""
        d = np.full(pts.shape[0], np.inf)
        for c in self.curves:
            for s in range(0, pts.shape[0], 4096):
                blk = pts[s:s + 4096]
                dd = np.sqrt(((blk[:, None, :] - c.xy[None, :, :]) ** 2).sum(-1)).min(1)
                d[s:s + 4096] = np.minimum(d[s:s + 4096], dd)
        return d


def _inside_curve(c: Curve, pts: np.ndarray) -> np.ndarray:
    p = c.params
    x = pts[:, 0] - p["center"][0]
    y = pts[:, 1] - p["center"][1]
    if c.kind == "circle":
        return x * x + y * y < p["r"] ** 2
    rot = p["rotation"]
    u = math.cos(rot) * x + math.sin(rot) * y
    v = -math.sin(rot) * x + math.cos(rot) * y
    return (u / p["a"]) ** 2 + (v / p["b"]) ** 2 < 1.0


def make_boundary(curves) -> Boundary:
    return Boundary(list(curves))


# ----------------------------------------------------------------------------
# Configurations (shapes and distributions of the paper's workloads)
# ----------------------------------------------------------------------------
def _cell_grid(lo, hi, m):
    h = (hi - lo) / m
    g = lo + h * (np.arange(m) + 0.5)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], axis=1)), h


def config_c0(n_nodes=256, m=64, dt=0.01):
    """Unit disk minus a hole of radius 0.3 at (0.2, 0); an m x m cell-centred
    grid over the box [-1, 1]^2 as volume points; manufactured solution
    u = exp(-2t) sin x sin y (F = 0), one backward-Euler step."""
    bnd = make_boundary([circle((0.0, 0.0), 1.0, n_nodes, ccw=True),
                         circle((0.2, 0.0), 0.3, n_nodes, ccw=False)])
    vol, h = _cell_grid(-1.0, 1.0, m)
    u0 = np.sin(vol[:, 0]) * np.sin(vol[:, 1])
    t1 = dt
    f_next = math.exp(-2.0 * t1) * np.sin(bnd.xy[:, 0]) * np.sin(bnd.xy[:, 1])
    region = bnd.region(vol)
    return dict(name="c0", bnd=bnd, vol=vol, vol_w=np.full(vol.shape[0], h * h), h=h,
                B=u0.copy(), u0=u0, f_next=f_next, dt=dt, alpha=math.sqrt(dt),
                region=region, grid=True,
                u_exact_next=math.exp(-2.0 * t1) * np.sin(vol[:, 0]) * np.sin(vol[:, 1]))


def _c1_boundary(n_nodes):
    cen = (0.5, 0.5)
    curves = [circle(cen, 0.5, n_nodes, ccw=True)]
    for k in range(5):
        t = 2.0 * np.pi * k / 5.0
        curves.append(circle((0.5 + 0.25 * math.cos(t), 0.5 + 0.25 * math.sin(t)),
                             0.06, n_nodes, ccw=False))
    return make_boundary(curves)


def config_c1(n_vol=1 << 20, n_nodes=4096, alpha=0.05, seed=1):
    """FMM throughput set: n_vol iid uniform points in the unit square with
    N(0,1) charges; outer circle (centre (0.5,0.5), radius 0.5) plus five
    circular holes of radius 0.06, n_nodes nodes per curve, N(0,1) dipole
    strengths."""
    rng = np.random.default_rng(seed)
    vol = rng.random((n_vol, 2))
    q = rng.standard_normal(n_vol)
    bnd = _c1_boundary(n_nodes)
    dip = rng.standard_normal(bnd.n)
    return dict(name="c1", bnd=bnd, vol=np.ascontiguousarray(vol), q=q, dip=dip, alpha=alpha)


def config_c2(alpha, n_vol=1 << 20, n_nodes=4096, seed=1):
    cfg = config_c1(n_vol, n_nodes, alpha, seed)
    cfg["name"] = "c2"
    # Dirichlet data of a synthetic solve: g = 1 - (volume potential on the nodes)
    # is formed by the caller; here only the raw sets are provided.
    return cfg


def _random_ellipses(rng, n_holes, n_nodes, amin, amax, gap, rmax=0.4, cen=(0.5, 0.5)):
    placed = []
    tries = 0
    while len(placed) < n_holes:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place holes")
        a = rng.uniform(amin, amax)
        b = rng.uniform(amin, amax)
        rot = rng.uniform(0.0, np.pi)
        rr = rmax * math.sqrt(rng.random())
        tt = rng.uniform(0, 2 * np.pi)
        c = (cen[0] + rr * math.cos(tt), cen[1] + rr * math.sin(tt))
        R = max(a, b)
        if math.hypot(c[0] - cen[0], c[1] - cen[1]) + R > 0.5 - gap:
            continue
        ok = all(math.hypot(c[0] - c2[0], c[1] - c2[1]) > R + R2 + gap for (c2, R2, *_r) in placed)
        if ok:
            placed.append((c, R, a, b, rot))
    return [ellipse(c, a, b, n_nodes, rot, ccw=False) for (c, R, a, b, rot) in placed]


def config_c3(m=1024, n_holes=10, n_nodes=2048, dt=1e-3, seed=3, n_outer=None):
    """Time-stepping set: unit square, n_holes random ellipses (semi-axes
    U[0.02,0.08], rotation U[0,pi)) with n_nodes nodes each inside an outer
    circle of radius 0.5 at (0.5,0.5); an m x m cell-centred grid;
    u_0 = 0 in the domain, u = 0 on the outer curve and u = c_k on hole k.
    The outer circle gets n_outer nodes, by default the power of two that makes
    its node spacing at most 0.4 grid cells, so that no curve is coarser than
    the grid (the trapezoid double layer is inaccurate within about two node
    spacings of its curve)."""
    rng = np.random.default_rng(seed)
    if n_outer is None:
        n_outer = 1 << int(math.ceil(math.log2(2 * math.pi * 0.5 / (0.4 / m))))
    curves = [circle((0.5, 0.5), 0.5, n_outer, ccw=True)]
    curves += _random_ellipses(rng, n_holes, n_nodes, 0.02, 0.08, 0.02)
    bnd = make_boundary(curves)
    vol, h = _cell_grid(0.0, 1.0, m)
    consts = np.concatenate([[0.0], rng.choice([-1.0, -0.5, 0.5, 1.0], size=n_holes)])
    region = bnd.region(vol)
    f_bnd = np.repeat(consts, np.diff(bnd.offset))
    return dict(name="c3", bnd=bnd, vol=vol, vol_w=np.full(vol.shape[0], h * h), h=h,
                consts=consts, region=region, f_bnd=f_bnd, dt=dt, alpha=math.sqrt(dt),
                u0=np.zeros(vol.shape[0]), grid=True)


def _mixture_density(x, y, mu, sg):
    """Density of an equal-weight mixture of isotropic Gaussians at (x, y)."""
    p = np.zeros_like(x)
    for g in range(len(sg)):
        d2 = (x - mu[g, 0]) ** 2 + (y - mu[g, 1]) ** 2
        p += np.exp(-d2 / (2 * sg[g] ** 2)) / (2 * np.pi * sg[g] ** 2)
    return p / len(sg)


def adaptive_cells(target, density, max_level=16, refine=None):
    """Square cells of an adaptive quadtree over the unit square: a cell of side
    h is split while h > 1/sqrt(target * density(centre)), or while
    refine(cx, cy, h) holds (and its level is below max_level).  Returns the
    cell centres and sides."""
    cx, cy = np.array([0.5]), np.array([0.5])
    ox, oy, oh = [], [], []
    for level in range(max_level + 1):
        h = 2.0 ** -level
        split = h * h * target * density(cx, cy) > 1.0
        if refine is not None:
            split |= refine(cx, cy, h)
        if level == max_level:
            split[:] = False
        ox.append(cx[~split])
        oy.append(cy[~split])
        oh.append(np.full(int((~split).sum()), h))
        sx, sy, q = cx[split], cy[split], h / 4
        if sx.size == 0:
            break
        cx = np.concatenate([sx - q, sx + q, sx - q, sx + q])
        cy = np.concatenate([sy - q, sy - q, sy + q, sy + q])
    return np.concatenate(ox), np.concatenate(oy), np.concatenate(oh)


def graded_leaves(centre=(0.5, 0.5), radius=0.3, lo=6, hi=10, K=2.0):
    """Leaves (level, ix, iy) of a quadtree over the unit square refined towards
    a circle: a box of level l splits while l < lo, or while l < hi and its
    distance to the circle is below K times its side.  With K >= sqrt(2) two
    touching leaves differ by at most one level (a split box of level l + 1
    touching a leaf of level l would bring the circle within K/2 + sqrt(2)/2
    sides of level l of the leaf), so the set is 2:1 balanced."""
    cx, cy = centre
    ix, iy = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
    out_l, out_x, out_y = [], [], []
    for level in range(hi + 1):
        s = 2.0 ** -level
        x0, y0 = ix * s, iy * s
        dx = np.maximum(np.maximum(x0 - cx, cx - (x0 + s)), 0.0)
        dy = np.maximum(np.maximum(y0 - cy, cy - (y0 + s)), 0.0)
        dmin = np.hypot(dx, dy)
        dmax = np.hypot(np.maximum(np.abs(x0 - cx), np.abs(x0 + s - cx)),
                        np.maximum(np.abs(y0 - cy), np.abs(y0 + s - cy)))
        dist = np.where(radius < dmin, dmin - radius, np.where(radius > dmax, radius - dmax, 0.0))
        split = (level < lo) | ((level < hi) & (dist < K * s))
        out_l.append(np.full(int((~split).sum()), level, dtype=np.int32))
        out_x.append(ix[~split].astype(np.int32))
        out_y.append(iy[~split].astype(np.int32))
        sx, sy = ix[split], iy[split]
        ix = np.concatenate([2 * sx, 2 * sx + 1, 2 * sx, 2 * sx + 1])
        iy = np.concatenate([2 * sy, 2 * sy, 2 * sy + 1, 2 * sy + 1])
        if ix.size == 0:
            break
    return np.concatenate(out_l), np.concatenate(out_x), np.concatenate(out_y)


def leaf_cell_centres(level, ix, iy):
    """The 16 cell centres of every leaf (cell t = jj 4 + ii), [n_leaves * 16][2]."""
    s = 2.0 ** -level.astype(np.float64)
    t = np.arange(16)
    u, v = (t & 3) + 0.5, (t >> 2) + 0.5
    x = (ix[:, None] + u[None, :] / 4.0) * s[:, None]
    y = (iy[:, None] + v[None, :] / 4.0) * s[:, None]
    return np.stack([x.ravel(), y.ravel()], axis=1)


def config_c4(n_vol=1 << 24, n_holes=20, n_nodes=8192, alpha=1e-3, seed=4, n_gauss=8):
    """Large adaptive set: the centres of about n_vol square cells of an
    adaptive quadtree over the unit square, refined where a mixture of n_gauss
    isotropic Gaussians (means U[0.2,0.8]^2, widths log-uniform on
    [0.01, 0.1]) is dense (side about 1/sqrt(T p(x)), T set by two coarse
    trials so that the count comes out near n_vol), and to side <= alpha / 4
    within 12 alpha of every curve (the boundary layer of width ~alpha that B
    acquires there, which the paper's refinement by B's interpolation error
    would resolve); weights the cell areas (the heat step adds each cell's own
    integral); n_holes circular holes r ~ U[0.01, 0.05]."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.2, 0.8, size=(n_gauss, 2))
    sg = np.exp(rng.uniform(math.log(0.01), math.log(0.1), size=n_gauss))
    dens = lambda x, y: _mixture_density(x, y, mu, sg)
    placed = []
    while len(placed) < n_holes:
        r = rng.uniform(0.01, 0.05)
        rr = 0.4 * math.sqrt(rng.random())
        tt = rng.uniform(0, 2 * np.pi)
        c = (0.5 + rr * math.cos(tt), 0.5 + rr * math.sin(tt))
        if rr + r > 0.48:
            continue
        if all(math.hypot(c[0] - c2[0], c[1] - c2[1]) > r + r2 + 0.02 for c2, r2 in placed):
            placed.append((c, r))
    circles = [((0.5, 0.5), 0.5)] + placed
    band = 12.0 * alpha

    def near_curves(cx, cy, h):
        if h <= alpha / 4:
            return np.zeros(cx.shape, dtype=bool)
        out = np.zeros(cx.shape, dtype=bool)
        reach = band + 0.7072 * h
        for (ccx, ccy), rad in circles:
            out |= np.abs(np.hypot(cx - ccx, cy - ccy) - rad) < reach
        return out

    # the count grows with T about linearly (plus the cells the curves add):
    # two trials and two secant steps put it near n_vol
    ts = [n_vol / 64.0, n_vol / 32.0]
    cs = [adaptive_cells(t, dens, refine=near_curves)[0].size for t in ts]
    for _ in range(2):
        a = (cs[-1] - cs[-2]) / (ts[-1] - ts[-2])
        ts.append(max(ts[0], ts[-1] + (n_vol - cs[-1]) / a))
        cs.append(adaptive_cells(ts[-1], dens, refine=near_curves)[0].size)
    x, y, h = adaptive_cells(ts[-1], dens, refine=near_curves)
    pts = np.ascontiguousarray(np.stack([x, y], axis=1))
    w = h * h
    curves = [circle((0.5, 0.5), 0.5, n_nodes, ccw=True)]
    curves += [circle(c, r, n_nodes, ccw=False) for c, r in placed]
    bnd = make_boundary(curves)
    consts = np.concatenate([[0.0], rng.choice([-1.0, -0.5, 0.5, 1.0], size=n_holes)])
    return dict(name="c4", bnd=bnd, vol=pts, vol_w=w, consts=consts, alpha=alpha,
                dt=alpha * alpha, grid=True)


def small_fmm_case(n_vol=4096, n_nodes=256, alpha=0.05, seed=11, n_holes=5, clustered=False):
    """A C1-shaped case small enough for the oracle's direct sums."""
    rng = np.random.default_rng(seed)
    if clustered:
        k = rng.integers(0, 3, size=n_vol)
        mu = np.array([[0.3, 0.3], [0.7, 0.6], [0.45, 0.8]])
        vol = np.clip(mu[k] + 0.05 * rng.standard_normal((n_vol, 2)), 1e-6, 1 - 1e-6)
    else:
        vol = rng.random((n_vol, 2))
    q = rng.standard_normal(n_vol)
    cen = (0.5, 0.5)
    curves = [circle(cen, 0.5, n_nodes, ccw=True)]
    for k in range(n_holes):
        t = 2.0 * np.pi * k / max(n_holes, 1)
        curves.append(circle((0.5 + 0.25 * math.cos(t), 0.5 + 0.25 * math.sin(t)),
                             0.06, n_nodes, ccw=False))
    bnd = make_boundary(curves)
    dip = rng.standard_normal(bnd.n)
    return dict(name="small", bnd=bnd, vol=np.ascontiguousarray(vol), q=q, dip=dip, alpha=alpha)


def sample_targets(n_total: int, k: int, seed: int = 0) -> np.ndarray:
    """k distinct target indices drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    k = min(k, n_total)
    return np.sort(rng.choice(n_total, size=k, replace=False)).astype(np.int64)


# ----------------------------------------------------------------------------
# The paper's examples (Sec. 4)
# ----------------------------------------------------------------------------
def grid_box(lo, hi, m):
    """(x0, y0, h, nx, ny) of an m x m cell-centred grid over [lo, hi]^2 and its points."""
    h = (hi - lo) / m
    pts, _ = _cell_grid(lo, hi, m)
    return (lo, lo, h, m, m), pts


def example1(m=256, n_outer=1024, n_inner=512, lo=-0.5, hi=0.5):
    """Example 1: the annulus 0.1 < |x| < 0.4 (outer circle counter-clockwise,
    hole clockwise), forcing F = 400 cos(20 r) + 20 sin(20 r) / r, Dirichlet
    data cos 8 on r = 0.4 and cos 2 on r = 0.1, exact solution
      u = exp(-lam^2 t) [Y0(0.1 lam) J0(lam r) - J0(0.1 lam) Y0(lam r)] + cos(20 r)
    with lam the first root of Y0(0.1 lam) J0(0.4 lam) = J0(0.1 lam) Y0(0.4 lam)
    (lam ~ 10.244, so the transient vanishes on both circles).  Volume points:
    an m x m cell-centred grid over [lo, hi]^2; F is given everywhere, u is
    extended by the boundary constants (region 0 outside, 1 in the hole)."""
    from scipy import optimize, special
    bnd = make_boundary([circle((0.0, 0.0), 0.4, n_outer, ccw=True),
                         circle((0.0, 0.0), 0.1, n_inner, ccw=False)])
    grid, pts = grid_box(lo, hi, m)
    f = lambda l: special.y0(0.1 * l) * special.j0(0.4 * l) - special.j0(0.1 * l) * special.y0(0.4 * l)
    lam = optimize.brentq(f, 9.0, 11.5, xtol=1e-15)
    r = np.hypot(pts[:, 0], pts[:, 1])
    F = 400.0 * np.cos(20.0 * r) + 20.0 * np.sin(20.0 * r) / r

    def exact(xy, t):
        rr = np.hypot(xy[:, 0], xy[:, 1])
        z = (special.y0(0.1 * lam) * special.j0(lam * rr) - special.j0(0.1 * lam) * special.y0(lam * rr))
        return math.exp(-lam * lam * t) * z + np.cos(20.0 * rr)

    consts = np.array([math.cos(8.0), math.cos(2.0)])
    f_bnd = np.concatenate([np.full(n_outer, consts[0]), np.full(n_inner, consts[1])])
    return dict(name="example1", bnd=bnd, grid=grid, pts=pts, F=F, lam=lam, exact=exact,
                consts=consts, f_bnd=f_bnd, region=bnd.region(pts))


def example3(m=256, n_outer=1024, n_inner=512, seed=3, lo=-0.5, hi=0.5):
    """Example 3's setting (and Example 2's domain): an elliptical region with
    an off-centre elliptical hole, u = 0 on both curves, random initial data
    uniform on [-1/2, 1/2] inside; the Allen-Cahn reaction u (1 - u^2) with
    eps = 1e-5 and dt = 1 (alpha^2 = eps dt for the Euler scheme)."""
    rng = np.random.default_rng(seed)
    bnd = make_boundary([ellipse((0.0, 0.0), 0.45, 0.32, n_outer, rotation=0.2, ccw=True),
                         ellipse((0.12, 0.04), 0.12, 0.07, n_inner, rotation=0.6, ccw=False)])
    grid, pts = grid_box(lo, hi, m)
    region = bnd.region(pts)
    u0 = np.where(region < 0, rng.uniform(-0.5, 0.5, pts.shape[0]), 0.0)
    return dict(name="example3", bnd=bnd, grid=grid, pts=pts, region=region, u0=u0,
                consts=np.zeros(2), f_bnd=np.zeros(bnd.n), eps=1e-5, dt=1.0)
