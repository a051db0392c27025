"""Box-code volume quadrature on a uniform grid -- TEST INFRASTRUCTURE ONLY.

Only the tests may import this module; it shares no code with the GPU library.
It follows Sec. 3.1 (eq. volume_potential and the leaf polynomials): the grid's
cells are grouped into leaves of 4 x 4 cells; on each leaf the density is the
least-squares cubic (ten monomials) through its 16 cell-centre values, and

    V(x) = sum over leaves  int_leaf K0(|x - y| / alpha) / (2 pi) p_leaf(y) dy

(the library's normalisation: U^p = V / alpha^2).  Each (target, leaf)
integral is taken by quadrature: tensor Gauss-Legendre over the leaf when the
target is at least a leaf side away (on sub-squares no wider than 4 alpha);
otherwise the leaf is written, by
inclusion-exclusion, as signed rectangles with a corner at the target, each
split at its diagonal into two triangles integrated in polar coordinates about
the target (radius r = R s^2, Gauss-Legendre in s and in the angle), which
takes the logarithmic singularity of K0 out.  K0 is dropped beyond 40 alpha
(below 1e-18).  U^p at a point of a leaf is its
leaf polynomial fitted to the values of U^p at the leaf's cells.
"""
from __future__ import annotations

import numpy as np
from scipy.special import k0 as _k0

NPOLAR = 96     # Gauss-Legendre points in s and in the angle, per triangle
NTENSOR = 16    # per direction over each sub-square of a leaf (well separated targets)
CUT = 40.0      # K0(r/alpha) is taken as zero beyond r = CUT alpha (K0(40) < 1e-18)

_gl_cache = {}


def _gl(n):
    if n not in _gl_cache:
        _gl_cache[n] = np.polynomial.legendre.leggauss(n)
    return _gl_cache[n]


def monomials(u, v):
    """The cubic basis 1, u, v, u^2, uv, v^2, u^3, u^2 v, u v^2, v^3 (last axis)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    return np.stack([np.ones_like(u), u, v, u * u, u * v, v * v, u ** 3, u * u * v, u * v * v, v ** 3], -1)


# the 16 cell centres of a leaf in its scaled coordinates (leaf = [-1, 1]^2)
_OFFS = np.array([-0.75, -0.25, 0.25, 0.75])


def fit(values, nx, ny):
    """Per-leaf least-squares cubic coefficients [ny/4, nx/4, 10] of the cell
    values (point j nx + i at cell (i, j))."""
    vals = np.asarray(values, dtype=np.float64).reshape(ny, nx)
    uu, vv = np.meshgrid(_OFFS, _OFFS, indexing="xy")      # [row j][col i]
    Vm = monomials(uu.ravel(), vv.ravel())                  # 16 x 10, cell (i, j) at j*4 + i
    blocks = vals.reshape(ny // 4, 4, nx // 4, 4).transpose(0, 2, 1, 3).reshape(ny // 4, nx // 4, 16)
    coef, *_ = np.linalg.lstsq(Vm, blocks.reshape(-1, 16).T, rcond=None)
    return coef.T.reshape(ny // 4, nx // 4, 10)


def _corner_rect(tx, ty, X, Y, alpha, cx, cy, H):
    """Signed integral of K0(r/alpha) m(y) over the rectangle with corners
    (tx, ty) and (tx + X, ty + Y) (X, Y signed), m the ten monomials in the
    leaf coordinates ((y - c) / H).  Returns [10]."""
    if X == 0.0 or Y == 0.0:
        return np.zeros(10)
    sgn = np.sign(X) * np.sign(Y)
    ax, ay = abs(X), abs(Y)
    sx, sy = np.sign(X), np.sign(Y)
    xs, ws = _gl(NPOLAR)
    out = np.zeros(10)
    # triangle 1: angle 0 .. atan(ay/ax) (bounded by x = ax); triangle 2: the rest (y = ay)
    th_d = np.arctan2(ay, ax)
    for lo, hi, edge in ((0.0, th_d, "x"), (th_d, np.pi / 2, "y")):
        th = 0.5 * (hi - lo) * (xs + 1) + lo
        wth = 0.5 * (hi - lo) * ws
        R = ax / np.cos(th) if edge == "x" else ay / np.sin(th)
        R = np.minimum(R, CUT * alpha)   # the kernel is negligible beyond
        s = 0.5 * (xs + 1)
        wsr = 0.5 * ws
        # r = R s^2: dr = 2 R s ds
        r = R[:, None] * s[None, :] ** 2
        jac = 2.0 * R[:, None] * s[None, :]
        px = tx + sx * r * np.cos(th)[:, None]
        py = ty + sy * r * np.sin(th)[:, None]
        m = monomials((px - cx) / H, (py - cy) / H)        # [nth, ns, 10]
        f = _k0(r / alpha) * r * jac                        # [nth, ns]
        out += np.einsum("a,b,ab,abk->k", wth, wsr, f, m)
    return sgn * out


def leaf_integrals(tx, ty, cx, cy, H, alpha):
    """[10]: int over the leaf [cx - H, cx + H] x [cy - H, cy + H] of
    K0(|t - y|/alpha) m_k((y - c)/H) dy (no 1/(2 pi))."""
    dx = max(abs(tx - cx) - H, 0.0)
    dy = max(abs(ty - cy) - H, 0.0)
    if np.hypot(dx, dy) > CUT * alpha:
        return np.zeros(10)
    if max(dx, dy) >= 2.0 * H:
        # sub-squares no wider than 4 alpha (K0 varies on the scale alpha)
        k = int(min(16, max(1, np.ceil(2.0 * H / (4.0 * alpha)))))
        xs, ws = _gl(NTENSOR)
        e = -H + (2.0 * H / k) * (np.arange(k)[:, None] + 0.5 * (xs[None, :] + 1))   # [k][n] nodes
        g = (np.outer(np.ones(k), ws) * (H / k)).ravel()
        gx, gy = cx + e.ravel(), cy + e.ravel()
        X, Y = np.meshgrid(gx, gy, indexing="ij")
        w = np.outer(g, g)
        r = np.hypot(tx - X, ty - Y)
        m = monomials((X - cx) / H, (Y - cy) / H)
        return np.einsum("ab,ab,abk->k", w, _k0(r / alpha), m)
    # inclusion-exclusion over the four corners of the leaf
    x0, x1, y0, y1 = cx - H, cx + H, cy - H, cy + H
    out = np.zeros(10)
    for X, sxs in ((x1, 1.0), (x0, -1.0)):
        for Y, sys_ in ((y1, 1.0), (y0, -1.0)):
            out += sxs * sys_ * _corner_rect(tx, ty, X - tx, Y - ty, alpha, cx, cy, H)
    return out


def potential(values, grid, alpha, targets):
    """V at the target points [m][2] of the piecewise-cubic density fitted to
    the cell values (grid = (x0, y0, h, nx, ny))."""
    x0, y0, h, nx, ny = grid
    coef = fit(values, nx, ny)
    H = 2.0 * h
    out = np.zeros(len(targets))
    for k, (tx, ty) in enumerate(np.asarray(targets, dtype=np.float64)):
        acc = 0.0
        for J in range(ny // 4):
            for I in range(nx // 4):
                cx, cy = x0 + (4 * I + 2) * h, y0 + (4 * J + 2) * h
                acc += leaf_integrals(tx, ty, cx, cy, H, alpha) @ coef[J, I]
        out[k] = acc / (2.0 * np.pi)
    return out


def leaf_eval(values, grid, pts):
    """The leaf polynomial (fitted to the cell values) of the leaf holding each point."""
    x0, y0, h, nx, ny = grid
    coef = fit(values, nx, ny)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    I = np.clip(np.floor((pts[:, 0] - x0) / (4 * h)).astype(int), 0, nx // 4 - 1)
    J = np.clip(np.floor((pts[:, 1] - y0) / (4 * h)).astype(int), 0, ny // 4 - 1)
    cx, cy = x0 + (4 * I + 2) * h, y0 + (4 * J + 2) * h
    m = monomials((pts[:, 0] - cx) / (2 * h), (pts[:, 1] - cy) / (2 * h))
    return np.einsum("nk,nk->n", m, coef[J, I])


# ---------------------------------------------------------------------------
# Adaptive leaves: childless boxes of a quad-tree over the square
# [x0, x0 + side]^2, leaf k at level l_k with integer position (ix_k, iy_k),
# each with its own 4 x 4 cell-centred grid (Sec. 3.1)
# ---------------------------------------------------------------------------
def leaf_cells(levels, ix, iy, root):
    """Cell centres [n_leaves * 16][2] (cell t = jj 4 + ii of leaf k at 16 k + t)."""
    x0, y0, side = root
    s = side / (2.0 ** np.asarray(levels, dtype=np.float64))
    out = np.zeros((len(s), 16, 2))
    for t in range(16):
        out[:, t, 0] = x0 + (np.asarray(ix) + ((t & 3) + 0.5) / 4.0) * s
        out[:, t, 1] = y0 + (np.asarray(iy) + ((t >> 2) + 0.5) / 4.0) * s
    return out.reshape(-1, 2)


def fit_cells(values16):
    """Per-leaf least-squares cubic coefficients [n][10] of 16 cell values each."""
    uu, vv = np.meshgrid(_OFFS, _OFFS, indexing="xy")
    Vm = monomials(uu.ravel(), vv.ravel())
    coef, *_ = np.linalg.lstsq(Vm, np.asarray(values16, dtype=np.float64).reshape(-1, 16).T, rcond=None)
    return coef.T


def potential_leaves(levels, ix, iy, root, values16, alpha, targets):
    """V at the targets of the piecewise cubic fitted on every leaf."""
    x0, y0, side = root
    coef = fit_cells(values16)
    s = side / (2.0 ** np.asarray(levels, dtype=np.float64))
    cx = x0 + (np.asarray(ix) + 0.5) * s
    cy = y0 + (np.asarray(iy) + 0.5) * s
    out = np.zeros(len(targets))
    for k, (tx, ty) in enumerate(np.asarray(targets, dtype=np.float64)):
        acc = 0.0
        for j in range(len(s)):
            acc += leaf_integrals(tx, ty, cx[j], cy[j], 0.5 * s[j], alpha) @ coef[j]
        out[k] = acc / (2.0 * np.pi)
    return out


def refine_flags(values16, values64, tol):
    """Sec. 3.1's refinement test: a leaf is split when its cubic fitted to the
    16 cell values misses the values at the 64 cell centres of its four
    children (children's 4 x 4 grids, child q = qy 2 + qx, cell t) by more
    than tol.  Returns the flags and the errors."""
    coef = fit_cells(values16)
    v64 = np.asarray(values64, dtype=np.float64).reshape(-1, 4, 16)
    err = np.zeros(len(coef))
    for q in range(4):
        qx, qy = q & 1, q >> 1
        for t in range(16):
            # child cell centre in the parent's scaled coordinates [-1, 1]
            u = -1.0 + (qx * 4 + (t & 3) + 0.5) / 4.0
            v = -1.0 + (qy * 4 + (t >> 2) + 0.5) / 4.0
            e = np.abs(monomials(u, v) @ coef.T - v64[:, q, t])
            err = np.maximum(err, e)
    return err > tol, err


def balanced_leaves(root, centre, depth_max, depth_min=2):
    """A 2:1 balanced leaf set refined towards a point (test input): levels
    from depth_min to depth_max, finer closer to `centre`.  Returns levels,
    ix, iy."""
    x0, y0, side = root
    cx, cy = centre
    leaves = {}

    def want(l, i, j):
        s = side / 2 ** l
        bx, by = x0 + (i + 0.5) * s, y0 + (j + 0.5) * s
        d = max(abs(bx - cx), abs(by - cy))
        return l < depth_min or (l < depth_max and d < 1.5 * s)

    def build(l, i, j):
        if want(l, i, j):
            for q in range(4):
                build(l + 1, 2 * i + (q & 1), 2 * j + (q >> 1))
        else:
            leaves[(l, i, j)] = True

    build(0, 0, 0)
    # 2:1 balance: split a leaf touched by a leaf two or more levels finer
    changed = True
    while changed:
        changed = False
        for (l, i, j) in list(leaves):
            if (l, i, j) not in leaves:
                continue
            s = 1.0 / 2 ** l
            hit = False
            for (l2, i2, j2) in leaves:
                if l2 < l + 2:
                    continue
                s2 = 1.0 / 2 ** l2
                if (i2 * s2 <= (i + 1) * s and i * s <= (i2 + 1) * s2 and
                        j2 * s2 <= (j + 1) * s and j * s <= (j2 + 1) * s2):
                    hit = True
                    break
            if hit:
                del leaves[(l, i, j)]
                for q in range(4):
                    leaves[(l + 1, 2 * i + (q & 1), 2 * j + (q >> 1))] = True
                changed = True
    keys = sorted(leaves)
    return (np.array([k[0] for k in keys], dtype=np.int32), np.array([k[1] for k in keys], dtype=np.int32),
            np.array([k[2] for k in keys], dtype=np.int32))


def balanced_leaves_by(root, want, depth_max):
    """A 2:1 balanced leaf set (test input): a box (l, i, j) is split while
    want(l, i, j) holds (up to depth_max), then leaves touched by leaves two
    or more levels finer are split.  Returns levels, ix, iy."""
    leaves = set()

    def build(l, i, j):
        if l < depth_max and want(l, i, j):
            for q in range(4):
                build(l + 1, 2 * i + (q & 1), 2 * j + (q >> 1))
        else:
            leaves.add((l, i, j))

    build(0, 0, 0)
    changed = True
    while changed:
        changed = False
        by_level = {}
        for (l, i, j) in leaves:
            by_level.setdefault(l, set()).add((i, j))
        for (l, i, j) in sorted(leaves):
            hit = False
            for l2 in range(l + 2, depth_max + 1):
                f = 2 ** (l2 - l)
                ring = [(i * f + a, j * f + b) for a in range(-1, f + 1) for b in range(-1, f + 1)
                        if not (0 <= a < f and 0 <= b < f)]
                if any(c in by_level.get(l2, ()) for c in ring):
                    hit = True
                    break
            if hit:
                leaves.discard((l, i, j))
                for q in range(4):
                    leaves.add((l + 1, 2 * i + (q & 1), 2 * j + (q >> 1)))
                changed = True
                break
    keys = sorted(leaves)
    return (np.array([k[0] for k in keys], dtype=np.int32), np.array([k[1] for k in keys], dtype=np.int32),
            np.array([k[2] for k in keys], dtype=np.int32))
