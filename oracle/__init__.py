"""CPU FP64 oracle for the Yukawa heat step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library (it neither
imports it nor links it), and the library never calls it.

It computes, plainly and slowly (Kropinski & Quaife, arXiv 1007.5335):
  * direct O(N_t N_s) sums of K0(|x-y|/alpha)/(2 pi) and of the double-layer
    kernel (Sec. 2; library-sum normalisation without the 1/alpha^2 of G);
  * the dense matrix of the trapezoid discretisation of the second-kind
    equation (Sec. 3.2, eq. discrete_sys) and its LU solve; the diagonal
    carries the generalised Euler-Maclaurin correction of the kernel's
    t^2 log|t| term, which makes the rule fifth order (in place of the
    paper's Alpert rule, whose node tables are not reproduced here);
  * one backward-Euler step (Sec. 2: alpha^2 = dt, B = u^N + dt F^N), split
    into volume potential plus double layer (eqs. particular, mod_helm_hom,
    vol_potential), evaluated as weighted point sums with a self-cell
    correction for grid points.
Parity pins for every function live in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "yk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C part with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    for name in ("yko_k0", "yko_k1", "yko_i0", "yko_i1"):
        f = getattr(lib, name)
        f.restype = ctypes.c_double
        f.argtypes = [ctypes.c_double]
    lib.yko_dl_kernel.restype = ctypes.c_double
    lib.yko_dl_kernel.argtypes = [ctypes.c_double] * 7
    lib.yko_dl_diag.restype = ctypes.c_double
    lib.yko_dl_diag.argtypes = [ctypes.c_double] * 3
    lib.yko_lattice_k0_sum.restype = ctypes.c_double
    lib.yko_lattice_k0_sum.argtypes = [ctypes.c_double]
    for name in ("yko_k0_vec", "yko_k1_vec", "yko_i0_vec", "yko_i1_vec"):
        f = getattr(lib, name)
        f.restype = None
        f.argtypes = [i64, dp, dp]
    lib.yko_volume_sum.restype = None
    lib.yko_volume_sum.argtypes = [i64, dp, i64, dp, dp, ctypes.c_double, ctypes.c_int, dp]
    lib.yko_dl_sum.restype = None
    lib.yko_dl_sum.argtypes = [i64, dp, i64, dp, dp, dp, ctypes.c_double, dp]
    lib.yko_set_threads.restype = None
    lib.yko_set_threads.argtypes = [ctypes.c_int]
    lib.yko_max_threads.restype = ctypes.c_int
    lib.yko_max_threads.argtypes = []
    lib.yko_dl_matrix.restype = None
    lib.yko_dl_matrix.argtypes = [i64, dp, dp, dp, dp, ctypes.c_double, dp]
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    """Number of OpenMP threads of the direct sums (timing only)."""
    _load().yko_set_threads(int(n))


def max_threads() -> int:
    return int(_load().yko_max_threads())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# Special functions
# ---------------------------------------------------------------------------
def k0(z):
    z = _f64(np.atleast_1d(z)); out = np.empty_like(z)
    _load().yko_k0_vec(z.size, _p(z), _p(out)); return out


def k1(z):
    z = _f64(np.atleast_1d(z)); out = np.empty_like(z)
    _load().yko_k1_vec(z.size, _p(z), _p(out)); return out


def i0(z):
    z = _f64(np.atleast_1d(z)); out = np.empty_like(z)
    _load().yko_i0_vec(z.size, _p(z), _p(out)); return out


def i1(z):
    z = _f64(np.atleast_1d(z)); out = np.empty_like(z)
    _load().yko_i1_vec(z.size, _p(z), _p(out)); return out


def dl_kernel(x, y, n, alpha) -> float:
    """d/dnu_y K0(|x-y|/alpha) for one target x, node y with unit normal n."""
    return _load().yko_dl_kernel(float(x[0]), float(x[1]), float(y[0]), float(y[1]),
                                 float(n[0]), float(n[1]), float(alpha))


# ---------------------------------------------------------------------------
# Direct sums (Sec. 2 kernels, library normalisation: no 1/alpha^2)
# ---------------------------------------------------------------------------
def volume_sum(src_xy, q, alpha, tgt_xy=None) -> np.ndarray:
    """V[q](t_i) = sum_j q_j K0(|t_i - s_j|/alpha)/(2 pi); tgt_xy None means
    targets are the sources and the self pair is skipped by index."""
    s = _f64(src_xy); q = _f64(q)
    same = tgt_xy is None
    t = s if same else _f64(tgt_xy)
    out = np.empty(t.shape[0])
    _load().yko_volume_sum(t.shape[0], _p(t), s.shape[0], _p(s), _p(q), float(alpha),
                           1 if same else 0, _p(out))
    return out


def dl_sum(bxy, bnormal, d, alpha, tgt_xy) -> np.ndarray:
    """DL[d](t_i) = sum_j d_j D(t_i, y_j)/(2 pi), off-surface (pairs with r = 0 skipped)."""
    b = _f64(bxy); n = _f64(bnormal); d = _f64(d); t = _f64(tgt_xy)
    out = np.empty(t.shape[0])
    _load().yko_dl_sum(t.shape[0], _p(t), b.shape[0], _p(b), _p(n), _p(d), float(alpha), _p(out))
    return out


def dl_diag(w, kappa, alpha):
    """Diagonal kernel value of the corrected trapezoid rule: the limit -kappa/2
    (Sec. 2) plus zeta(3) kappa w^2 / (8 pi^2 alpha^2), the generalised
    Euler-Maclaurin error of the kernel's t^2 log|t| term along the curve
    (derivation at yko_dl_diag in yk_oracle.c)."""
    return np.array([_load().yko_dl_diag(float(a), float(b), float(alpha))
                     for a, b in zip(np.atleast_1d(w), np.atleast_1d(kappa))])


def dl_matrix(bxy, bnormal, w, kappa, alpha) -> np.ndarray:
    """A = I - 2 [w_n D(y_j, y_n)/(2 pi)], diagonal D = dl_diag (eq. discrete_sys,
    corrected trapezoid rule)."""
    b = _f64(bxy); n = _f64(bnormal); w = _f64(w); k = _f64(kappa)
    nb = b.shape[0]
    A = np.empty((nb, nb))
    _load().yko_dl_matrix(nb, _p(b), _p(n), _p(w), _p(k), float(alpha), _p(A))
    return A


def dl_on_surface(bxy, bnormal, w, kappa, sigma, alpha) -> np.ndarray:
    """On-surface DL[w sigma](y_j) with the corrected diagonal (the matrix action
    of (I - A)/2 written as a sum)."""
    off = dl_sum(bxy, bnormal, _f64(w) * _f64(sigma), alpha, bxy)
    return off + _f64(w) * dl_diag(w, kappa, alpha) * _f64(sigma) / (2.0 * math.pi)


def apply_bie(bxy, bnormal, w, kappa, sigma, alpha) -> np.ndarray:
    """(A sigma)_j = sigma_j - 2 DL[w sigma](y_j)."""
    return _f64(sigma) - 2.0 * dl_on_surface(bxy, bnormal, w, kappa, sigma, alpha)


# ---------------------------------------------------------------------------
# Self-cell correction for grid points
# ---------------------------------------------------------------------------
def lattice_k0_sum(eps: float) -> float:
    """sum over the nonzero points j of Z^2 with |j| eps <= 40 of K0(|j| eps)."""
    return float(_load().yko_lattice_k0_sum(float(eps)))


def self_cell(h: float, alpha: float, n_gauss: int = 48) -> float:
    """(1/2pi) int over the h x h cell centred at the target of K0(|y|/alpha) dA.

    Split the square into 8 right triangles with apex at the centre; along a
    ray at angle theta the radius ends at R = (h/2)/cos(theta), and
    int_0^R K0(r/alpha) r dr = alpha^2 - alpha R K1(R/alpha)."""
    x, wq = np.polynomial.legendre.leggauss(n_gauss)
    th = (x + 1.0) * (math.pi / 8.0)
    wt = wq * (math.pi / 8.0)
    R = 0.5 * h / np.cos(th)
    inner = alpha * alpha - alpha * R * k1(R / alpha)
    return float(8.0 * np.sum(wt * inner) / (2.0 * math.pi))


# ---------------------------------------------------------------------------
# Backward-Euler heat step (Sec. 2 and Sec. 3)
# ---------------------------------------------------------------------------
class DenseBIE:
    """LU factorisation of A (fixed across steps for a fixed geometry and alpha)."""

    def __init__(self, bxy, bnormal, w, kappa, alpha):
        import scipy.linalg as sla
        self.A = dl_matrix(bxy, bnormal, w, kappa, alpha)
        self.lu = sla.lu_factor(self.A)
        self.alpha = alpha

    def solve(self, g):
        import scipy.linalg as sla
        return sla.lu_solve(self.lu, -2.0 * self.alpha ** 2 * _f64(g))


def heat_step(bnd_xy, bnd_normal, bnd_w, bnd_kappa, vol_xy, vol_w, B, f_next, dt,
              grid_h=None, bie=None, tgt_mask=None, offsets=None, near=True):
    """One step with alpha^2 = dt (backward Euler; pass 2 dt / 3 for the
    extrapolated Gear scheme), B already extended to all volume points.
    Returns (u_next at the targets, sigma, U^p on the nodes).

      q      = W * B
      U^p    = (V[q] + B * C_self) / alpha^2   (C_self only for grid points:
               the constant-exact lattice weight, grid.self_weight)
      g      = f^{N+1} - U^p on the nodes (for grid points, the cells within
               two sides of a node enter with their integral,
               grid.node_cell_correction)
      sigma  = A^{-1} (-2 alpha^2 g)
      u^{N+1} = U^p + DL[w sigma] / alpha^2, and at targets within a few node
               spacings of a curve U^h from grid.near_values (when the curve
               offsets are given and near is true)
    """
    from . import grid as _grid
    alpha = math.sqrt(dt)
    vol_xy = _f64(vol_xy); B = _f64(B)
    q = _f64(vol_w) * B
    tx = vol_xy if tgt_mask is None else vol_xy[tgt_mask]
    if tgt_mask is None:
        Vv = volume_sum(vol_xy, q, alpha)
        Bt = B
    else:
        # targets are a subset of the sources: skip self pair by exact distance
        Vv = volume_sum(vol_xy, q, alpha, tgt_xy=tx)
        Bt = B[tgt_mask]
    if grid_h is not None:
        Vv = Vv + Bt * _grid.self_weight(grid_h, alpha)
    Vb = volume_sum(vol_xy, q, alpha, tgt_xy=bnd_xy)
    if grid_h is not None:
        # cells next to a node enter with their integral (grid.node_cell_correction)
        Vb = Vb + _grid.node_cell_correction(bnd_xy, vol_xy, vol_w, B, alpha)
    up_b = Vb / alpha ** 2
    g = _f64(f_next) - up_b
    if bie is None:
        bie = DenseBIE(bnd_xy, bnd_normal, bnd_w, bnd_kappa, alpha)
    sigma = bie.solve(g)
    uh = dl_sum(bnd_xy, bnd_normal, _f64(bnd_w) * sigma, alpha, tx) / alpha ** 2
    if near and offsets is not None:
        off = np.asarray(offsets, dtype=np.int64)
        ncj = np.repeat(np.diff(off), np.diff(off))
        speed = _f64(bnd_w) * ncj / (2.0 * math.pi)
        nt = _grid.near_targets(bnd_xy, bnd_normal, speed, off, tx)
        uh[nt[0]] = _grid.near_values(bnd_xy, bnd_normal, off, sigma, g, alpha, tx, nt)
    return Vv / alpha ** 2 + uh, sigma, up_b
