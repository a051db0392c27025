"""Thin ctypes binding of libyk (include/yk.h), same names as the C ABI.

Only argument marshalling happens here: every array is a contiguous FP64 (or
int32) torch tensor on the GPU, passed to the library by its device address.
Every computation runs in the library's HIP kernels.  If the built library is
missing, loading fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libyk.so")

YK_OK = 0
YK_ERR_ARG = -1
YK_ERR_HIP = -2
YK_ERR_NOMEM = -3
YK_ERR_NOCONV = -4
YK_ERR_NONFINITE = -5
YK_ERR_INTERNAL = -6

YK_PREC_FP64 = 0
YK_PREC_MIXED = 1
YK_PREC_FP32 = 2

YK_TREE_UNIFORM = 0
YK_TREE_ADAPTIVE = 1
YK_TREE_AUTO = 2

HEAT_GRID_SELF_CELL = 1
HEAT_ZERO_GUESS = 2
HEAT_NO_NEAR = 4
HEAT_BOX_CODE = 8

SCHEME_EULER = 0
SCHEME_GEAR = 1
REACTION_NONE = 0
REACTION_ALLEN_CAHN = 1

EXPORTS = (
    "yk_default_options", "yk_create", "yk_destroy", "yk_set_stream", "yk_set_options",
    "yk_last_error", "yk_invalidate_geometry", "yk_volume_potential", "yk_double_layer_apply",
    "yk_gmres_density", "yk_heat_step", "yk_rhs_backward_euler", "yk_fmm_potential",
    "yk_plan_info_get", "yk_timing_enable", "yk_timing_read",
    "yk_ws_default_options", "yk_ws_create", "yk_ws_destroy", "yk_ws_observe", "yk_ws_train",
    "yk_ws_predict", "yk_set_warm_start", "yk_ws_num_params", "yk_ws_get_params",
    "yk_ws_set_params", "yk_ws_loss_grad", "yk_ws_forward", "yk_ws_adam_step",
    "yk_gmres_density_noalloc", "yk_plan_tree_export", "yk_rhs_imex", "yk_heat_step_grid",
    "yk_near_info", "yk_plan_adaptive_export", "yk_box_potential", "yk_box_potential_adaptive",
    "yk_box_refine", "yk_heat_step_leaves",
)

STAGES = ("gather", "p2m", "m2m", "m2l", "l2l", "leaf", "scatter", "direct", "l2p", "near_build")


class yk_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("fmm_tol", ctypes.c_double), ("p", ctypes.c_int),
                ("leaf_size", ctypes.c_int), ("direct", ctypes.c_int), ("gmres_m", ctypes.c_int),
                ("debug_flags", ctypes.c_int), ("near_cache_mb", ctypes.c_int), ("tree", ctypes.c_int)]


class yk_boundary(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("offset", ctypes.POINTER(ctypes.c_int64)),
                ("xy", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("speed", ctypes.c_void_p), ("curvature", ctypes.c_void_p)]


class yk_grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("h", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64)]


class yk_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("guess_used", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("res0", ctypes.c_double), ("res_final", ctypes.c_double),
                ("ms", ctypes.c_double * 8)]

    def as_dict(self):
        return dict(iters=self.iters, outer_iters=self.outer_iters, guess_used=self.guess_used,
                    matvecs=self.matvecs, res0=self.res0, res_final=self.res_final,
                    ms=list(self.ms))


class yk_plan_info(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_int32), ("leaf_level", ctypes.c_int32), ("lmin", ctypes.c_int32),
                ("p", ctypes.c_int32), ("P", ctypes.c_int32), ("Pp", ctypes.c_int32),
                ("n_points", ctypes.c_int64), ("n_boxes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("pairs_charge", ctypes.c_int64), ("pairs_dipole", ctypes.c_int64),
                ("m2l_translations", ctypes.c_int64), ("m2l_slots", ctypes.c_int64),
                ("p2m_points", ctypes.c_int64), ("l2p_points", ctypes.c_int64),
                ("near_terms", ctypes.c_int32), ("nser", ctypes.c_int32),
                ("build_ms", ctypes.c_double), ("m2l_sparse", ctypes.c_int32),
                ("near_sym", ctypes.c_int32), ("near_charge_values", ctypes.c_int64),
                ("near_incoming", ctypes.c_int64), ("p_initial", ctypes.c_int32),
                ("order_check_err", ctypes.c_double), ("m2m_children", ctypes.c_int64),
                ("l2l_children", ctypes.c_int64), ("n_ulist", ctypes.c_int64),
                ("tables_ms", ctypes.c_double), ("order_check_ms", ctypes.c_double),
                ("tree", ctypes.c_int32), ("max_u", ctypes.c_int32), ("n_wlist", ctypes.c_int64),
                ("n_xboxes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class yk_ws_options(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int), ("batch", ctypes.c_int), ("steps", ctypes.c_int),
                ("lr", ctypes.c_double), ("max_obs", ctypes.c_int), ("seed", ctypes.c_uint64)]


class YkError(RuntimeError):
    def __init__(self, status, msg, stats=None):
        super().__init__(f"libyk status {status}: {msg}")
        self.status = status
        self.stats = stats


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libyk.so (built in-tree by paper_1007_5335_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libyk.so not found at {path}; build it with "
                          f"`python -m paper_1007_5335_amd.build` (no fallback exists)")
    # torch brings its own HIP runtime; loaded first, it is the one libyk
    # binds to (loaded the other way round, the library's calls find no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, dbl, ip = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    i32 = ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "yk_default_options": (None, [P(yk_options)]),
        "yk_create": (ip, [P(yk_options), P(vp)]),
        "yk_destroy": (ip, [vp]),
        "yk_set_stream": (ip, [vp, vp]),
        "yk_set_options": (ip, [vp, P(yk_options)]),
        "yk_last_error": (ctypes.c_char_p, [vp]),
        "yk_invalidate_geometry": (ip, [vp]),
        "yk_volume_potential": (ip, [vp, i64, vp, vp, i64, vp, dbl, vp]),
        "yk_double_layer_apply": (ip, [vp, P(yk_boundary), vp, i64, vp, dbl, vp]),
        "yk_gmres_density": (ip, [vp, P(yk_boundary), dbl, vp, vp, dbl, ip, vp, P(yk_stats)]),
        "yk_heat_step": (ip, [vp, P(yk_boundary), i64, vp, vp, vp, ip, vp, dbl, dbl, vp, vp,
                              P(yk_stats)]),
        "yk_rhs_backward_euler": (ip, [vp, i64, vp, vp, vp, ip, P(dbl), dbl, vp]),
        "yk_fmm_potential": (ip, [vp, i64, vp, vp, P(yk_boundary), vp, dbl, vp, vp]),
        "yk_plan_info_get": (ip, [vp, ip, P(yk_plan_info)]),
        "yk_timing_enable": (ip, [vp, ip]),
        "yk_timing_read": (ip, [vp, P(dbl), P(i64), ip]),
        "yk_ws_default_options": (None, [P(yk_ws_options)]),
        "yk_ws_create": (ip, [vp, P(yk_boundary), P(yk_ws_options), P(vp)]),
        "yk_ws_destroy": (ip, [vp]),
        "yk_ws_observe": (ip, [vp, vp, vp]),
        "yk_ws_train": (ip, [vp, P(dbl)]),
        "yk_ws_predict": (ip, [vp, vp, vp]),
        "yk_set_warm_start": (ip, [vp, vp]),
        "yk_ws_num_params": (i64, [vp, P(ip), P(ip)]),
        "yk_ws_get_params": (ip, [vp, vp]),
        "yk_ws_set_params": (ip, [vp, vp]),
        "yk_ws_loss_grad": (ip, [vp, i64, vp, vp, vp, P(dbl)]),
        "yk_ws_forward": (ip, [vp, i64, vp, vp]),
        "yk_ws_adam_step": (ip, [vp, vp]),
        "yk_gmres_density_noalloc": (ip, [vp, P(yk_boundary), dbl, vp, vp, dbl, ip, vp, P(yk_stats)]),
        "yk_plan_tree_export": (ip, [vp, ip, P(dbl), P(i64), vp, vp, vp, vp, vp, vp, vp, vp]),
        "yk_plan_adaptive_export": (ip, [vp, ip, vp, vp, vp, vp, vp, vp, vp]),
        "yk_box_potential": (ip, [vp, P(yk_grid), vp, dbl, vp, i64, vp, vp]),
        "yk_box_potential_adaptive": (ip, [vp, P(dbl), i64, P(i32), P(i32), P(i32), vp, dbl, vp]),
        "yk_box_refine": (ip, [vp, i64, vp, vp, dbl, vp, vp]),
        "yk_heat_step_leaves": (ip, [vp, P(yk_boundary), P(dbl), i64, P(i32), P(i32), P(i32), vp, ip, vp, dbl,
                                     dbl, vp, vp, P(yk_stats)]),
        "yk_rhs_imex": (ip, [vp, ip, ip, i64, vp, vp, vp, vp, vp, ip, P(dbl), dbl, vp]),
        "yk_heat_step_grid": (ip, [vp, P(yk_boundary), P(yk_grid), vp, ip, vp, dbl, dbl, vp, vp, P(yk_stats)]),
        "yk_near_info": (ip, [vp, P(i64), P(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# argument helpers
# ---------------------------------------------------------------------------
def _dev(t, name, dtype="float64", shape_last=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    want = {"float64": torch.float64, "float32": torch.float32, "int32": torch.int32}[dtype]
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape [n, {shape_last}]")
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, status, stats=None):
    if status != YK_OK:
        msg = load_library().yk_last_error(ctx)
        raise YkError(status, msg.decode() if msg else "", stats)


class Boundary:
    """Device-resident boundary (curve 0 outer, holes after) and its C view."""

    def __init__(self, xy, normal, speed, curvature, offset):
        import torch
        dev = "cuda"
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
        self.xy = f(xy) if not isinstance(xy, torch.Tensor) else xy
        self.normal = f(normal) if not isinstance(normal, torch.Tensor) else normal
        self.speed = f(speed) if not isinstance(speed, torch.Tensor) else speed
        self.curvature = f(curvature) if not isinstance(curvature, torch.Tensor) else curvature
        self.offset = np.ascontiguousarray(offset, dtype=np.int64)
        self.n = int(self.offset[-1])
        self.n_curves = len(self.offset) - 1
        self._c = yk_boundary(self.n_curves,
                              self.offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              _dev(self.xy, "xy", shape_last=2), _dev(self.normal, "normal", shape_last=2),
                              _dev(self.speed, "speed"), _dev(self.curvature, "curvature"))

    @classmethod
    def from_workload(cls, bnd):
        return cls(bnd.xy, bnd.normal, bnd.speed, bnd.curvature, bnd.offset)

    @property
    def struct(self):
        return self._c


# ---------------------------------------------------------------------------
# C ABI, same names
# ---------------------------------------------------------------------------
def yk_default_options() -> yk_options:
    o = yk_options()
    load_library().yk_default_options(ctypes.byref(o))
    return o


def yk_create(opt: yk_options | None = None, **kw):
    if opt is None:
        opt = yk_default_options()
    for k, v in kw.items():
        setattr(opt, k, v)
    h = ctypes.c_void_p()
    lib = load_library()
    st = lib.yk_create(ctypes.byref(opt), ctypes.byref(h))
    if st != YK_OK:
        raise YkError(st, "yk_create failed: " + lib.yk_last_error(None).decode(errors="replace"))
    import torch
    yk_set_stream(h, torch.cuda.current_stream())
    return h


def yk_destroy(ctx):
    load_library().yk_destroy(ctx)


def yk_set_stream(ctx, stream=None):
    ptr = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(ctx, load_library().yk_set_stream(ctx, ptr))


def yk_set_options(ctx, opt: yk_options):
    _check(ctx, load_library().yk_set_options(ctx, ctypes.byref(opt)))


def yk_last_error(ctx) -> str:
    m = load_library().yk_last_error(ctx)
    return m.decode() if m else ""


def yk_invalidate_geometry(ctx):
    _check(ctx, load_library().yk_invalidate_geometry(ctx))


def yk_volume_potential(ctx, src_xy, q, tgt_xy, alpha, out):
    n_tgt = 0 if tgt_xy is None else tgt_xy.shape[0]
    _check(ctx, load_library().yk_volume_potential(
        ctx, src_xy.shape[0], _dev(src_xy, "src_xy", shape_last=2), _dev(q, "q"), n_tgt,
        _dev(tgt_xy, "tgt_xy", shape_last=2), float(alpha), _dev(out, "out")))
    return out


def yk_double_layer_apply(ctx, bnd: Boundary, sigma, tgt_xy, alpha, out):
    n_tgt = 0 if tgt_xy is None else tgt_xy.shape[0]
    _check(ctx, load_library().yk_double_layer_apply(
        ctx, ctypes.byref(bnd.struct), _dev(sigma, "sigma"), n_tgt,
        _dev(tgt_xy, "tgt_xy", shape_last=2), float(alpha), _dev(out, "out")))
    return out


def yk_gmres_density(ctx, bnd: Boundary, alpha, g, sigma0, tol, max_iter, sigma,
                     raise_on_noconv=True):
    st = yk_stats()
    s = load_library().yk_gmres_density(ctx, ctypes.byref(bnd.struct), float(alpha), _dev(g, "g"),
                                        _dev(sigma0, "sigma0"), float(tol), int(max_iter),
                                        _dev(sigma, "sigma"), ctypes.byref(st))
    if s == YK_ERR_NOCONV and not raise_on_noconv:
        return st
    _check(ctx, s, st)
    return st


def yk_gmres_density_noalloc(ctx, bnd: Boundary, alpha, g, sigma0, tol, max_iter, sigma,
                             raise_on_noconv=True):
    st = yk_stats()
    s = load_library().yk_gmres_density_noalloc(ctx, ctypes.byref(bnd.struct), float(alpha), _dev(g, "g"),
                                                _dev(sigma0, "sigma0"), float(tol), int(max_iter),
                                                _dev(sigma, "sigma"), ctypes.byref(st))
    if s == YK_ERR_NOCONV and not raise_on_noconv:
        return st
    _check(ctx, s, st)
    return st


def yk_heat_step(ctx, bnd: Boundary, vol_xy, vol_w, B, flags, f_next, dt, tol, sigma_io, u_next,
                 raise_on_noconv=True):
    st = yk_stats()
    s = load_library().yk_heat_step(ctx, ctypes.byref(bnd.struct), vol_xy.shape[0],
                                    _dev(vol_xy, "vol_xy", shape_last=2), _dev(vol_w, "vol_w"),
                                    _dev(B, "B"), int(flags), _dev(f_next, "f_next"), float(dt),
                                    float(tol), _dev(sigma_io, "sigma_io"), _dev(u_next, "u_next"),
                                    ctypes.byref(st))
    if s == YK_ERR_NOCONV and not raise_on_noconv:
        return st
    _check(ctx, s, st)
    return st


def yk_rhs_backward_euler(ctx, u, F, region, consts, dt, B):
    c = np.ascontiguousarray(consts, dtype=np.float64)
    _check(ctx, load_library().yk_rhs_backward_euler(
        ctx, u.shape[0], _dev(u, "u"), _dev(F, "F"), _dev(region, "region", dtype="int32"),
        int(c.size), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt), _dev(B, "B")))
    return B


def alpha2_of(scheme, dt, nu=1.0):
    """alpha^2 of the scheme for u_t - nu Lap u = F: nu dt (Euler), 2 nu dt / 3 (Gear)."""
    return nu * dt if scheme == SCHEME_EULER else 2.0 * nu * dt / 3.0


def yk_rhs_imex(ctx, scheme, reaction, u, u_prev, F, F_prev, region, consts, dt, B):
    c = np.ascontiguousarray(consts, dtype=np.float64)
    _check(ctx, load_library().yk_rhs_imex(
        ctx, int(scheme), int(reaction), u.shape[0], _dev(u, "u"), _dev(u_prev, "u_prev"), _dev(F, "F"),
        _dev(F_prev, "F_prev"), _dev(region, "region", dtype="int32"), int(c.size),
        c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt), _dev(B, "B")))
    return B


def make_grid(x0, y0, h, nx, ny) -> yk_grid:
    return yk_grid(float(x0), float(y0), float(h), int(nx), int(ny))


def yk_heat_step_grid(ctx, bnd: Boundary, grid: yk_grid, B, flags, f_next, alpha2, tol, sigma_io, u_next,
                      raise_on_noconv=True):
    st = yk_stats()
    if B.shape[0] != grid.nx * grid.ny or u_next.shape[0] != grid.nx * grid.ny:
        raise ValueError("B and u_next need one value per grid cell")
    s = load_library().yk_heat_step_grid(ctx, ctypes.byref(bnd.struct), ctypes.byref(grid), _dev(B, "B"),
                                         int(flags), _dev(f_next, "f_next"), float(alpha2), float(tol),
                                         _dev(sigma_io, "sigma_io"), _dev(u_next, "u_next"), ctypes.byref(st))
    if s == YK_ERR_NOCONV and not raise_on_noconv:
        return st
    _check(ctx, s, st)
    return st


def yk_box_potential(ctx, grid: yk_grid, B, alpha, V, pts=None, pts_vals=None):
    if B.shape[0] != grid.nx * grid.ny or V.shape[0] != grid.nx * grid.ny:
        raise ValueError("B and V need one value per grid cell")
    n = 0 if pts is None else int(pts.shape[0])
    _check(ctx, load_library().yk_box_potential(ctx, ctypes.byref(grid), _dev(B, "B"), float(alpha), _dev(V, "V"),
                                                n, _dev(pts, "pts") if n else None,
                                                _dev(pts_vals, "pts_vals") if n else None))


def yk_box_potential_adaptive(ctx, root, level, ix, iy, vals, alpha, V):
    import numpy as np
    lv = np.ascontiguousarray(level, dtype=np.int32)
    jx = np.ascontiguousarray(ix, dtype=np.int32)
    jy = np.ascontiguousarray(iy, dtype=np.int32)
    n = lv.shape[0]
    if vals.shape[0] != 16 * n or V.shape[0] != 16 * n:
        raise ValueError("vals and V need 16 values per leaf")
    rt = (ctypes.c_double * 3)(*[float(v) for v in root])
    i32p = ctypes.POINTER(ctypes.c_int32)
    _check(ctx, load_library().yk_box_potential_adaptive(ctx, rt, n, lv.ctypes.data_as(i32p),
                                                         jx.ctypes.data_as(i32p), jy.ctypes.data_as(i32p),
                                                         _dev(vals, "vals"), float(alpha), _dev(V, "V")))


def yk_heat_step_leaves(ctx, bnd: Boundary, root, level, ix, iy, B, flags, f_next, alpha2, tol, sigma_io, u_next):
    import numpy as np
    lv = np.ascontiguousarray(level, dtype=np.int32)
    jx = np.ascontiguousarray(ix, dtype=np.int32)
    jy = np.ascontiguousarray(iy, dtype=np.int32)
    n = lv.shape[0]
    if B.shape[0] != 16 * n or u_next.shape[0] != 16 * n:
        raise ValueError("B and u_next need 16 values per leaf")
    st = yk_stats()
    rt = (ctypes.c_double * 3)(*[float(v) for v in root])
    i32p = ctypes.POINTER(ctypes.c_int32)
    s = load_library().yk_heat_step_leaves(ctx, ctypes.byref(bnd.struct), rt, n, lv.ctypes.data_as(i32p),
                                           jx.ctypes.data_as(i32p), jy.ctypes.data_as(i32p), _dev(B, "B"),
                                           int(flags), _dev(f_next, "f_next"), float(alpha2), float(tol),
                                           _dev(sigma_io, "sigma_io"), _dev(u_next, "u_next"), ctypes.byref(st))
    _check(ctx, s, st)
    return st


def yk_box_refine(ctx, v16, v64, tol, flags, err=None):
    n = int(v16.shape[0]) // 16
    _check(ctx, load_library().yk_box_refine(ctx, n, _dev(v16, "v16"), _dev(v64, "v64"), float(tol),
                                             _dev(flags, "flags", "int32"), _dev(err, "err")))


def yk_near_info(ctx):
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(ctx, load_library().yk_near_info(ctx, ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def yk_fmm_potential(ctx, vol_xy, q, bnd: Boundary, d, alpha, out_vol, out_bnd):
    _check(ctx, load_library().yk_fmm_potential(
        ctx, vol_xy.shape[0], _dev(vol_xy, "vol_xy", shape_last=2), _dev(q, "q"),
        ctypes.byref(bnd.struct), _dev(d, "d"), float(alpha), _dev(out_vol, "out_vol"),
        _dev(out_bnd, "out_bnd")))
    return out_vol, out_bnd


def yk_plan_info_get(ctx, slot=0) -> yk_plan_info:
    info = yk_plan_info()
    _check(ctx, load_library().yk_plan_info_get(ctx, int(slot), ctypes.byref(info)))
    return info


def yk_timing_enable(ctx, enable=True):
    _check(ctx, load_library().yk_timing_enable(ctx, 1 if enable else 0))


def yk_timing_read(ctx, reset=False):
    ms = (ctypes.c_double * len(STAGES))()
    calls = (ctypes.c_int64 * len(STAGES))()
    _check(ctx, load_library().yk_timing_read(ctx, ms, calls, 1 if reset else 0))
    return {name: (ms[i], calls[i]) for i, name in enumerate(STAGES)}


# ---------------------------------------------------------------------------
# learned warm start
# ---------------------------------------------------------------------------
class WarmStartHandle:
    """A yk_ws together with the context that owns it (destroy it first)."""

    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h


def yk_ws_default_options() -> yk_ws_options:
    o = yk_ws_options()
    load_library().yk_ws_default_options(ctypes.byref(o))
    return o


def yk_ws_create(ctx, bnd: Boundary, opt: yk_ws_options | None = None, **kw) -> WarmStartHandle:
    if opt is None:
        opt = yk_ws_default_options()
    for k, v in kw.items():
        setattr(opt, k, v)
    h = ctypes.c_void_p()
    _check(ctx, load_library().yk_ws_create(ctx, ctypes.byref(bnd.struct), ctypes.byref(opt), ctypes.byref(h)))
    return WarmStartHandle(ctx, h)


def yk_ws_destroy(ws: WarmStartHandle):
    load_library().yk_ws_destroy(ws.h)


def yk_ws_observe(ws: WarmStartHandle, g, sigma):
    _check(ws.ctx, load_library().yk_ws_observe(ws.h, _dev(g, "g"), _dev(sigma, "sigma")))


def yk_ws_train(ws: WarmStartHandle) -> float:
    loss = ctypes.c_double()
    _check(ws.ctx, load_library().yk_ws_train(ws.h, ctypes.byref(loss)))
    return loss.value


def yk_ws_predict(ws: WarmStartHandle, g_next, sigma_out):
    _check(ws.ctx, load_library().yk_ws_predict(ws.h, _dev(g_next, "g_next"), _dev(sigma_out, "sigma_out")))
    return sigma_out


def yk_set_warm_start(ctx, ws: WarmStartHandle | None):
    _check(ctx, load_library().yk_set_warm_start(ctx, ws.h if ws is not None else None))


def yk_ws_num_params(ws: WarmStartHandle):
    H, Fp = ctypes.c_int(), ctypes.c_int()
    n = load_library().yk_ws_num_params(ws.h, ctypes.byref(H), ctypes.byref(Fp))
    return int(n), H.value, Fp.value


def yk_ws_get_params(ws: WarmStartHandle, out):
    _check(ws.ctx, load_library().yk_ws_get_params(ws.h, _dev(out, "params", dtype="float32")))
    return out


def yk_ws_set_params(ws: WarmStartHandle, params):
    _check(ws.ctx, load_library().yk_ws_set_params(ws.h, _dev(params, "params", dtype="float32")))


def yk_ws_loss_grad(ws: WarmStartHandle, X, t, grad) -> float:
    loss = ctypes.c_double()
    _check(ws.ctx, load_library().yk_ws_loss_grad(ws.h, X.shape[0], _dev(X, "X", dtype="float32"),
                                                  _dev(t, "t", dtype="float32"),
                                                  _dev(grad, "grad", dtype="float32"), ctypes.byref(loss)))
    return loss.value


def yk_ws_forward(ws: WarmStartHandle, X, y):
    _check(ws.ctx, load_library().yk_ws_forward(ws.h, X.shape[0], _dev(X, "X", dtype="float32"),
                                                _dev(y, "y", dtype="float32")))
    return y


def yk_ws_adam_step(ws: WarmStartHandle, grad):
    _check(ws.ctx, load_library().yk_ws_adam_step(ws.h, _dev(grad, "grad", dtype="float32")))


def yk_plan_tree_export(ctx, slot=0):
    """The cached tree of `slot` as numpy arrays (keys, perm, box codes,
    parents, leaf ranges, U lists, V lists) plus the bounding square."""
    import numpy as np
    import torch
    info = yk_plan_info_get(ctx, slot)
    if not info.valid:
        raise YkError(YK_ERR_ARG, "no tree cached in this slot")
    N, nb, nl, L = info.n_points, info.n_boxes, info.n_leaves, info.leaf_level
    dev = lambda n, dt: torch.empty(max(int(n), 1), dtype=dt, device="cuda")
    keys, perm = dev(N, torch.int32), dev(N, torch.int32)
    code, parent = dev(nb, torch.int32), dev(nb, torch.int32)
    lr, uoff, ul = dev(nl * 6, torch.int32), dev(nl + 1, torch.int32), dev(info.n_ulist, torch.int32)
    vl = dev(nb * 27, torch.int32)
    sq = (ctypes.c_double * 3)()
    lb = (ctypes.c_int64 * (L + 2))()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    _check(ctx, load_library().yk_plan_tree_export(ctx, int(slot), sq, lb, ptr(keys), ptr(perm), ptr(code),
                                                   ptr(parent), ptr(lr), ptr(uoff), ptr(ul), ptr(vl)))
    h = lambda t, n: t.cpu().numpy()[:int(n)]
    return dict(square=(sq[0], sq[1], sq[2]), level_begin=np.array(lb[:], dtype=np.int64), leaf_level=L,
                lmin=info.lmin, keys=h(keys, N).view(np.uint32), perm=h(perm, N), box_code=h(code, nb).view(np.uint32),
                parent=h(parent, nb), leaf_range=h(lr, nl * 6).reshape(nl, 6), ulist_off=h(uoff, nl + 1),
                ulist=h(ul, info.n_ulist), vlist=h(vl, nb * 27).reshape(nb, 27))


def yk_plan_adaptive_export(ctx, slot=0):
    """The adaptive parts of the cached tree of `slot` as numpy arrays: each
    leaf's box, each box's level, the W lists (CSR over leaves) and the X
    lists (CSR over the boxes that have one)."""
    import torch
    info = yk_plan_info_get(ctx, slot)
    if not info.valid:
        raise YkError(YK_ERR_ARG, "no tree cached in this slot")
    nb, nl, nw, nx = info.n_boxes, info.n_leaves, info.n_wlist, info.n_xboxes
    dev = lambda n: torch.empty(max(int(n), 1), dtype=torch.int32, device="cuda")
    lb, bl, wo, wl, xb, xo, xl = dev(nl), dev(nb), dev(nl + 1), dev(nw), dev(nx), dev(nx + 1), dev(nw)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    _check(ctx, load_library().yk_plan_adaptive_export(ctx, int(slot), ptr(lb), ptr(bl), ptr(wo), ptr(wl),
                                                       ptr(xb), ptr(xo), ptr(xl)))
    h = lambda t, n: t.cpu().numpy()[:int(n)]
    return dict(leaf_box=h(lb, nl), box_level=h(bl, nb), wlist_off=h(wo, nl + 1), wlist=h(wl, nw),
                xbox=h(xb, nx), xlist_off=h(xo, nx + 1), xlist=h(xl, nw))
