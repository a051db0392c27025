"""The time schemes, the grid step and the near-boundary evaluation on the GPU:
element by element against the oracle on small cases, against closed forms
at larger ones, and the paper's Example 1 temporal study (Sec. 4, Table 1)."""
import math
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import dev, elem_err, host

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def yk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1007_5335_amd.yk as yk
    yk.load_library()
    return yk


CTX = [None]


@pytest.fixture(scope="module", autouse=True)
def _ctx(yk):
    CTX[0] = yk.yk_create()
    yield
    yk.yk_destroy(CTX[0])


def table1():
    rows = np.loadtxt(os.path.join(HERE, "golden", "example1_table1.txt"))
    return rows[:, 0], rows[:, 1], rows[:, 2]


@pytest.mark.parametrize("scheme,reaction", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_rhs_imex_matches_oracle(yk, scheme, reaction):
    from oracle import grid as G
    rng = np.random.default_rng(11 + scheme + 2 * reaction)
    n = 5003
    u, up = rng.standard_normal(n), rng.standard_normal(n)
    F, Fp = rng.standard_normal(n), rng.standard_normal(n)
    reg = rng.integers(-1, 4, size=n).astype(np.int32)
    c = np.array([0.25, -1.0, 0.5])
    dt = 0.013
    import torch
    B = torch.empty(n, dtype=torch.float64, device="cuda")
    yk.yk_rhs_imex(CTX[0], scheme, reaction, dev(u), dev(up), dev(F), dev(Fp), dev(reg), c, dt, B)
    ref = G.rhs_imex(scheme, reaction, u, up, F, Fp, reg, c, dt)
    assert np.max(np.abs(host(B) - ref)) <= 4e-16 * np.max(np.abs(ref))


def _grid_case(n0=256, n1=128):
    b = W.make_boundary([W.circle((0.0, 0.0), 0.4, n0), W.circle((0.0, 0.0), 0.1, n1, ccw=False)])
    grid, pts = W.grid_box(-0.5, 0.5, 48)
    uf = lambda p: np.sin(3 * p[:, 0]) * np.sin(2 * p[:, 1]) + 1.0
    return b, grid, pts, uf


@pytest.mark.parametrize("direct,nodes", [(1, (256, 128)), (0, (256, 128)), (0, (250, 130))])
def test_grid_step_matches_oracle(yk, direct, nodes):
    """One grid step (U^p on the grid, bicubic U^p on the nodes, the density,
    U^h with the near-boundary rule) element by element against the oracle;
    power-of-two curves take the LDS FFTs, the others the direct sums."""
    import torch
    from oracle import grid as G
    b, grid, pts, uf = _grid_case(*nodes)
    a2 = 2.5e-3
    B = (1 + 13 * a2) * uf(pts) - 13 * a2
    f = uf(b.xy)
    ref_u, ref_s, _, _, nt = G.heat_step_grid(b.xy, b.normal, b.weights(), b.curvature, b.speed, b.offset,
                                              grid, B, f, a2)
    ctx = yk.yk_create(direct=direct, leaf_size=16)
    try:
        bd = yk.Boundary.from_workload(b)
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        u = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
        print(f"grid step direct={direct} {pts.shape[0]} cells, {b.n} nodes", flush=True)
        st = yk.yk_heat_step_grid(ctx, bd, yk.make_grid(*grid), dev(B), yk.HEAT_ZERO_GUESS, dev(f), a2, 1e-13,
                                  sig, u)
        n_near, setup_ms = yk.yk_near_info(ctx)
    finally:
        yk.yk_destroy(ctx)
    print(f"  iters {st.iters}, near {n_near} (oracle {nt[0].size}), setup {setup_ms:.1f} ms", flush=True)
    assert n_near == nt[0].size
    assert elem_err(host(sig), ref_s) <= 1e-10
    assert elem_err(host(u), ref_u) <= 1e-10


def test_grid_step_closed_form(yk):
    """u = sin(3x) sin(2y) + 1 is reproduced by one step at every cell inside
    the annulus, the near-boundary ones included; without the near-boundary
    rule the cells next to the curves are far off."""
    import torch
    b = W.make_boundary([W.circle((0.0, 0.0), 0.4, 1024), W.circle((0.0, 0.0), 0.1, 512, ccw=False)])
    grid, pts = W.grid_box(-0.5, 0.5, 512)
    uf = lambda p: np.sin(3 * p[:, 0]) * np.sin(2 * p[:, 1]) + 1.0
    a2 = 1e-3
    B = (1 + 13 * a2) * uf(pts) - 13 * a2
    inside = b.region(pts) < 0
    ctx = yk.yk_create()
    errs = {}
    try:
        bd = yk.Boundary.from_workload(b)
        for flags in (yk.HEAT_ZERO_GUESS, yk.HEAT_ZERO_GUESS | yk.HEAT_NO_NEAR):
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            u = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
            yk.yk_heat_step_grid(ctx, bd, yk.make_grid(*grid), dev(B), flags, dev(uf(b.xy)), a2, 1e-12, sig, u)
            errs[flags] = np.max(np.abs(host(u) - uf(pts))[inside])
        n_near, ms = yk.yk_near_info(ctx)
    finally:
        yk.yk_destroy(ctx)
    print(f"closed form: max error {errs}, near {n_near}, setup {ms:.1f} ms", flush=True)
    assert errs[yk.HEAT_ZERO_GUESS] < 1e-6
    assert errs[yk.HEAT_ZERO_GUESS | yk.HEAT_NO_NEAR] > 100 * errs[yk.HEAT_ZERO_GUESS]


def run_example1(yk, scheme, dt, m=2048, n_outer=1024, n_inner=512, T=1e-2, tol=1e-12, flags=0):
    """Max error over the cells inside the annulus at t = T (Sec. 4, Example 1);
    Gear starts from the exact values at t = 0 and dt."""
    import torch
    e = W.example1(m=m, n_outer=n_outer, n_inner=n_inner)
    b, pts = e["bnd"], e["pts"]
    nsteps = int(round(T / dt))
    a2 = yk.alpha2_of(scheme, dt)
    ctx = yk.yk_create()
    try:
        bd = yk.Boundary.from_workload(b)
        grid = yk.make_grid(*e["grid"])
        F, reg, fb = dev(e["F"]), dev(e["region"]), dev(e["f_bnd"])
        u = dev(e["exact"](pts, 0.0))
        up = None
        k0 = 0
        if scheme == yk.SCHEME_GEAR:
            up, u = u, dev(e["exact"](pts, dt))
            k0 = 1
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        B = torch.empty_like(u)
        for _ in range(k0, nsteps):
            yk.yk_rhs_imex(ctx, scheme, yk.REACTION_NONE, u, up, F, F, reg, e["consts"], dt, B)
            un = torch.empty_like(u)
            yk.yk_heat_step_grid(ctx, bd, grid, B, flags, fb, a2, tol, sig, un)
            up, u = u, un
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    ins = e["region"] < 0
    return float(np.max(np.abs(host(u) - e["exact"](pts, T))[ins]))


@pytest.mark.parametrize("scheme", [0, 1])
def test_example1_temporal_order(yk, scheme):
    """Sec. 4, Example 1: errors at t = 1e-2 for dt = 2e-3 .. 2.5e-4 fall by 2
    per halving for Euler and by 4 for extrapolated Gear, and agree with
    Table 1 (tests/golden/example1_table1.txt) to within 10%; 2048^2 cells,
    1024 + 512 nodes."""
    dts, e_euler, e_gear = table1()
    want = e_euler if scheme == 0 else e_gear
    errs = []
    for dt in dts:
        print(f"example 1 scheme {scheme} dt {dt:g}", flush=True)
        errs.append(run_example1(yk, scheme, dt))
        print(f"  error {errs[-1]:.4e} (Table 1: {want[len(errs) - 1]:.3g})", flush=True)
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    target = 2.0 if scheme == 0 else 4.0
    assert np.all(np.abs(ratios - target) < 0.2 * target), ratios
    assert np.all(np.abs(errs / want - 1.0) < 0.1), errs / want


def test_example1_box_code(yk):
    """Example 1 with the box code (cubic leaf fits, exact near integrals):
    extrapolated Gear at dt = 5e-4 and 2.5e-4 agrees with Table 1 to within
    10% and keeps the factor 4 per halving, as the lattice rule does."""
    dts, _, e_gear = table1()
    errs = []
    for dt, want in zip(dts[2:], e_gear[2:]):
        errs.append(run_example1(yk, 1, dt, flags=yk.HEAT_BOX_CODE))
        print(f"  box code, Gear dt {dt:g}: error {errs[-1]:.4e} (Table 1: {want:.3g})", flush=True)
        assert abs(errs[-1] / want - 1.0) < 0.1
    assert abs(errs[0] / errs[1] - 4.0) < 0.8


def test_allen_cahn_steps_match_oracle(yk):
    """Two Allen-Cahn steps (Sec. 4, Example 3: eps = 1e-5, dt = 1, u = 0 on the
    curves) on a small grid, GPU against the oracle element by element."""
    import torch
    from oracle import grid as G
    e = W.example3(m=48, n_outer=256, n_inner=128)
    b, pts = e["bnd"], e["pts"]
    a2 = G.alpha2_of(G.SCHEME_EULER, e["dt"], e["eps"])
    u_ref = e["u0"].copy()
    for _ in range(2):
        B = G.rhs_imex(G.SCHEME_EULER, G.REACTION_ALLEN_CAHN, u_ref, None, None, None, e["region"], e["consts"],
                       e["dt"])
        u_ref, s_ref, _, _, _ = G.heat_step_grid(b.xy, b.normal, b.weights(), b.curvature, b.speed, b.offset,
                                                 e["grid"], B, e["f_bnd"], a2)
    ctx = yk.yk_create(direct=1)
    try:
        bd = yk.Boundary.from_workload(b)
        u = dev(e["u0"])
        B = torch.empty_like(u)
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        for _ in range(2):
            yk.yk_rhs_imex(ctx, yk.SCHEME_EULER, yk.REACTION_ALLEN_CAHN, u, None, None, None, dev(e["region"]),
                           e["consts"], e["dt"], B)
            un = torch.empty_like(u)
            yk.yk_heat_step_grid(ctx, bd, yk.make_grid(*e["grid"]), B, 0, dev(e["f_bnd"]), a2, 1e-13, sig, un)
            u = un
    finally:
        yk.yk_destroy(ctx)
    ins = e["region"] < 0
    assert elem_err(host(u)[ins], u_ref[ins]) <= 1e-10
    assert elem_err(host(sig), s_ref) <= 1e-9


def test_allen_cahn_hundred_steps(yk):
    """Example 3 at 512^2 cells: 100 steps of dt = 1.  The semi-implicit step
    keeps |u| <= max|2u - u^3| on [-1, 1] (about 1.089; the smoothing operator
    is a contraction in the maximum norm), and the solution coarsens towards
    +-1 (the mean |u| inside grows past 0.8)."""
    import torch
    e = W.example3(m=512, n_outer=2048, n_inner=1024)
    b, pts = e["bnd"], e["pts"]
    a2 = yk.alpha2_of(yk.SCHEME_EULER, e["dt"], e["eps"])
    ctx = yk.yk_create()
    ins = e["region"] < 0
    try:
        bd = yk.Boundary.from_workload(b)
        u = dev(e["u0"])
        reg = dev(e["region"])
        B = torch.empty_like(u)
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        fb = dev(e["f_bnd"])
        grid = yk.make_grid(*e["grid"])
        umax = []
        for step in range(100):
            yk.yk_rhs_imex(ctx, yk.SCHEME_EULER, yk.REACTION_ALLEN_CAHN, u, None, None, None, reg, e["consts"],
                           e["dt"], B)
            un = torch.empty_like(u)
            yk.yk_heat_step_grid(ctx, bd, grid, B, 0, fb, a2, 1e-10, sig, un)
            u = un
            if step % 20 == 19:
                h = host(u)[ins]
                umax.append(np.max(np.abs(h)))
                print(f"allen-cahn step {step + 1}: max|u| {umax[-1]:.4f} mean|u| {np.mean(np.abs(h)):.4f}",
                      flush=True)
    finally:
        yk.yk_destroy(ctx)
    h = host(u)[ins]
    assert max(umax) <= 1.09
    assert np.mean(np.abs(h)) > 0.8
