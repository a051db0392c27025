"""The box code (Sec. 3.1, eq. volume_potential and the leaf polynomials) on
the GPU against the oracle's box code (oracle/box.py): the volume potential of
the leaves' cubic fits at sampled cells, element by element, on grids whose
leaf counts are and are not powers of two, with and without a far field; the
leaf polynomials at points; and the grid heat step run with it."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, elem_err, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1007_5335_amd.yk as yk
    yk.load_library()
    return yk


def _cells(grid):
    x0, y0, h, nx, ny = grid
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    return np.stack([x0 + (i.ravel() + 0.5) * h, y0 + (j.ravel() + 0.5) * h], 1)


@pytest.mark.parametrize("grid,alpha", [((0.0, 0.0, 1 / 32, 32, 32), 0.1),
                                        ((0.0, 0.0, 1 / 32, 32, 32), 0.02),
                                        ((-0.3, 0.2, 0.025, 40, 24), 0.05),
                                        ((0.0, 0.0, 1 / 128, 128, 128), 0.01),
                                        ((0.1, -0.2, 0.05, 4, 4), 0.03),
                                        ((0.0, 0.0, 0.05, 8, 4), 0.2)])
def test_box_potential_vs_oracle(yk, grid, alpha):
    """Rough cell values (noise of 0.3 on a smooth field), so the leaf fits
    carry large high-order terms; every sampled cell within 1e-10 of the
    largest value."""
    import torch
    from oracle import box as X
    c = _cells(grid)
    rng = np.random.default_rng(7)
    B = np.cos(3 * c[:, 0] - c[:, 1]) + 0.3 * rng.standard_normal(len(c))   # rough: the fits differ from B
    ctx = yk.yk_create()
    try:
        V = torch.empty(len(c), dtype=torch.float64, device="cuda")
        print(f"box grid {grid}, alpha {alpha}", flush=True)
        yk.yk_box_potential(ctx, yk.make_grid(grid[0], grid[1], grid[2], grid[3], grid[4]), dev(B), alpha, V)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    got = host(V)
    idx = np.unique(np.concatenate([rng.choice(len(c), min(24, len(c)), replace=False),
                                    [0, len(c) - 1, grid[3] - 1]]))
    ref = X.potential(B, grid, alpha, c[idx])
    err = elem_err(got[idx], ref)
    print(f"  max err / max |ref| over {len(idx)} cells: {err:.2e}", flush=True)
    assert err <= 1e-10


def test_box_leaf_polynomials_vs_oracle(yk):
    import torch
    from oracle import box as X
    grid = (-0.3, 0.2, 0.025, 40, 24)
    c = _cells(grid)
    rng = np.random.default_rng(3)
    B = np.sin(2 * c[:, 0]) * np.exp(c[:, 1]) + 0.1 * rng.standard_normal(len(c))
    pts = np.stack([grid[0] + rng.random(500) * 40 * 0.025, grid[1] + rng.random(500) * 24 * 0.025], 1)
    ctx = yk.yk_create()
    try:
        V = torch.empty(len(c), dtype=torch.float64, device="cuda")
        pv = torch.empty(len(pts), dtype=torch.float64, device="cuda")
        yk.yk_box_potential(ctx, yk.make_grid(*grid), dev(B), 0.05, V, dev(pts), pv)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    ref = X.leaf_eval(host(V), grid, pts)
    assert elem_err(host(pv), ref) <= 1e-12


def test_grid_step_box_code_closed_form(yk):
    """u = sin(3x) sin(2y) + 1 by one step of the grid form with the box code:
    every cell inside the annulus within 1e-6, like the lattice rule."""
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
        for flags in (yk.HEAT_ZERO_GUESS, yk.HEAT_ZERO_GUESS | yk.HEAT_BOX_CODE):
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            u = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
            yk.yk_heat_step_grid(ctx, bd, yk.make_grid(*grid), dev(B), flags, dev(uf(b.xy)), a2, 1e-12, sig, u)
            errs[flags] = np.max(np.abs(host(u) - uf(pts))[inside])
    finally:
        yk.yk_destroy(ctx)
    print(f"closed form: max error lattice {errs[yk.HEAT_ZERO_GUESS]:.2e}, "
          f"box code {errs[yk.HEAT_ZERO_GUESS | yk.HEAT_BOX_CODE]:.2e}", flush=True)
    assert errs[yk.HEAT_ZERO_GUESS | yk.HEAT_BOX_CODE] < 1e-6


def test_box_rejects_sides_not_multiple_of_four(yk):
    import torch
    ctx = yk.yk_create()
    try:
        B = torch.zeros(30, dtype=torch.float64, device="cuda")
        V = torch.empty(30, dtype=torch.float64, device="cuda")
        with pytest.raises(yk.YkError) as ei:
            yk.yk_box_potential(ctx, yk.make_grid(0.0, 0.0, 0.1, 6, 5), B, 0.1, V)
        assert ei.value.status == yk.YK_ERR_ARG
    finally:
        yk.yk_destroy(ctx)


@pytest.mark.parametrize("depth,alpha", [(5, 0.05), (7, 0.01), (3, 0.2)])
def test_adaptive_box_potential_vs_oracle(yk, depth, alpha):
    """The box code on 2:1-balanced adaptive leaves (refined towards a point,
    levels 2 .. depth): V at sampled cells against the oracle's box code on
    the same leaves; the tree's leaves are the given ones (near tables per
    level pair, W and X lists through polynomial multipoles and tables)."""
    import torch
    from oracle import box as X
    root = (-0.2, 0.1, 1.3)
    lv, ix, iy = X.balanced_leaves(root, (0.2, 0.5), depth)
    cells = X.leaf_cells(lv, ix, iy, root)
    rng = np.random.default_rng(depth)
    B = np.cos(2 * cells[:, 0]) * np.exp(cells[:, 1]) + 0.2 * rng.standard_normal(len(cells))
    ctx = yk.yk_create()
    try:
        V = torch.empty(len(cells), dtype=torch.float64, device="cuda")
        print(f"adaptive box: {len(lv)} leaves, levels {lv.min()}..{lv.max()}, alpha {alpha}", flush=True)
        yk.yk_box_potential_adaptive(ctx, root, lv, ix, iy, dev(B), alpha, V)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    got = host(V)
    idx = np.unique(np.concatenate([rng.choice(len(cells), 20, replace=False), [0, len(cells) - 1]]))
    ref = X.potential_leaves(lv, ix, iy, root, B, alpha, cells[idx])
    err = elem_err(got[idx], ref)
    print(f"  max err / max |ref| over {len(idx)} cells: {err:.2e}", flush=True)
    assert err <= 1e-10


def test_adaptive_box_rejects_unbalanced_leaves(yk):
    import torch
    # quadrant (0, 0) in four level-2 leaves, the one at (1, 1) split again:
    # its level-3 leaves at x = 3/8 .. 1/2 touch the level-1 leaf at (1, 0)
    lv = [1, 1, 1] + [2] * 3 + [3] * 4
    ix = [1, 0, 1] + [0, 1, 0] + [2, 3, 2, 3]
    iy = [0, 1, 1] + [0, 0, 1] + [2, 2, 3, 3]
    n = len(lv)
    ctx = yk.yk_create()
    try:
        B = torch.zeros(16 * n, dtype=torch.float64, device="cuda")
        V = torch.empty(16 * n, dtype=torch.float64, device="cuda")
        with pytest.raises(yk.YkError) as ei:
            yk.yk_box_potential_adaptive(ctx, (0.0, 0.0, 1.0), lv, ix, iy, B, 0.1, V)
        assert ei.value.status == yk.YK_ERR_ARG
    finally:
        yk.yk_destroy(ctx)


def test_box_refinement_test_vs_oracle(yk):
    import torch
    from oracle import box as X
    rng = np.random.default_rng(11)
    n = 300
    v16 = rng.standard_normal(16 * n)
    v64 = rng.standard_normal(64 * n) * 0.01
    ref_f, ref_e = X.refine_flags(v16, v64, 1.0)
    ctx = yk.yk_create()
    try:
        fl = torch.empty(n, dtype=torch.int32, device="cuda")
        er = torch.empty(n, dtype=torch.float64, device="cuda")
        yk.yk_box_refine(ctx, dev(v16), dev(v64), 1.0, fl, er)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    assert elem_err(host(er), ref_e) <= 1e-13
    assert np.array_equal(host(fl).astype(bool), ref_f)


def test_heat_step_on_adaptive_leaves_closed_form(yk):
    """One step on adaptive leaves refined towards the annulus's two circles
    (levels 6 .. 8, 2:1 balanced): u = sin(3x) sin(2y) + 1 at every cell
    inside, box code for U^p, leaf polynomials on the nodes, the density
    solve and the near-boundary evaluation."""
    import torch
    from oracle import box as X
    b = W.make_boundary([W.circle((0.0, 0.0), 0.4, 1024), W.circle((0.0, 0.0), 0.1, 512, ccw=False)])
    root = (-0.5, -0.5, 1.0)

    def want(l, i, j):
        s = 2.0 ** -l
        r = np.hypot(root[0] + (i + 0.5) * s, root[1] + (j + 0.5) * s)
        return l < 6 or min(abs(r - 0.4), abs(r - 0.1)) < s

    lv, ix, iy = X.balanced_leaves_by(root, want, 8)
    cells = X.leaf_cells(lv, ix, iy, root)
    uf = lambda p: np.sin(3 * p[:, 0]) * np.sin(2 * p[:, 1]) + 1.0
    a2 = 1e-3
    B = (1 + 13 * a2) * uf(cells) - 13 * a2
    inside = b.region(cells) < 0
    ctx = yk.yk_create()
    try:
        bd = yk.Boundary.from_workload(b)
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        u = torch.empty(len(cells), dtype=torch.float64, device="cuda")
        print(f"leaves {len(lv)}, cells {len(cells)}", flush=True)
        st = yk.yk_heat_step_leaves(ctx, bd, root, lv, ix, iy, dev(B), yk.HEAT_ZERO_GUESS, dev(uf(b.xy)), a2,
                                    1e-12, sig, u)
    finally:
        yk.yk_destroy(ctx)
    err = np.max(np.abs(host(u) - uf(cells))[inside])
    print(f"  adaptive leaves: max error inside {err:.2e}, {st.iters} iterations", flush=True)
    assert err < 1e-6
