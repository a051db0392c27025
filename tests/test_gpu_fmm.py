"""GPU parity of the FMM path against the CPU oracle's direct sums and dense solves."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import dev, elem_err, host, rel_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1007_5335_amd.yk as yk
    yk.load_library()
    return yk


def _ctx(yk, **kw):
    kw.setdefault("direct", 0)
    return yk.yk_create(**kw)


def _oracle_fmm_potential(oracle_lib, c):
    b = c["bnd"]
    vol, q, dip, al = c["vol"], c["q"], c["dip"], c["alpha"]
    # dipole strength d_j with unit normal: pass weights 1 via dl_sum(d)
    ov = oracle_lib.volume_sum(vol, q, al) + oracle_lib.dl_sum(b.xy, b.normal, dip, al, vol)
    ob = oracle_lib.volume_sum(vol, q, al, tgt_xy=b.xy) + oracle_lib.dl_sum(b.xy, b.normal, dip, al, b.xy)
    return ov, ob


@pytest.mark.parametrize("alpha,leaf,clustered", [(0.05, 64, False), (0.05, 16, False),
                                                  (0.01, 64, False), (0.2, 32, False),
                                                  (0.05, 32, True)])
def test_fmm_potential_vs_direct(yk, oracle_lib, alpha, leaf, clustered):
    import torch
    c = W.small_fmm_case(n_vol=6000, n_nodes=256, alpha=alpha, seed=5, clustered=clustered)
    b = c["bnd"]
    ctx = _ctx(yk, leaf_size=leaf, fmm_tol=1e-10, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
        ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
        print(f"case alpha={alpha} leaf={leaf} clustered={clustered}", flush=True)
        yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(c["q"]), bd, dev(c["dip"]), alpha, ov, ob)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    rv, rb = _oracle_fmm_potential(oracle_lib, c)
    ev, eb = elem_err(host(ov), rv), elem_err(host(ob), rb)
    print(f"  max err / max |ref|: volume {ev:.2e} nodes {eb:.2e}", flush=True)
    assert ev <= 1e-10 and eb <= 1e-10


@pytest.mark.parametrize("n_src,n_tgt", [(1, 0), (5, 0), (5, 7), (100, 0), (300, 33)])
def test_fmm_tiny_trees(yk, oracle_lib, n_src, n_tgt):
    """Degenerate trees: a single point (zero extent, no pair at all: the self
    pair is left out, so the output is exactly zero), depth 0 and depth 1
    (every pair in the near field, no expansion used), and the smallest sizes
    with a far field, against the oracle's direct sums."""
    import torch
    rng = np.random.default_rng(100 + n_src)
    src = rng.random((n_src, 2)); q = rng.standard_normal(n_src)
    tgt = rng.random((n_tgt, 2)) * 1.2 - 0.1 if n_tgt else None
    n_out = n_tgt if n_tgt else n_src
    ctx = _ctx(yk, leaf_size=64, fmm_tol=1e-10, debug_flags=1)
    try:
        print(f"case n_src={n_src} n_tgt={n_tgt}", flush=True)
        out = torch.full((n_out,), float("nan"), dtype=torch.float64, device="cuda")
        yk.yk_volume_potential(ctx, dev(src), dev(q), dev(tgt) if n_tgt else None, 0.07, out)
        torch.cuda.synchronize()
        info = yk.yk_plan_info_get(ctx, 2)   # (the stand-alone sums' tree)
    finally:
        yk.yk_destroy(ctx)
    got = host(out)
    print(f"  leaf level {info.leaf_level}, far field from level {info.lmin}", flush=True)
    if n_src + n_tgt <= 64:
        assert info.leaf_level == 0
    assert np.all(np.isfinite(got))
    if n_src == 1 and not n_tgt:
        assert np.all(got == 0.0)
        return
    ref = oracle_lib.volume_sum(src, q, 0.07, tgt_xy=tgt) if n_tgt else oracle_lib.volume_sum(src, q, 0.07)
    err = elem_err(got, ref)
    print(f"  max err / max |ref| {err:.2e}", flush=True)
    assert err <= 1e-10


def test_fmm_volume_potential_separate_targets(yk, oracle_lib):
    import torch
    rng = np.random.default_rng(8)
    src = rng.random((5000, 2)); q = rng.standard_normal(5000)
    tgt = rng.random((1500, 2)) * 1.2 - 0.1          # some targets outside the sources' box
    ctx = _ctx(yk, leaf_size=32, debug_flags=1)
    try:
        out = torch.empty(1500, dtype=torch.float64, device="cuda")
        yk.yk_volume_potential(ctx, dev(src), dev(q), dev(tgt), 0.07, out)
        out2 = torch.empty(5000, dtype=torch.float64, device="cuda")
        yk.yk_volume_potential(ctx, dev(src), dev(q), None, 0.07, out2)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    assert elem_err(host(out), oracle_lib.volume_sum(src, q, 0.07, tgt_xy=tgt)) <= 1e-10
    assert elem_err(host(out2), oracle_lib.volume_sum(src, q, 0.07)) <= 1e-10


def test_fmm_double_layer_on_surface(yk, oracle_lib):
    import torch
    c = W.small_fmm_case(n_vol=16, n_nodes=512, alpha=0.05, seed=2)
    b = c["bnd"]
    sig = np.cos(5 * b.xy[:, 0]) + b.xy[:, 1]
    ctx = _ctx(yk, leaf_size=32, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        out = torch.empty(b.n, dtype=torch.float64, device="cuda")
        yk.yk_double_layer_apply(ctx, bd, dev(sig), None, 0.05, out)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    ref = oracle_lib.dl_on_surface(b.xy, b.normal, b.weights(), b.curvature, sig, 0.05)
    assert elem_err(host(out), ref) <= 1e-10


def test_sparse_m2l_boundary_tree(yk, oracle_lib):
    """A nodes-only tree (mostly empty V lists) takes the sparse M2L path; its
    sums on the surface still match the oracle's direct sums."""
    import torch
    c = W.small_fmm_case(n_vol=16, n_nodes=1024, alpha=0.02, seed=4)
    b = c["bnd"]
    sig = np.sin(3 * b.xy[:, 1]) + b.xy[:, 0] ** 2
    ctx = _ctx(yk, leaf_size=16)
    try:
        bd = yk.Boundary.from_workload(b)
        out = torch.empty(b.n, dtype=torch.float64, device="cuda")
        yk.yk_double_layer_apply(ctx, bd, dev(sig), None, 0.02, out)
        torch.cuda.synchronize()
        info = yk.yk_plan_info_get(ctx, 1)   # (on-surface sums use the nodes-only tree)
    finally:
        yk.yk_destroy(ctx)
    assert info.m2l_sparse == 1 and info.m2l_translations > 0, info.as_dict()
    assert info.m2l_slots == info.m2l_translations
    ref = oracle_lib.dl_on_surface(b.xy, b.normal, b.weights(), b.curvature, sig, 0.02)
    assert elem_err(host(out), ref) <= 1e-10


def test_fmm_gmres_vs_dense_lu(yk, oracle_lib):
    import torch
    c = W.small_fmm_case(n_vol=16, n_nodes=256, alpha=0.05, seed=2)
    b = c["bnd"]
    g = np.sin(4 * b.xy[:, 0]) * np.cos(3 * b.xy[:, 1])
    ctx = _ctx(yk, leaf_size=32, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        sig = torch.empty(b.n, dtype=torch.float64, device="cuda")
        st = yk.yk_gmres_density(ctx, bd, 0.05, dev(g), None, 1e-12, 200, sig)
    finally:
        yk.yk_destroy(ctx)
    ref = oracle_lib.DenseBIE(b.xy, b.normal, b.weights(), b.curvature, 0.05).solve(g)
    assert elem_err(host(sig), ref) <= 1e-10, st.as_dict()


def test_fmm_heat_step_c0(yk, oracle_lib):
    import torch
    cfg = W.config_c0()
    b = cfg["bnd"]
    ctx = _ctx(yk, leaf_size=32, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        n = cfg["vol"].shape[0]
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        st = yk.yk_heat_step(ctx, bd, dev(cfg["vol"]), dev(cfg["vol_w"]), dev(cfg["B"]),
                             yk.HEAT_GRID_SELF_CELL | yk.HEAT_ZERO_GUESS, dev(cfg["f_next"]),
                             cfg["dt"], 1e-13, sig, u)
    finally:
        yk.yk_destroy(ctx)
    u_ref, s_ref, _ = oracle_lib.heat_step(b.xy, b.normal, b.weights(), b.curvature, cfg["vol"],
                                           cfg["vol_w"], cfg["B"], cfg["f_next"], cfg["dt"],
                                           grid_h=cfg["h"], offsets=b.offset)
    assert elem_err(host(u), u_ref) <= 1e-10, st.as_dict()
    assert elem_err(host(sig), s_ref) <= 1e-10


def test_fmm_fp32_mode_accuracy(yk, oracle_lib):
    """FP32 near field and FP32 matrix-core M2L: error at FP32 level, stated."""
    import torch
    c = W.small_fmm_case(n_vol=6000, n_nodes=256, alpha=0.05, seed=5)
    b = c["bnd"]
    ctx = _ctx(yk, leaf_size=32, precision=yk.YK_PREC_FP32, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
        ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
        yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(c["q"]), bd, dev(c["dip"]), 0.05, ov, ob)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    rv, rb = _oracle_fmm_potential(oracle_lib, c)
    ev, eb = elem_err(host(ov), rv), elem_err(host(ob), rb)
    print(f"  fp32 max err / max |ref|: volume {ev:.2e} nodes {eb:.2e}", flush=True)
    assert ev < 2e-5 and eb < 2e-5


@pytest.mark.parametrize("p", [8, 16, 24, 31])
def test_fmm_order_sweep_small(yk, oracle_lib, p):
    """Each padded order (16/32/48/64 coefficients) runs and converges with p."""
    import torch
    c = W.small_fmm_case(n_vol=4000, n_nodes=128, alpha=0.05, seed=6)
    b = c["bnd"]
    ctx = _ctx(yk, leaf_size=16, p=p, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
        ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
        yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(c["q"]), bd, dev(c["dip"]), 0.05, ov, ob)
        torch.cuda.synchronize()
        info = yk.yk_plan_info_get(ctx, 0)
    finally:
        yk.yk_destroy(ctx)
    rv, rb = _oracle_fmm_potential(oracle_lib, c)
    err = elem_err(np.concatenate([host(ov), host(ob)]), np.concatenate([rv, rb]))
    print(f"  p={p} Pp={info.Pp} L={info.leaf_level} max err / max |ref| {err:.2e}", flush=True)
    bound = {8: 1e-3, 16: 1e-7, 24: 1e-10, 31: 1e-12}[p]
    assert err < bound


def test_mixed_precision_gmres_refines_to_fp64(yk, oracle_lib):
    import torch
    c = W.small_fmm_case(n_vol=16, n_nodes=256, alpha=0.05, seed=2)
    b = c["bnd"]
    g = np.sin(4 * b.xy[:, 0]) * np.cos(3 * b.xy[:, 1])
    ctx = _ctx(yk, leaf_size=32, precision=yk.YK_PREC_MIXED, debug_flags=1)
    try:
        bd = yk.Boundary.from_workload(b)
        sig = torch.empty(b.n, dtype=torch.float64, device="cuda")
        st = yk.yk_gmres_density(ctx, bd, 0.05, dev(g), None, 1e-12, 200, sig)
    finally:
        yk.yk_destroy(ctx)
    ref = oracle_lib.DenseBIE(b.xy, b.normal, b.weights(), b.curvature, 0.05).solve(g)
    print("  mixed", st.as_dict(), flush=True)
    assert st.res_final <= 1e-12 and st.outer_iters >= 1
    assert elem_err(host(sig), ref) <= 1e-10


@pytest.mark.parametrize("alpha", [0.01, 0.05, 0.2])
def test_mixed_density_solve_full_boundary(yk, oracle_lib, alpha):
    """The density solve on the full-size boundary (outer circle + 5 holes x
    4096 nodes) for each alpha, in plain FP64 and in mixed precision
    (FP32-operator corrections, FP64 residuals): the residual of each returned
    density under the oracle's own operator (direct sums, eq. discrete_sys)
    is within 1e-10 of the right-hand side."""
    import torch
    c = W.config_c1()
    b = c["bnd"]
    g = np.sin(40 * b.xy[:, 0]) * np.cos(30 * b.xy[:, 1]) + 1.0
    rhs = -2.0 * alpha * alpha * g
    w = b.weights()
    for prec in (yk.YK_PREC_FP64, yk.YK_PREC_MIXED):
        ctx = _ctx(yk, fmm_tol=1e-10, precision=prec)
        try:
            bd = yk.Boundary.from_workload(b)
            sig = torch.empty(b.n, dtype=torch.float64, device="cuda")
            print(f"full boundary alpha={alpha} precision={prec}", flush=True)
            st = yk.yk_gmres_density(ctx, bd, alpha, dev(g), None, 1e-11, 400, sig)
            torch.cuda.synchronize()
            info = yk.yk_plan_info_get(ctx, 1)
        finally:
            yk.yk_destroy(ctx)
        s_np = host(sig)
        res = rhs - oracle_lib.apply_bie(b.xy, b.normal, w, b.curvature, s_np, alpha)
        r = float(np.linalg.norm(res) / np.linalg.norm(rhs))
        print(f"  {st.as_dict()} p={info.p}; oracle residual {r:.2e}", flush=True)
        assert st.res_final <= 1e-11
        if prec == yk.YK_PREC_MIXED:
            assert st.outer_iters >= 1
        assert r <= 1e-10


def test_fmm_near_field_accuracy_tight(yk, oracle_lib):
    """Points packed so every near pair has t = r^2/(4 alpha^2) <= 1, and p = 31:
    the near field (own logarithm and series) and the far field agree with the
    direct sums to ~1e-13."""
    import torch
    rng = np.random.default_rng(21)
    src = rng.random((6000, 2)) * 0.05
    q = rng.standard_normal(6000)
    ctx = _ctx(yk, leaf_size=16, p=31, debug_flags=1)
    try:
        out = torch.empty(6000, dtype=torch.float64, device="cuda")
        yk.yk_volume_potential(ctx, dev(src), dev(q), None, 0.2, out)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    ref = oracle_lib.volume_sum(src, q, 0.2)
    assert elem_err(host(out), ref) < 5e-13


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fmm_full_size_sampled_vs_oracle(yk, oracle_lib, precision):
    """The benchmark's workload at full size (2^20 charges + 6 x 4096 dipoles,
    alpha = 0.05) in the benchmark's launch configuration; sampled outputs are
    compared one by one with the oracle's direct sums."""
    import torch
    c = W.config_c1()
    b = c["bnd"]
    prec = yk.YK_PREC_FP32 if precision == "fp32" else yk.YK_PREC_FP64
    ctx = yk.yk_create(fmm_tol=1e-10, leaf_size=64, precision=prec)
    try:
        bd = yk.Boundary.from_workload(b)
        ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
        ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
        print(f"full-size C1 {precision}", flush=True)
        for _ in range(2):      # second call reuses the cached tree
            yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(c["q"]), bd, dev(c["dip"]), c["alpha"], ov, ob)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    iv = W.sample_targets(c["vol"].shape[0], 24, seed=11)
    ib = W.sample_targets(b.n, 8, seed=12)
    tv, tb = c["vol"][iv], b.xy[ib]
    tgt = np.concatenate([tv, tb])
    ref = (oracle_lib.volume_sum(c["vol"], c["q"], c["alpha"], tgt_xy=tgt)
           + oracle_lib.dl_sum(b.xy, b.normal, c["dip"], c["alpha"], tgt))
    got = np.concatenate([host(ov)[iv], host(ob)[ib]])
    scale = float(np.sqrt(np.mean(ref ** 2)))
    err = float(np.max(np.abs(got - ref)) / scale)
    print(f"  max err / rms {err:.2e}", flush=True)
    assert err < (1e-9 if precision == "fp64" else 2e-5)


@pytest.mark.parametrize("p,bound", [(8, 1e-3), (16, 1e-6), (31, 1e-10)])
def test_fmm_full_size_orders_vs_oracle(yk, oracle_lib, p, bound):
    """Other expansion orders on the full-size tree (65,536 leaves, where P2M
    runs in two halves of the orders and adds the dipoles afterwards): sampled
    outputs against the oracle, within a bound set by the order's truncation
    (about 0.025 * 0.44^p relative)."""
    import torch
    c = W.config_c1()
    b = c["bnd"]
    ctx = _ctx(yk, p=p, leaf_size=64)
    try:
        bd = yk.Boundary.from_workload(b)
        ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
        ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
        print(f"full-size C1 p={p}", flush=True)
        yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(c["q"]), bd, dev(c["dip"]), c["alpha"], ov, ob)
        torch.cuda.synchronize()
        info = yk.yk_plan_info_get(ctx, 0)
    finally:
        yk.yk_destroy(ctx)
    assert info.p == p and info.n_leaves >= 8192
    iv = W.sample_targets(c["vol"].shape[0], 16, seed=21)
    ib = W.sample_targets(b.n, 8, seed=22)
    tgt = np.concatenate([c["vol"][iv], b.xy[ib]])
    ref = (oracle_lib.volume_sum(c["vol"], c["q"], c["alpha"], tgt_xy=tgt)
           + oracle_lib.dl_sum(b.xy, b.normal, c["dip"], c["alpha"], tgt))
    got = np.concatenate([host(ov)[iv], host(ob)[ib]])
    err = float(np.max(np.abs(got - ref)) / np.sqrt(np.mean(ref ** 2)))
    print(f"  max err / rms {err:.2e}", flush=True)
    assert err < bound


def _c4_like_pass_vs_oracle(yk, oracle_lib, c, nv, nb, seed, orders=(0,)):
    """One FMM pass per expansion order (0: chosen from fmm_tol = 1e-10);
    per-target and l2 relative errors against the oracle on sampled targets.
    The charges are a positive density times the cell areas (the form of
    q = W B with positive data): with areas spanning many orders of magnitude,
    zero-mean charges would make each target's potential a cancelling sum of
    much larger terms, and its relative error would measure the cancellation."""
    import torch
    b, vol = c["bnd"], c["vol"]
    n = vol.shape[0]
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.5, 1.5, n) * c["vol_w"] * np.sqrt(n)
    dip = rng.standard_normal(b.n) * 1e-3
    iv = W.sample_targets(n, nv, seed=seed + 1)
    ib = W.sample_targets(b.n, nb, seed=seed + 2)
    tgt = np.concatenate([vol[iv], b.xy[ib]])
    ref = (oracle_lib.volume_sum(vol, q, c["alpha"], tgt_xy=tgt)
           + oracle_lib.dl_sum(b.xy, b.normal, dip, c["alpha"], tgt))
    res = []
    for p in orders:
        ctx = _ctx(yk, fmm_tol=1e-10, leaf_size=64, p=p)
        try:
            bd = yk.Boundary.from_workload(b)
            ov = torch.empty(n, dtype=torch.float64, device="cuda")
            ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
            yk.yk_fmm_potential(ctx, dev(vol), dev(q), bd, dev(dip), c["alpha"], ov, ob)
            torch.cuda.synchronize()
            info = yk.yk_plan_info_get(ctx, 0)
        finally:
            yk.yk_destroy(ctx)
        got = np.concatenate([host(ov)[iv], host(ob)[ib]])
        err = np.abs(got - ref) / np.abs(ref)
        l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"  p={info.p} leaf level {info.leaf_level}, {info.n_leaves} leaves, lmin {info.lmin}, "
              f"tree build {info.build_ms:.0f} ms (tables {info.tables_ms:.0f}, order check "
              f"{info.order_check_ms:.0f}); "
              f"per-target relative errors {err}, l2 {l2:.2e}", flush=True)
        res.append((info, err, l2))
    return res


def test_clustered_small_alpha_pass_vs_oracle(yk, oracle_lib):
    """A reduced C4-shaped set (about 2^20 adaptive cells refined by a mixture
    of 8 Gaussians, 8 small holes of 4096 nodes in the gaps, alpha = 1e-3):
    many leaves hold no charges, which the large-tree P2M must not mistake for
    the ends of a block's run of charges.  At the default tolerance (1e-10)
    the tree's build-time order check raises the order until the far field of
    the small holes' dense dipoles meets it; every sampled output, volume
    cells and nodes alike, is then within 1e-10 of the oracle's direct sum
    relative to its own value."""
    c = W.config_c4(n_vol=1 << 20, n_holes=8, n_nodes=4096, seed=9)
    print("clustered 2^20, alpha 1e-3", flush=True)
    ((info, err, l2),) = _c4_like_pass_vs_oracle(yk, oracle_lib, c, 6, 6, 31)
    print(f"  order {info.p_initial} -> {info.p}, order check {info.order_check_err:.2e}", flush=True)
    assert info.n_leaves >= 8192
    assert np.max(err) <= 1e-10 and l2 <= 1e-10, err


def test_c4_full_size_pass_vs_oracle(yk, oracle_lib):
    """The large adaptive set at full size (about 2^24 adaptive cells refined by
    a mixture of 8 Gaussians, 20 holes x 8192 nodes, alpha = 1e-3): one FMM
    pass at the default tolerance (and the default, automatic tree form, which
    takes the adaptive quad-tree here), sampled outputs against the oracle's
    direct sums, each within 1e-10 relative to its own value."""
    c = W.config_c4()
    print("C4 full size", flush=True)
    ((info, err, l2),) = _c4_like_pass_vs_oracle(yk, oracle_lib, c, 2, 2, 41)
    print(f"  order {info.p_initial} -> {info.p}, order check {info.order_check_err:.2e}", flush=True)
    # the default (automatic) form takes the adaptive tree for this clustered set
    assert info.tree == yk.YK_TREE_ADAPTIVE and info.n_leaves > 200_000 and info.n_wlist > 0
    assert np.max(err) <= 1e-10 and l2 <= 1e-10, err


def test_c4_heat_steps_mixed_learned(yk):
    """Backward-Euler steps on the large adaptive set (about 2^24 adaptive
    cells with their areas as weights and their own integrals added, 20 holes
    x 8192 nodes, dt = alpha^2 = 1e-6, u = c_k on hole k, u = 0 at t = 0):
    plain FP64 with the previous-step guess against mixed precision with the
    learned warm start (trained after five steps).  Every step of both reaches
    the GMRES tolerance from one of the two guesses, the two agree to the
    solves' reach, and the solution stays within the boundary data's range
    (maximum principle: |u| <= max |c_k| = 1 inside the domain), which needs
    the near-boundary evaluation at cells closer to a curve than a few node
    spacings (the plain trapezoid sum there grows the solution step by step)."""
    import time
    import torch
    c = W.config_c4()
    b, vol = c["bnd"], c["vol"]
    region = torch.as_tensor(b.region(vol), dtype=torch.int32, device="cuda")
    f = dev(np.repeat(c["consts"], np.diff(b.offset)))
    n_steps = 7
    finals = {}
    inside = b.region(vol) < 0
    for name, prec, learned in (("fp64", yk.YK_PREC_FP64, False), ("mixed_learned", yk.YK_PREC_MIXED, True)):
        ctx = yk.yk_create(fmm_tol=1e-10, precision=prec)
        ws = None
        try:
            bd = yk.Boundary.from_workload(b)
            if learned:
                ws = yk.yk_ws_create(ctx, bd)
                yk.yk_set_warm_start(ctx, ws)
            vx, vw = dev(vol), dev(c["vol_w"])
            u = torch.zeros(vol.shape[0], dtype=torch.float64, device="cuda")
            B, un = torch.empty_like(u), torch.empty_like(u)
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            for step in range(1, n_steps + 1):
                if ws is not None and step == 6:
                    yk.yk_ws_train(ws)
                yk.yk_rhs_backward_euler(ctx, u, None, region, c["consts"], c["dt"], B)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = yk.yk_heat_step(ctx, bd, vx, vw, B, yk.HEAT_GRID_SELF_CELL, f, c["dt"], 1e-10, sig, un)
                torch.cuda.synchronize()
                umax = float(torch.max(torch.abs(un[torch.as_tensor(inside, device="cuda")])))
                print(f"C4 {name} step {step}: {(time.perf_counter() - t0) * 1e3:.1f} ms, "
                      f"{st.iters} iterations, res0 {st.res0:.2e}, guess {st.guess_used}, "
                      f"max|u| inside {umax:.4f}", flush=True)
                assert umax <= 1.02
                assert st.res_final <= 1e-10
                # the previous density or, once trained, whichever of it and
                # the network's prediction has the smaller residual
                assert st.guess_used in ((1, 2) if learned and step >= 6 else (1,))
                u, un = un, u
            finals[name] = host(u).copy()
        finally:
            if ws is not None:
                yk.yk_ws_destroy(ws)
            yk.yk_destroy(ctx)
    assert elem_err(finals["mixed_learned"], finals["fp64"]) < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_near_cache_matches_on_the_fly(yk, oracle_lib, precision):
    """The cached near-field values give the same sums as evaluating the
    kernels on the fly, also on a second call with new strengths (the cache
    holds geometry only)."""
    import torch
    c = W.small_fmm_case(n_vol=6000, n_nodes=256, alpha=0.05, seed=21, clustered=False)
    b = c["bnd"]
    rng = np.random.default_rng(22)
    strengths = ((c["q"], c["dip"]), (rng.standard_normal(c["q"].size), rng.standard_normal(b.n)))
    prec = yk.YK_PREC_FP32 if precision == "fp32" else yk.YK_PREC_FP64
    outs = {}
    for cache_mb in (16384, 0):
        ctx = _ctx(yk, leaf_size=32, fmm_tol=1e-10, precision=prec, near_cache_mb=cache_mb)
        try:
            bd = yk.Boundary.from_workload(b)
            res = []
            for q, dip in strengths:
                ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
                ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
                print(f"near cache {cache_mb} MiB {precision}", flush=True)
                yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(q), bd, dev(dip), c["alpha"], ov, ob)
                torch.cuda.synchronize()
                res.append(np.concatenate([host(ov), host(ob)]))
        finally:
            yk.yk_destroy(ctx)
        outs[cache_mb] = res
    tol = 1e-13 if precision == "fp64" else 2e-6
    for a, bb in zip(outs[16384], outs[0]):
        assert elem_err(a, bb) < tol
    rv, rb = _oracle_fmm_potential(oracle_lib, c)
    ref = np.concatenate([rv, rb])
    assert elem_err(outs[16384][0], ref) <= (1e-10 if precision == "fp64" else 2e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["few_items", "many_items", "clustered"])
def test_symmetric_near_field_matches_full_storage(yk, oracle_lib, precision, case):
    """Charge-to-charge near-field values stored once per pair of neighbouring
    leaves and applied both ways (the default when every leaf holds at most 64
    charges) give the sums of storing both orders (debug_flags bit 4), also on
    a second call with new strengths; they are read at about half the bytes.
    Few items run four wavefronts per item, many items one; the clustered set
    has leaves of more than 64 targets (nodes of the holes), split into
    several items."""
    import torch
    n_vol, leaf = {"few_items": (6000, 32), "many_items": (1 << 17, 16), "clustered": (20000, 32)}[case]
    c = W.small_fmm_case(n_vol=n_vol, n_nodes=256, alpha=0.05, seed=23, clustered=case == "clustered")
    b = c["bnd"]
    rng = np.random.default_rng(24)
    strengths = ((c["q"], c["dip"]), (rng.standard_normal(c["q"].size), rng.standard_normal(b.n)))
    prec = yk.YK_PREC_FP32 if precision == "fp32" else yk.YK_PREC_FP64
    outs, infos = {}, {}
    for flags in (0, 16):
        ctx = _ctx(yk, leaf_size=leaf, fmm_tol=1e-10, precision=prec, debug_flags=flags)
        try:
            bd = yk.Boundary.from_workload(b)
            res = []
            for q, dip in strengths:
                ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
                ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
                print(f"symmetric near field {case} {precision} flags {flags}", flush=True)
                yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(q), bd, dev(dip), c["alpha"], ov, ob)
                torch.cuda.synchronize()
                res.append(np.concatenate([host(ov), host(ob)]))
            infos[flags] = yk.yk_plan_info_get(ctx, 0)
        finally:
            yk.yk_destroy(ctx)
        outs[flags] = res
    full, sym = infos[16], infos[0]
    assert full.near_sym == 0 and full.near_charge_values == full.pairs_charge
    if case != "clustered":
        assert sym.near_sym == 1
    if sym.near_sym:
        assert sym.near_charge_values < 0.7 * sym.pairs_charge
        assert sym.near_incoming > 0
    tol = 1e-13 if precision == "fp64" else 2e-6
    for a, bb in zip(outs[0], outs[16]):
        assert elem_err(a, bb) < tol
    if case == "few_items":
        rv, rb = _oracle_fmm_potential(oracle_lib, c)
        assert elem_err(outs[0][0], np.concatenate([rv, rb])) <= (1e-10 if precision == "fp64" else 2e-5)


def test_heat_step_reuses_charge_multipoles(yk):
    """Two C3-size heat steps (1024^2 grid, 65,536 leaves): the second volume
    pass of each step starts from the charges' multipoles kept by the first
    and adds only the dipoles'; the result equals recomputing them (debug_flags
    bit 3) to rounding."""
    import torch
    cfg = W.config_c3(m=1024, n_holes=10, n_nodes=2048, dt=1e-3, seed=3)
    b = cfg["bnd"]
    runs = {}
    for flags in (0, 8):
        opt = yk.yk_default_options()
        opt.debug_flags = flags
        ctx = yk.yk_create(opt)
        try:
            bd = yk.Boundary.from_workload(b)
            vol, w, f = dev(cfg["vol"]), dev(cfg["vol_w"]), dev(cfg["f_bnd"])
            region = torch.as_tensor(cfg["region"], dtype=torch.int32, device="cuda")
            u = dev(cfg["u0"])
            B, un = torch.empty_like(u), torch.empty_like(u)
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            for step in range(2):
                print(f"C3 step {step} flags={flags}", flush=True)
                yk.yk_rhs_backward_euler(ctx, u, None, region, cfg["consts"], cfg["dt"], B)
                yk.yk_heat_step(ctx, bd, vol, w, B, yk.HEAT_GRID_SELF_CELL, f, cfg["dt"], 1e-10, sig, un)
                u, un = un, u
            torch.cuda.synchronize()
            info = yk.yk_plan_info_get(ctx, 0)
        finally:
            yk.yk_destroy(ctx)
        assert info.n_leaves >= 8192
        runs[flags] = (host(u).copy(), host(sig).copy())
    assert elem_err(runs[0][0], runs[8][0]) < 1e-12
    assert elem_err(runs[0][1], runs[8][1]) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_heat_steps_reuse_previous_residual(yk, precision):
    """Three steps of the C0 problem: passing back the returned density lets the
    context reuse A sigma for the next step's initial residual (one operator
    application fewer per step) with the same results as recomputing it (the
    memo is dropped by re-setting the options before every step)."""
    import torch
    cfg = W.config_c0()
    b = cfg["bnd"]
    prec = yk.YK_PREC_MIXED if precision == "mixed" else yk.YK_PREC_FP64
    runs = {}
    for reuse in (True, False):
        opt = yk.yk_default_options()
        opt.leaf_size, opt.precision = 32, prec
        ctx = yk.yk_create(opt)
        try:
            bd = yk.Boundary.from_workload(b)
            n = cfg["vol"].shape[0]
            vol, w, f = dev(cfg["vol"]), dev(cfg["vol_w"]), dev(cfg["f_next"])
            B = dev(cfg["B"])
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            u = torch.empty(n, dtype=torch.float64, device="cuda")
            mv, us = [], []
            for step in range(3):
                if not reuse:
                    yk.yk_set_options(ctx, opt)
                print(f"step {step} reuse={reuse} {precision}", flush=True)
                st = yk.yk_heat_step(ctx, bd, vol, w, B, yk.HEAT_GRID_SELF_CELL, f, cfg["dt"], 1e-12, sig, u)
                torch.cuda.synchronize()
                mv.append(st.matvecs)
                us.append(host(u).copy())
                B = u.clone()
        finally:
            yk.yk_destroy(ctx)
        runs[reuse] = (mv, us, host(sig))
    (mv1, u1, s1), (mv0, u0, s0) = runs[True], runs[False]
    for a, c in zip(u1, u0):
        assert elem_err(a, c) < 1e-11
    assert elem_err(s1, s0) < 1e-10
    # steps after the first skip one application of the FP64 operator
    assert sum(mv1[1:]) <= sum(mv0[1:]) - 2, (mv1, mv0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_density_operator_graph_replay(yk, oracle_lib, precision):
    """The density operator captured in a HIP graph and replayed (many times per
    solve, with the solver's own kernels and host synchronisations between
    replays, and again in a second solve) gives the eager operator's solution."""
    import torch
    c = W.small_fmm_case(n_vol=16, n_nodes=256, alpha=0.05, seed=2)
    b = c["bnd"]
    g1 = np.sin(4 * b.xy[:, 0]) * np.cos(3 * b.xy[:, 1])
    g2 = np.cos(2 * b.xy[:, 0]) + b.xy[:, 1] ** 2
    prec = yk.YK_PREC_MIXED if precision == "mixed" else yk.YK_PREC_FP64
    sols = {}
    for flags in (4, 0):          # 4: graph replay, 0: eager operator
        ctx = _ctx(yk, leaf_size=32, precision=prec, debug_flags=flags)
        try:
            bd = yk.Boundary.from_workload(b)
            out = []
            for g in (g1, g2, g1):
                sig = torch.empty(b.n, dtype=torch.float64, device="cuda")
                print(f"graph replay flags={flags} {precision}", flush=True)
                st = yk.yk_gmres_density(ctx, bd, 0.05, dev(g), None, 1e-12, 200, sig)
                torch.cuda.synchronize()
                out.append((host(sig).copy(), st.iters))
        finally:
            yk.yk_destroy(ctx)
        sols[flags] = out
    ref1 = oracle_lib.DenseBIE(b.xy, b.normal, b.weights(), b.curvature, 0.05).solve(g1)
    for (s_g, it_g), (s_e, it_e) in zip(sols[4], sols[0]):
        assert elem_err(s_g, s_e) < 1e-11
    assert elem_err(sols[4][0][0], ref1) <= 1e-10
    assert elem_err(sols[4][2][0], ref1) <= 1e-10
