"""GPU parity of the FMM heat step against the CPU oracle, element by element,
in every precision mode, over several steps of the time loop."""
import math

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


def _rhs(u, region, consts):
    """B = u inside the domain, the curve's constant outside it (Sec. 3.1)."""
    return np.where(region < 0, u, consts[np.maximum(region, 0)])


@pytest.fixture(scope="module")
def reduced_c3(oracle_lib):
    """A reduced time-stepping set: 128^2 grid (2^14 cells), 10 ellipses x 256
    nodes + 1024 on the outer circle, dt = 1e-3; four backward-Euler steps of
    the oracle (dense LU of the 3,584-node system, factored once)."""
    cfg = W.config_c3(m=128, n_holes=10, n_nodes=256, dt=1e-3, seed=3)
    b = cfg["bnd"]
    bie = oracle_lib.DenseBIE(b.xy, b.normal, b.weights(), b.curvature, cfg["alpha"])
    u = cfg["u0"].copy()
    steps = []
    for _ in range(4):
        B = _rhs(u, cfg["region"], cfg["consts"])
        u, sig, _ = oracle_lib.heat_step(b.xy, b.normal, b.weights(), b.curvature, cfg["vol"], cfg["vol_w"],
                                         B, cfg["f_bnd"], cfg["dt"], grid_h=cfg["h"], bie=bie, offsets=b.offset)
        steps.append((u.copy(), sig.copy()))
    return cfg, steps


@pytest.mark.parametrize("mode", ["fp64", "mixed", "mixed_learned"])
def test_reduced_c3_heat_steps_vs_oracle(yk, reduced_c3, mode):
    """Four steps on a tree of at least 8192 leaves (leaf size 4), where the
    volume passes take the large-tree path (charge multipoles in two halves of
    the orders, kept from the first pass for the second); every step's u and
    sigma element by element against the oracle within 1e-10 of their largest
    entry.  The learned mode trains the network after step 3 and offers its
    guess at step 4."""
    import torch
    cfg, ref = reduced_c3
    b = cfg["bnd"]
    prec = yk.YK_PREC_FP64 if mode == "fp64" else yk.YK_PREC_MIXED
    ctx = yk.yk_create(leaf_size=4, precision=prec)
    ws = None
    try:
        bd = yk.Boundary.from_workload(b)
        if mode == "mixed_learned":
            ws = yk.yk_ws_create(ctx, bd, steps=200)
            yk.yk_set_warm_start(ctx, ws)
        vol, w, f = dev(cfg["vol"]), dev(cfg["vol_w"]), dev(cfg["f_bnd"])
        region = torch.as_tensor(cfg["region"], dtype=torch.int32, device="cuda")
        u = dev(cfg["u0"])
        B, un = torch.empty_like(u), torch.empty_like(u)
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        for step, (u_ref, s_ref) in enumerate(ref, start=1):
            if ws is not None and step == 4:
                yk.yk_ws_train(ws)
            print(f"reduced C3 {mode} step {step}", flush=True)
            yk.yk_rhs_backward_euler(ctx, u, None, region, cfg["consts"], cfg["dt"], B)
            st = yk.yk_heat_step(ctx, bd, vol, w, B, yk.HEAT_GRID_SELF_CELL, f, cfg["dt"], 1e-12, sig, un)
            torch.cuda.synchronize()
            info = yk.yk_plan_info_get(ctx, 0)
            eu, es = elem_err(host(un), u_ref), elem_err(host(sig), s_ref)
            print(f"  iters {st.iters} guess {st.guess_used} leaves {info.n_leaves} p {info.p}: "
                  f"u err {eu:.2e}, sigma err {es:.2e}", flush=True)
            assert info.n_leaves >= 8192
            assert st.res_final <= 1e-12
            assert eu <= 1e-10 and es <= 1e-10
            if ws is not None and step == 4:
                assert st.guess_used in (1, 2)
            u, un = un, u
    finally:
        if ws is not None:
            yk.yk_ws_destroy(ws)
        yk.yk_destroy(ctx)


def test_mixed_heat_step_few_volume_points_many_nodes(yk, oracle_lib):
    """Fewer volume points (256) than boundary nodes (4,096) in mixed precision:
    the density solve takes workspaces larger than the volume charges, which
    live in a buffer of their own; u and sigma against the oracle."""
    import torch
    cfg = W.config_c0(n_nodes=2048, m=16)
    b = cfg["bnd"]
    ctx = yk.yk_create(leaf_size=32, precision=yk.YK_PREC_MIXED)
    try:
        bd = yk.Boundary.from_workload(b)
        n = cfg["vol"].shape[0]
        sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        print(f"mixed heat step n_vol={n} nodes={b.n}", flush=True)
        st = yk.yk_heat_step(ctx, bd, dev(cfg["vol"]), dev(cfg["vol_w"]), dev(cfg["B"]),
                             yk.HEAT_GRID_SELF_CELL | yk.HEAT_ZERO_GUESS, dev(cfg["f_next"]),
                             cfg["dt"], 1e-12, sig, u)
        torch.cuda.synchronize()
    finally:
        yk.yk_destroy(ctx)
    u_ref, s_ref, _ = oracle_lib.heat_step(b.xy, b.normal, b.weights(), b.curvature, cfg["vol"],
                                           cfg["vol_w"], cfg["B"], cfg["f_next"], cfg["dt"], grid_h=cfg["h"], offsets=b.offset)
    assert st.outer_iters >= 1
    assert elem_err(host(u), u_ref) <= 1e-10
    assert elem_err(host(sig), s_ref) <= 1e-10


def test_warm_start_for_another_boundary_is_rejected(yk):
    """A warm start made for one boundary and attached to a heat step on
    another is refused with YK_ERR_ARG before any work (its feature kernels
    would index the other boundary's arrays with its own sizes)."""
    import torch
    c_small = W.config_c0(n_nodes=128, m=16)
    c_big = W.config_c0(n_nodes=256, m=16)
    ctx = yk.yk_create(direct=1)
    try:
        bd_small = yk.Boundary.from_workload(c_small["bnd"])
        bd_big = yk.Boundary.from_workload(c_big["bnd"])
        ws = yk.yk_ws_create(ctx, bd_small)
        try:
            yk.yk_set_warm_start(ctx, ws)
            n = c_big["vol"].shape[0]
            sig = torch.zeros(c_big["bnd"].n, dtype=torch.float64, device="cuda")
            u = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
            with pytest.raises(yk.YkError) as ei:
                yk.yk_heat_step(ctx, bd_big, dev(c_big["vol"]), dev(c_big["vol_w"]), dev(c_big["B"]),
                                yk.HEAT_GRID_SELF_CELL, dev(c_big["f_next"]), c_big["dt"], 1e-12, sig, u)
            assert ei.value.status == yk.YK_ERR_ARG
            assert "another boundary" in str(ei.value)
            assert torch.all(u == 7.0)
        finally:
            yk.yk_ws_destroy(ws)
    finally:
        yk.yk_destroy(ctx)


def test_heat_steps_are_bitwise_reproducible(yk, reduced_c3):
    """The same four steps (mixed precision, learned warm start trained after
    step 3, on the small-tree boundary operator whose sparse M2L sums its
    translations in a fixed order) in two fresh contexts give bitwise equal
    densities and solutions at every step."""
    import torch
    cfg, _ = reduced_c3
    b = cfg["bnd"]
    runs = []
    for rep in range(2):
        ctx = yk.yk_create(leaf_size=16, precision=yk.YK_PREC_MIXED)
        ws = None
        try:
            bd = yk.Boundary.from_workload(b)
            ws = yk.yk_ws_create(ctx, bd, steps=50)
            yk.yk_set_warm_start(ctx, ws)
            vol, w, f = dev(cfg["vol"]), dev(cfg["vol_w"]), dev(cfg["f_bnd"])
            region = torch.as_tensor(cfg["region"], dtype=torch.int32, device="cuda")
            u = dev(cfg["u0"])
            B, un = torch.empty_like(u), torch.empty_like(u)
            sig = torch.zeros(b.n, dtype=torch.float64, device="cuda")
            rec = []
            for step in range(1, 5):
                if step == 4:
                    yk.yk_ws_train(ws)
                print(f"reproducibility run {rep} step {step}", flush=True)
                yk.yk_rhs_backward_euler(ctx, u, None, region, cfg["consts"], cfg["dt"], B)
                st = yk.yk_heat_step(ctx, bd, vol, w, B, yk.HEAT_GRID_SELF_CELL, f, cfg["dt"], 1e-10, sig, un)
                rec.append((host(un).copy(), host(sig).copy(), st.iters, st.guess_used))
                u, un = un, u
            info = yk.yk_plan_info_get(ctx, 1)
        finally:
            if ws is not None:
                yk.yk_ws_destroy(ws)
            yk.yk_destroy(ctx)
        runs.append(rec)
    assert info.m2l_sparse == 1
    for (u0, s0, i0, g0), (u1, s1, i1, g1) in zip(*runs):
        assert i0 == i1 and g0 == g1
        assert np.array_equal(u0, u1) and np.array_equal(s0, s1)
