"""The library's quad-tree (keys, sort, leaf level, boxes, parents, leaf ranges,
U and V lists, built by the GPU kernels) against the numpy reference, bit for
bit: this is integer work."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1007_5335_amd.yk as yk
    yk.load_library()
    return yk


def _compare(got, ref):
    assert got["leaf_level"] == ref["leaf_level"] and got["lmin"] == ref["lmin"]
    for k in ("keys", "perm", "level_begin", "box_code", "parent", "leaf_range", "ulist_off", "ulist", "vlist"):
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        bad = np.flatnonzero((a != b).ravel())
        assert bad.size == 0, (k, bad[:5], a.ravel()[bad[:5]], b.ravel()[bad[:5]])


def _square_ok(sets, sq):
    pts = np.concatenate([np.asarray(s).reshape(-1, 2) for s in sets])
    x0, y0, side = sq
    assert np.all(pts[:, 0] >= x0) and np.all(pts[:, 1] >= y0)
    assert np.all(pts[:, 0] <= x0 + side) and np.all(pts[:, 1] <= y0 + side)
    ext = np.max(pts.max(0) - pts.min(0))
    assert ext <= side <= ext * (1 + 1e-8)


@pytest.mark.parametrize("case", ["uniform", "clustered_targets", "c1_full"])
def test_tree_and_lists_match_reference(yk, case):
    import torch
    from oracle import tree as T
    if case == "c1_full":
        c = W.config_c1()
        alpha, leaf = c["alpha"], 64
    else:
        c = W.small_fmm_case(n_vol=20000, n_nodes=512, alpha=0.02, seed=31, clustered=case != "uniform")
        alpha, leaf = 0.02, 16
    b = c["bnd"]
    ctx = yk.yk_create(leaf_size=leaf, p=8, near_cache_mb=0, tree=yk.YK_TREE_UNIFORM)
    try:
        print(f"tree {case}: {c['vol'].shape[0]} + {b.n} points", flush=True)
        if case == "clustered_targets":
            # charges and separate targets (sets 0 and 2) through the stand-alone sum
            rng = np.random.default_rng(5)
            tgt = rng.random((3000, 2)) * 1.2 - 0.1
            out = torch.empty(3000, dtype=torch.float64, device="cuda")
            yk.yk_volume_potential(ctx, dev(c["vol"]), dev(c["q"]), dev(tgt), alpha, out)
            slot, sets = 2, [c["vol"], np.zeros((0, 2)), tgt]
        else:
            bd = yk.Boundary.from_workload(b)
            ov = torch.empty(c["vol"].shape[0], dtype=torch.float64, device="cuda")
            ob = torch.empty(b.n, dtype=torch.float64, device="cuda")
            yk.yk_fmm_potential(ctx, dev(c["vol"]), dev(c["q"]), bd, dev(c["dip"]), alpha, ov, ob)
            slot, sets = 0, [c["vol"], b.xy]
        torch.cuda.synchronize()
        got = yk.yk_plan_tree_export(ctx, slot)
        info = yk.yk_plan_info_get(ctx, slot)
    finally:
        yk.yk_destroy(ctx)
    _square_ok(sets, got["square"])
    ref = T.build(sets, got["square"], leaf, alpha)
    print(f"  leaf level {info.leaf_level}, {info.n_boxes} boxes, {info.n_leaves} leaves, "
          f"{info.n_ulist} U entries, build {info.build_ms:.1f} ms", flush=True)
    _compare(got, ref)
