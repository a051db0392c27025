"""Pins of the adaptive quad-tree reference (oracle/tree.py, build_adaptive)
by brute force on small sets: the refinement rule, 2:1 balance, the leaves'
partition of the points, and the classical completeness of the adaptive FMM
lists -- every (target leaf, source leaf) pair is reached by exactly one of
U, V (between ancestors), W and X, the rest lying beyond the far cut-off."""
import numpy as np
import pytest

from oracle import tree as T


def _case(seed=3, n=2500, cluster=400):
    rng = np.random.default_rng(seed)
    vol = rng.random((n, 2))
    vol[:cluster] = 0.3 + 0.02 * rng.random((cluster, 2))          # a dense cluster
    th = np.linspace(0, 6.2, 300)
    bnd = 0.5 + 0.3 * np.stack([np.cos(th), np.sin(th)], 1)
    tgt = rng.random((150, 2)) * 1.1 - 0.05
    sets = [vol, bnd, tgt]
    lo = np.min(np.concatenate(sets), 0)
    ext = np.max(np.max(np.concatenate(sets), 0) - lo) * (1 + 1e-9)
    return sets, (lo[0], lo[1], ext)


@pytest.fixture(scope="module", params=[(16, 1.0), (8, 0.002)])
def tree(request):
    s, alpha = request.param
    sets, sq = _case()
    return sets, sq, s, alpha, T.build_adaptive(sets, sq, s, alpha)


def _geom(t):
    x0, y0, sz = T._square_of(t["box_code"], t["box_level"])
    return x0, y0, sz


def _touch(g, a, b):
    x0, y0, sz = g
    return ((x0[a] <= x0[b] + sz[b]) & (x0[b] <= x0[a] + sz[a]) &
            (y0[a] <= y0[b] + sz[b]) & (y0[b] <= y0[a] + sz[a]))


def _gap(g, a, b):
    """Chebyshev gap between the closed squares of boxes a and b (level-15 units)."""
    x0, y0, sz = g
    gx = np.maximum(0, np.maximum(x0[a] - (x0[b] + sz[b]), x0[b] - (x0[a] + sz[a])))
    gy = np.maximum(0, np.maximum(y0[a] - (y0[b] + sz[b]), y0[b] - (y0[a] + sz[a])))
    return np.maximum(gx, gy)


def _points_in(t, k):
    lr = t["leaf_range"][k]
    return sum(int(lr[2 * s + 1] - lr[2 * s]) for s in range(3))


def test_refinement_rule_and_minimal_balance(tree):
    sets, sq, s, alpha, t = tree
    lev, code = t["box_level"], t["box_code"]
    # a leaf holds at most s points unless it is at the finest level
    for k, b in enumerate(t["leaf_box"]):
        assert _points_in(t, k) <= s or lev[b] == T.MAX_LEVEL
    # each split box either holds more than s points or touches an existing
    # box two levels finer (its split was forced by the balance)
    codes15 = (t["keys"] & np.uint32(0x3FFFFFFF)).astype(np.uint64)
    g = _geom(t)
    for b in np.flatnonzero(~t["is_leaf"]):
        n = np.sum((codes15 >> np.uint64(2 * (T.MAX_LEVEL - lev[b]))) == np.uint64(code[b]))
        if n > s:
            continue
        finer = np.flatnonzero(lev == lev[b] + 2)
        assert np.any(_touch(g, finer, np.full(finer.size, b))), b
    # every split box has at least one child, every child's parent is split
    par = t["parent"]
    assert np.all(~t["is_leaf"][par[par >= 0]])
    assert set(np.flatnonzero(~t["is_leaf"])) <= set(par[par >= 0])


def test_touching_leaves_differ_by_at_most_one_level(tree):
    sets, sq, s, alpha, t = tree
    g = _geom(t)
    lb = t["leaf_box"]
    T_ = _touch(g, lb[:, None], lb[None, :])
    dl = np.abs(t["box_level"][lb][:, None] - t["box_level"][lb][None, :])
    assert np.all(dl[T_] <= 1)
    # hence at most 12 neighbours besides the leaf itself
    assert np.diff(t["ulist_off"]).max() <= 13


def test_leaves_partition_the_points(tree):
    sets, sq, s, alpha, t = tree
    N = len(t["keys"])
    cover = np.zeros(N, dtype=np.int64)
    codes15 = (t["keys"] & np.uint32(0x3FFFFFFF)).astype(np.uint64)
    for k, b in enumerate(t["leaf_box"]):
        lev = t["box_level"][b]
        for st in range(3):
            a, e = t["leaf_range"][k, 2 * st], t["leaf_range"][k, 2 * st + 1]
            cover[a:e] += 1
            assert np.all((t["keys"][a:e] >> np.uint32(30)) == st)
            assert np.all((codes15[a:e] >> np.uint64(2 * (T.MAX_LEVEL - lev))) == np.uint64(t["box_code"][b]))
    assert np.all(cover == 1)
    # leaves are disjoint and in Morton order of their first cell
    lev = t["box_level"][t["leaf_box"]].astype(np.uint64)
    first = t["box_code"][t["leaf_box"]].astype(np.uint64) << (np.uint64(2) * (np.uint64(T.MAX_LEVEL) - lev))
    size = np.uint64(1) << (np.uint64(2) * (np.uint64(T.MAX_LEVEL) - lev))
    assert np.all(first[1:] >= first[:-1] + size[:-1])


def _anc(t, b):
    out = []
    while b >= 0:
        out.append(int(b))
        b = t["parent"][b]
    return out


def test_lists_reach_every_leaf_pair_exactly_once(tree):
    sets, sq, s, alpha, t = tree
    g = _geom(t)
    lb = t["leaf_box"]
    nleaf = len(lb)
    lev = t["box_level"]
    anc = [_anc(t, b) for b in lb]
    box_leaf = -np.ones(len(lev), dtype=np.int64)
    box_leaf[lb] = np.arange(nleaf)
    V = [set(v[v >= 0].tolist()) for v in t["vlist"]]
    W = [set(t["wlist"][t["wlist_off"][k]:t["wlist_off"][k + 1]].tolist()) for k in range(nleaf)]
    X = {int(d): set(t["xlist"][t["xlist_off"][i]:t["xlist_off"][i + 1]].tolist()) for i, d in enumerate(t["xbox"])}
    U = [set(t["ulist"][t["ulist_off"][k]:t["ulist_off"][k + 1]].tolist()) for k in range(nleaf)]
    side15 = float(1 << T.MAX_LEVEL)
    cut = 40.0 * alpha * side15 / sq[2]          # the far cut-off in level-15 units
    for kb in range(nleaf):
        ab = anc[kb]
        by_level_b = {int(lev[a]): a for a in ab}
        for kc in range(nleaf):
            ac = anc[kc]
            n = int(kc in U[kb])
            n += sum(1 for e in ac if int(lev[e]) in by_level_b and e in V[by_level_b[int(lev[e])]])
            n += sum(1 for e in ac if e in W[kb])
            n += sum(1 for a in ab if kc in X.get(a, ()))
            if n == 0:
                # only pairs beyond the cut-off may be left out
                assert t["lmin"] > 2 and _gap(g, lb[kb], lb[kc]) >= cut, (kb, kc)
            else:
                assert n == 1, (kb, kc, n)


def test_w_and_x_pairs_are_separated_and_one_level_apart_at_least(tree):
    sets, sq, s, alpha, t = tree
    g = _geom(t)
    lev = t["box_level"]
    for k, b in enumerate(t["leaf_box"]):
        w = t["wlist"][t["wlist_off"][k]:t["wlist_off"][k + 1]]
        if w.size:
            assert np.all(lev[w] > lev[b]) and np.all(lev[w] >= t["lmin"])
            # at least one box of the finer size between them
            assert np.all(_gap(g, w, np.full(w.size, b)) >= (1 << (T.MAX_LEVEL - lev[w])))
            assert np.all(_touch(g, t["parent"][w], np.full(w.size, b)))
    for i, d in enumerate(t["xbox"]):
        x = t["xlist"][t["xlist_off"][i]:t["xlist_off"][i + 1]]
        k = np.searchsorted(t["xbox"], d)
        assert k == i
        for c in x:
            w = t["wlist"][t["wlist_off"][c]:t["wlist_off"][c + 1]]
            assert d in w


def test_uniform_points_give_one_leaf_level():
    # a 64 x 64 lattice of cell centres with 4 points per leaf at level 5:
    # every box splits to the same depth, no balance refinement
    n = 64
    g = (np.arange(n) + 0.5) / n
    xy = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    t = T.build_adaptive([xy, np.zeros((0, 2)), np.zeros((0, 2))], (0.0, 0.0, 1.0), 4, 1.0)
    assert np.all(t["box_level"][t["leaf_box"]] == 5) and len(t["leaf_box"]) == 1024
    assert len(t["xbox"]) == 0 and len(t["wlist"]) == 0
    ref = T.build([xy, np.zeros((0, 2)), np.zeros((0, 2))], (0.0, 0.0, 1.0), 4, 1.0)
    # the same leaves as the uniform tree at level 5 (Morton order), the same
    # U lists (the uniform tree keeps them in row order, the adaptive one sorted)
    assert ref["leaf_level"] == 5
    assert np.array_equal(t["box_code"][t["leaf_box"]], ref["box_code"][ref["level_begin"][5]:])
    assert np.array_equal(t["ulist_off"], ref["ulist_off"])
    for k in range(1024):
        a, e = t["ulist_off"][k], t["ulist_off"][k + 1]
        assert np.array_equal(t["ulist"][a:e], np.sort(ref["ulist"][a:e]))
