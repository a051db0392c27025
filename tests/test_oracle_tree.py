"""Pins of the numpy quad-tree reference (oracle/tree.py) by brute force:
Morton interleaving, the stable order, leaf ranges, parents, and the U and V
lists checked pair by pair against their geometric definitions."""
import numpy as np
import pytest

from oracle import tree as T


def test_morton_interleaving_small_values_and_round_trip():
    assert int(T.morton(1, 0)) == 1 and int(T.morton(0, 1)) == 2
    assert int(T.morton(3, 3)) == 15 and int(T.morton(2, 0)) == 4 and int(T.morton(0, 2)) == 8
    rng = np.random.default_rng(0)
    v = rng.integers(0, 1 << 15, 1000)
    assert np.array_equal(T.compact(T.spread(v)), v)
    ix, iy = rng.integers(0, 1 << 15, 1000), rng.integers(0, 1 << 15, 1000)
    c = T.morton(ix, iy)
    assert np.array_equal(T.compact(c), ix) and np.array_equal(T.compact(c >> np.uint64(1)), iy)


@pytest.fixture(scope="module")
def small_tree():
    rng = np.random.default_rng(3)
    vol = rng.random((2500, 2))
    vol[:400] = 0.3 + 0.02 * rng.random((400, 2))          # a dense cluster
    bnd = 0.5 + 0.3 * np.stack([np.cos(np.linspace(0, 6.2, 300)), np.sin(np.linspace(0, 6.2, 300))], 1)
    tgt = rng.random((150, 2)) * 1.1 - 0.05
    sets = [vol, bnd, tgt]
    lo = np.min(np.concatenate(sets), 0)
    ext = np.max(np.max(np.concatenate(sets), 0) - lo) * (1 + 1e-9)
    sq = (lo[0], lo[1], ext)
    return sets, sq, T.build(sets, sq, 16, 0.004)


def _cell(t, b, lev):
    c = np.uint64(t["box_code"][b])
    return int(T.compact(c)), int(T.compact(c >> np.uint64(1)))


def _level_of(t, b):
    return int(np.searchsorted(t["level_begin"], b, side="right") - 1)


def test_order_is_stable_and_perm_maps_back(small_tree):
    sets, sq, t = small_tree
    raw = T.keys_of(sets, sq)
    starts = np.concatenate([[0], np.cumsum([len(s) for s in sets])])
    sid = (t["keys"] >> np.uint32(30)).astype(np.int64)
    assert np.all(np.diff(t["keys"].astype(np.int64)) >= 0)
    assert np.array_equal(raw[starts[sid] + t["perm"]], t["keys"])
    # within equal keys, increasing original index (stable)
    g = starts[sid] + t["perm"]
    same = t["keys"][1:] == t["keys"][:-1]
    assert np.all(g[1:][same] > g[:-1][same])


def test_leaf_ranges_cover_every_point_once(small_tree):
    sets, sq, t = small_tree
    L = t["leaf_level"]
    lr = t["leaf_range"]
    owner = np.full(len(t["keys"]), -1)
    for li in range(lr.shape[0]):
        for s in range(3):
            a, b = lr[li, 2 * s], lr[li, 2 * s + 1]
            assert np.all(owner[a:b] == -1)
            owner[a:b] = li
            codes = (t["keys"][a:b] & np.uint32(0x3FFFFFFF)).astype(np.uint64) >> np.uint64(2 * (15 - L))
            assert np.all(codes == t["box_code"][t["level_begin"][L] + li])
            assert np.all((t["keys"][a:b] >> np.uint32(30)) == s)
    assert np.all(owner >= 0)


def test_parents_hold_their_children(small_tree):
    _, _, t = small_tree
    for b in range(t["level_begin"][1], len(t["box_code"])):
        p = t["parent"][b]
        assert _level_of(t, p) == _level_of(t, b) - 1
        assert int(t["box_code"][p]) == int(t["box_code"][b]) >> 2


def test_ulists_are_the_adjacent_leaves_both_ways(small_tree):
    _, _, t = small_tree
    L = t["leaf_level"]
    nl = len(t["ulist_off"]) - 1
    cells = [_cell(t, t["level_begin"][L] + i, L) for i in range(nl)]
    for i in range(nl):
        got = list(t["ulist"][t["ulist_off"][i]:t["ulist_off"][i + 1]])
        want = [j for j in range(nl)
                if max(abs(cells[j][0] - cells[i][0]), abs(cells[j][1] - cells[i][1])) <= 1]
        # row by row: sorted by (dy, dx)
        key = lambda j: (cells[j][1] - cells[i][1], cells[j][0] - cells[i][0])
        assert got == sorted(want, key=key)
        assert i in got
        for j in got:
            assert i in t["ulist"][t["ulist_off"][j]:t["ulist_off"][j + 1]]


def test_vlists_are_the_separated_children_of_the_parents_neighbours(small_tree):
    _, _, t = small_tree
    lb = t["level_begin"]
    for lev in range(max(t["lmin"], 2), t["leaf_level"] + 1):
        boxes = range(lb[lev], lb[lev + 1])
        cells = {b: _cell(t, b, lev) for b in boxes}
        for b in boxes:
            bx, by = cells[b]
            want = set()
            for j in boxes:
                jx, jy = cells[j]
                parent_adjacent = max(abs(jx // 2 - bx // 2), abs(jy // 2 - by // 2)) <= 1
                if parent_adjacent and max(abs(jx - bx), abs(jy - by)) > 1:
                    want.add(j)
            got = [v for v in t["vlist"][b] if v >= 0]
            assert len(got) == len(set(got))
            assert set(got) == want
    for b in range(lb[max(t["lmin"], 2)]):
        assert np.all(t["vlist"][b] == -1)
