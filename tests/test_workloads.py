"""The seeded input generators that are not pinned elsewhere: the graded leaf
sets the box-code benchmark uses must tile the unit square and be 2:1
balanced (the library rejects any other leaf set)."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("lo,hi,radius", [(3, 7, 0.3), (4, 8, 0.21), (6, 10, 0.3)])
def test_graded_leaves_tile_and_balance(lo, hi, radius):
    lv, ix, iy = W.graded_leaves(centre=(0.5, 0.5), radius=radius, lo=lo, hi=hi)
    assert lv.min() >= lo and lv.max() == hi
    n = 1 << hi
    grid = np.full((n, n), -1, dtype=np.int16)
    for level in range(int(lv.min()), hi + 1):
        f = 1 << (hi - level)
        for a, b in zip(ix[lv == level], iy[lv == level]):
            cell = grid[b * f:(b + 1) * f, a * f:(a + 1) * f]
            assert (cell == -1).all()          # no overlap
            cell[...] = level
    assert (grid >= 0).all()                   # the square is covered
    g = grid.astype(int)
    # touching leaves (edges and corners) differ by at most one level
    assert np.abs(np.diff(g, axis=0)).max() <= 1
    assert np.abs(np.diff(g, axis=1)).max() <= 1
    assert np.abs(g[1:, 1:] - g[:-1, :-1]).max() <= 1
    assert np.abs(g[1:, :-1] - g[:-1, 1:]).max() <= 1


def test_leaf_cell_centres_layout():
    lv = np.array([1, 2], dtype=np.int32)
    ix = np.array([1, 0], dtype=np.int32)
    iy = np.array([0, 3], dtype=np.int32)
    c = W.leaf_cell_centres(lv, ix, iy)
    assert c.shape == (32, 2)
    # leaf 0: side 1/2 at (1/2, 0), cell t = jj 4 + ii of side 1/8
    assert np.allclose(c[0], [0.5 + 1 / 16, 1 / 16])
    assert np.allclose(c[5], [0.5 + 3 / 16, 3 / 16])
    # leaf 1: side 1/4 at (0, 3/4); its last cell
    assert np.allclose(c[31], [3.5 / 16, 0.75 + 3.5 / 16])
