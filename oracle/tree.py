"""Plain numpy quad-tree and FMM interaction lists -- TEST INFRASTRUCTURE ONLY.

Only the tests may import this module.  It shares no code with the GPU
library.  From point coordinates and a bounding square it builds, by the
definitions (Sec. 3.1's quad-tree; the classical FMM lists):

  * keys: the level-15 cell (ix, iy) = floor((x - x0) 2^15 / side), clamped
    to [0, 2^15), interleaved into a Morton code (x bits even, y bits odd),
    with the point set id (0 charges, 1 nodes, 2 targets) above bit 30;
  * the stable sort of the keys (so each set is one block, Morton-ordered);
  * the leaf level: the smallest level whose point-weighted occupancy
    sum_i n_i^2 / N (n_i the points per non-empty box) is at most the leaf size;
  * the non-empty boxes of every level down to the leaf level, sorted by code,
    with their parents;
  * per leaf and set, the range of sorted positions it owns;
  * U lists (the non-empty leaves of a leaf's 3 x 3 block, row by row) and
    V lists (27 slots per box: the 6 x 6 block of the parent's neighbours'
    children minus the box's own 3 x 3 block, row by row, -1 where empty).
"""
from __future__ import annotations

import numpy as np

MAX_LEVEL = 15


def spread(v):
    """Interleave the 15 low bits of v with zeros (bit k -> bit 2k)."""
    v = np.asarray(v, dtype=np.uint64)
    out = np.zeros_like(v)
    for k in range(MAX_LEVEL):
        out |= ((v >> np.uint64(k)) & np.uint64(1)) << np.uint64(2 * k)
    return out


def compact(c):
    """Inverse of spread: the even bits of c packed together."""
    c = np.asarray(c, dtype=np.uint64)
    out = np.zeros_like(c)
    for k in range(MAX_LEVEL):
        out |= ((c >> np.uint64(2 * k)) & np.uint64(1)) << np.uint64(k)
    return out


def morton(ix, iy):
    return (spread(ix) | (spread(iy) << np.uint64(1))).astype(np.uint64)


def keys_of(sets, square):
    """Keys of the concatenated point sets [(n_s, 2) arrays] for the square (x0, y0, side)."""
    x0, y0, side = square
    inv = float(1 << MAX_LEVEL) / side
    out = []
    for s, xy in enumerate(sets):
        xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
        ix = np.clip(np.floor((xy[:, 0] - x0) * inv), 0, (1 << MAX_LEVEL) - 1).astype(np.int64)
        iy = np.clip(np.floor((xy[:, 1] - y0) * inv), 0, (1 << MAX_LEVEL) - 1).astype(np.int64)
        out.append((np.uint64(s) << np.uint64(30)) | morton(ix, iy))
    return np.concatenate(out).astype(np.uint32)


def build(sets, square, leaf_size, alpha, far_cut=40.0):
    """The tree of the point sets; see the module docstring."""
    keys = keys_of(sets, square)
    n_set = [len(np.asarray(x).reshape(-1, 2)) for x in sets]
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    set_start = np.concatenate([[0], np.cumsum(n_set)])
    perm = order - set_start[(skeys >> np.uint32(30)).astype(np.int64)]
    codes15 = (skeys & np.uint32(0x3FFFFFFF)).astype(np.uint64)
    N = len(skeys)
    # leaf level by point-weighted occupancy
    L = MAX_LEVEL
    for lev in range(MAX_LEVEL + 1):
        _, cnt = np.unique(codes15 >> np.uint64(2 * (MAX_LEVEL - lev)), return_counts=True)
        if np.sum(cnt.astype(np.float64) ** 2) / N <= leaf_size:
            L = lev
            break
    # boxes per level
    level_codes = [np.unique(codes15 >> np.uint64(2 * (MAX_LEVEL - lev))) for lev in range(L + 1)]
    level_begin = np.concatenate([[0], np.cumsum([len(c) for c in level_codes])]).astype(np.int64)
    box_code = np.concatenate(level_codes).astype(np.uint32)
    parent = np.full(len(box_code), -1, dtype=np.int32)
    for lev in range(1, L + 1):
        idx = np.searchsorted(level_codes[lev - 1], level_codes[lev] >> np.uint64(2))
        parent[level_begin[lev]:level_begin[lev + 1]] = level_begin[lev - 1] + idx
    # leaf ranges per set
    leaf = level_codes[L]
    nleaf = len(leaf)
    lrange = np.zeros((nleaf, 6), dtype=np.int32)
    lc = codes15 >> np.uint64(2 * (MAX_LEVEL - L))
    li = np.searchsorted(leaf, lc)
    st = (skeys >> np.uint32(30)).astype(np.int64)
    change = np.concatenate([[True], (st[1:] != st[:-1]) | (li[1:] != li[:-1])])
    first = np.flatnonzero(change)                      # first sorted position of each (set, leaf) run
    last = np.concatenate([first[1:], [N]])             # one past its last
    lrange[li[first], 2 * st[first]] = first
    lrange[li[first], 2 * st[first] + 1] = last
    # lists
    def lookup(lev, jx, jy):
        """Index (within the level) of the boxes at (jx, jy), -1 where absent."""
        ns = 1 << lev
        ok = (jx >= 0) & (jy >= 0) & (jx < ns) & (jy < ns)
        c = morton(np.where(ok, jx, 0), np.where(ok, jy, 0))
        pos = np.searchsorted(level_codes[lev], c)
        pos_c = np.minimum(pos, len(level_codes[lev]) - 1)
        hit = ok & (level_codes[lev][pos_c] == c)
        return np.where(hit, pos_c, -1)
    lx, ly = compact(leaf).astype(np.int64), compact(leaf >> np.uint64(1)).astype(np.int64)
    cols = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            cols.append(lookup(L, lx + dx, ly + dy))
    cols = np.stack(cols, axis=1)
    ulist_off = np.zeros(nleaf + 1, dtype=np.int32)
    ulist_off[1:] = np.cumsum((cols >= 0).sum(axis=1))
    ulist = cols[cols >= 0].astype(np.int32)          # row-major: each leaf's 3 x 3 in order
    lmin = 2
    while lmin <= L and square[2] / (1 << lmin) >= far_cut * alpha:
        lmin += 1
    vlist = np.full((len(box_code), 27), -1, dtype=np.int32)
    for lev in range(max(lmin, 2), L + 1):
        c = level_codes[lev]
        ix, iy = compact(c).astype(np.int64), compact(c >> np.uint64(1)).astype(np.int64)
        cxs, cys = ix & 1, iy & 1
        # the 6 x 6 block of the parent's neighbours' children, row by row,
        # relative to the box: offsets -2 - c .. 3 - c in each direction
        cand, near = [], []
        for ody in range(6):
            for odx in range(6):
                dx, dy = odx - 2 - cxs, ody - 2 - cys
                j = lookup(lev, ix + dx, iy + dy)
                cand.append(np.where(j >= 0, level_begin[lev] + j, -1))
                near.append((np.abs(dx) <= 1) & (np.abs(dy) <= 1))
        cand, near = np.stack(cand, axis=1), np.stack(near, axis=1)   # [nb, 36]
        assert np.all(near.sum(axis=1) == 9)
        vlist[level_begin[lev]:level_begin[lev + 1]] = cand[~near].reshape(len(c), 27)
    return dict(keys=skeys, perm=perm.astype(np.int32), leaf_level=L, lmin=lmin, level_begin=level_begin,
                box_code=box_code, parent=parent, leaf_range=lrange, ulist_off=ulist_off, ulist=ulist,
                vlist=vlist)
