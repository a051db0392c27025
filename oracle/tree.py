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

build_adaptive() gives the adaptive form of Sec. 3.1's quad-tree (boxes
refined box by box, childless boxes at any level) with the lists of the
adaptive FMM:

  * a box is split while it holds more than max_points points (level 15 at
    most); then, until nothing changes, a leaf is split when an existing box
    two levels finer touches it (2:1 balance: touching leaves differ by at
    most one level);
  * leaves are numbered in Morton order of their first level-15 cell;
  * U(b), b a leaf: the leaves touching b, b itself included;
  * V(b): as above, among the existing boxes of b's level;
  * W(b), b a leaf: the boxes d finer than b whose parent touches b and which
    do not touch b themselves (the far part of the colleagues' subtrees);
  * X(d): the leaves b with d in W(b).
"Touch" is the intersection of the closed squares.  Lists are sorted by
index; W and X keep only boxes at levels >= lmin (coarser pairs are further
apart than the far cut-off).
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


def _square_of(code, lev):
    """Level-15 integer extent [x0, x0 + size] x [y0, y0 + size] of boxes (code, lev)."""
    code = np.asarray(code, dtype=np.uint64)
    k = MAX_LEVEL - np.asarray(lev, dtype=np.int64)
    x0 = compact(code).astype(np.int64) << k
    y0 = compact(code >> np.uint64(1)).astype(np.int64) << k
    return x0, y0, np.left_shift(np.int64(1), k)


def build_adaptive(sets, square, max_points, alpha, far_cut=40.0):
    """The adaptive tree of the point sets; see the module docstring."""
    keys = keys_of(sets, square)
    n_set = [len(np.asarray(x).reshape(-1, 2)) for x in sets]
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    set_start = np.concatenate([[0], np.cumsum(n_set)])
    perm = order - set_start[(skeys >> np.uint32(30)).astype(np.int64)]
    codes15 = (skeys & np.uint32(0x3FFFFFFF)).astype(np.uint64)
    N = len(skeys)
    # non-empty boxes of every level and their point counts
    codes, counts = [], []
    for lev in range(MAX_LEVEL + 1):
        c, n = np.unique(codes15 >> np.uint64(2 * (MAX_LEVEL - lev)), return_counts=True)
        codes.append(c)
        counts.append(n)
    # state per non-empty box: 0 not in the tree (inside a leaf), 1 leaf, 2 split
    ABSENT, LEAF, SPLIT = 0, 1, 2
    state = []
    for lev in range(MAX_LEVEL + 1):
        if lev == 0:
            exists = np.ones(len(codes[0]), dtype=bool)
        else:
            par = np.searchsorted(codes[lev - 1], codes[lev] >> np.uint64(2))
            exists = state[lev - 1][par] == SPLIT
        split = (counts[lev] > max_points) & (lev < MAX_LEVEL)
        state.append(np.where(exists, np.where(split, SPLIT, LEAF), ABSENT).astype(np.int8))

    def exists_at(lev, jx, jy):
        ns = 1 << lev
        ok = (jx >= 0) & (jy >= 0) & (jx < ns) & (jy < ns)
        c = morton(np.where(ok, jx, 0), np.where(ok, jy, 0))
        pos = np.minimum(np.searchsorted(codes[lev], c), len(codes[lev]) - 1)
        return ok & (codes[lev][pos] == c) & (state[lev][pos] != ABSENT)

    # 2:1 balance: the 20 cells two levels finer that ring a leaf touch it
    ring = [(i, j) for j in range(-1, 5) for i in range(-1, 5) if not (0 <= i <= 3 and 0 <= j <= 3)]
    changed = True
    while changed:
        changed = False
        for lev in range(MAX_LEVEL - 1):
            idx = np.flatnonzero(state[lev] == LEAF)
            if idx.size == 0:
                continue
            bx = compact(codes[lev][idx]).astype(np.int64)
            by = compact(codes[lev][idx] >> np.uint64(1)).astype(np.int64)
            hit = np.zeros(idx.size, dtype=bool)
            for i, j in ring:
                hit |= exists_at(lev + 2, 4 * bx + i, 4 * by + j)
            if not hit.any():
                continue
            changed = True
            state[lev][idx[hit]] = SPLIT
            par = np.searchsorted(codes[lev], codes[lev + 1] >> np.uint64(2))
            newly = np.isin(par, idx[hit])
            state[lev + 1][newly] = LEAF   # their counts are at most the parent's
    # the tree: existing boxes per level (down to the deepest one present)
    L = max(lev for lev in range(MAX_LEVEL + 1) if np.any(state[lev] != ABSENT))
    level_codes = [codes[lev][state[lev] != ABSENT] for lev in range(L + 1)]
    level_state = [state[lev][state[lev] != ABSENT] for lev in range(L + 1)]
    level_begin = np.concatenate([[0], np.cumsum([len(c) for c in level_codes])]).astype(np.int64)
    box_code = np.concatenate(level_codes).astype(np.uint32)
    box_level = np.concatenate([np.full(len(c), lev) for lev, c in enumerate(level_codes)]).astype(np.int64)
    is_leaf = np.concatenate(level_state) == LEAF
    nbox = len(box_code)
    parent = np.full(nbox, -1, dtype=np.int32)
    for lev in range(1, L + 1):
        idx = np.searchsorted(level_codes[lev - 1], level_codes[lev] >> np.uint64(2))
        parent[level_begin[lev]:level_begin[lev + 1]] = level_begin[lev - 1] + idx
    # leaves in Morton order of their first level-15 cell
    lb = np.flatnonzero(is_leaf)
    start = box_code[lb].astype(np.uint64) << (np.uint64(2) * (MAX_LEVEL - box_level[lb]).astype(np.uint64))
    o = np.argsort(start, kind="stable")
    leaf_box = lb[o].astype(np.int32)
    start = start[o]
    nleaf = len(leaf_box)
    # each point's leaf, and the leaves' ranges per set
    li = np.searchsorted(start, codes15, side="right") - 1
    lrange = np.zeros((nleaf, 6), dtype=np.int32)
    st = (skeys >> np.uint32(30)).astype(np.int64)
    change = np.concatenate([[True], (st[1:] != st[:-1]) | (li[1:] != li[:-1])])
    first = np.flatnonzero(change)
    last = np.concatenate([first[1:], [N]])
    lrange[li[first], 2 * st[first]] = first
    lrange[li[first], 2 * st[first] + 1] = last
    # geometry of every box in level-15 units
    bx0, by0, bsz = _square_of(box_code, box_level)

    def touch(a, b):
        """Closed squares of boxes a and b (index arrays, broadcast) intersect."""
        return ((bx0[a] <= bx0[b] + bsz[b]) & (bx0[b] <= bx0[a] + bsz[a]) &
                (by0[a] <= by0[b] + bsz[b]) & (by0[b] <= by0[a] + bsz[a]))

    lmin = 2
    while lmin <= L and square[2] / (1 << lmin) >= far_cut * alpha:
        lmin += 1
    # U: touching leaves
    T = touch(leaf_box[:, None], leaf_box[None, :])
    ulist_off = np.zeros(nleaf + 1, dtype=np.int32)
    ulist_off[1:] = np.cumsum(T.sum(axis=1))
    ulist = np.nonzero(T)[1].astype(np.int32)          # row by row, ascending within a row
    # V: as in the uniform tree, among the existing boxes of each level
    vlist = np.full((nbox, 27), -1, dtype=np.int32)
    for lev in range(max(lmin, 2), L + 1):
        c = level_codes[lev]
        if len(c) == 0:
            continue
        ix, iy = compact(c).astype(np.int64), compact(c >> np.uint64(1)).astype(np.int64)
        cxs, cys = ix & 1, iy & 1
        cand, near = [], []
        for ody in range(6):
            for odx in range(6):
                dx, dy = odx - 2 - cxs, ody - 2 - cys
                jx, jy = ix + dx, iy + dy
                ns = 1 << lev
                ok = (jx >= 0) & (jy >= 0) & (jx < ns) & (jy < ns)
                cc = morton(np.where(ok, jx, 0), np.where(ok, jy, 0))
                pos = np.minimum(np.searchsorted(c, cc), len(c) - 1)
                hit = ok & (c[pos] == cc)
                cand.append(np.where(hit, level_begin[lev] + pos, -1))
                near.append((np.abs(dx) <= 1) & (np.abs(dy) <= 1))
        cand, near = np.stack(cand, axis=1), np.stack(near, axis=1)
        vlist[level_begin[lev]:level_begin[lev + 1]] = cand[~near].reshape(len(c), 27)
    # W: boxes finer than the leaf whose parent touches it and which do not
    d_all = np.arange(nbox)
    has_par = parent >= 0
    W = np.zeros((nleaf, nbox), dtype=bool)
    for k, b in enumerate(leaf_box):
        cand = has_par & (box_level > box_level[b]) & (box_level >= lmin)
        pt = np.zeros(nbox, dtype=bool)
        pt[has_par] = touch(np.maximum(parent[has_par], 0), np.full(has_par.sum(), b))
        W[k] = cand & pt & ~touch(d_all, np.full(nbox, b))
    wlist_off = np.zeros(nleaf + 1, dtype=np.int32)
    wlist_off[1:] = np.cumsum(W.sum(axis=1))
    wlist = np.nonzero(W)[1].astype(np.int32)
    # X: the transpose of W
    WT = W.T
    xbox = np.flatnonzero(WT.any(axis=1)).astype(np.int32)
    xlist_off = np.zeros(len(xbox) + 1, dtype=np.int32)
    xlist_off[1:] = np.cumsum(WT[xbox].sum(axis=1))
    xlist = np.nonzero(WT[xbox])[1].astype(np.int32)
    return dict(keys=skeys, perm=perm.astype(np.int32), leaf_level=L, lmin=lmin, level_begin=level_begin,
                box_code=box_code, box_level=box_level, parent=parent, is_leaf=is_leaf, leaf_box=leaf_box,
                leaf_range=lrange, ulist_off=ulist_off, ulist=ulist, vlist=vlist, wlist_off=wlist_off,
                wlist=wlist, xbox=xbox, xlist_off=xlist_off, xlist=xlist,
                point_leaf=li.astype(np.int32), counts=(codes, counts))
