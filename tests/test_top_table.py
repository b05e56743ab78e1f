"""Host-side model of the top-table flags the library builds (no GPU).

The GPU tests check the flags' effect; this test pins the rule itself on
trees where the table level equals the depth, where the last finest cell of
a coarse leaf has exactly one leaf in its one-cell table cell."""

import numpy as np

import workloads as W

FULL, ONE, INDEX = 0x80000000, 0x40000000, 0x3FFFFFFF


def build_table(tree, lt):
    """Python statement of the table: entry = leaf holding the cell's first
    finest cell, flagged FULL (cell refined to depth D) or ONE (one leaf
    covers the cell)."""
    D = tree.depth
    shift = 3 * (D - lt)
    base = np.arange(8 ** lt + 1, dtype=np.uint64) << np.uint64(shift)
    top = np.searchsorted(tree.keys, base[:-1], side="right") - 1
    top = np.append(top, tree.n).astype(np.int64)
    flags = np.zeros(8 ** lt, dtype=np.int64)
    for c in range(8 ** lt):
        lo, nx = top[c], top[c + 1]
        if nx - lo == 1 << shift and tree.levels[lo] == D:
            flags[c] = FULL
        elif tree.levels[lo] <= lt:
            flags[c] = ONE
    return top, flags


def lookup(tree, top, flags, lt, k):
    D = tree.depth
    shift = 3 * (D - lt)
    c = k >> shift
    lo = top[c]
    if flags[c] == FULL:
        return lo + (k & ((1 << shift) - 1)), D
    if flags[c] != ONE:
        hi = top[c + 1]
        lo = lo + int(np.searchsorted(tree.keys[lo:hi], np.uint64(k), side="right")) - 1
    return lo, int(tree.levels[lo])


def test_flags_match_the_plain_lookup():
    for seed, D, p in ((2, 3, 0.7), (5, 4, 0.4), (9, 3, 0.2)):
        t = W.random_octree(D, p, seed, min_level=1)
        for lt in range(0, D + 1):
            top, flags = build_table(t, lt)
            for k in range(8 ** D):
                want = int(np.searchsorted(t.keys, np.uint64(k), side="right")) - 1
                got, lvl = lookup(t, top, flags, lt, k)
                assert got == want and lvl == t.levels[want], (seed, D, lt, k)
