"""Leaf-only linear octrees over the unit box (the paper's contribution grid).

The contribution grid is an AMR Cartesian grid stored as compact arrays of
its leaves only: Morton key, refinement level and cell value (paper
Sec. 2.3.1).  Conventions used throughout this repository:

* the tree has a global maximum depth D (1 <= D <= 21); a cell at level L has
  edge 2**(D-L) in units of the finest cell h = 2**-D;
* a leaf's key is the Morton code, at depth D, of its minimum corner: bit b of
  the integer x coordinate goes to key bit 3b, y to 3b+1, z to 3b+2;
* leaves are sorted by key and tile [0, 8**D) without gaps or overlaps, so
  leaf i covers the key range [key[i], key[i] + 8**(D-level[i])).

This module only *constructs* such arrays (from a density field and a
refinement rule, sec. 2.3.1 and sec. 2.4's density/uniformity criterion); it
does not search or walk them.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Octree:
    depth: int                 # global maximum depth D
    keys: np.ndarray           # uint64 [n], sorted ascending
    levels: np.ndarray         # uint8 [n]
    rho: np.ndarray            # float64 [n], cell value (volume mean)
    info: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.keys.shape[0])

    def anchors(self):
        """Integer minimum corners [n, 3] at depth D."""
        return morton_decode(self.keys, self.depth)

    def sizes(self):
        """Edge length of every leaf in finest cells (int64 [n])."""
        return np.left_shift(np.int64(1), (self.depth - self.levels.astype(np.int64)))


def morton_encode(ix, iy, iz, nbits):
    """Interleave nbits bits of three integer arrays into uint64 Morton keys."""
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    key = np.zeros(np.broadcast(ix, iy, iz).shape, dtype=np.uint64)
    one = np.uint64(1)
    for b in range(nbits):
        sb = np.uint64(b)
        key |= ((ix >> sb) & one) << np.uint64(3 * b)
        key |= ((iy >> sb) & one) << np.uint64(3 * b + 1)
        key |= ((iz >> sb) & one) << np.uint64(3 * b + 2)
    return key


def morton_decode(keys, nbits):
    """Inverse of morton_encode: uint64 keys -> int64 [n, 3] coordinates."""
    keys = np.asarray(keys, dtype=np.uint64)
    out = np.zeros(keys.shape + (3,), dtype=np.int64)
    one = np.uint64(1)
    for b in range(nbits):
        for a in range(3):
            bit = (keys >> np.uint64(3 * b + a)) & one
            out[..., a] |= bit.astype(np.int64) << b
    return out


# child offsets of a cell in Morton order: child c has (c & 1, c >> 1 & 1, c >> 2)
_CHILD = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int32)


def morton_coords(level):
    """Integer coordinates of all cells of a uniform 2**level grid, in Morton order.

    Built by recursion on the key's top digit (index s = 8*parent + child), so
    it is exact and fast for large grids (int32 [8**level, 3]).
    """
    c = np.zeros((1, 3), dtype=np.int32)
    for _ in range(level):
        c = (2 * c[:, None, :] + _CHILD[None, :, :]).reshape(-1, 3)
    return c


def _pyramid(grid, depth):
    """max / min / mean of the fine grid over every cell of every level."""
    mx = {depth: grid}
    mn = {depth: grid}
    mean = {depth: grid}
    for L in range(depth - 1, -1, -1):
        m = 1 << L
        mx[L] = mx[L + 1].reshape(m, 2, m, 2, m, 2).max(axis=(1, 3, 5))
        mn[L] = mn[L + 1].reshape(m, 2, m, 2, m, 2).min(axis=(1, 3, 5))
        mean[L] = mean[L + 1].reshape(m, 2, m, 2, m, 2).mean(axis=(1, 3, 5))
    return mx, mn, mean


def _leaves_from_rule(grid, depth, refine):
    """Top-down construction: a cell is split iff refine(L, mx, mn) says so.

    refine(L, mx_L, mn_L) returns a boolean array over the level-L cells.  A
    cell becomes a leaf when it exists (all its ancestors were split) and is
    not split itself, or when it reaches the maximum depth.
    """
    n = 1 << depth
    assert grid.shape == (n, n, n)
    mx, mn, mean = _pyramid(grid, depth)
    active = np.ones((1, 1, 1), dtype=bool)
    keys, levels, vals = [], [], []
    counts = {}
    for L in range(depth + 1):
        if L == depth:
            leaf = active
            nxt = None
        else:
            split = np.asarray(refine(L, mx[L], mn[L]), dtype=bool)
            leaf = active & ~split
            nxt = active & split
        ix, iy, iz = np.nonzero(leaf)
        s = depth - L
        keys.append(morton_encode(ix.astype(np.int64) << s, iy.astype(np.int64) << s,
                                  iz.astype(np.int64) << s, depth))
        levels.append(np.full(ix.shape[0], L, dtype=np.uint8))
        vals.append(mean[L][ix, iy, iz])
        counts[L] = int(ix.shape[0])
        if nxt is None:
            break
        active = nxt.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)
    keys = np.concatenate(keys)
    levels = np.concatenate(levels)
    vals = np.concatenate(vals)
    order = np.argsort(keys, kind="stable")
    return Octree(depth, keys[order], levels[order], np.ascontiguousarray(vals[order], dtype=np.float64),
                  {"leaves_per_level": counts})


def uniform_octree(depth, rho_morton):
    """Single-level tree: every cell of a uniform 2**depth grid is a leaf.

    rho_morton holds the cell values in Morton order (leaf order)."""
    n = 8 ** depth
    rho = np.ascontiguousarray(rho_morton, dtype=np.float64)
    assert rho.shape == (n,)
    keys = np.arange(n, dtype=np.uint64)
    levels = np.full(n, depth, dtype=np.uint8)
    return Octree(depth, keys, levels, rho, {"leaves_per_level": {depth: n}})


def grid_to_morton(grid):
    """Reorder an [ix,iy,iz] grid of side 2**L into Morton order."""
    level = int(round(np.log2(grid.shape[0])))
    c = morton_coords(level)
    return grid[c[:, 0], c[:, 1], c[:, 2]]


def threshold_refined_octree(grid, base_level, threshold):
    """AMR tree: uniform down to base_level, then split wherever the cell's
    maximum fine-grid value exceeds threshold, down to the grid's depth."""
    depth = int(round(np.log2(grid.shape[0])))

    def refine(L, mx, mn):
        if L < base_level:
            return np.ones(mx.shape, dtype=bool)
        return mx > threshold

    t = _leaves_from_rule(grid, depth, refine)
    t.info.update({"rule": "threshold", "base_level": base_level, "threshold": float(threshold)})
    return t


def uniformity_merged_octree(grid, density_floor, rel_uniformity=0.01):
    """Tree from the paper's density + uniformity criterion (sec. 2.4).

    A cell is split only if its maximum fine value reaches density_floor and
    its relative variation (max - min) / max reaches rel_uniformity; otherwise
    it is kept as a leaf (equivalently: eight sibling leaves are merged when
    they are all below the floor or agree within rel_uniformity)."""
    depth = int(round(np.log2(grid.shape[0])))

    def refine(L, mx, mn):
        return (mx >= density_floor) & ((mx - mn) >= rel_uniformity * mx)

    t = _leaves_from_rule(grid, depth, refine)
    t.info.update({"rule": "uniformity", "density_floor": float(density_floor),
                   "rel_uniformity": rel_uniformity})
    return t


def random_octree(depth, p_split, seed, min_level=0, value_sampler=None):
    """Random topology for tests: each cell above the maximum depth is split
    with probability p_split (always below min_level).  Values are lognormal
    unless value_sampler(rng, n) is given."""
    rng = np.random.default_rng(seed)
    n = 1 << depth
    grid = np.zeros((n, n, n))

    draws = {}

    def refine(L, mx, mn):
        if L < min_level:
            return np.ones(mx.shape, dtype=bool)
        r = rng.random(mx.shape) < p_split
        draws[L] = r
        return r

    t = _leaves_from_rule(grid, depth, refine)
    if value_sampler is None:
        t.rho = np.exp(rng.standard_normal(t.n))
    else:
        t.rho = np.ascontiguousarray(value_sampler(rng, t.n), dtype=np.float64)
    t.info.update({"rule": "random", "p_split": p_split, "seed": seed})
    return t


def split_leaf(tree, i):
    """Replace leaf i by its eight children, each carrying the parent's value.

    The new tree covers the same space with the same piecewise-constant
    density, so every column through it is unchanged."""
    L = int(tree.levels[i])
    assert L < tree.depth
    child_span = np.uint64(8 ** (tree.depth - L - 1))
    kids = tree.keys[i] + child_span * np.arange(8, dtype=np.uint64)
    keys = np.concatenate([tree.keys[:i], kids, tree.keys[i + 1:]])
    levels = np.concatenate([tree.levels[:i], np.full(8, L + 1, dtype=np.uint8), tree.levels[i + 1:]])
    rho = np.concatenate([tree.rho[:i], np.full(8, tree.rho[i]), tree.rho[i + 1:]])
    return Octree(tree.depth, keys, levels, rho, dict(tree.info))


def sparse_random_octree(depth, n_splits, seed, focus=None):
    """Deep trees without a dense grid: starting from the root, n_splits
    times pick a random leaf above the maximum depth (or, with focus = a
    point in [0,1)^3, the leaf holding that point) and split it into its
    eight children.  Values are lognormal."""
    rng = np.random.default_rng(seed)
    leaves = {0: 0}  # key -> level
    for _ in range(n_splits):
        if focus is not None:
            cell = [int(np.floor(f * (1 << depth))) for f in focus]
            k = int(morton_encode(cell[0], cell[1], cell[2], depth))
            key = max(kk for kk in leaves if kk <= k)
        else:
            cand = [kk for kk, L in leaves.items() if L < depth]
            if not cand:
                break
            key = cand[int(rng.integers(len(cand)))]
        L = leaves[key]
        if L >= depth:
            continue
        span = 8 ** (depth - L - 1)
        for c in range(8):
            leaves[key + c * span] = L + 1
    keys = np.array(sorted(leaves), dtype=np.uint64)
    levels = np.array([leaves[int(k)] for k in keys], dtype=np.uint8)
    rho = np.exp(rng.standard_normal(len(keys)))
    return Octree(depth, keys, levels, rho, {"rule": "sparse_random", "seed": seed})
