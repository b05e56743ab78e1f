"""Source points (the paper's source grid, sec. 2.2): where rays start.

All points lie in the half-open unit box [0, 1)**3.  Arrays are float64
[S, 3], C-contiguous.
"""

import numpy as np

from .octree import morton_coords, morton_encode

_BELOW_ONE = np.nextafter(1.0, 0.0)


def cell_centres(level):
    """Centres (i + 1/2) / 2**level of a uniform grid, in Morton order.

    Consecutive sources are then spatially compact (8, 64, 512 ... points fill
    cubes), which keeps rays of neighbouring lanes close together."""
    c = morton_coords(level).astype(np.float64)
    c += 0.5
    c *= 1.0 / (1 << level)
    return np.ascontiguousarray(c)


def leaf_centres(tree):
    """Centre of every leaf of an octree, in leaf (Morton) order."""
    a = tree.anchors().astype(np.float64)
    s = tree.sizes().astype(np.float64)[:, None]
    return np.ascontiguousarray((a + 0.5 * s) * (1.0 / (1 << tree.depth)))


def _morton_sort(points, depth):
    cell = np.floor(points * (1 << depth)).astype(np.int64)
    key = morton_encode(cell[:, 0], cell[:, 1], cell[:, 2], depth)
    order = np.argsort(key, kind="stable")
    return np.ascontiguousarray(points[order])


def density_weighted_points(tree, count, seed, sort=True):
    """Poisson-like sample of the density: leaf k is drawn with probability
    proportional to rho_k * volume_k, then a point is placed uniformly inside
    it.  The points are finally sorted by the Morton key of their finest cell
    so that consecutive sources are spatially close."""
    rng = np.random.default_rng(seed)
    w = tree.rho * tree.sizes().astype(np.float64) ** 3
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    pick = np.searchsorted(cdf, rng.random(count), side="right")
    pick = np.minimum(pick, tree.n - 1)
    a = tree.anchors()[pick].astype(np.float64)
    s = tree.sizes()[pick].astype(np.float64)[:, None]
    u = rng.random((count, 3))
    pts = (a + u * s) * (1.0 / (1 << tree.depth))
    pts = np.minimum(pts, _BELOW_ONE)
    if sort:
        pts = _morton_sort(pts, tree.depth)
    return np.ascontiguousarray(pts)


def random_points(count, seed, lo=0.0, hi=1.0):
    """Uniform random points in [lo, hi)**3 (clamped below 1)."""
    rng = np.random.default_rng(seed)
    pts = lo + (hi - lo) * rng.random((count, 3))
    return np.ascontiguousarray(np.minimum(pts, _BELOW_ONE))
