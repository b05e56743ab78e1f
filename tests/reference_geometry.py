"""Independent references used to pin the oracle (test helpers).

None of these share code with the oracle or the GPU library.  They state
what a column is in other ways:

* exit_time: the distance from Q along m to the unit box's boundary;
* bruteforce_chords: the plain definition N = sum_k rho_k |segment cap AABB_k|,
  intersecting the segment [0, t_exit] with every leaf box by the slab test,
  vectorised over all leaves (no traversal at all);
* amanatides_woo: the textbook incremental grid walk (Amanatides & Woo 1987)
  on a uniform grid, which yields the ordered sequence of crossed cells;
* fnv_sequence_hash: the 64-bit FNV-1a-style hash of a leaf-index sequence
  (FNV offset basis 0xcbf29ce484222325, prime 0x100000001b3, one 64-bit word
  per index), used to compare visited sequences at scale.
"""

import numpy as np

FNV_OFFSET = 0xCBF29CE484222325
FNV_PRIME = 0x100000001B3
MASK64 = (1 << 64) - 1


def fnv_sequence_hash(indices):
    h = FNV_OFFSET
    for i in indices:
        h = ((h ^ (int(i) & MASK64)) * FNV_PRIME) & MASK64
    return h


def exit_time(Q, m):
    """t at which Q + m t leaves [0,1]^3.  An axis bounds iff 1/m_a is finite:
    m_a = 0 never bounds, and neither does a subnormal m_a (the reading of
    rays parallel to an axis that the walk follows; it differs from the
    exact geometry only for a source closer to the face such an axis would
    leave through than |m_a|, that is on it or a subnormal distance away)."""
    t = np.inf
    for a in range(3):
        with np.errstate(divide="ignore", over="ignore"):
            bounding = np.isfinite(1.0 / m[a])
        if not bounding:
            continue
        if m[a] > 0:
            t = min(t, (1.0 - Q[a]) / m[a])
        else:
            t = min(t, (0.0 - Q[a]) / m[a])
    return t


def leaf_boxes(tree):
    a = tree.anchors().astype(np.float64)
    s = tree.sizes().astype(np.float64)[:, None]
    h = 1.0 / (1 << tree.depth)
    return a * h, (a + s) * h


def bruteforce_chords(tree, Q, m, boxes=None):
    """Chord of the segment Q + m t, t in [0, t_exit], in every leaf box."""
    lo, hi = boxes if boxes is not None else leaf_boxes(tree)
    Q = np.asarray(Q, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    te = exit_time(Q, m)
    t_in = np.zeros(lo.shape[0])
    t_out = np.full(lo.shape[0], te)
    for a in range(3):
        # the bounding rule of exit_time: an axis bounds iff 1/m_a is finite
        with np.errstate(divide="ignore", over="ignore"):
            bounding = np.isfinite(1.0 / m[a])
        if bounding:
            t1 = (lo[:, a] - Q[a]) / m[a]
            t2 = (hi[:, a] - Q[a]) / m[a]
            t_in = np.maximum(t_in, np.minimum(t1, t2))
            t_out = np.minimum(t_out, np.maximum(t1, t2))
        else:
            # a ray parallel to the axis (m_a zero or subnormal) stays in the
            # plane through Q; inside a face plane it belongs to the cells
            # above it: cells are half-open, [lo, hi)
            inside = (lo[:, a] <= Q[a]) & (Q[a] < hi[:, a])
            t_out = np.where(inside, t_out, -np.inf)
    chord = np.maximum(t_out - t_in, 0.0)
    entry = np.where(chord > 0, t_in, np.inf)
    return chord, entry, te


def amanatides_woo(n, Q, m):
    """Ordered cells (ix, iy, iz) of an n^3 uniform grid over [0,1)^3 crossed
    by Q + m t, t >= 0 (textbook incremental traversal)."""
    cell = [int(np.floor(Q[a] * n)) for a in range(3)]
    step, t_max, t_delta = [0] * 3, [np.inf] * 3, [np.inf] * 3
    for a in range(3):
        if m[a] > 0:
            step[a] = 1
            t_max[a] = ((cell[a] + 1) / n - Q[a]) / m[a]
            t_delta[a] = 1.0 / (n * m[a])
        elif m[a] < 0:
            step[a] = -1
            t_max[a] = (cell[a] / n - Q[a]) / m[a]
            t_delta[a] = -1.0 / (n * m[a])
    out = [tuple(cell)]
    while True:
        a = int(np.argmin(t_max))
        cell[a] += step[a]
        if cell[a] < 0 or cell[a] >= n:
            return out
        t_max[a] += t_delta[a]
        out.append(tuple(cell))


def random_unit_vectors(count, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]
