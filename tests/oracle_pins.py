"""Pins of the CPU oracle: checks against things other than the oracle itself.

Each ``pin_*`` function takes the oracle module and a loaded library handle
and raises AssertionError when the oracle disagrees with the pin.  The
regular tests run them on the real oracle; the mutation tests run them on
copies of the oracle with a planted mistake and require that some pin fails.

Which pin covers which oracle function:
  healpix_ring  pin_healpix_golden_nside1, pin_healpix_structure
  healpix_nested pin_healpix_nested
  check_tiling  pin_tiling
  walk_one      pin_walk_golden, pin_uniform_closed_form, pin_chord_invariants,
                pin_bruteforce, pin_amanatides_woo, pin_negation, pin_edge_cases,
                pin_deep_tree, pin_kahan_compensation
  columns       pin_linearity_and_refinement, pin_columns_consistency, pin_kahan_bound
  gradient      pin_gradient
  nested_reference pin_nested_reference
  grid_tree     pin_grid_tree_closed_forms, pin_grid_tree_rule
  shielding     pin_shielding_integrals, pin_line_depth_constants,
                pin_escape_probability, pin_av_eff, pin_shielding_edge_cases
"""

import os

import numpy as np

import workloads as W
from reference_geometry import (amanatides_woo, bruteforce_chords, exit_time, fnv_sequence_hash,
                                leaf_boxes, random_unit_vectors)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _frac(s):
    if "/" in s:
        a, b = s.split("/")
        return float(a) / float(b)
    return float(s)


# ---------------------------------------------------------------- HEALPix

def pin_healpix_golden_nside1(orc, lib):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "healpix_nside1.txt"))
            if ln.strip() and not ln.startswith("#")]
    d = orc.healpix_ring(1, lib=lib)
    assert d.shape == (12, 3)
    for pix, zs, ps in rows:
        z = _frac(zs)
        phi = np.pi * _frac(ps)
        st = np.sqrt(1.0 - z * z)
        want = np.array([st * np.cos(phi), st * np.sin(phi), z])
        assert np.abs(d[int(pix)] - want).max() <= 1e-15, (pix, d[int(pix)], want)


def pin_healpix_structure(orc, lib):
    for nside in (1, 2, 3, 4, 8):
        d = orc.healpix_ring(nside, lib=lib)
        npix = 12 * nside * nside
        assert d.shape == (npix, 3)
        assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() <= 1e-15
        assert np.abs(d.sum(axis=0)).max() <= 1e-13
        # closed under negation
        for v in d:
            assert np.abs(d + v).sum(axis=1).min() <= 1e-14
        # rings: consecutive pixels with equal z; sizes 4i (caps) / 4 nside (belt)
        z = d[:, 2]
        breaks = np.nonzero(np.diff(z) != 0)[0] + 1
        rings = np.split(np.arange(npix), breaks)
        assert len(rings) == 4 * nside - 1
        before = 0
        for i, r in enumerate(rings, start=1):
            want = 4 * min(i, nside, 4 * nside - i)
            assert len(r) == want, (nside, i, len(r), want)
            zi = z[r[0]]
            # equal-area zone identity: area fraction north of the ring centre
            frac = (before + 0.5 * len(r)) / npix
            assert abs((1.0 - zi) / 2.0 - frac) <= 1e-15, (nside, i)
            # azimuths ascend with constant spacing 2 pi / (ring size)
            phi = np.mod(np.arctan2(d[r, 1], d[r, 0]), 2 * np.pi)
            if len(r) > 1:
                assert np.abs(np.diff(phi) - 2 * np.pi / len(r)).max() <= 1e-12
            before += len(r)
        # z strictly decreasing from ring to ring (north to south)
        assert np.all(np.diff(z[[r[0] for r in rings]]) < 0)


# ---------------------------------------------------------------- tiling

def _match_ring(nest, ring):
    """Index of the RING centre nearest to each NESTED centre, and the
    distance to it."""
    from scipy.spatial import cKDTree

    dist, idx = cKDTree(ring).query(nest)
    return idx, dist


def pin_healpix_nested(orc, lib):
    """NESTED order, which the oracle reaches through the continuous HEALPix
    projection, a route independent of its RING table: the same centres as
    RING to a few ulp (nside 1 in the same order; above, every NESTED centre
    matches a distinct RING centre), and the hierarchy -- the 4 pixels
    4p .. 4p+3 at 2 nside surround pixel p: their mean direction lies within
    0.2 pixel of p's centre and each of them within 1.1 pixel (child pixel
    scale sqrt(4 pi / npix)); in-face neighbours (indices differing in bit 0
    or bit 1) are adjacent pixels; and the face coordinates have the
    orientation of the definition."""
    one = orc.healpix_nested(1, lib=lib)
    assert np.abs(one - orc.healpix_ring(1, lib=lib)).max() <= 1e-15
    for ns in (2, 4, 8, 16, 64):
        ring = orc.healpix_ring(ns, lib=lib)
        nest = orc.healpix_nested(ns, lib=lib)
        idx, dist = _match_ring(nest, ring)
        assert np.array_equal(np.sort(idx), np.arange(ring.shape[0])), ns
        assert dist.max() <= 2e-15, (ns, dist.max())
        if ns > 16:
            continue
        parent = orc.healpix_nested(ns // 2, lib=lib)
        scale = np.sqrt(4 * np.pi / nest.shape[0])
        kids = nest.reshape(-1, 4, 3)
        mean = kids.mean(1)
        mean /= np.linalg.norm(mean, axis=1)[:, None]
        off = np.arccos(np.clip((mean * parent).sum(1), -1, 1)) / scale
        assert off.max() < 0.2, (ns, off.max())
        dist = np.arccos(np.clip((kids * parent[:, None, :]).sum(2), -1, 1)) / scale
        assert dist.max() < 1.1, (ns, dist.max())
        for bit in (1, 2):
            q = np.arange(nest.shape[0]) ^ bit
            step = np.arccos(np.clip((nest * nest[q]).sum(1), -1, 1)) / scale
            assert step.max() < 1.6 and step.min() > 0.5, (ns, bit, step.min(), step.max())
    # orientation: face coordinates start at the face's south corner, x runs
    # toward its east corner and y toward its west corner, so of the 4 pixels
    # of a face at nside 2, 4f is southmost, 4f+3 northmost, and 4f+1 lies
    # east of 4f+2 on the same ring
    d2 = orc.healpix_nested(2, lib=lib).reshape(12, 4, 3)
    z = d2[:, :, 2]
    assert np.all(z[:, 0] < z[:, 1]) and np.all(z[:, 1] == z[:, 2]) and np.all(z[:, 3] > z[:, 1])
    phi = np.arctan2(d2[:, :, 1], d2[:, :, 0])
    east = np.mod(phi[:, 1] - phi[:, 2], 2 * np.pi)
    assert np.all((east > 0) & (east < np.pi)), east


def pin_tiling(orc, lib):
    t = W.random_octree(4, 0.4, 11, min_level=1)
    assert orc.check_tiling(t.keys, t.levels, 4, lib=lib) == orc.OK
    u = W.uniform_octree(2, np.ones(64))
    assert orc.check_tiling(u.keys, u.levels, 2, lib=lib) == orc.OK
    k, L = t.keys.copy(), t.levels.copy()
    k[[3, 4]] = k[[4, 3]]
    L[[3, 4]] = L[[4, 3]]
    assert orc.check_tiling(k, L, 4, lib=lib) == orc.ERR_UNSORTED
    # gap: drop a leaf
    assert orc.check_tiling(np.delete(t.keys, 5), np.delete(t.levels, 5), 4, lib=lib) == orc.ERR_TILING
    # overlap: make a leaf coarser than its span
    i = int(np.nonzero(t.levels == 4)[0][1])
    L = t.levels.copy()
    L[i] = 3
    assert orc.check_tiling(t.keys, L, 4, lib=lib) == orc.ERR_TILING
    # misaligned key (level-3 leaf moved by one fine cell)
    j = int(np.nonzero(t.levels <= 3)[0][2])
    k = t.keys.copy()
    k[j] += np.uint64(1)
    assert orc.check_tiling(k, t.levels, 4, lib=lib) != orc.OK
    # wrong end: last leaf missing
    assert orc.check_tiling(t.keys[:-1], t.levels[:-1], 4, lib=lib) == orc.ERR_TILING
    # level beyond depth
    L = u.levels.copy()
    L[0] = 3
    assert orc.check_tiling(u.keys, L, 2, lib=lib) != orc.OK


# ---------------------------------------------------------------- walks

def golden_trees():
    t1 = W.Octree(1, np.arange(8, dtype=np.uint64), np.full(8, 1, dtype=np.uint8),
                  np.arange(1, 9, dtype=np.float64))
    keys = np.concatenate([np.arange(8), 8 * np.arange(1, 8)]).astype(np.uint64)
    levels = np.array([2] * 8 + [1] * 7, dtype=np.uint8)
    rho = np.concatenate([1.0 + np.arange(8) / 10.0, 10.0 * np.arange(1, 8)])
    t2 = W.Octree(2, keys, levels, rho)
    return {"T1": t1, "T2": t2}


def pin_walk_golden(orc, lib):
    trees = golden_trees()
    r3 = np.sqrt(3.0)

    def val(s):
        if s == "d":
            return 1.0 / r3
        if s.endswith("r3"):
            return float(s[:-2]) * r3
        return float(s)

    for ln in open(os.path.join(GOLDEN, "walk_examples.txt")):
        if not ln.strip() or ln.startswith("#"):
            continue
        f = ln.split()
        tree = trees[f[1]]
        Q = [val(x) for x in f[2:5]]
        m = [val(x) for x in f[5:8]]
        N, tx = val(f[8]), val(f[9])
        vis = [int(x) for x in f[10].split(",")]
        r = orc.walk_one(tree, Q, m, lib=lib)
        assert r["status"] == orc.OK, f[0]
        assert list(r["visited"]) == vis, (f[0], list(r["visited"]), vis)
        assert abs(r["N"] - N) <= 1e-15 * N, (f[0], r["N"], N)
        assert abs(r["texit"] - tx) <= 1e-15 * tx, (f[0], r["texit"], tx)


def _test_rays(seed, count):
    rng = np.random.default_rng(seed)
    Q = rng.random((count, 3))
    m = random_unit_vectors(count, seed + 1)
    return Q, m


def _special_dirs(orc, lib):
    axis = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    diag = np.array([[1, 1, 1], [-1, 1, -1], [1, -1, 0], [0, 1, 1]], float)
    diag /= np.linalg.norm(diag, axis=1)[:, None]
    return np.vstack([axis, diag, orc.healpix_ring(2, lib=lib)])


def pin_uniform_closed_form(orc, lib):
    t = W.random_octree(5, 0.45, 21, min_level=1)
    rho0 = 2.5
    t.rho = np.full(t.n, rho0)
    Q, m = _test_rays(22, 150)
    dirs = _special_dirs(orc, lib)
    cases = list(zip(Q, m)) + [(Q[i % len(Q)], d) for i, d in enumerate(dirs)]
    # cell-centre and face-aligned sources with HEALPix directions
    for q in ([0.5, 0.5, 0.5], [0.25, 0.0, 0.75], [1 / 64, 3 / 64, 5 / 64]):
        cases += [(np.array(q), d) for d in dirs]
    for q, d in cases:
        r = orc.walk_one(t, q, d, lib=lib)
        te = exit_time(q, d)
        assert r["status"] == orc.OK
        assert abs(r["N"] - rho0 * te) <= 1e-13 * rho0 * te, (q, d, r["N"], rho0 * te)
        assert abs(r["texit"] - te) <= 1e-13 * te


def pin_chord_invariants(orc, lib):
    t = W.random_octree(5, 0.45, 31, min_level=1)
    sizes = t.sizes() / float(1 << t.depth)
    Q, m = _test_rays(32, 150)
    dirs = _special_dirs(orc, lib)
    cases = list(zip(Q, m)) + [(np.array([0.5, 0.5, 0.5]), d) for d in dirs]
    for q, d in cases:
        r = orc.walk_one(t, q, d, lib=lib)
        te = exit_time(q, d)
        c = r["chords"]
        assert r["status"] == orc.OK and r["steps"] == len(c)
        assert np.all(c >= 0.0)
        assert abs(c.sum() - te) <= 1e-13 * te
        assert np.all(c <= np.sqrt(3.0) * sizes[r["visited"]] * (1 + 1e-12))
    # generic rays never need the clamp; it only absorbs rounding at exact
    # lattice crossings (the source at the box centre above)
    for q, d in zip(Q, m):
        assert orc.walk_one(t, q, d, lib=lib)["clamps"] == 0


def pin_bruteforce(orc, lib):
    for seed, D, p in ((41, 4, 0.5), (42, 3, 0.7), (43, 4, 0.3)):
        t = W.random_octree(D, p, seed, min_level=1)
        boxes = leaf_boxes(t)
        Q, m = _test_rays(seed + 100, 120)
        dirs = _special_dirs(orc, lib)
        h = 1.0 / (1 << D)
        face = np.array([3 * h, 0.5, 5 * h])
        cases = list(zip(Q, m)) + [(face, d) for d in dirs] + [(np.array([0.5 * h] * 3), d) for d in dirs]
        # a subnormal component never bounds: sources on the z = 0 face and
        # on the box's corner heading up y with m_z = -2.2e-311
        sub = np.array([0.0, 1.0, -2.22507386e-311])
        cases += [(np.array([3 * h, 5 * h, 0.0]), sub), (np.zeros(3), sub)]
        for q, d in cases:
            r = orc.walk_one(t, q, d, lib=lib)
            chord, entry, te = bruteforce_chords(t, q, d, boxes)
            assert r["status"] == orc.OK
            nb = float(np.dot(t.rho, chord))
            assert abs(r["N"] - nb) <= 1e-12 * nb, (seed, q, d, r["N"], nb)
            # per-leaf chords agree; every leaf with a positive chord is visited
            walk_chord = np.zeros(t.n)
            np.add.at(walk_chord, r["visited"], r["chords"])
            assert np.abs(walk_chord - chord).max() <= 1e-12
            assert set(np.nonzero(chord > 1e-12)[0]) <= set(r["visited"].tolist())
            # order of the positive-chord leaves follows the entry times
            pos = [i for i, c in zip(r["visited"], r["chords"]) if c > 1e-12]
            assert pos == sorted(pos, key=lambda i: entry[i])


def pin_amanatides_woo(orc, lib):
    for D in (3, 4):
        n = 1 << D
        t = W.uniform_octree(D, np.exp(np.random.default_rng(D).standard_normal(8 ** D)))
        Q, m = _test_rays(50 + D, 150)
        for q, d in zip(Q, m):
            r = orc.walk_one(t, q, d, lib=lib)
            cells = amanatides_woo(n, q, d)
            want = [int(W.morton_encode(c[0], c[1], c[2], D)) for c in cells]
            assert list(r["visited"]) == want, (D, q, d)


def pin_negation(orc, lib):
    t = W.random_octree(4, 0.5, 61, min_level=1)
    rho0 = 0.75
    t.rho = np.full(t.n, rho0)
    Q, m = _test_rays(62, 100)
    for q, d in zip(Q, m):
        a = orc.walk_one(t, q, d, lib=lib)["N"]
        b = orc.walk_one(t, q, -d, lib=lib)["N"]
        full = rho0 * (exit_time(q, d) + exit_time(q, -d))
        assert abs(a + b - full) <= 1e-13 * full


def pin_linearity_and_refinement(orc, lib):
    t = W.random_octree(4, 0.5, 71, min_level=1)
    rng = np.random.default_rng(72)
    r1, r2 = np.exp(rng.standard_normal(t.n)), np.exp(rng.standard_normal(t.n))
    Q, m = _test_rays(73, 40)
    dirs = orc.healpix_ring(1, lib=lib)
    a, b = 0.3, 1.7
    n1 = orc.columns(t, Q, dirs, rho=r1, lib=lib)["N"]
    n2 = orc.columns(t, Q, dirs, rho=r2, lib=lib)["N"]
    n12 = orc.columns(t, Q, dirs, rho=a * r1 + b * r2, lib=lib)["N"]
    assert np.abs(n12 - (a * n1 + b * n2)).max() <= 1e-12 * np.abs(n12).max()
    t.rho = r1
    coarse = [int(i) for i in np.nonzero(t.levels < t.depth)[0][:5]]
    for i in coarse:
        s = W.split_leaf(t, i)
        assert orc.check_tiling(s.keys, s.levels, s.depth, lib=lib) == orc.OK
        ns = orc.columns(s, Q, dirs, lib=lib)["N"]
        assert np.abs(ns - n1).max() <= 1e-12 * np.abs(n1).max()
    # random directions too
    for q, d in zip(Q, m):
        base = orc.walk_one(t, q, d, lib=lib)["N"]
        s = W.split_leaf(t, coarse[0])
        assert abs(orc.walk_one(s, q, d, lib=lib)["N"] - base) <= 1e-12 * base


def pin_columns_consistency(orc, lib):
    """columns() equals walk_one() ray by ray; the hash is FNV over the
    visited sequence; A = exp(-kappa N)."""
    t = W.random_octree(4, 0.5, 81, min_level=1)
    Q, _ = _test_rays(82, 10)
    dirs = orc.healpix_ring(2, lib=lib)
    kappa = 0.7
    out = orc.columns(t, Q, dirs, kappa, rho32=t.rho.astype(np.float32), lib=lib)
    assert out["status"] == orc.OK and out["clamps"] == 0
    for s in range(len(Q)):
        for d in range(len(dirs)):
            r = orc.walk_one(t, Q[s], dirs[d], rho32=t.rho.astype(np.float32), lib=lib)
            assert out["N"][s, d] == r["N"] and out["steps"][s, d] == r["steps"]
            assert out["N32"][s, d] == r["N32"]
            assert int(out["hash"][s, d]) == r["hash"] == fnv_sequence_hash(r["visited"])
            assert abs(out["A"][s, d] - np.exp(-kappa * r["N"])) <= 1e-15
            assert abs(out["A32"][s, d] - np.exp(-kappa * r["N32"])) <= 3e-7 * out["A32"][s, d]


def pin_edge_cases(orc, lib):
    # minimal tree, D = 1
    t = W.uniform_octree(1, np.arange(1.0, 9.0))
    r = orc.walk_one(t, [0.5, 0.5, 0.5], [1, 0, 0], lib=lib)
    assert r["status"] == orc.OK and list(r["visited"]) == [7] and r["N"] == 8 * 0.5
    # source on the lower face, walking down: leaves at once
    r = orc.walk_one(t, [0.0, 0.25, 0.25], [-1, 0, 0], lib=lib)
    assert r["status"] == orc.OK and r["steps"] == 1 and r["N"] == 0.0
    # last representable coordinate below 1
    top = np.nextafter(1.0, 0.0)
    r = orc.walk_one(t, [top, top, top], [1, 0, 0], lib=lib)
    assert r["status"] == orc.OK and list(r["visited"]) == [7]
    assert abs(r["N"] - 8 * (1.0 - top)) <= 1e-30
    # a denormal direction component does not bound the walk
    r = orc.walk_one(t, [0.25, 0.25, 0.25], [1e-310, 0, 1], lib=lib)
    assert r["status"] == orc.OK and list(r["visited"]) == [0, 4]
    # a ray running inside the face plane z = 1/2 belongs to the upper cells
    r = orc.walk_one(t, [0.25, 0.25, 0.5], [1, 0, 0], lib=lib)
    assert list(r["visited"]) == [4, 5]
    # errors: source outside [0,1)^3, zero or non-finite direction
    assert orc.walk_one(t, [1.0, 0.5, 0.5], [1, 0, 0], lib=lib)["status"] == orc.ERR_RANGE
    assert orc.walk_one(t, [-1e-300, 0.5, 0.5], [1, 0, 0], lib=lib)["status"] == orc.ERR_RANGE
    assert orc.walk_one(t, [np.nan, 0.5, 0.5], [1, 0, 0], lib=lib)["status"] == orc.ERR_RANGE
    assert orc.walk_one(t, [0.5, 0.5, 0.5], [0, 0, 0], lib=lib)["status"] == orc.ERR_ARG
    assert orc.walk_one(t, [0.5, 0.5, 0.5], [np.inf, 0, 0], lib=lib)["status"] == orc.ERR_ARG


def deep_tree(depth=21):
    """The cell at the origin corner is split at every level; all others are
    leaves.  7 leaves per level plus 8 at the maximum depth."""
    keys, levels = [], []
    for L in range(depth):
        span = 8 ** (depth - L - 1)
        for c in range(1, 8):
            keys.append(c * span)
            levels.append(L + 1)
    keys.append(0)
    levels.append(depth)
    # the origin cell at the maximum depth has 7 siblings already listed at level `depth`
    order = np.argsort(np.array(keys, dtype=np.uint64), kind="stable")
    k = np.array(keys, dtype=np.uint64)[order]
    lv = np.array(levels, dtype=np.uint8)[order]
    rho = np.exp(np.random.default_rng(depth).standard_normal(len(k)))
    return W.Octree(depth, k, lv, rho)


def pin_deep_tree(orc, lib):
    t = deep_tree(21)
    assert orc.check_tiling(t.keys, t.levels, 21, lib=lib) == orc.OK
    boxes = leaf_boxes(t)
    h = 2.0 ** -21
    cases = [([0.3 * h, 0.7 * h, 0.2 * h], d) for d in random_unit_vectors(30, 91)]
    cases += [([0.9, 0.9, 0.9], -np.ones(3) / np.sqrt(3.0)), ([h, 2 * h, 3 * h], [1, 0, 0])]
    for q, d in cases:
        r = orc.walk_one(t, q, d, lib=lib)
        chord, _, te = bruteforce_chords(t, np.array(q), np.array(d, float), boxes)
        nb = float(np.dot(t.rho, chord))
        assert r["status"] == orc.OK
        assert abs(r["N"] - nb) <= 1e-12 * nb
        assert abs(r["texit"] - te) <= 1e-13 * te


def pin_kahan_compensation(orc, lib):
    """A ray whose first product is 2**17 ulps larger than each later one by a
    factor that rounds them away in plain FP32 summation; the compensated sum
    keeps them (error within 2 ulps of the exact sum of the FP32 products)."""
    D = 7
    n = 1 << D
    grid = np.zeros((n, n, n))
    grid[:, 0, 0] = 10.0
    t = W.threshold_refined_octree(grid, 0, 1.0)
    row = np.nonzero((t.levels == D) & np.all(t.anchors()[:, 1:] == 0, axis=1))[0]
    assert len(row) == n
    rho = np.ones(t.n)
    rho[row] = 7.8e-4
    rho[row[0]] = 32768.0
    t.rho = rho
    r32 = rho.astype(np.float32)
    q = np.array([0.5 / n, 0.5 / n, 0.5 / n])
    r = orc.walk_one(t, q, [1, 0, 0], rho32=r32, lib=lib)
    terms = [np.float32(r32[i]) * np.float32(c) for i, c in zip(r["visited"], r["chords"])]
    exact = float(np.sum(np.array(terms, dtype=np.float64)))
    naive = np.float32(0)
    for x in terms:
        naive = np.float32(naive + x)
    assert abs(float(naive) - exact) > 20 * 2.0 ** -24 * exact  # the case discriminates
    assert abs(r["N32"] - exact) <= 2 * 2.0 ** -24 * exact


def pin_kahan_bound(orc, lib):
    """FP32 compensated columns stay within 1e-5 (relative) of FP64 on a
    lognormal AMR cloud."""
    g = W.gaussian_random_field(32, -4.0, 5)
    rho = W.lognormal(g, 2.0)
    t = W.threshold_refined_octree(rho, 3, 2.0 * rho.mean())
    src = W.random_points(30, 6)
    out = orc.columns(t, src, orc.healpix_ring(2, lib=lib), 1.0, rho32=t.rho.astype(np.float32),
                      lib=lib)
    rel = np.abs(out["N32"].astype(np.float64) - out["N"]) / out["N"]
    assert rel.max() <= 1e-5


def pin_gradient(orc, lib):
    t = W.random_octree(3, 0.5, 101, min_level=1)
    src = W.random_points(12, 102)
    dirs = orc.healpix_ring(1, lib=lib)
    g = np.random.default_rng(103).standard_normal((len(src), len(dirs)))
    grad = orc.gradient(t, src, dirs, g, lib=lib)
    boxes = leaf_boxes(t)
    want = np.zeros(t.n)
    for s in range(len(src)):
        for d in range(len(dirs)):
            want += g[s, d] * bruteforce_chords(t, src[s], dirs[d], boxes)[0]
    scale = np.abs(want).max()
    assert np.abs(grad - want).max() <= 1e-12 * scale
    N = orc.columns(t, src, dirs, lib=lib)["N"]
    assert abs(np.dot(t.rho, grad) - np.sum(g * N)) <= 1e-12 * np.sum(np.abs(g * N))
    # central differences (N is linear in rho: exact up to rounding)
    for k in (0, t.n // 2, t.n - 1):
        h = 1e-3 * t.rho[k]
        rp, rm = t.rho.copy(), t.rho.copy()
        rp[k] += h
        rm[k] -= h
        dp = orc.columns(t, src, dirs, rho=rp, lib=lib)["N"]
        dm = orc.columns(t, src, dirs, rho=rm, lib=lib)["N"]
        fd = float(np.sum(g * (dp - dm) / (2 * h)))
        assert abs(fd - grad[k]) <= 1e-8 * scale


def pin_nested_reference(orc, lib):
    """Reference of a coarse NESTED pixel = mean of its 4^k finer pixels:
    with the fine values equal to their own index the mean of pixel q is
    q 4^k + (4^k - 1) / 2 exactly; two stages of coarsening equal one; the
    error is 0 for coarse = reference and 1 for coarse = 2 reference."""
    S = 3
    for dc, k in ((12, 1), (12, 2), (48, 1), (12, 3)):
        r = 4 ** k
        fine = np.tile(np.arange(dc * r, dtype=np.float64), (S, 1)) + np.arange(S)[:, None] * 1e6
        want = np.arange(dc) * r + (r - 1) / 2.0 + np.arange(S)[:, None] * 1e6
        ref, err = orc.nested_reference(fine, want, lib=lib)
        assert np.array_equal(ref, want) and np.all(err == 0.0)
        _, err2 = orc.nested_reference(fine, 2 * want[:, :], lib=lib)
        pos = want > 0
        assert np.all(err2[pos] == 1.0)
        if k >= 2:
            mid, _ = orc.nested_reference(fine, np.zeros((S, dc * r // 4)), lib=lib)
            two, _ = orc.nested_reference(mid, want, lib=lib)
            assert np.array_equal(two, ref)


def pin_grid_tree_closed_forms(orc, lib):
    """A uniform grid, or one below the floor, is one leaf (the root) with
    the grid's value; one hot cell in a uniform background above the floor
    splits exactly its D ancestors, giving 1 + 7 D leaves with the hot cell
    alone at level D; the split tests are inclusive (max == floor splits,
    (max - min) == rel max splits)."""
    D = 3
    n = 8 ** D
    k, lv, v = orc.grid_tree(np.full(n, 2.5), D, 1.0, 0.01, lib=lib)
    assert list(k) == [0] and list(lv) == [0] and v[0] == 2.5
    rng = np.random.default_rng(91)
    k, lv, v = orc.grid_tree(rng.random(n) * 0.5, D, 1.0, 0.01, lib=lib)
    assert list(k) == [0] and list(lv) == [0]
    hot = 300
    g = np.full(n, 4.0)
    g[hot] = 8.0
    k, lv, v = orc.grid_tree(g, D, 1.0, 0.01, lib=lib)
    assert len(k) == 1 + 7 * D
    assert orc.check_tiling(k, lv, D, lib=lib) == orc.OK
    assert np.sum(lv == D) == 8 and k[lv == D].min() <= hot <= k[lv == D].max()
    assert v[list(k).index(hot)] == 8.0
    # the mean of a leaf covering the hot cell's siblings and itself
    parent = hot & ~7
    assert np.sum((k >= parent) & (k < parent + 8)) == 8
    # inclusive tests: two values 1.0 and 0.75 in one level-2 cell
    g = np.full(n, 1.0)
    g[:8] = 0.75
    for rel, floor, want_split in ((0.25, 1.0, True), (0.2500001, 1.0, False), (0.25, 1.0000001, False)):
        k, lv, v = orc.grid_tree(g, D, floor, rel, lib=lib)
        assert (len(k) > 1) == want_split, (rel, floor, len(k))


def pin_grid_tree_rule(orc, lib):
    """On lognormal clouds: the leaves tile the box; every leaf fails the
    rule (or is at level D) and every leaf's parent passes it, with max and
    min taken directly over the covered fine cells; each value is the mean
    of the covered fine cells (to 1e-14); keys and levels equal those of the
    numpy generator of the workloads, an independent implementation."""
    for n, seed, q in ((16, 92, 60.0), (32, 93, 75.0)):
        D = int(np.log2(n))
        rho = W.lognormal(W.gaussian_random_field(n, -4.0, seed), 2.0)
        grid = W.octree.grid_to_morton(rho)
        floor = float(np.percentile(rho, q))
        k, lv, v = orc.grid_tree(grid, D, floor, 0.01, lib=lib)
        assert orc.check_tiling(k, lv, D, lib=lib) == orc.OK
        ref = W.uniformity_merged_octree(rho, floor, 0.01)
        assert np.array_equal(k, ref.keys) and np.array_equal(lv, ref.levels)

        def rule(key, level):
            span = 8 ** (D - int(level))
            block = grid[int(key): int(key) + span]
            mx, mn = block.max(), block.min()
            return mx >= floor and (mx - mn) >= 0.01 * mx

        for key, level, val in zip(k, lv, v):
            span = 8 ** (D - int(level))
            block = grid[int(key): int(key) + span]
            assert abs(val - block.mean()) <= 1e-14 * abs(block.mean())
            assert int(level) == D or not rule(key, level)
            if int(level) > 0:
                pspan = 8 ** (D - int(level) + 1)
                assert rule(int(key) // pspan * pspan, int(level) - 1)


# ---------------------------------------------------------------- several fields per leaf

AXES = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
# CGS constants (CODATA 2018) and the speed of light: A = 8 pi and nu = c make
# the line prefactor A c^3 / (8 pi nu^3) exactly 1 (the same roundings in
# numerator and denominator); T = 0 and vturb = 1 make du = 1.
C_LIGHT = 2.99792458e10
UNIT_LINE = dict(line_A=8.0 * np.pi, line_nu=C_LIGHT)


def _unit_lines(k):
    return dict(line_A=[UNIT_LINE["line_A"]] * k, line_nu=[UNIT_LINE["line_nu"]] * k)


def pin_shielding_integrals(orc, lib):
    """With a unit line prefactor and du = 1, the per-ray values are the
    columns of each field alone (the single-field walk, pinned above), times
    the length unit, bit for bit."""
    t = W.random_octree(4, 0.45, 201, min_level=1)
    rng = np.random.default_rng(202)
    F = np.stack([t.rho, rng.standard_normal(t.n), rng.random(t.n) * 3.0], 1)
    src = W.random_points(9, 203)
    dirs = orc.healpix_ring(2, lib=lib)
    L = 3.0
    out = orc.shielding(t, F, src, dirs, length=L, temp=np.zeros(len(src)), vturb=1.0,
                        **_unit_lines(2), lib=lib)
    assert out["status"] == orc.OK
    for f in range(3):
        N = orc.columns(t, src, dirs, rho=F[:, f], lib=lib)["N"]
        assert np.array_equal(out["rays"][:, :, f], L * N), f


def pin_line_depth_constants(orc, lib):
    """tau = A c^3 / (8 pi nu^3) N / du: exactly N for the unit prefactor;
    linear in A, falling as nu^-3, and 1/du with du the quadrature sum of
    the mean thermal speed sqrt(8 kB T / (pi m_p)) and vturb (for protons at
    100 K the mean speed is 1.450 km/s)."""
    t = W.uniform_octree(2, np.full(64, 1.0))
    src = np.array([[0.5, 0.5, 0.5]])
    N_ref = 0.5 * 7.0  # column of field 1 along an axis from the centre, length 7
    F = np.stack([np.ones(64), np.ones(64)], 1)

    def tau(A, nu, T, vt):
        o = orc.shielding(t, F, src, AXES[:1], length=7.0, temp=[T], vturb=vt, line_A=[A],
                          line_nu=[nu], lib=lib)
        assert o["status"] == orc.OK
        return o["rays"][0, 0, 1]

    A1, nu1 = UNIT_LINE["line_A"], UNIT_LINE["line_nu"]
    assert tau(A1, nu1, 0.0, 1.0) == N_ref
    base = tau(7.2e-8, 1.15e11, 0.0, 1.0e5)
    assert abs(tau(2 * 7.2e-8, 1.15e11, 0.0, 1.0e5) / base - 2.0) <= 1e-15
    assert abs(tau(7.2e-8, 2 * 1.15e11, 0.0, 1.0e5) / base - 0.125) <= 1e-15
    assert abs(tau(7.2e-8, 1.15e11, 0.0, 4.0e5) / base - 0.25) <= 1e-15
    du_thermal = N_ref / tau(A1, nu1, 100.0, 0.0)
    assert abs(du_thermal - 1.450e5) <= 0.001e5, du_thermal
    # quadrature: thermal speed equal to vturb gives sqrt(2) vturb
    du_both = N_ref / tau(A1, nu1, 100.0, du_thermal)
    assert abs(du_both / (np.sqrt(2.0) * du_thermal) - 1.0) <= 1e-14


def _axis_beta(orc, lib, value, length=2.0):
    """beta at the centre of a uniform field: all six axis rays see
    tau = value * 0.5 * length (unit prefactor, du = 1)."""
    t = W.uniform_octree(2, np.ones(64))
    F = np.stack([np.ones(64), np.full(64, value)], 1)
    o = orc.shielding(t, F, [[0.5, 0.5, 0.5]], AXES, length=length, temp=[0.0], vturb=1.0,
                      **_unit_lines(1), lib=lib)
    assert o["status"] == orc.OK
    assert np.all(o["rays"][0, :, 1] == value * 0.5 * length)
    return o["beta"][0, 0]


def pin_escape_probability(orc, lib):
    """beta = mean over directions of (1 - e^-tau) / tau: 1 - 1/e at tau = 1,
    e - 1 at tau = -1 (inverted populations), 1 at tau = 0, 1 - tau/2 for
    tiny tau (the naive quotient loses digits there), 1/tau for large tau,
    and the average of two directions with different depths."""
    assert abs(_axis_beta(orc, lib, 1.0) - 0.6321205588285577) <= 2e-16
    assert abs(_axis_beta(orc, lib, -1.0) - 1.718281828459045) <= 4e-16
    assert _axis_beta(orc, lib, 0.0) == 1.0
    b = _axis_beta(orc, lib, 1e-12)
    assert abs(b - (1.0 - 0.5e-12)) <= 2e-16
    assert abs(_axis_beta(orc, lib, 800.0) - 1.0 / 800.0) <= 1e-18
    # field 1 only in x < 1/2: from (1/2, 1/2, 1/2) the +x ray sees tau = 0,
    # the -x ray tau = 2 (length 4, chord 1/2)
    t = W.uniform_octree(1, np.ones(8))
    x_low = (np.arange(8) & 1) == 0  # Morton bit 0 is x
    F = np.stack([np.ones(8), np.where(x_low, 1.0, 0.0)], 1)
    o = orc.shielding(t, F, [[0.5, 0.5, 0.5]], AXES[:2], length=4.0, temp=[0.0], vturb=1.0,
                      **_unit_lines(1), lib=lib)
    assert abs(o["beta"][0, 0] - 0.7161661791908468) <= 2e-16


def pin_av_eff(orc, lib):
    """AV_eff = -(1/gamma) ln(mean_d exp(-gamma av0 N_d)): av0 N when all
    directions agree (also where exp(-gamma av0 N) underflows), ln 2 / gamma
    for one clear and one opaque direction, between the smallest and the
    mean av0 N in general, and the mean in the limit gamma -> 0."""
    gamma, av0 = 3.02, 6.29e-22
    t = W.uniform_octree(2, np.ones(64))
    centre = [[0.5, 0.5, 0.5]]
    for nh in (1.0, 1e21, 3e24):  # gamma av0 N = 1.9e-21, 0.95, 2850
        o = orc.shielding(t, np.full(64, nh), centre, AXES, length=2.0, gamma=gamma, av0=av0,
                          lib=lib)
        want = av0 * nh  # N = nh * 0.5 * 2
        assert o["status"] == orc.OK
        assert abs(o["av_eff"][0] - want) <= 1e-14 * want, (nh, o["av_eff"][0], want)
    t1 = W.uniform_octree(1, np.ones(8))
    x_low = (np.arange(8) & 1) == 0
    o = orc.shielding(t1, np.where(x_low, 1e26, 0.0), centre, AXES[:2], gamma=gamma, av0=av0,
                      lib=lib)
    assert abs(o["av_eff"][0] - np.log(2.0) / gamma) <= 1e-15
    tr = W.random_octree(4, 0.45, 211, min_level=1)
    nh = tr.rho * 1e22
    src = W.random_points(20, 212)
    dirs = orc.healpix_ring(2, lib=lib)
    o = orc.shielding(tr, nh, src, dirs, gamma=gamma, av0=av0, lib=lib)
    av = av0 * o["rays"][:, :, 0]
    assert np.all(o["av_eff"] >= av.min(1) * (1 - 1e-14))
    assert np.all(o["av_eff"] <= av.mean(1) * (1 + 1e-14))
    assert np.all(o["av_eff"] < av.mean(1))  # strict: the columns differ
    o = orc.shielding(tr, nh, src, dirs, gamma=1e-9, av0=av0, lib=lib)
    assert np.all(np.abs(o["av_eff"] / av.mean(1) - 1.0) <= 1e-6)


def pin_shielding_edge_cases(orc, lib):
    """A source outside the box, or du not > 0, gives NaN for that source
    only and an error; an empty field gives AV_eff = 0 and beta = 1."""
    t = W.uniform_octree(2, np.ones(64))
    F = np.stack([np.zeros(64), np.zeros(64)], 1)
    src = np.array([[0.3, 0.3, 0.3], [1.0, 0.5, 0.5], [0.6, 0.6, 0.6]])
    o = orc.shielding(t, F, src, AXES, temp=[10.0, 10.0, 10.0], vturb=0.0, **_unit_lines(1),
                      lib=lib)
    assert o["status"] == orc.ERR_RANGE
    assert np.all(np.isnan(o["rays"][1])) and np.isnan(o["av_eff"][1]) and np.isnan(o["beta"][1, 0])
    assert np.all(o["av_eff"][[0, 2]] == 0.0) and np.all(o["beta"][[0, 2], 0] == 1.0)
    o = orc.shielding(t, F, src[[0, 2]], AXES, temp=[0.0, 10.0], vturb=0.0, **_unit_lines(1),
                      lib=lib)
    assert o["status"] == orc.ERR_RANGE
    assert np.isnan(o["av_eff"][0]) and o["av_eff"][1] == 0.0


ALL_PINS = [
    pin_healpix_golden_nside1,
    pin_healpix_structure,
    pin_healpix_nested,
    pin_tiling,
    pin_walk_golden,
    pin_uniform_closed_form,
    pin_chord_invariants,
    pin_bruteforce,
    pin_amanatides_woo,
    pin_negation,
    pin_linearity_and_refinement,
    pin_columns_consistency,
    pin_edge_cases,
    pin_deep_tree,
    pin_kahan_compensation,
    pin_kahan_bound,
    pin_gradient,
    pin_nested_reference,
    pin_grid_tree_closed_forms,
    pin_grid_tree_rule,
    pin_shielding_integrals,
    pin_line_depth_constants,
    pin_escape_probability,
    pin_av_eff,
    pin_shielding_edge_cases,
]
