"""Contribution grid built on the GPU (rt_grid_tree) vs the oracle.

Bar: bit-exact keys, levels, values and leaf count (the split decisions and
the level-by-level means are the same FP64 operations in the same order on
both sides).
"""

import time

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def _build(rt, grid, depth, floor, rel):
    g = torch.as_tensor(np.ascontiguousarray(grid, dtype=np.float64)).to("cuda")
    k, lv, v = rt.grid_tree(g, depth, floor, rel)
    torch.cuda.synchronize()
    return k.cpu().numpy().view(np.uint64), lv.cpu().numpy(), v.cpu().numpy()


def _compare(rt, orc, grid, depth, floor, rel=0.01):
    got = _build(rt, grid, depth, floor, rel)
    want = orc.grid_tree(grid, depth, floor, rel)
    assert len(got[0]) == len(want[0])
    for g, w, name in zip(got, want, ("keys", "levels", "values")):
        assert np.array_equal(g, w), name
    return got


@pytest.mark.parametrize("n,seed,q", [(2, 1, 50.0), (4, 2, 60.0), (8, 3, 75.0), (16, 4, 75.0),
                                      (32, 5, 70.0), (64, 6, 80.0)])
def test_lognormal_clouds(rt, orc, n, seed, q):
    depth = int(np.log2(n))
    if n >= 8:
        rho = W.lognormal(W.gaussian_random_field(n, -4.0, seed), 2.0)
    else:
        rho = np.random.default_rng(seed).lognormal(0.0, 2.0, (n, n, n))
    grid = W.octree.grid_to_morton(rho)
    k, lv, _ = _compare(rt, orc, grid, depth, float(np.percentile(rho, q)))
    assert orc.check_tiling(k, lv, depth) == orc.OK


@pytest.mark.parametrize("depth", [1, 3, 4, 7])
def test_degenerate_grids(rt, orc, depth):
    n = 8 ** depth
    # uniform: one leaf; all split: every fine cell a leaf; one hot cell
    k, lv, v = _compare(rt, orc, np.full(n, 3.0), depth, 1.0)
    assert len(k) == 1 and lv[0] == 0 and v[0] == 3.0
    grid = np.random.default_rng(depth).random(n) + 1.0
    k, lv, _ = _compare(rt, orc, grid, depth, -1e300, 0.0)
    assert len(k) == n and np.all(lv == depth)
    hot = np.full(n, 2.0)
    hot[n // 3] = 5.0
    k, _, _ = _compare(rt, orc, hot, depth, 1.0)
    assert len(k) == 1 + 7 * depth


def test_argument_errors(rt):
    lib = rt._abi.load()
    E = rt._abi.RT_ERR_ARG
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    assert rt._abi.rt_grid_tree_workspace_bytes(0) == 0
    assert rt._abi.rt_grid_tree_workspace_bytes(11) == 0
    assert lib.rt_grid_tree(p, 0, 1.0, 0.01, p, 1 << 20, p, p, p, p, None) == E
    assert lib.rt_grid_tree(p, 11, 1.0, 0.01, p, 1 << 20, p, p, p, p, None) == E
    assert lib.rt_grid_tree(None, 2, 1.0, 0.01, p, 1 << 20, p, p, p, p, None) == E
    assert lib.rt_grid_tree(p, 2, float("nan"), 0.01, p, 1 << 20, p, p, p, p, None) == E
    assert lib.rt_grid_tree(p, 2, 1.0, 0.01, p, 16, p, p, p, p, None) == rt._abi.RT_ERR_WORKSPACE
    assert lib.rt_grid_tree(p, 2, 1.0, 0.01, p + 8, 1 << 20, p, p, p, p, None) == \
        rt._abi.RT_ERR_WORKSPACE


def test_merged512_fullsize(rt, orc):
    """The benchmark cloud's 512^3 grid: the GPU tree equals the oracle's
    and the workload generator's (so every walk over it is the same)."""
    g = W.gaussian_random_field(512, -4.0, 1004)
    rho = W.lognormal(g, 2.0)
    del g
    floor = float(np.percentile(rho, 75.0))
    grid = W.octree.grid_to_morton(rho)
    del rho
    dev = torch.device("cuda")
    gd = torch.as_tensor(grid).to(dev)
    rt.grid_tree(gd, 9, floor, 0.01)  # warm up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, lv, v = rt.grid_tree(gd, 9, floor, 0.01)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    print(f"512^3 grid -> {k.numel()} leaves in {ms:.2f} ms (incl. the count read-back)")
    got = (k.cpu().numpy().view(np.uint64), lv.cpu().numpy(), v.cpu().numpy())
    want = orc.grid_tree(grid, 9, floor, 0.01)
    for a, b, name in zip(got, want, ("keys", "levels", "values")):
        assert np.array_equal(a, b), name
    assert got[0].shape[0] == 38961931
    # the same tree as the workload's host generator, so the same walks
    w = W.make_workload(4)
    assert np.array_equal(got[0], w.tree.keys) and np.array_equal(got[1], w.tree.levels)


def _regions(tree):
    """Bytes of the staged keys, levels and top table of an Octree."""
    n, D = tree.n, tree.depth
    ksize = 4 if D <= 10 else 8
    lt = 0
    while lt < D and lt < 9 and 8 ** (lt + 1) <= 2 * n:
        lt += 1
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    kb, lb = al(ksize * (n + 1)), al(n)
    off = (-tree._ws.data_ptr()) % 256
    ws = tree._ws[off:]
    return (ws[:ksize * (n + 1)], ws[kb:kb + n], ws[kb + lb:kb + lb + 4 * (8 ** lt + 1)])


@pytest.mark.parametrize("case", ["random5", "random7", "sparse11", "sparse14", "sparse21", "single"])
def test_device_octree_equals_host(rt, case):
    if case.startswith("random"):
        t = W.random_octree(int(case[6:]), 0.4, 31, min_level=1)
    elif case == "single":
        t = W.Octree(3, np.zeros(1, np.uint64), np.zeros(1, np.uint8), np.ones(1))
    else:
        t = W.sparse_random_octree(int(case[6:]), 30, 32)
    dev = torch.device("cuda")
    host = rt.Octree(t.keys, t.levels, t.depth, dev)
    k = torch.as_tensor(t.keys.view(np.int64)).to(dev)
    lv = torch.as_tensor(t.levels).to(dev)
    devt = rt.Octree.from_device(k, lv, t.depth)
    torch.cuda.synchronize()
    for a, b, name in zip(_regions(host), _regions(devt), ("keys", "levels", "top")):
        assert torch.equal(a, b), (case, name)


def test_device_octree_errors(rt):
    t = W.random_octree(4, 0.5, 41, min_level=1)
    dev = torch.device("cuda")
    E = rt._abi

    def build(keys, levels, depth=t.depth):
        return rt.Octree.from_device(torch.as_tensor(np.asarray(keys, np.uint64).view(np.int64)).to(dev),
                                     torch.as_tensor(np.asarray(levels, np.uint8)).to(dev), depth)

    def status(keys, levels, depth=t.depth):
        try:
            build(keys, levels, depth)
        except E.RtError as e:
            return e.status
        return E.RT_OK

    k, lv = t.keys.copy(), t.levels.copy()
    sw = k.copy()
    sw[[3, 4]] = sw[[4, 3]]
    assert status(sw, lv) == E.RT_ERR_UNSORTED
    assert status(np.delete(k, 5), np.delete(lv, 5)) == E.RT_ERR_TILING      # gap
    bad = lv.copy()
    bad[2] = t.depth + 1
    assert status(k, bad) == E.RT_ERR_TILING                                  # level > D
    mis = k.copy()
    mis[7] += 1
    assert status(mis, lv) in (E.RT_ERR_TILING, E.RT_ERR_UNSORTED)          # misaligned
    assert status(k[1:], lv[1:]) == E.RT_ERR_TILING                           # first key not 0
    assert status(k[:-1], lv[:-1]) == E.RT_ERR_TILING                         # ends early
    assert status(k, lv) == E.RT_OK


def test_grid_to_walk_on_device(rt, orc):
    """Grid -> tree -> octree handle -> columns, all on the device, equals
    the same walk over the host-built tree and the oracle."""
    rho = W.lognormal(W.gaussian_random_field(64, -4.0, 51), 2.0)
    grid = W.octree.grid_to_morton(rho)
    floor = float(np.percentile(rho, 70.0))
    dev = torch.device("cuda")
    keys, levels, values = rt.grid_tree(torch.as_tensor(grid).to(dev), 6, floor)
    tree_d = rt.Octree.from_device(keys, levels, 6)
    ref_tree = W.uniformity_merged_octree(rho, floor, 0.01)
    src = W.random_points(500, 52)
    dirs = orc.healpix_ring(2)
    N_dev, _ = rt.columns(tree_d, values, torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev))
    ok, ov, oval = orc.grid_tree(grid, 6, floor)
    ref = orc.columns(W.Octree(6, ok, ov, oval), src, dirs, threads=8)
    assert np.array_equal(N_dev.cpu().numpy(), ref["N"])
    assert np.array_equal(ok, ref_tree.keys)
