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
