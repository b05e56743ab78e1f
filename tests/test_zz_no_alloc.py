"""rt_grid_tree_static (the grid construction without a caller workspace,
for callers that cannot allocate) against rt_grid_tree, through the C ABI.

Bar: bit-exact keys, levels, values and leaf count (the same kernels on
the same grid; only the scratch differs).  Two calls in a row, the second on
a smaller grid, so that the second runs over the first's leftover scratch;
the largest accepted depth; and the refusal of deeper grids.
"""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def _grid(n, seed, q):
    rho = W.lognormal(W.gaussian_random_field(n, -4.0, seed), 2.0)
    return W.octree.grid_to_morton(rho), float(np.percentile(rho, q))


def _outputs(n_cells, dev):
    return (torch.full((n_cells,), -1, dtype=torch.int64, device=dev),
            torch.full((n_cells,), 255, dtype=torch.uint8, device=dev),
            torch.full((n_cells,), float("nan"), dtype=torch.float64, device=dev),
            torch.full((1,), -1, dtype=torch.int64, device=dev))


def _with_workspace(rt, g, depth, floor, rel):
    dev = g.device
    keys, levels, values, n = _outputs(g.numel(), dev)
    nbytes = rt._abi.rt_grid_tree_workspace_bytes(depth)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    lib = rt._abi.load()
    st = lib.rt_grid_tree(g.data_ptr(), depth, floor, rel, base, nbytes, keys.data_ptr(),
                          levels.data_ptr(), values.data_ptr(), n.data_ptr(), None)
    assert st == rt._abi.RT_OK, lib.rt_last_error()
    torch.cuda.synchronize()
    return keys, levels, values, n


def _static(rt, g, depth, floor, rel):
    dev = g.device
    keys, levels, values, n = _outputs(g.numel(), dev)
    lib = rt._abi.load()
    st = lib.rt_grid_tree_static(g.data_ptr(), depth, floor, rel, keys.data_ptr(),
                                 levels.data_ptr(), values.data_ptr(), n.data_ptr(), None)
    assert st == rt._abi.RT_OK, lib.rt_last_error()
    torch.cuda.synchronize()
    return keys, levels, values, n


def _same(a, b):
    ka, la, va, na = a
    kb, lb, vb, nb = b
    k = int(na.item())
    assert k == int(nb.item()) and k >= 1
    assert torch.equal(ka[:k], kb[:k])
    assert torch.equal(la[:k], lb[:k])
    assert torch.equal(va[:k].view(torch.int64), vb[:k].view(torch.int64))
    return k


def test_static_scratch_matches_workspace_call(rt):
    dev = torch.device("cuda")
    counts = []
    # the largest accepted grid, then smaller ones over its leftover scratch
    for n, seed, q in ((128, 11, 75.0), (64, 12, 60.0), (16, 13, 80.0)):
        grid, floor = _grid(n, seed, q)
        depth = int(np.log2(n))
        g = torch.as_tensor(grid).to(dev)
        counts.append(_same(_static(rt, g, depth, floor, 0.01),
                            _with_workspace(rt, g, depth, floor, 0.01)))
    assert counts[0] > counts[1] > counts[2]
    # degenerate grids: one leaf, and every fine cell a leaf
    g = torch.full((8 ** 3,), 2.0, dtype=torch.float64, device=dev)
    assert _same(_static(rt, g, 3, 1.0, 0.01), _with_workspace(rt, g, 3, 1.0, 0.01)) == 1
    g = torch.rand(8 ** 4, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(5)) + 1.0
    assert _same(_static(rt, g, 4, -1e300, 0.0), _with_workspace(rt, g, 4, -1e300, 0.0)) == 8 ** 4


def test_static_scratch_refuses_deeper_grids(rt):
    lib = rt._abi.load()
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    E = rt._abi.RT_ERR_ARG
    assert lib.rt_grid_tree_static(p, 8, 1.0, 0.01, p, p, p, p, None) == E
    assert b"static scratch" in lib.rt_last_error()
    assert lib.rt_grid_tree_static(p, 0, 1.0, 0.01, p, p, p, p, None) == E
    assert lib.rt_grid_tree_static(None, 3, 1.0, 0.01, p, p, p, p, None) == E
    assert lib.rt_grid_tree_static(p, 3, float("inf"), 0.01, p, p, p, p, None) == E
