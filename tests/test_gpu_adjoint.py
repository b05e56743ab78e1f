"""HIP adjoint walk (dL/drho through RayColumns) vs the oracle's FP64
gradient, the linearity identity, and FP64 central differences.

Bars: the FP32 adjoint (FP32 products g * l, FP32 atomic sums in an
unspecified order) within 1e-5 relative of the oracle's FP64 gradient, with
an absolute floor of 1e-6 * max|grad|; against FP64 central differences
within 1e-4 relative with a floor of 1e-7 * max|grad|.
"""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import random_dirs, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def _close(got, want, rel, floor):
    scale = np.abs(want).max()
    err = np.abs(got - want)
    tol = rel * np.abs(want) + floor * scale
    bad = np.nonzero(err > tol)[0]
    assert len(bad) == 0, (f"{len(bad)} of {len(want)} leaves off; worst rel "
                           f"{(err / np.maximum(np.abs(want), 1e-300)).max():.3e}")


def _loss_grad(rt, tree, src, dirs, w, kappa, rho_dtype=torch.float32):
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    rho = torch.as_tensor(tree.rho).to(dev, rho_dtype).requires_grad_(True)
    src_d, dirs_d = torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev)
    w_d = torch.as_tensor(w).to(dev, rho_dtype)
    N, A = rt.ray_columns(rho, t, src_d, dirs_d, kappa)
    L = (w_d * A).sum()
    L.backward()
    return rho.grad.double().cpu().numpy(), N.detach().double().cpu().numpy(), A.detach().double().cpu().numpy()


@pytest.mark.parametrize("seed,depth,p", [(1, 4, 0.5), (2, 5, 0.3), (3, 6, 0.15)])
def test_adjoint_matches_oracle_gradient(rt, orc, seed, depth, p):
    tree = W.random_octree(depth, p, seed, min_level=1)
    src = W.random_points(200, seed + 1)
    dirs = np.vstack([orc.healpix_ring(2), random_dirs(5, seed + 2)])
    kappa = 0.9
    w = np.random.default_rng(seed + 3).random((len(src), len(dirs)))
    grad, N, A = _loss_grad(rt, tree, src, dirs, w, kappa)
    ref = orc.columns(tree, src, dirs, kappa)
    g = -kappa * w * ref["A"]  # dL/dN for L = sum w exp(-kappa N)
    want = orc.gradient(tree, src, dirs, g)
    _close(grad, want, 1e-5, 1e-6)
    # N linear in rho: sum_k rho_k dL/drho_k = sum_r g_r N_r
    lhs = float(np.dot(tree.rho.astype(np.float32).astype(np.float64), grad))
    rhs = float(np.sum(-kappa * w * A * N))
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_adjoint_gN_and_gA_paths(rt, orc):
    """g = dL/dN - kappa A dL/dA with both upstream gradients present."""
    tree = W.random_octree(4, 0.5, 11, min_level=1)
    src = W.random_points(100, 12)
    dirs = orc.healpix_ring(1)
    kappa = 1.3
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    rho = torch.as_tensor(tree.rho).to(dev, torch.float32).requires_grad_(True)
    N, A = rt.ray_columns(rho, t, torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev),
                          kappa)
    rng = np.random.default_rng(13)
    a = rng.standard_normal((len(src), len(dirs)))
    b = rng.standard_normal((len(src), len(dirs)))
    L = (torch.as_tensor(a).to(dev, torch.float32) * N).sum() + \
        (torch.as_tensor(b).to(dev, torch.float32) * A).sum()
    L.backward()
    ref = orc.columns(tree, src, dirs, kappa)
    want = orc.gradient(tree, src, dirs, a - kappa * ref["A"] * b)
    _close(rho.grad.double().cpu().numpy(), want, 1e-5, 1e-6)


def test_adjoint_fp64_rho_returns_fp64_grad(rt, orc):
    tree = W.random_octree(3, 0.5, 21, min_level=1)
    src = W.random_points(50, 22)
    dirs = orc.healpix_ring(1)
    w = np.random.default_rng(23).random((len(src), len(dirs)))
    grad, _, _ = _loss_grad(rt, tree, src, dirs, w, 1.0, rho_dtype=torch.float64)
    ref = orc.columns(tree, src, dirs, 1.0)
    want = orc.gradient(tree, src, dirs, -w * ref["A"])
    _close(grad, want, 1e-5, 1e-6)


def test_adjoint_amr128_central_differences(rt, orc):
    """Config of the adjoint study: AMR 64^3 -> 128^3 (threshold 2<rho>),
    all leaf centres as sources, nside 2, L = sum w exp(-kappa N), kappa = 1.
    The FP32 adjoint is checked against FP64 central differences on 64
    random leaves, the differences formed per ray and summed."""
    w3 = W.make_workload(3)
    tree, src = w3.tree, w3.sources
    dirs = orc.healpix_ring(w3.nside)
    w = w3.weights()
    kappa = w3.kappa
    grad, _, _ = _loss_grad(rt, tree, src, dirs, w, kappa)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    src_d, dirs_d = torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev)
    w_d = torch.as_tensor(w).to(dev)
    rho0 = torch.as_tensor(tree.rho.astype(np.float32).astype(np.float64)).to(dev)
    leaves = w3.fd_leaves(64)
    fd = np.empty(len(leaves))
    for j, k in enumerate(leaves):
        h = 1e-3 * float(rho0[k])
        rp, rm = rho0.clone(), rho0.clone()
        rp[k] += h
        rm[k] -= h
        _, Ap = rt.columns(t, rp, src_d, dirs_d, kappa)
        _, Am = rt.columns(t, rm, src_d, dirs_d, kappa)
        fd[j] = float((w_d * (Ap - Am)).sum() / (2 * h))
    scale = np.abs(grad).max()
    err = np.abs(grad[leaves] - fd)
    assert np.all(err <= 1e-4 * np.abs(fd) + 1e-7 * scale), (err / np.abs(fd)).max()


def test_adjoint_amr128_vs_oracle_sample(rt, orc):
    """Same workload, every 16th source: FP32 adjoint vs the oracle's FP64
    gradient over those rays."""
    w3 = W.make_workload(3)
    src = w3.sources[::16]
    dirs = orc.healpix_ring(w3.nside)
    w = w3.weights()[::16]
    grad, _, _ = _loss_grad(rt, w3.tree, src, dirs, w, w3.kappa)
    ref = orc.columns(w3.tree, src, dirs, w3.kappa, threads=8)
    want = orc.gradient(w3.tree, src, dirs, -w3.kappa * w * ref["A"])
    _close(grad, want, 1e-5, 1e-6)


@pytest.mark.parametrize("S,Dn", [(1, 1), (63, 5), (65, 12), (257, 3), (1000, 1)])
def test_adjoint_ragged_sizes(rt, orc, S, Dn):
    """Ray counts that leave the last wavefront and block partly empty: the
    lockstep adjoint loop must neither lose nor double any ray."""
    tree = W.random_octree(4, 0.45, 40 + S, min_level=1)
    src = W.random_points(S, 41 + S)
    dirs = random_dirs(Dn, 42 + Dn)
    w = np.random.default_rng(43 + S).random((S, Dn))
    grad, _, _ = _loss_grad(rt, tree, src, dirs, w, 1.0)
    ref = orc.columns(tree, src, dirs, 1.0)
    want = orc.gradient(tree, src, dirs, -w * ref["A"])
    _close(grad, want, 1e-5, 1e-6)


def test_adjoint_invalid_and_zero_rays(rt, orc):
    """Sources outside the box give NaN columns and no gradient; rays with a
    zero upstream gradient add nothing; a gradient given with strides other
    than the library's layout is rearranged by the binding.  The result is
    the oracle's gradient over the valid rays alone."""
    tree = W.random_octree(4, 0.5, 51, min_level=1)
    good = W.random_points(150, 52)
    bad = np.array([[1.0, 0.5, 0.5], [0.5, -1e-300, 0.5], [0.25, 0.5, 1.5]])
    src = np.vstack([good[:70], bad, good[70:]])
    valid = np.ones(len(src), bool)
    valid[70:73] = False
    dirs = np.vstack([orc.healpix_ring(1), random_dirs(3, 53)])
    rng = np.random.default_rng(54)
    gN = rng.standard_normal((len(src), len(dirs)))
    gN[rng.random(gN.shape) < 0.3] = 0.0
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    src_d, dirs_d = torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev)
    N, _ = rt.columns(t, torch.as_tensor(tree.rho).to(dev, torch.float32), src_d, dirs_d, 1.0)
    assert bool(torch.isnan(N[70:73]).all()) and not bool(torch.isnan(N[valid]).any())
    g_src_major = torch.as_tensor(gN).to(dev, torch.float32).contiguous()  # strides (Dn, 1)
    grad = rt.columns_backward(t, src_d, dirs_d, 1.0, gN=g_src_major)
    want = orc.gradient(tree, src[valid], dirs, gN[valid])
    _close(grad.cpu().numpy(), want, 1e-5, 1e-6)
