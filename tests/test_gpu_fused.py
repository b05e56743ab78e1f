"""The forward and its adjoint in one pass (rt_columns_with_adjoint) for a
loss linear in N and A, against the separate calls and the oracle.

Bars: N and A bit-identical to rt_columns (RT_FP32_KAHAN); the gradient
within 1e-5 relative of the oracle's FP64 gradient (floor 1e-6 max|grad|),
as for rt_columns_backward, and within the same bar of the separate
rt_columns_backward call, whose additions run in another order.
"""

import os

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import edge_sources, random_dirs, random_seeds, require_gpu, special_dirs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def _close(got, want, rel=1e-5, floor=1e-6):
    scale = np.abs(want).max()
    err = np.abs(got - want)
    bad = np.nonzero(err > rel * np.abs(want) + floor * scale)[0]
    assert len(bad) == 0, f"{len(bad)} of {len(want)} leaves off"


def _same(a, b):
    """Equal values, NaN where the other has NaN (invalid rays)."""
    return np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True)


def _run(rt, orc, tree, src, dirs, kappa, wN, wA):
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    r32 = torch.as_tensor(tree.rho.astype(np.float32)).to(dev)
    src_d, dirs_d = torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev)
    tw = lambda x: None if x is None else torch.as_tensor(x).to(dev, torch.float32)  # noqa: E731
    N, A, grad = rt.columns_with_adjoint(t, r32, src_d, dirs_d, kappa, wN=tw(wN), wA=tw(wA))
    N0, A0 = rt.columns(t, r32, src_d, dirs_d, kappa)
    assert _same(N, N0) and _same(A, A0), "N and A differ from rt_columns"
    sep = rt.columns_backward(t, src_d, dirs_d, kappa, gN=tw(wN), gA=tw(wA), A=A0)
    torch.cuda.synchronize()
    got, sep = grad.cpu().numpy(), sep.cpu().numpy()
    valid = ~np.isnan(N0.cpu().numpy()).any(axis=1)
    ref = orc.columns(tree, src[valid], dirs, kappa, rho32=tree.rho.astype(np.float32))
    g = np.zeros((int(valid.sum()), len(dirs)))
    if wN is not None:
        g = g + wN[valid]
    if wA is not None:
        g = g - kappa * ref["A32"].astype(np.float64) * wA[valid]
    want = orc.gradient(tree, src[valid], dirs, g)
    _close(got, want)
    _close(got, sep)
    return got


@pytest.mark.parametrize("seed,depth,p", [(1, 4, 0.5), (2, 6, 0.2), (3, 7, 0.1)])
def test_random_trees(rt, orc, seed, depth, p):
    tree = W.random_octree(depth, p, seed, min_level=1)
    src = np.vstack([W.random_points(300, seed + 1), edge_sources(depth)])
    dirs = np.vstack([orc.healpix_ring(2), special_dirs(), random_dirs(5, seed + 2)])
    rng = np.random.default_rng(seed + 3)
    wA = rng.random((len(src), len(dirs)))
    wN = rng.standard_normal((len(src), len(dirs)))
    _run(rt, orc, tree, src, dirs, 0.8, None, wA)
    _run(rt, orc, tree, src, dirs, 1.1, wN, wA)
    _run(rt, orc, tree, src, dirs, 1.0, wN, None)


@pytest.mark.parametrize("S,Dn", [(1, 1), (63, 5), (65, 12), (257, 3)])
def test_ragged_sizes(rt, orc, S, Dn):
    tree = W.random_octree(4, 0.45, 60 + S, min_level=1)
    src = W.random_points(S, 61 + S)
    dirs = random_dirs(Dn, 62 + Dn)
    wA = np.random.default_rng(63 + S).random((S, Dn))
    _run(rt, orc, tree, src, dirs, 1.0, None, wA)


def test_invalid_sources_and_zero_weights(rt, orc):
    """Sources outside the box get N = A = NaN and add nothing; zero weights
    add nothing."""
    tree = W.random_octree(4, 0.5, 71, min_level=1)
    good = W.random_points(120, 72)
    src = np.vstack([good[:50], [[1.0, 0.5, 0.5], [0.5, -1e-300, 0.5]], good[50:]])
    dirs = orc.healpix_ring(1)
    rng = np.random.default_rng(73)
    wA = rng.random((len(src), len(dirs)))
    wA[rng.random(wA.shape) < 0.3] = 0.0
    _run(rt, orc, tree, src, dirs, 1.0, None, wA)


@pytest.mark.parametrize("depth", [10, 14])
def test_deep_trees(rt, orc, depth):
    """10: the deepest tree with 32-bit keys and the LDS spread table; 14:
    64-bit keys."""
    tree = W.sparse_random_octree(depth, 30, 81)
    src = W.random_points(200, 82)
    dirs = np.vstack([orc.healpix_ring(1), special_dirs()])
    wA = np.random.default_rng(83).random((len(src), len(dirs)))
    _run(rt, orc, tree, src, dirs, 1.0, None, wA)


@pytest.mark.parametrize("seed", random_seeds())
def test_random_configurations(rt, orc, seed):
    """Seeded random trees (depth 1..9), sources with face and corner
    points, directions, kappa, and loss weights on A alone or on N and A."""
    rng = np.random.default_rng(seed + 77)
    depth = int(rng.integers(1, 10))
    tree = W.random_octree(depth, float(rng.uniform(0.05, 0.6)), seed + 5, min_level=min(1, depth))
    src = np.vstack([W.random_points(int(rng.integers(1, 300)), seed + 6), edge_sources(depth)])
    dirs = np.vstack([random_dirs(int(rng.integers(1, 30)), seed + 7), special_dirs()])
    wA = rng.random((len(src), len(dirs)))
    wN = rng.random((len(src), len(dirs))) if seed % 2 else None
    _run(rt, orc, tree, src, dirs, float(rng.uniform(0.1, 2.0)), wN, wA)


def test_without_weights_only_the_forward_runs(rt):
    tree = W.random_octree(3, 0.5, 91, min_level=1)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    r32 = torch.as_tensor(tree.rho.astype(np.float32)).to(dev)
    src = torch.as_tensor(W.random_points(70, 92)).to(dev)
    dirs = torch.as_tensor(random_dirs(3, 93)).to(dev)
    grad = torch.full((tree.n,), 2.5, dtype=torch.float64, device=dev)
    N, A, g = rt.columns_with_adjoint(t, r32, src, dirs, 1.0, grad=grad)
    N0, A0 = rt.columns(t, r32, src, dirs, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(N, N0) and torch.equal(A, A0)
    assert g is grad and bool((grad == 2.5).all())


def test_argument_errors(rt):
    tree = W.random_octree(3, 0.5, 95, min_level=1)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    r32 = torch.as_tensor(tree.rho.astype(np.float32)).to(dev)
    src = torch.rand(4, 3, dtype=torch.float64, device=dev)
    dirs = torch.as_tensor(random_dirs(2, 96)).to(dev)
    buf = torch.empty(8, dtype=torch.float32, device=dev)
    grad = torch.zeros(tree.n, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    lib = rt._abi.load()
    E = rt._abi.RT_ERR_ARG
    args = [t.handle, r32.data_ptr(), src.data_ptr(), 4, dirs.data_ptr(), 2, 1.0, buf.data_ptr(),
            None, buf.data_ptr(), None, 1, 4, grad.data_ptr(), s]
    for i, v in ((1, None), (9, None), (13, None), (6, float("nan")), (3, 0), (11, -1)):
        a = list(args)
        a[i] = v
        assert lib.rt_columns_with_adjoint(*a) == E, i
    with pytest.raises(TypeError):
        rt.columns_with_adjoint(t, r32.double(), src, dirs, 1.0, wA=torch.ones(4, 2))


def test_merged512_fullsize(rt, orc):
    """The benchmark's pass at full size (1.6e9 rays): N and A bit-identical to
    rt_columns on every ray, the gradient equal to the separate adjoint's
    within 1e-5 (the order of additions differs), the identity
    sum_k rho_k grad_k = sum_r g_r N_r over every ray, and the oracle's
    gradient of a 1/4096 source subsample walked by both paths."""
    w = W.make_workload(4)
    dev = torch.device("cuda")
    t = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    r32 = torch.as_tensor(w.tree.rho.astype(np.float32)).to(dev)
    src = torch.as_tensor(w.sources).to(dev)
    dirs = torch.as_tensor(rt.healpix_dirs(w.nside)).to(dev)
    S, Dn = src.shape[0], dirs.shape[0]
    gen = torch.Generator(device=dev)
    gen.manual_seed(3004)
    wA = torch.rand((Dn, S), device=dev, generator=gen).t()
    N, A, grad = rt.columns_with_adjoint(t, r32, src, dirs, w.kappa, wA=wA)
    N0, A0 = rt.columns(t, r32, src, dirs, w.kappa)
    assert torch.equal(N, N0) and torch.equal(A, A0)
    del N0
    sep = rt.columns_backward(t, src, dirs, w.kappa, gA=wA, A=A0)
    _close(grad.cpu().numpy(), sep.cpu().numpy())
    g = -w.kappa * A.double() * wA.double()
    rhs = float((g * N.double()).sum())
    lhs = float((r32.double() * grad).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs)
    # the oracle on a subsample: both paths on those sources only
    sub = w.sources[::4096]
    wsub = wA[::4096].cpu().numpy().astype(np.float64)
    _, _, gsub = rt.columns_with_adjoint(t, r32, torch.as_tensor(sub).to(dev), dirs, w.kappa,
                                         wA=torch.as_tensor(wsub).to(dev, torch.float32))
    ref = orc.columns(w.tree, sub, dirs.cpu().numpy(), w.kappa, rho32=w.tree.rho.astype(np.float32),
                      threads=8)
    want = orc.gradient(w.tree, sub, dirs.cpu().numpy(), -w.kappa * ref["A32"].astype(np.float64) * wsub)
    _close(gsub.cpu().numpy(), want)


def test_A_output_is_optional(rt):
    """With d_A = NULL the kernel still forms A for g = -kappa A wA; the
    gradient equals the one of the call that stores A."""
    tree = W.random_octree(4, 0.4, 97, min_level=1)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    r32 = torch.as_tensor(tree.rho.astype(np.float32)).to(dev)
    S, Dn = 300, 12
    src = torch.as_tensor(W.random_points(S, 98)).to(dev)
    dirs = torch.as_tensor(random_dirs(Dn, 99)).to(dev)
    wA = torch.rand((Dn, S), device=dev)
    N = torch.empty((Dn, S), dtype=torch.float32, device=dev)
    g1 = torch.zeros(tree.n, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    rt._abi.rt_columns_with_adjoint(t.handle, r32.data_ptr(), src.data_ptr(), S, dirs.data_ptr(), Dn,
                                    1.0, None, wA.data_ptr(), N.data_ptr(), None, 1, S,
                                    g1.data_ptr(), s)
    N2, _, g2 = rt.columns_with_adjoint(t, r32, src, dirs, 1.0, wA=wA.t())
    torch.cuda.synchronize()
    assert torch.equal(N.t(), N2)
    _close(g1.cpu().numpy(), g2.cpu().numpy())


@pytest.mark.timeout(1200)
@pytest.mark.skipif(not os.environ.get("RAYWALK_GRADIENT_512"),
                    reason='about 25 minutes of oracle work on 16 cores, run in parts: set '
                           'RAYWALK_GRADIENT_512="a:b" for the rays of sources a..b-1')
def test_gradient_of_every_ray_merged_512(rt, orc):
    """The fused pass's gradient for the rays of sources a..b-1 of the 512^3
    cloud (RAYWALK_GRADIENT_512 = "a:b"; all: 0:134217728) against the
    oracle's FP64 gradient of the same rays, leaf by leaf.  The loss is
    L = sum wN N with the benchmark's seeded weights, so g = wN is known to
    both sides without a forward pass; the A term is covered by the tests
    above.  The oracle's gradient is summed over source blocks walked on every
    core (its calls release the interpreter's lock) and reports as it goes."""
    import concurrent.futures as cf
    import time

    a0, b0 = (int(x) for x in os.environ["RAYWALK_GRADIENT_512"].split(":"))
    w = W.make_workload(4)
    S = w.sources.shape[0]
    assert 0 <= a0 < b0 <= S
    dev = torch.device("cuda")
    t = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    r32 = torch.as_tensor(w.tree.rho.astype(np.float32)).to(dev)
    dirs_h = rt.healpix_dirs(w.nside)
    assert np.array_equal(dirs_h, orc.healpix_ring(w.nside))
    dirs = torch.as_tensor(dirs_h).to(dev)
    Dn = dirs.shape[0]
    gen = torch.Generator(device=dev)
    gen.manual_seed(3004)
    wN = torch.rand((Dn, S), device=dev, generator=gen).t()[a0:b0]
    src = torch.as_tensor(w.sources[a0:b0]).to(dev)
    _, _, grad = rt.columns_with_adjoint(t, r32, src, dirs, w.kappa, wN=wN)
    got = grad.cpu().numpy()
    g = wN.cpu().numpy().astype(np.float64)
    del grad, wN, src
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    bounds = np.linspace(0, b0 - a0, 8 * cores + 1).astype(np.int64)
    want = np.zeros(w.tree.n)
    t0 = time.perf_counter()

    def block(j):
        a, b = int(bounds[j]), int(bounds[j + 1])
        return orc.gradient(w.tree, w.sources[a0 + a:a0 + b], dirs_h, g[a:b])

    with cf.ThreadPoolExecutor(cores) as pool:
        futures = [pool.submit(block, j) for j in range(len(bounds) - 1)]
        for k, f in enumerate(cf.as_completed(futures)):
            want += f.result()
            if k % cores == cores - 1:
                print(f"[{w.name}] oracle gradient: {k + 1} of {len(futures)} source blocks, "
                      f"{time.perf_counter() - t0:.0f} s", flush=True)
    _close(got, want)
    print(f"[{w.name}] sources {a0}..{b0}: every leaf within the bar", flush=True)
