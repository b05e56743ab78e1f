"""HIP forward walk vs the oracle, element by element, on the same inputs.

Bar: bit-exact N (FP64), N32 (FP32-Kahan: same traversal and chords, same
FP32 recurrence), step counts and visited-sequence hashes; A within a few
ulp (two different exp implementations); FP32 within 1e-5 of FP64.  The
direction tables fed to both sides are the oracle's.
"""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import (assert_attenuation, assert_bitexact, assert_fp32_vs_fp64, edge_sources,
                        gpu_walk, random_dirs, random_seeds, require_gpu, special_dirs)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def _compare(rt, orc, tree, src, dirs, kappa=1.0, sample=None, cap=0):
    ref = orc.columns(tree, src, dirs, kappa, rho32=tree.rho.astype(np.float32), threads=8)
    got = gpu_walk(rt, tree, src, dirs, kappa, sample=sample, cap=cap)
    assert_bitexact(got, ref)
    finite = np.isfinite(ref["N"])
    assert_attenuation({k: v[finite] for k, v in got.items() if k in ("A", "A32")},
                       {k: v[finite] for k, v in ref.items() if k in ("A", "A32")})
    return got, ref


def test_uniform32_iid_full(rt, orc):
    """32^3 uniform tree, all 32768 cell centres, 12 HEALPix directions."""
    w = W.make_workload(0)
    dirs = orc.healpix_ring(1)
    S = w.sources.shape[0]
    rng = np.random.default_rng(7)
    sample = rng.choice(S * len(dirs), 64, replace=False)
    cap = 3 * 32 + 3
    got, ref = _compare(rt, orc, w.tree, w.sources, dirs, sample=sample, cap=cap)
    assert_fp32_vs_fp64(got)
    assert ref["clamps"] == 0
    # full visited sequences of sampled rays (ray id r = d * S + s)
    for j, r in enumerate(sample):
        d, s = divmod(int(r), S)
        want = orc.walk_one(w.tree, w.sources[s], dirs[d])["visited"]
        seq = got["visited"][j]
        assert list(seq[:len(want)]) == list(want)
        assert np.all(seq[len(want):] == -1)


@pytest.mark.parametrize("depth,p,seed", [(1, 0.0, 1), (3, 0.7, 2), (4, 0.5, 3), (5, 0.35, 4),
                                          (6, 0.25, 5), (7, 0.12, 6)])
def test_random_amr_trees(rt, orc, depth, p, seed):
    tree = W.random_octree(depth, p, seed, min_level=min(1, depth))
    src = np.vstack([W.random_points(301, seed + 10), edge_sources(depth)])
    dirs = np.vstack([orc.healpix_ring(2), special_dirs(), random_dirs(17, seed + 20)])
    got, _ = _compare(rt, orc, tree, src, dirs, kappa=0.8)
    assert_fp32_vs_fp64(got)


@pytest.mark.parametrize("depth,splits,seed", [(8, 300, 34), (9, 300, 35), (10, 300, 36)])
def test_deep_trees_narrow_keys(rt, orc, depth, splits, seed):
    """Depths 8..10 use 32-bit keys and the LDS spread table; 10 is the
    deepest they cover (8^10 keys, a 1024-entry table).  Sparse trees keep
    the top table shallow, so most lookups take the key search."""
    tree = W.sparse_random_octree(depth, splits, seed)
    deep = W.sparse_random_octree(depth, 60, seed + 1, focus=[0.7, 0.2, 0.9])
    for t in (tree, deep):
        src = np.vstack([W.random_points(97, seed + 2), edge_sources(depth),
                         np.array([[0.7, 0.2, 0.9], [1.0 - 2.0 ** -depth, 0.0, 1.0 - 2.0 ** -53]])])
        dirs = np.vstack([orc.healpix_ring(1), special_dirs(), random_dirs(9, seed + 3)])
        got, _ = _compare(rt, orc, t, src, dirs)
        assert_fp32_vs_fp64(got)


@pytest.mark.parametrize("depth,splits,seed", [(11, 400, 31), (14, 300, 32), (21, 250, 33)])
def test_deep_trees_wide_keys(rt, orc, depth, splits, seed):
    """Depth > 10 uses 64-bit keys on the device."""
    tree = W.sparse_random_octree(depth, splits, seed)
    deep = W.sparse_random_octree(depth, 60, seed + 1, focus=[0.3, 0.6, 0.2])
    for t in (tree, deep):
        src = np.vstack([W.random_points(97, seed + 2), edge_sources(depth),
                         np.array([[0.3, 0.6, 0.2]])])
        dirs = np.vstack([orc.healpix_ring(1), special_dirs(), random_dirs(9, seed + 3)])
        got, _ = _compare(rt, orc, t, src, dirs)
        assert_fp32_vs_fp64(got)


def test_invalid_rays_give_nan(rt, orc):
    tree = W.random_octree(4, 0.5, 41, min_level=1)
    src = np.array([[0.5, 0.5, 0.5], [1.0, 0.5, 0.5], [-1e-300, 0.2, 0.2], [np.nan, 0.1, 0.1],
                    [0.2, 0.3, 0.4]])
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [np.inf, 0.0, 0.0], [0.6, 0.0, 0.8]])
    got = gpu_walk(rt, tree, src, dirs)
    ref = orc.columns(tree, src, dirs, rho32=tree.rho.astype(np.float32))
    bad_src = np.array([False, True, True, True, False])
    bad_dir = np.array([False, True, True, False])
    bad = bad_src[:, None] | bad_dir[None, :]
    assert np.all(np.isnan(got["N"][bad])) and np.all(np.isnan(got["A"][bad]))
    assert np.all(np.isnan(got["N32"][bad]))
    assert np.all(got["steps"][bad] == -1) and np.all(ref["steps"][bad] == -1)
    assert np.array_equal(got["steps"], ref["steps"]) and np.array_equal(got["hash"], ref["hash"])
    assert np.array_equal(got["N"][~bad], ref["N"][~bad])
    assert np.array_equal(got["N32"][~bad], ref["N32"][~bad])


def test_strided_outputs_and_determinism(rt, orc):
    tree = W.random_octree(5, 0.4, 51, min_level=1)
    src = W.random_points(1000, 52)
    dirs = orc.healpix_ring(2)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    rho = torch.as_tensor(tree.rho).to(dev)
    src_d, dirs_d = torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev)
    N1, A1 = rt.columns(t, rho, src_d, dirs_d, 1.0)
    N2, A2 = rt.columns(t, rho, src_d, dirs_d, 1.0)
    assert torch.equal(N1, N2) and torch.equal(A1, A2)
    # source-major layout [S][Dn] through the raw ABI strides
    S, Dn = src.shape[0], dirs.shape[0]
    Nr = torch.full((S, Dn), -1.0, dtype=torch.float64, device=dev)
    rt._abi.rt_columns(t.handle, rho.data_ptr(), rt._abi.RT_FP64, src_d.data_ptr(), S,
                       dirs_d.data_ptr(), Dn, 1.0, Nr.data_ptr(), None, Dn, 1,
                       torch.cuda.current_stream().cuda_stream)
    assert torch.equal(Nr, N1)
    # padded layout: every third slot written, the rest untouched
    P = torch.full((S * Dn * 3,), -7.0, dtype=torch.float64, device=dev)
    rt._abi.rt_columns(t.handle, rho.data_ptr(), rt._abi.RT_FP64, src_d.data_ptr(), S,
                       dirs_d.data_ptr(), Dn, 1.0, P.data_ptr(), None, 3, 3 * S,
                       torch.cuda.current_stream().cuda_stream)
    P = P.view(Dn, S, 3)
    assert torch.equal(P[:, :, 0].t(), N1)
    assert torch.all(P[:, :, 1:] == -7.0)


@pytest.mark.parametrize("S,Dn", [(1, 1), (63, 1), (65, 3), (257, 12), (4097, 5)])
def test_ragged_sizes(rt, orc, S, Dn):
    tree = W.random_octree(4, 0.5, 61, min_level=1)
    src = W.random_points(S, 62 + S)
    dirs = random_dirs(Dn, 63 + Dn)
    _compare(rt, orc, tree, src, dirs)


def test_argument_errors(rt):
    tree = W.random_octree(3, 0.5, 71, min_level=1)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    rho = torch.as_tensor(tree.rho).to(dev)
    src = torch.rand(4, 3, dtype=torch.float64, device=dev)
    dirs = torch.as_tensor(random_dirs(2, 1)).to(dev)
    N = torch.empty(8, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(rt._abi.RtError) as e:
        rt._abi.rt_columns(t.handle, rho.data_ptr(), 0, src.data_ptr(), 0, dirs.data_ptr(), 2,
                           1.0, N.data_ptr(), None, 1, 4, s)
    assert e.value.status == rt._abi.RT_ERR_ARG
    with pytest.raises(rt._abi.RtError):
        rt._abi.rt_columns(t.handle, rho.data_ptr(), 5, src.data_ptr(), 4, dirs.data_ptr(), 2,
                           1.0, N.data_ptr(), None, 1, 4, s)
    with pytest.raises(rt._abi.RtError):
        rt._abi.rt_columns(t.handle, rho.data_ptr(), 0, src.data_ptr(), 4, dirs.data_ptr(), 2,
                           1.0, N.data_ptr(), None, -1, 4, s)
    with pytest.raises(rt._abi.RtError):
        rt._abi.rt_columns(t.handle, rho.data_ptr(), 0, src.data_ptr(), 4, dirs.data_ptr(), 2,
                           float("nan"), N.data_ptr(), None, 1, 4, s)
    with pytest.raises(rt._abi.RtError):
        rt._abi.rt_columns(t.handle, rho.data_ptr(), 0, src.data_ptr(), 1 << 62, dirs.data_ptr(),
                           1 << 3, 1.0, N.data_ptr(), None, 1, 4, s)
    with pytest.raises(ValueError):
        rt.columns(t, rho[:-1].contiguous(), src, dirs)


def test_buffers_on_another_device_are_refused(rt):
    """The kernels take raw pointers, so the binding refuses, before any
    launch, a buffer that is not on the octree's GPU (a host tensor here)."""
    tree = W.random_octree(3, 0.5, 72, min_level=1)
    t = rt.Octree(tree.keys, tree.levels, tree.depth, "cuda")
    assert t.device == torch.device("cuda", torch.cuda.current_device())
    src = torch.rand(4, 3, dtype=torch.float64)
    dirs = random_dirs(2, 1)
    g = torch.ones(4, 2, dtype=torch.float32)
    with pytest.raises(ValueError, match="grad is on cpu"):
        rt.columns_backward(t, src, dirs, 1.0, gN=g, grad=torch.zeros(tree.n, dtype=torch.float64))
    with pytest.raises(ValueError):
        rt.columns(t, torch.as_tensor(tree.rho), src, dirs)
    with pytest.raises(TypeError):
        rt.shielding(t, torch.as_tensor(tree.rho), src, dirs, 1.0)
    # the same calls with device buffers run
    grad = rt.columns_backward(t, src, dirs, 1.0, gN=g)
    torch.cuda.synchronize()
    assert grad.device == t.device and bool(torch.isfinite(grad).all())


@pytest.mark.parametrize("seed", random_seeds())
def test_random_configurations(rt, orc, seed):
    """Seeded random trees (depth 1..9, random refinement), random sources
    (with face and corner points) and directions: bit-exact columns, step
    counts and hashes, and the several-fields walk within its bar."""
    from gpu_common import assert_shielding
    rng = np.random.default_rng(seed)
    depth = int(rng.integers(1, 10))
    p = float(rng.uniform(0.05, 0.6))
    tree = W.random_octree(depth, p, seed, min_level=min(int(rng.integers(0, 3)), depth))
    src = np.vstack([W.random_points(int(rng.integers(1, 400)), seed + 1), edge_sources(depth)])
    dirs = np.vstack([random_dirs(int(rng.integers(1, 40)), seed + 2), special_dirs()])
    _compare(rt, orc, tree, src, dirs, kappa=float(rng.uniform(0.1, 3.0)))
    K = int(rng.integers(1, 9))
    inp = W.line_inputs(tree, src, K - 1, seed + 3)
    ref = orc.shielding(tree, inp["fields"], src, dirs, length=inp["length"], temp=inp["temp"],
                        vturb=inp["vturb"], line_A=inp["line_A"], line_nu=inp["line_nu"], threads=8)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    got = rt.shielding(t, torch.as_tensor(inp["fields"]).to(dev), torch.as_tensor(src).to(dev),
                       torch.as_tensor(dirs).to(dev), inp["length"], temp=inp["temp"],
                       vturb=inp["vturb"], line_A=inp["line_A"], line_nu=inp["line_nu"], rays=True)
    torch.cuda.synchronize()
    assert_shielding({k: v.cpu().numpy() for k, v in got.items()}, ref, len(dirs))


def test_more_rays_than_one_dispatch(rt, orc):
    """2^28 sources x 17 directions = 4.56e9 rays, more work items than one
    dispatch counts (2^32 - 1): the launches cap their grids and stride.
    Sampled rays beyond index 2^32 (and the last one) against the oracle,
    bit for bit, with their visited lists, and the adjoint's linearity
    identity over every ray."""
    dev = torch.device("cuda")
    tree = W.random_octree(3, 0.5, 61, min_level=1)
    rho32_h = tree.rho.astype(np.float32)
    S, Dn = 1 << 28, 17
    gen = torch.Generator(device=dev)
    gen.manual_seed(62)
    src = torch.rand((S, 3), generator=gen, device=dev, dtype=torch.float64)
    dirs = random_dirs(Dn, 63)
    dirs_d = torch.as_tensor(dirs).to(dev)
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    rho32 = torch.as_tensor(rho32_h).to(dev)
    N32, A32 = rt.columns(t, rho32, src, dirs_d, 1.0)
    total = S * Dn
    rng = np.random.default_rng(64)
    sample = np.concatenate([rng.integers(1 << 32, total, 300), rng.integers(0, total, 100),
                             [total - 1, (1 << 32) - 1, 1 << 32]]).astype(np.int64)
    cap = 3 * 8 + 3
    sample_d = torch.as_tensor(sample).to(dev)
    visited = torch.empty((len(sample), cap), dtype=torch.int32, device=dev)
    # the visited lists of the sampled rays only (no per-ray steps or hashes)
    rt._abi.rt_columns_trace(t.handle, src.data_ptr(), S, dirs_d.data_ptr(), Dn, None, None, 1, S,
                             sample_d.data_ptr(), len(sample), visited.data_ptr(), cap,
                             torch.cuda.current_stream().cuda_stream)
    d_idx, s_idx = np.divmod(sample, S)
    si = torch.as_tensor(s_idx).to(dev)
    got = N32[si, torch.as_tensor(d_idx).to(dev)].cpu().numpy()
    src_h = src[si].cpu().numpy()
    vis = visited.cpu().numpy()
    for j in range(len(sample)):
        r = orc.walk_one(tree, src_h[j], dirs[d_idx[j]], rho32=rho32_h)
        assert got[j] == np.float32(r["N32"]), (int(sample[j]), got[j], r["N32"])
        k = len(r["visited"])
        assert list(vis[j, :k]) == list(r["visited"]) and np.all(vis[j, k:] == -1)
    del N32
    # adjoint over every ray: sum_k rho_k grad_k = sum_r g_r N_r, g = -A (w = 1),
    # with N from the FP64 walk; the sums run one direction at a time
    ones = torch.ones((Dn, S), dtype=torch.float32, device=dev).t()
    grad = rt.columns_backward(t, src, dirs_d, 1.0, gA=ones, A=A32)
    del ones
    N64, _ = rt.columns(t, rho32.double(), src, dirs_d, 1.0, with_A=False)
    lhs = float((rho32.double() * grad).sum())
    rhs = -sum(float((A32[:, d].double() * N64[:, d]).sum()) for d in range(Dn))
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
