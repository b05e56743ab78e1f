"""HIP several-fields walk (rt_shielding) vs the oracle, on the same inputs.

Bar (derived from the arithmetic of both sides):
  * per-ray N_H: bit-exact (the same walk, the same FP64 sum, one product);
  * per-ray tau: within 4 ulp (the same products and quotients, and a
    square root that is correctly rounded on both sides: the slack only
    guards the quotient and root implementations);
  * beta: each term -expm1(-tau)/tau within about 2 ulp between the two
    libm implementations, summed in the same order over Dn positive terms:
    relative (2 Dn + 8) eps;
  * A_V,eff: the oracle takes min and sum in two passes, the kernel keeps a
    running minimum and rescales its sum; the mean of exponentials then
    agrees to about (2 Dn + 4) eps relative, so ln(mean) / gamma to that
    over gamma, absolute, plus 8 eps relative of the value.
"""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import assert_shielding, edge_sources, random_dirs, require_gpu, special_dirs

pytestmark = pytest.mark.gpu

GAMMA, AV0 = 3.02, 6.29e-22


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def gpu_shielding(rt, tree, fields, src, dirs, inp, rays=True, av_eff=True, beta=True,
                  gamma=GAMMA, av0=AV0, f32=False):
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    F = torch.as_tensor(np.ascontiguousarray(fields, dtype=np.float32 if f32 else np.float64)).to(dev)
    out = rt.shielding(t, F, torch.as_tensor(src).to(dev), torch.as_tensor(dirs).to(dev),
                       inp["length"], temp=inp.get("temp"), vturb=inp.get("vturb", 0.0),
                       line_A=inp.get("line_A", ()), line_nu=inp.get("line_nu", ()),
                       gamma=gamma, av0=av0, rays=rays, av_eff=av_eff, beta=beta)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_shielding(orc, tree, fields, src, dirs, inp, gamma=GAMMA, av0=AV0):
    return orc.shielding(tree, fields, src, dirs, length=inp["length"], temp=inp.get("temp"),
                         vturb=inp.get("vturb", 0.0), line_A=inp.get("line_A", ()),
                         line_nu=inp.get("line_nu", ()), gamma=gamma, av0=av0, threads=8)


def _inputs(tree, src, n_lines, seed):
    inp = W.line_inputs(tree, src, n_lines, seed)
    return inp["fields"], inp


@pytest.mark.parametrize("depth,p,seed,n_lines", [(1, 0.0, 11, 0), (3, 0.6, 12, 1), (4, 0.5, 13, 3),
                                                   (5, 0.35, 14, 7), (6, 0.2, 15, 2), (4, 0.45, 16, 4),
                                                   (5, 0.3, 17, 5), (3, 0.5, 18, 6)])
def test_random_amr_trees(rt, orc, depth, p, seed, n_lines):
    tree = W.random_octree(depth, p, seed, min_level=min(1, depth))
    src = np.vstack([W.random_points(200, seed + 10), edge_sources(depth),
                     [[1.0, 0.5, 0.5], [0.5, -1e-300, 0.5]]])  # two sources outside the box
    dirs = np.vstack([orc.healpix_ring(2), special_dirs(), random_dirs(9, seed + 20)])
    fields, inp = _inputs(tree, src, n_lines, seed + 30)
    ref = oracle_shielding(orc, tree, fields, src, dirs, inp)
    assert ref["status"] == orc.ERR_RANGE  # the two outside sources
    got = gpu_shielding(rt, tree, fields, src, dirs, inp)
    assert_shielding(got, ref, len(dirs))
    assert np.isnan(got["av_eff"][-2:]).all() and not np.isnan(got["av_eff"][:-2]).any()


@pytest.mark.parametrize("depth", [10, 11, 14, 21])
def test_deep_trees_wide_keys(rt, orc, depth):
    """10 is the deepest tree with 32-bit keys; beyond, 64-bit keys."""
    tree = W.sparse_random_octree(depth, 40, 300 + depth)
    tree.rho = np.random.default_rng(depth).lognormal(0.0, 1.0, tree.n)
    src = np.vstack([W.random_points(150, 310 + depth), [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]])
    dirs = np.vstack([orc.healpix_ring(1), special_dirs()])
    fields, inp = _inputs(tree, src, 3, 320 + depth)
    ref = oracle_shielding(orc, tree, fields, src, dirs, inp)
    got = gpu_shielding(rt, tree, fields, src, dirs, inp)
    assert_shielding(got, ref, len(dirs))


def test_uniform32_full(rt, orc):
    """All 32768 cell centres of the 32^3 cloud, 12 directions, 4 fields."""
    w = W.make_workload(0)
    dirs = orc.healpix_ring(1)
    fields, inp = _inputs(w.tree, w.sources, 3, 6000)
    ref = oracle_shielding(orc, w.tree, fields, w.sources, dirs, inp)
    got = gpu_shielding(rt, w.tree, fields, w.sources, dirs, inp)
    assert_shielding(got, ref, len(dirs))


@pytest.mark.parametrize("S,Dn", [(1, 1), (63, 5), (65, 12), (257, 3), (1000, 48)])
def test_ragged_sizes(rt, orc, S, Dn):
    tree = W.random_octree(4, 0.4, 41, min_level=1)
    src = W.random_points(S, 42 + S)
    dirs = random_dirs(Dn, 43 + Dn)
    fields, inp = _inputs(tree, src, 2, 44)
    ref = oracle_shielding(orc, tree, fields, src, dirs, inp)
    got = gpu_shielding(rt, tree, fields, src, dirs, inp)
    assert_shielding(got, ref, Dn)


def test_optional_outputs_and_extremes(rt, orc):
    """Each output alone equals the same output of the full call; a huge
    density (gamma av0 N in the thousands, where exp underflows) and
    gamma = 1e-9 stay within the bar."""
    tree = W.random_octree(4, 0.45, 51, min_level=1)
    src = W.random_points(300, 52)
    dirs = orc.healpix_ring(2)
    fields, inp = _inputs(tree, src, 2, 53)
    full = gpu_shielding(rt, tree, fields, src, dirs, inp)
    only_av = gpu_shielding(rt, tree, fields, src, dirs, inp, rays=False, beta=False)
    only_beta = gpu_shielding(rt, tree, fields, src, dirs, inp, rays=False, av_eff=False)
    assert set(only_av) == {"av_eff"} and set(only_beta) == {"beta"}
    assert np.array_equal(only_av["av_eff"], full["av_eff"])
    assert np.array_equal(only_beta["beta"], full["beta"])
    for scale, gamma in ((1e6, GAMMA), (1.0, 1e-9)):
        f = fields.copy()
        f[:, 0] *= scale
        ref = oracle_shielding(orc, tree, f, src, dirs, inp, gamma=gamma)
        got = gpu_shielding(rt, tree, f, src, dirs, inp, gamma=gamma)
        assert np.isfinite(got["av_eff"]).all()
        assert_shielding(got, ref, len(dirs), gamma=gamma)


def test_single_field_needs_no_lines(rt, orc):
    tree = W.random_octree(3, 0.5, 61, min_level=1)
    src = W.random_points(100, 62)
    dirs = orc.healpix_ring(1)
    inp = {"length": 2.0e20}
    ref = oracle_shielding(orc, tree, tree.rho * 30.0, src, dirs, inp)
    got = gpu_shielding(rt, tree, tree.rho[:, None] * 30.0, src, dirs, inp)
    assert "beta" not in got
    assert_shielding(got, ref, len(dirs))


@pytest.mark.parametrize("depth,p,seed,n_lines", [(3, 0.6, 112, 0), (4, 0.5, 113, 3),
                                                   (5, 0.35, 114, 7), (6, 0.2, 115, 1)])
def test_f32_fields(rt, orc, depth, p, seed, n_lines):
    """rt_shielding_f32: against the oracle fed the same FP32 values (to the
    bar above), and bit for bit against rt_shielding on those values widened
    to FP64 (the kernel widens each field exactly before the same
    arithmetic)."""
    tree = W.random_octree(depth, p, seed, min_level=1)
    src = np.vstack([W.random_points(200, seed + 10), edge_sources(depth)])
    dirs = np.vstack([orc.healpix_ring(2), special_dirs(), random_dirs(5, seed + 20)])
    fields, inp = _inputs(tree, src, n_lines, seed + 30)
    f32 = fields.astype(np.float32)
    ref = oracle_shielding(orc, tree, f32.astype(np.float64), src, dirs, inp)
    got = gpu_shielding(rt, tree, f32, src, dirs, inp, f32=True)
    assert_shielding(got, ref, len(dirs))
    wide = gpu_shielding(rt, tree, f32.astype(np.float64), src, dirs, inp)
    for k in got:
        a, b = got[k], wide[k]
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), k


def test_f32_deep_tree_and_ragged(rt, orc):
    tree = W.sparse_random_octree(14, 40, 414)
    src = W.random_points(65, 415)
    dirs = random_dirs(7, 416)
    fields, inp = _inputs(tree, src, 2, 417)
    f32 = fields.astype(np.float32)
    ref = oracle_shielding(orc, tree, f32.astype(np.float64), src, dirs, inp)
    got = gpu_shielding(rt, tree, f32, src, dirs, inp, f32=True)
    assert_shielding(got, ref, len(dirs))


def test_argument_errors(rt):
    dev = torch.device("cuda")
    tree = W.random_octree(2, 0.5, 71, min_level=1)
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    src = torch.full((4, 3), 0.5, dtype=torch.float64, device=dev)
    dirs = torch.as_tensor(special_dirs()).to(dev)
    ok = dict(temp=np.full(4, 20.0), vturb=1e5, line_A=[1e-7], line_nu=[1e11])
    F2 = torch.ones((tree.n, 2), dtype=torch.float64, device=dev)
    Err = rt._abi.RtError
    for bad in (dict(line_nu=[0.0]), dict(line_nu=[-1e11]), dict(line_A=[float("nan")]),
                dict(vturb=float("inf"))):
        with pytest.raises(Err):
            rt.shielding(t, F2, src, dirs, 1.0, **{**ok, **bad})
    with pytest.raises(Err):
        rt.shielding(t, F2, src, dirs, 1.0, gamma=0.0, **ok)
    with pytest.raises(Err):
        rt.shielding(t, F2, src, dirs, float("nan"), **ok)
    F9 = torch.ones((tree.n, 9), dtype=torch.float64, device=dev)
    with pytest.raises(Err):
        rt.shielding(t, F9, src, dirs, 1.0, temp=ok["temp"], line_A=[1e-7] * 8, line_nu=[1e11] * 8)
    lib = rt._abi.load()
    av = torch.empty(4, dtype=torch.float64, device=dev)
    # lines without temperatures, and no fields, are refused by the library itself
    assert lib.rt_shielding(t.handle, F2.data_ptr(), 2, src.data_ptr(), 4, dirs.data_ptr(),
                            dirs.shape[0], 1.0, None, 0.0, None, None, GAMMA, AV0, None,
                            av.data_ptr(), None, None) == rt._abi.RT_ERR_ARG
    assert lib.rt_shielding(t.handle, None, 1, src.data_ptr(), 4, dirs.data_ptr(), dirs.shape[0],
                            1.0, None, 0.0, None, None, GAMMA, AV0, None, av.data_ptr(), None,
                            None) == rt._abi.RT_ERR_ARG
    assert lib.rt_shielding_f32(t.handle, None, 1, src.data_ptr(), 4, dirs.data_ptr(), dirs.shape[0],
                                1.0, None, 0.0, None, None, GAMMA, AV0, None, av.data_ptr(), None,
                                None) == rt._abi.RT_ERR_ARG
    F2f = torch.ones((tree.n, 2), dtype=torch.float32, device=dev)
    assert lib.rt_shielding_f32(t.handle, F2f.data_ptr(), 2, src.data_ptr(), 4, dirs.data_ptr(),
                                dirs.shape[0], 1.0, None, 0.0, None, None, GAMMA, AV0, None,
                                av.data_ptr(), None, None) == rt._abi.RT_ERR_ARG
    with pytest.raises(TypeError):
        rt.shielding(t, F2.to(torch.float16), src, dirs, 1.0, **ok)
    assert lib.rt_shielding(t.handle, F2.data_ptr(), 0, src.data_ptr(), 4, dirs.data_ptr(),
                            dirs.shape[0], 1.0, None, 0.0, None, None, GAMMA, AV0, None,
                            av.data_ptr(), None, None) == rt._abi.RT_ERR_ARG
