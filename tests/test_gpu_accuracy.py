"""The angular-resolution comparison (rt_nested_reference and the study
functions built on it) against the oracle, on the same inputs.

Bar: reference means and relative errors bit-exact (both sides sum the
4^k values in index order and divide once); e_N of a sky map bit-exact (the
columns are); e_AV within the A_V,eff bar of the several-fields walk carried
through the quotient.  The oracle's NESTED table is fed to both sides.
"""

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import require_gpu

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


@pytest.mark.parametrize("S,dc,k", [(1, 12, 0), (1, 12, 3), (7, 48, 1), (1000, 12, 2), (257, 3, 1)])
def test_nested_reference_kernel(rt, orc, S, dc, k):
    from paper_2605_09882_amd import accuracy
    rng = np.random.default_rng(S + dc + k)
    df = dc * 4 ** k
    fine = rng.lognormal(0.0, 1.0, (S, df))
    coarse = rng.lognormal(0.0, 1.0, (S, dc))
    dev = torch.device("cuda")
    # direction-major buffers with [S, D] views, as columns() returns them
    f = torch.as_tensor(np.ascontiguousarray(fine.T)).to(dev).t()
    c = torch.as_tensor(np.ascontiguousarray(coarse.T)).to(dev).t()
    ref, err = accuracy.nested_reference(f, c)
    want_ref, want_err = orc.nested_reference(fine, coarse)
    assert np.array_equal(ref.cpu().numpy(), want_ref)
    assert np.array_equal(err.cpu().numpy(), want_err)


def test_nested_reference_errors(rt):
    lib = rt._abi.load()
    dev = torch.device("cuda")
    buf = torch.ones(64, dtype=torch.float64, device=dev)
    out = torch.empty(64, dtype=torch.float64, device=dev)
    p = buf.data_ptr()
    E = rt._abi.RT_ERR_ARG
    assert lib.rt_nested_reference(p, 24, p, 12, 1, out.data_ptr(), None, None) == E  # ratio 2
    assert lib.rt_nested_reference(p, 96, p, 12, 1, out.data_ptr(), None, None) == E  # ratio 8
    assert lib.rt_nested_reference(p, 6, p, 12, 1, out.data_ptr(), None, None) == E   # fine < coarse
    assert lib.rt_nested_reference(p, 13, p, 12, 1, out.data_ptr(), None, None) == E  # not a multiple
    assert lib.rt_nested_reference(None, 48, p, 12, 1, out.data_ptr(), None, None) == E
    assert lib.rt_nested_reference(p, 48, None, 12, 1, None, out.data_ptr(), None) == E
    assert lib.rt_nested_reference(p, 48, p, 12, 0, out.data_ptr(), None, None) == E


def _cloud(n=32, seed=77):
    g = W.gaussian_random_field(n, -4.0, seed)
    nh = 10.0 * W.lognormal(g, 2.0)
    return W.uniformity_merged_octree(nh, 1.0, 0.01), nh


@pytest.mark.parametrize("point", [[0.5, 0.5, 0.5], [0.3, 0.61, 0.47]])
def test_sky_map_errors(rt, orc, point):
    from paper_2605_09882_amd import accuracy
    tree_h, _ = _cloud()
    dev = torch.device("cuda")
    tree = rt.Octree(tree_h.keys, tree_h.levels, tree_h.depth, dev)
    rho = torch.as_tensor(tree_h.rho).to(dev)
    dirs_of = lambda lv: orc.healpix_nested(1 << lv)  # noqa: E731
    got = accuracy.sky_map_errors(tree, rho, point, levels=(0, 1, 2), ref_level=4, dirs_of=dirs_of)
    Nref = orc.columns(tree_h, [point], dirs_of(4))["N"]
    for lv in (0, 1, 2):
        N = orc.columns(tree_h, [point], dirs_of(lv))["N"]
        _, want = orc.nested_reference(Nref, N)
        assert np.array_equal(got[lv]["e_N"], want[0]), lv
        assert got[lv]["rays"] == 12 * 4 ** lv


def test_av_eff_errors(rt, orc):
    from paper_2605_09882_amd import accuracy
    tree_h, _ = _cloud(16, 78)
    dev = torch.device("cuda")
    tree = rt.Octree(tree_h.keys, tree_h.levels, tree_h.depth, dev)
    nh = torch.as_tensor(tree_h.rho).to(dev)
    cells = W.cell_centres(4)
    length = 3.0e20
    dirs_of = lambda lv: orc.healpix_nested(1 << lv)  # noqa: E731
    got, ref = accuracy.av_eff_errors(tree, nh, cells, length, levels=(0, 1), ref_level=3,
                                      dirs_of=dirs_of)
    want_ref = orc.shielding(tree_h, tree_h.rho, cells, dirs_of(3), length=length, rays=False,
                             threads=8)["av_eff"]
    tol_ref = (2 * 768 + 4) * EPS / 3.02 + 8 * EPS * want_ref
    assert np.all(np.abs(ref - want_ref) <= tol_ref)
    for lv in (0, 1):
        av = orc.shielding(tree_h, tree_h.rho, cells, dirs_of(lv), length=length, rays=False,
                           threads=8)["av_eff"]
        want = np.abs(av - want_ref) / want_ref
        tol_av = (2 * 12 * 4 ** lv + 4) * EPS / 3.02 + 8 * EPS * av
        # the quotient moves by at most the two A_V,eff tolerances over the reference
        tol = (tol_av + tol_ref * (1 + want)) / want_ref + 4 * EPS * want
        assert np.all(np.abs(got[lv]["e_AV"] - want) <= tol), lv


def test_study_sky_map_fullsize(rt, orc):
    """The study's 128^3 cloud, sky map from the centre at levels 0..3
    against level 6 (49152 rays), as the study runs it, bit for bit."""
    from paper_2605_09882_amd import accuracy
    g = W.gaussian_random_field(128, -4.0, 1005)
    nh = 10.0 * W.lognormal(g, 2.0)
    tree_h = W.uniformity_merged_octree(nh, 1.0, 0.01)
    dev = torch.device("cuda")
    tree = rt.Octree(tree_h.keys, tree_h.levels, tree_h.depth, dev)
    rho = torch.as_tensor(tree_h.rho).to(dev)
    dirs_of = lambda lv: orc.healpix_nested(1 << lv)  # noqa: E731
    got = accuracy.sky_map_errors(tree, rho, [0.5, 0.5, 0.5], dirs_of=dirs_of)
    Nref = orc.columns(tree_h, [[0.5, 0.5, 0.5]], dirs_of(6), threads=8)["N"]
    for lv in (0, 1, 2, 3):
        N = orc.columns(tree_h, [[0.5, 0.5, 0.5]], dirs_of(lv))["N"]
        _, want = orc.nested_reference(Nref, N)
        assert np.array_equal(got[lv]["e_N"], want[0]), lv
    # the error shrinks with resolution on average
    means = [got[lv]["e_N"].mean() for lv in (0, 1, 2, 3)]
    assert means[3] < means[0]
