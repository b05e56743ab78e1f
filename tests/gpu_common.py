"""Shared helpers of the GPU tests (HIP path vs oracle on the same inputs)."""

import os

import numpy as np
import pytest
import torch

import workloads as W

_EPS = np.finfo(np.float64).eps


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X (run with -m 'not gpu' on CPU)")
    import paper_2605_09882_amd as rt

    rt._abi.load()  # raises if the HIP library was not built
    return rt


def gpu_walk(rt, tree, src, dirs, kappa=1.0, rho64=None, rho32=None, trace=True, sample=None,
             cap=0):
    """Runs the HIP path (FP64 and FP32-Kahan forwards, trace) and returns
    host arrays [S, Dn]."""
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    r64 = torch.as_tensor(tree.rho if rho64 is None else rho64, dtype=torch.float64).to(dev)
    r32 = torch.as_tensor(tree.rho.astype(np.float32) if rho32 is None else rho32).to(dev)
    src_d = torch.as_tensor(np.ascontiguousarray(src)).to(dev)
    dirs_d = torch.as_tensor(np.ascontiguousarray(dirs)).to(dev)
    out = {}
    N, A = rt.columns(t, r64, src_d, dirs_d, kappa)
    out["N"], out["A"] = N.cpu().numpy(), A.cpu().numpy()
    N32, A32 = rt.columns(t, r32, src_d, dirs_d, kappa)
    out["N32"], out["A32"] = N32.cpu().numpy(), A32.cpu().numpy()
    if trace:
        steps, h, vis = rt.columns_trace(t, src_d, dirs_d, sample=sample, cap=cap)
        out["steps"] = steps.cpu().numpy().astype(np.int64)
        out["hash"] = h.cpu().numpy().view(np.uint64)
        if vis is not None:
            out["visited"] = vis.cpu().numpy()
    torch.cuda.synchronize()
    return out


def assert_bitexact(gpu, ref, keys=("N", "N32", "steps", "hash")):
    for k in keys:
        g, r = gpu[k], ref[k]
        assert g.shape == r.shape, k
        if g.dtype.kind == "f":
            same = (g == r) | (np.isnan(g) & np.isnan(r))
        else:
            same = g == r
        if not same.all():
            bad = np.argwhere(~same)
            s, d = bad[0]
            raise AssertionError(f"{k}: {len(bad)} of {g.size} rays differ; first (s={s}, d={d}): "
                                 f"gpu={g[s, d]!r} oracle={r[s, d]!r}")


def assert_attenuation(gpu, ref):
    """A = exp(-kappa N): FP64 within 2 ulp of the oracle's libm exp, FP32
    within 4 ulp of expf of the same N32."""
    a, b = gpu["A"], ref["A"]
    assert np.all(np.abs(a - b) <= 4.5e-16 * np.abs(b))
    a32, b32 = gpu["A32"].astype(np.float64), ref["A32"].astype(np.float64)
    assert np.all(np.abs(a32 - b32) <= 4.8e-7 * np.abs(b32))


def assert_fp32_vs_fp64(gpu):
    n64 = gpu["N"]
    rel = np.abs(gpu["N32"].astype(np.float64) - n64) / np.maximum(n64, 1e-300)
    assert rel.max() <= 1e-5, rel.max()


def edge_sources(depth):
    """Sources on cell faces, edges and corners, at 0 and just below 1."""
    h = 1.0 / (1 << depth)
    top = np.nextafter(1.0, 0.0)
    pts = [[0.5, 0.5, 0.5], [0.0, 0.0, 0.0], [top, top, top], [0.0, 0.5, top],
           [3 * h, 5 * h, 0.5], [0.5 * h, 0.5 * h, 0.5 * h], [0.25, 0.75, 0.125 + 0.5 * h],
           [1 - h, h, 0.5 - h]]
    return np.minimum(np.mod(np.array(pts, dtype=np.float64), 1.0), top)


def special_dirs():
    axis = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    diag = np.array([[1, 1, 1], [-1, 1, -1], [1, -1, 0], [0, 1, 1], [3, -4, 12]], float)
    diag /= np.linalg.norm(diag, axis=1)[:, None]
    return np.vstack([axis, diag])


def assert_shielding(got, ref, n_dirs, gamma=3.02, rays=True):
    """rt_shielding outputs against the oracle's, to the bar derived in
    test_gpu_shielding.py."""
    bad = np.isnan(ref["av_eff"])
    assert np.array_equal(np.isnan(got["av_eff"]), bad)
    ok = ~bad
    if rays:
        g, r = got["rays"], ref["rays"]
        assert g.shape == r.shape
        assert np.all(np.isnan(g[bad])) and not np.isnan(g[ok]).any()
        nh_g, nh_r = g[ok][..., 0], r[ok][..., 0]
        diff = nh_g != nh_r
        assert not diff.any(), f"N_H differs on {diff.sum()} rays: {nh_g[diff][:4]} vs {nh_r[diff][:4]}"
        tg, tr = g[ok][..., 1:], r[ok][..., 1:]
        assert np.all(np.abs(tg - tr) <= 4 * _EPS * np.abs(tr)), np.max(np.abs(tg - tr) / np.abs(tr))
    a, b = got["av_eff"][ok], ref["av_eff"][ok]
    tol = (2 * n_dirs + 4) * _EPS / abs(gamma) + 8 * _EPS * np.abs(b)
    assert np.all(np.abs(a - b) <= tol), np.max(np.abs(a - b) - tol)
    if ref["beta"].shape[1] > 0:
        assert np.all(np.isnan(got["beta"][bad]))
        a, b = got["beta"][ok], ref["beta"][ok]
        assert np.all(np.abs(a - b) <= (2 * n_dirs + 8) * _EPS * np.abs(b)), \
            np.max(np.abs(a - b) / np.abs(b))


def random_dirs(count, seed):
    v = np.random.default_rng(seed).standard_normal((count, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def random_seeds():
    """The seeds of the random-configuration tests: 100..119, or the range
    "a:b" given in RAYWALK_RANDOM_SEEDS for a longer sweep."""
    a, b = (int(x) for x in os.environ.get("RAYWALK_RANDOM_SEEDS", "100:120").split(":"))
    return range(a, b)
