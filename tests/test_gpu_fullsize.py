"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (whole-workload launches, the library's own HEALPix table where it is
bit-identical to the oracle's).

The oracle cannot walk 1.6e9 rays, so: (i) a seeded sample of rays is
walked one by one by the oracle and compared bit for bit; (ii) properties
that hold at any size are checked on every ray (FP32 vs FP64 within 1e-5,
finite non-negative columns, the uniform-density closed form N = t_exit on
the workload's own topology); (iii) the adjoint is checked against the
oracle's FP64 gradient on a source subsample, through the linearity
identity sum_k rho_k dL/drho_k = sum_r g_r N_r on every ray, and against
FP64 central differences on sampled leaves; (iv) the several-fields walk
(n_H and three lines) is compared with the oracle on a seeded source
sample of every workload, and on every source A_V,eff lies between the
smallest and the mean of its directions' extinctions from the FP64 column
walk.
"""

import os
import time

import numpy as np
import pytest
import torch

import workloads as W
from gpu_common import assert_shielding, require_gpu

pytestmark = pytest.mark.gpu

N_SAMPLE_RAYS = 1500
N_SAMPLE_SOURCES = 3000
SHIELD_LINES = 3  # n_H and three lines: the configuration bench.py times


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


_cache = {}


def _workload(i):
    if i not in _cache:
        _cache.clear()
        _cache[i] = W.make_workload(i)
    return _cache[i]


def _dirs(rt, orc, nside):
    """The library's table when it equals the oracle's bit for bit (as it
    does for nside 1 and 2), else the oracle's for both sides."""
    mine, ref = rt.healpix_dirs(nside), orc.healpix_ring(nside)
    return (mine, True) if np.array_equal(mine, ref) else (ref, False)


def _exit_time(src, m):
    """Distance along m from every source to the unit box boundary [S]."""
    t = torch.full((src.shape[0],), float("inf"), dtype=torch.float64, device=src.device)
    for a in range(3):
        if m[a] > 0:
            t = torch.minimum(t, (1.0 - src[:, a]) / m[a])
        elif m[a] < 0:
            t = torch.minimum(t, (0.0 - src[:, a]) / m[a])
    return t


@pytest.mark.parametrize("index", [1, 2, 3, 4])
def test_fullsize_forward(rt, orc, index):
    w = _workload(index)
    dev = torch.device("cuda")
    dirs, same_table = _dirs(rt, orc, w.nside)
    if w.nside <= 2:
        assert same_table
    tree = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    src = torch.as_tensor(w.sources).to(dev)
    dirs_d = torch.as_tensor(dirs).to(dev)
    rho64 = torch.as_tensor(w.tree.rho).to(dev)
    rho32 = torch.as_tensor(w.tree.rho.astype(np.float32)).to(dev)
    S, Dn = src.shape[0], dirs.shape[0]
    N64, _ = rt.columns(tree, rho64, src, dirs_d, w.kappa, with_A=False)
    N32, A32 = rt.columns(tree, rho32, src, dirs_d, w.kappa)
    rng = np.random.default_rng(5000 + index)
    sample = np.sort(rng.choice(S * Dn, N_SAMPLE_RAYS, replace=False))
    steps, h, vis = rt.columns_trace(tree, src, dirs_d, sample=sample, cap=3 * (1 << w.tree.depth) + 3)
    d_idx, s_idx = np.divmod(sample, S)
    g64 = N64[s_idx, d_idx].cpu().numpy()
    g32 = N32[s_idx, d_idx].cpu().numpy()
    a32 = A32[s_idx, d_idx].cpu().numpy()
    gst = steps[s_idx, d_idx].cpu().numpy()
    gh = h[s_idx, d_idx].cpu().numpy().view(np.uint64)
    vis = vis.cpu().numpy()
    r32 = w.tree.rho.astype(np.float32)
    for j in range(len(sample)):
        s, d = int(s_idx[j]), int(d_idx[j])
        ref = orc.walk_one(w.tree, w.sources[s], dirs[d], rho32=r32)
        assert ref["status"] == orc.OK
        assert g64[j] == ref["N"], (index, s, d, g64[j], ref["N"])
        assert g32[j] == np.float32(ref["N32"]), (index, s, d)
        assert gst[j] == ref["steps"] and int(gh[j]) == ref["hash"]
        assert np.array_equal(vis[j, :ref["steps"]], ref["visited"])
        assert abs(a32[j] - np.exp(-w.kappa * ref["N32"])) <= 4.8e-7 * a32[j] + 1e-38
    # properties on every ray
    assert bool(torch.isfinite(N64).all()) and float(N64.min()) >= 0.0
    assert int(steps.min()) >= 1
    rel = ((N32.double() - N64).abs() / N64.clamp_min(1e-300)).max()
    assert float(rel) <= 1e-5
    # uniform density on the same topology: N = t_exit exactly up to rounding
    ones = torch.ones(w.tree.n, dtype=torch.float64, device=dev)
    Nu, _ = rt.columns(tree, ones, src, dirs_d, w.kappa, with_A=False)
    for d in range(Dn):
        te = _exit_time(src, dirs[d])
        err = ((Nu[:, d] - te).abs() / te).max()
        assert float(err) <= 1e-13, (index, d, float(err))
    torch.cuda.synchronize()


def test_fullsize_adjoint_merged512(rt, orc):
    """The paper-scale workload's adjoint (FP32-Kahan forward, L = sum w A)."""
    w = _workload(4)
    dev = torch.device("cuda")
    dirs, _ = _dirs(rt, orc, w.nside)
    tree = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    src = torch.as_tensor(w.sources).to(dev)
    dirs_d = torch.as_tensor(dirs).to(dev)
    S, Dn = src.shape[0], dirs.shape[0]
    rho32 = torch.as_tensor(w.tree.rho.astype(np.float32)).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(3004)
    wgt = torch.rand((Dn, S), generator=gen, device=dev, dtype=torch.float32).t()
    _, A = rt.columns(tree, rho32, src, dirs_d, w.kappa)
    grad = rt.columns_backward(tree, src, dirs_d, w.kappa, gA=wgt, A=A)
    # identity on every ray: sum_k rho_k grad_k = sum_r g_r N_r, g = -kappa A w
    rho_d = rho32.double()
    N64, A64 = rt.columns(tree, rho_d, src, dirs_d, w.kappa)
    lhs = float((rho_d * grad).sum())
    rhs = float((-w.kappa * A.double() * wgt.double() * N64).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
    # oracle FP64 gradient over every 4096th source (all directions)
    sub = slice(0, S, 4096)
    src_s = w.sources[sub]
    w_s = wgt[sub].cpu().numpy().astype(np.float64)
    grad_s = rt.columns_backward(tree, torch.as_tensor(src_s).to(dev), dirs_d, w.kappa,
                                 gA=wgt[sub].contiguous(), A=A[sub].contiguous()).cpu().numpy()
    rho_w = W.Octree(w.tree.depth, w.tree.keys, w.tree.levels,
                     w.tree.rho.astype(np.float32).astype(np.float64))
    ref = orc.columns(rho_w, src_s, dirs, w.kappa, threads=8)
    want = orc.gradient(rho_w, src_s, dirs, -w.kappa * w_s * ref["A"])
    scale = np.abs(want).max()
    assert np.all(np.abs(grad_s - want) <= 1e-5 * np.abs(want) + 1e-6 * scale)
    # FP64 central differences on sampled leaves (loss from the FP64 walk)
    g_full = grad.cpu().numpy()
    leaves = w.fd_leaves(8)
    for k in leaves:
        hstep = 1e-3 * float(rho_d[k])
        rp, rm = rho_d.clone(), rho_d.clone()
        rp[k] += hstep
        rm[k] -= hstep
        _, Ap = rt.columns(tree, rp, src, dirs_d, w.kappa)
        _, Am = rt.columns(tree, rm, src, dirs_d, w.kappa)
        fd = float((wgt.double() * (Ap - Am)).sum() / (2 * hstep))
        assert abs(g_full[k] - fd) <= 1e-4 * abs(fd) + 1e-7 * np.abs(g_full).max(), (k, g_full[k], fd)


@pytest.mark.parametrize("index", [1, 2])
def test_fullsize_adjoint_identity(rt, orc, index):
    """The adjoint on the AMR and the uniform 128^3 workloads: the linearity
    identity on every ray and the oracle's FP64 gradient on a source
    subsample."""
    w = _workload(index)
    dev = torch.device("cuda")
    dirs, _ = _dirs(rt, orc, w.nside)
    tree = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    src = torch.as_tensor(w.sources).to(dev)
    dirs_d = torch.as_tensor(dirs).to(dev)
    S, Dn = src.shape[0], dirs.shape[0]
    rho32 = torch.as_tensor(w.tree.rho.astype(np.float32)).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(3000 + index)
    wgt = torch.rand((Dn, S), generator=gen, device=dev, dtype=torch.float32).t()
    _, A = rt.columns(tree, rho32, src, dirs_d, w.kappa)
    grad = rt.columns_backward(tree, src, dirs_d, w.kappa, gA=wgt, A=A)
    rho_d = rho32.double()
    N64, _ = rt.columns(tree, rho_d, src, dirs_d, w.kappa, with_A=False)
    lhs = float((rho_d * grad).sum())
    rhs = float((-w.kappa * A.double() * wgt.double() * N64).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
    step = max(1, S // 2000)
    sub = slice(0, S, step)
    src_s = w.sources[sub]
    w_s = wgt[sub].cpu().numpy().astype(np.float64)
    grad_s = rt.columns_backward(tree, torch.as_tensor(src_s).to(dev), dirs_d, w.kappa,
                                 gA=wgt[sub].contiguous(), A=A[sub].contiguous()).cpu().numpy()
    rho_w = W.Octree(w.tree.depth, w.tree.keys, w.tree.levels,
                     w.tree.rho.astype(np.float32).astype(np.float64))
    ref = orc.columns(rho_w, src_s, dirs, w.kappa, threads=8)
    want = orc.gradient(rho_w, src_s, dirs, -w.kappa * w_s * ref["A"])
    scale = np.abs(want).max()
    assert np.all(np.abs(grad_s - want) <= 1e-5 * np.abs(want) + 1e-6 * scale)
    torch.cuda.synchronize()


@pytest.mark.parametrize("index,f32", [(4, False), (4, True), (2, False), (2, True), (1, False),
                                       (3, False)])
def test_fullsize_shielding(rt, orc, index, f32):
    """The several-fields walk at full size (FP64 fields, and FP32 fields for
    the coherent workloads, the oracle then fed the same FP32 values)."""
    w = _workload(index)
    dev = torch.device("cuda")
    dirs, _ = _dirs(rt, orc, w.nside)
    tree = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    src = torch.as_tensor(w.sources).to(dev)
    dirs_d = torch.as_tensor(dirs).to(dev)
    S, Dn = src.shape[0], dirs.shape[0]
    inp = W.line_inputs(w.tree, w.sources, SHIELD_LINES, 6000 + index)
    if f32:
        inp["fields"] = inp["fields"].astype(np.float32)
    F = torch.as_tensor(inp["fields"]).to(dev)
    if f32:
        inp["fields"] = inp["fields"].astype(np.float64)  # the oracle's copy: the same values
    T = torch.as_tensor(inp["temp"]).to(dev)
    gamma, av0 = 3.02, 6.29e-22
    out = rt.shielding(tree, F, src, dirs_d, inp["length"], temp=T, vturb=inp["vturb"],
                       line_A=inp["line_A"], line_nu=inp["line_nu"], gamma=gamma, av0=av0)
    av = out["av_eff"]
    beta = out["beta"].cpu().numpy()
    assert bool(torch.isfinite(av).all()) and bool((av >= 0).all())
    assert np.isfinite(beta).all() and (beta > 0).all()
    # every source: min_d av0 N_H <= A_V,eff <= mean_d av0 N_H (Jensen)
    N, _ = rt.columns(tree, F[:, 0].to(torch.float64).contiguous(), src, dirs_d, with_A=False)
    avd = av0 * (inp["length"] * N)
    lo, hi = avd.min(dim=1).values, avd.mean(dim=1)
    slack = 1e-12 * hi + (2 * Dn + 4) * 2.3e-16 / gamma
    assert bool((av >= lo - slack).all()) and bool((av <= hi + slack).all())
    del N, avd
    # seeded sample against the oracle
    rng = np.random.default_rng(7000 + index)
    idx = np.sort(rng.choice(S, N_SAMPLE_SOURCES, replace=False))
    ref = orc.shielding(w.tree, inp["fields"], w.sources[idx], dirs, length=inp["length"],
                        temp=inp["temp"][idx], vturb=inp["vturb"], line_A=inp["line_A"],
                        line_nu=inp["line_nu"], gamma=gamma, av0=av0, rays=False, threads=8)
    assert ref["status"] == orc.OK
    got = {"av_eff": av.cpu().numpy()[idx], "beta": beta[idx]}
    assert_shielding(got, ref, Dn, gamma=gamma, rays=False)
    torch.cuda.synchronize()


@pytest.mark.timeout(1200)
@pytest.mark.skipif(not os.environ.get("RAYWALK_SHIELDING_512"),
                    reason='about 25 minutes of oracle work on 16 cores, run in parts: set '
                           'RAYWALK_SHIELDING_512="a:b" to compare sources a..b-1')
def test_every_source_shielding_merged_512(rt, orc):
    """The several-fields walk with FP32-stored fields (n_H and three lines,
    the configuration the benchmark times) on every source a..b-1 of the
    512^3 cloud named in RAYWALK_SHIELDING_512 ("a:b"; all: 0:134217728),
    against the oracle fed the same values, in chunks of 2^21 sources."""
    a0, b0 = (int(x) for x in os.environ["RAYWALK_SHIELDING_512"].split(":"))
    w = _workload(4)
    S = w.sources.shape[0]
    assert 0 <= a0 < b0 <= S
    dev = torch.device("cuda")
    dirs, _ = _dirs(rt, orc, w.nside)
    tree = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    dirs_d = torch.as_tensor(dirs).to(dev)
    inp = W.line_inputs(w.tree, w.sources, SHIELD_LINES, 6004)
    f32 = inp["fields"].astype(np.float32)
    F = torch.as_tensor(f32).to(dev)
    f64 = f32.astype(np.float64)  # the oracle's copy: the same values
    gamma, av0 = 3.02, 6.29e-22
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    t0 = time.perf_counter()
    for a in range(a0, b0, 1 << 21):
        b = min(a + (1 << 21), b0)
        src = torch.as_tensor(w.sources[a:b]).to(dev)
        T = torch.as_tensor(inp["temp"][a:b]).to(dev)
        out = rt.shielding(tree, F, src, dirs_d, inp["length"], temp=T, vturb=inp["vturb"],
                           line_A=inp["line_A"], line_nu=inp["line_nu"], gamma=gamma, av0=av0)
        got = {"av_eff": out["av_eff"].cpu().numpy(), "beta": out["beta"].cpu().numpy()}
        ref = orc.shielding(w.tree, f64, w.sources[a:b], dirs, length=inp["length"],
                            temp=inp["temp"][a:b], vturb=inp["vturb"], line_A=inp["line_A"],
                            line_nu=inp["line_nu"], gamma=gamma, av0=av0, rays=False, threads=cores)
        assert ref["status"] == orc.OK
        assert_shielding(got, ref, len(dirs), gamma=gamma, rays=False)
        print(f"[{w.name}] sources {a}..{b}: within the bar; {time.perf_counter() - t0:.0f} s",
              flush=True)
