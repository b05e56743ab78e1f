"""The walk calls on streams other than the default one: two calls running
at once on two streams over one octree, and the forward and the fused
forward-and-adjoint pass captured in HIP graphs and replayed with new inputs
between the replays.  Every launch goes to the stream the caller passes
(torch's current stream here); none of these calls synchronises, allocates
or clears memory itself, so they can be captured.

Bar: N and A bit for bit against eager calls on the default stream; the
gradient within 1e-12 of its largest entry (its FP64 atomic additions come
in a different order from run to run).
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


@pytest.fixture(scope="module")
def case(rt):
    tree = W.random_octree(6, 0.3, 611, min_level=2)
    dev = torch.device("cuda")
    t = rt.Octree(tree.keys, tree.levels, tree.depth, dev)
    src = torch.as_tensor(W.random_points(4096, 612)).to(dev)
    dirs = torch.as_tensor(rt.healpix_dirs(2)).to(dev)
    r32 = torch.as_tensor(tree.rho.astype(np.float32)).to(dev)
    r64 = torch.as_tensor(tree.rho).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(613)
    w = torch.rand((src.shape[0], dirs.shape[0]), generator=g, device=dev, dtype=torch.float32)
    return t, src, dirs, r32, r64, w


def _grad_close(a, b):
    scale = float(b.abs().max())
    assert scale > 0
    assert float((a - b).abs().max()) <= 1e-12 * scale


def test_two_streams_at_once(rt, case):
    t, src, dirs, r32, r64, w = case
    N32, A32 = rt.columns(t, r32, src, dirs, 0.7)
    N64, A64 = rt.columns(t, r64, src, dirs, 0.7)
    Nf, Af, gf = rt.columns_with_adjoint(t, r32, src, dirs, 0.7, wA=w)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out1, out2 = [], []
    with torch.cuda.stream(s1):
        for _ in range(3):
            out1.append(rt.columns(t, r64, src, dirs, 0.7))
    with torch.cuda.stream(s2):
        for _ in range(3):
            grad = torch.zeros(t.n, dtype=torch.float64, device=src.device)
            out2.append(rt.columns_with_adjoint(t, r32, src, dirs, 0.7, wA=w, grad=grad))
    torch.cuda.synchronize()
    for N, A in out1:
        assert torch.equal(N, N64) and torch.equal(A, A64)
    for N, A, g in out2:
        assert torch.equal(N, Nf) and torch.equal(A, Af)
        assert torch.equal(N, N32) and torch.equal(A, A32)
        _grad_close(g, gf)


def _warm(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()


def test_forward_in_a_graph(rt, case):
    t, src, dirs, r32, r64, w = case
    rho = r64.clone()
    _warm(lambda: rt.columns(t, rho, src, dirs, 0.7))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        N_g, A_g = rt.columns(t, rho, src, dirs, 0.7)
    for k in range(4):
        # eager work between the replays: new leaf values in the captured input
        rho.copy_(r64 * (1.0 + 0.5 * k))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        N_e, A_e = rt.columns(t, rho, src, dirs, 0.7)
        torch.cuda.synchronize()
        assert torch.equal(N_g, N_e) and torch.equal(A_g, A_e)


def test_fused_pass_in_a_graph(rt, case):
    t, src, dirs, r32, r64, w = case
    rho = r32.clone()
    wA = w.clone()
    grad = torch.zeros(t.n, dtype=torch.float64, device=src.device)

    def step():
        grad.zero_()  # a fill kernel, captured with the walk
        return rt.columns_with_adjoint(t, rho, src, dirs, 0.7, wA=wA, grad=grad)

    _warm(step)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        N_g, A_g, _ = step()
    for k in range(4):
        rho.copy_(r32 * (1.0 + 0.25 * k))
        wA.copy_(w.flip(0))
        if k % 2:
            wA.copy_(w)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        g_graph = grad.clone()
        ref = torch.zeros_like(grad)
        N_e, A_e, _ = rt.columns_with_adjoint(t, rho, src, dirs, 0.7, wA=wA, grad=ref)
        torch.cuda.synchronize()
        assert torch.equal(N_g, N_e) and torch.equal(A_g, A_e)
        _grad_close(g_graph, ref)
