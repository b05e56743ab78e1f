"""The measurement probes (include/raytheia_calib.h) on the GPU, through the
C ABI: the copy moves every byte, the read probe combines every word it
reads, and the VALU probes run the requested number of iterations.  The
roofline figures rest on these kernels doing the work they are timed for.

Bars: copy and read bit-exact; the integer VALU probe bit-exact against a
host model of its chains; the FP32 and FP64 probes against host models of
the same chains without fusion, within one unit of the truncated integer
they write (fused and unfused results differ in the last bits, which can
move a sum that lies on an integer across it).
"""

import numpy as np
import pytest
import torch

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    return require_gpu()


def _words(nbytes, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, generator=g)


@pytest.mark.parametrize("granules", [1, 3, 1000])
def test_copy_moves_every_byte(rt, granules):
    gr = rt._abi.rt_calib_stream_granule()
    assert gr == 16384
    host = _words(granules * gr, 11 + granules)
    src = host.cuda()
    dst = torch.full((host.numel() + 4096,), 0x5a5a5a5a, dtype=torch.int32, device="cuda")
    rt._abi.rt_calib_copy(src.data_ptr(), dst.data_ptr(), granules * gr, None)
    torch.cuda.synchronize()
    out = dst.cpu()
    assert torch.equal(out[:host.numel()], host)
    assert bool((out[host.numel():] == 0x5a5a5a5a).all())
    assert torch.equal(src.cpu(), host)


@pytest.mark.parametrize("granules", [1, 5, 777])
def test_read_combines_every_word(rt, granules):
    gr = rt._abi.rt_calib_stream_granule()
    host = _words(granules * gr, 23 + granules)
    src = host.cuda()
    sink = torch.zeros(granules + 1, dtype=torch.int32, device="cuda")
    sink[-1] = 0x2468ace
    rt._abi.rt_calib_read(src.data_ptr(), granules * gr, sink.data_ptr(), None)
    torch.cuda.synchronize()
    blocks = host.numpy().view(np.uint32).reshape(granules, gr // 4)
    want = np.bitwise_xor.reduce(blocks, axis=1)
    got = sink.cpu().numpy().view(np.uint32)
    assert np.array_equal(got[:granules], want)
    assert got[granules] == 0x2468ace


def _host_i32(n, iters):
    tid = np.arange(n, dtype=np.uint32)
    a = [(tid * np.uint32(7) + np.uint32(j)).astype(np.uint32) for j in range(8)]
    k = [(np.uint32((0x9E3779B9 * (j + 1)) & 0xFFFFFFFF) ^ tid).astype(np.uint32) for j in range(8)]
    for _ in range(iters):
        a = [((a[j] ^ k[j]) + a[(j + 1) % 8]).astype(np.uint32) for j in range(8)]
    s = np.zeros(n, dtype=np.uint32)
    for j in range(8):
        s ^= a[j]
    return s


def _host_float(n, iters, dtype, eps):
    tid = np.arange(n)
    m = (dtype(1.0) - dtype(eps) * (tid % 256 & 7).astype(dtype)).astype(dtype)
    c = (dtype(1e-3) * (tid & 15).astype(dtype)).astype(dtype)
    a = [(tid + j).astype(dtype) for j in range(8)]
    for _ in range(iters):
        a = [(a[j] * m + c).astype(dtype) for j in range(8)]
    s = np.zeros(n, dtype=dtype)
    for j in range(8):
        s = (s + a[j]).astype(dtype)
    return np.trunc(s.astype(np.float64)).astype(np.int64)


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("n_threads,iters", [(256, 1), (1024, 37), (4096, 100)])
def test_valu_probes_run_their_chains(rt, kind, n_threads, iters):
    out = torch.full((n_threads + 64,), -7, dtype=torch.int32, device="cuda")
    rt._abi.rt_calib_valu(kind, n_threads, iters, out.data_ptr(), None)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert (got[n_threads:] == -7).all()
    got = got[:n_threads]
    if kind == 1:
        assert np.array_equal(got.view(np.uint32), _host_i32(n_threads, iters))
    else:
        want = (_host_float(n_threads, iters, np.float64, 1e-9) if kind == 0
                else _host_float(n_threads, iters, np.float32, 1e-7))
        assert np.abs(got.astype(np.int64) - want).max() <= 1


def test_probe_argument_errors(rt):
    lib = rt._abi.load()
    gr = rt._abi.rt_calib_stream_granule()
    buf = torch.zeros(2 * gr // 4, dtype=torch.int32, device="cuda")
    p = buf.data_ptr()
    assert lib.rt_calib_copy(p, p + gr, gr + 16, None) == rt._abi.RT_ERR_ARG
    assert lib.rt_calib_copy(p, p + gr // 2, gr, None) == rt._abi.RT_ERR_ARG
    assert lib.rt_calib_read(p + 4, gr, p, None) == rt._abi.RT_ERR_ARG
    assert lib.rt_calib_valu(3, 256, 1, p, None) == rt._abi.RT_ERR_ARG
    assert lib.rt_calib_valu(0, 255, 1, p, None) == rt._abi.RT_ERR_ARG
    assert lib.rt_calib_valu(0, 256, 0, p, None) == rt._abi.RT_ERR_ARG
