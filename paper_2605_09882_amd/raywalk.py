"""Torch-facing binding of the reverse ray-walk library.

PyTorch supplies device memory and the current HIP stream; every step of the
walk runs in the library's HIP kernels.  Outputs are [S, Dn] views over
direction-major [Dn, S] buffers (stride_src = 1, stride_dir = S), the layout
with coalesced stores.

The adjoint follows from N being linear in rho: dN(s,d)/drho_k is the chord
of ray (s, d) in leaf k (sec. 2.3: I = sum_k f_k r_k), so
dL/drho_k = sum over rays of g * r_k with g = dL/dN - kappa A dL/dA.
"""

import numpy as np
import torch

from . import _abi

_PREC = {torch.float64: _abi.RT_FP64, torch.float32: _abi.RT_FP32_KAHAN}


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _gpu(device):
    """device with its index filled in (a bare "cuda" is the current GPU), so
    that it compares equal to the device of the tensors allocated there."""
    device = torch.device(device)
    if device.type == "cuda" and device.index is None:
        device = torch.device("cuda", torch.cuda.current_device())
    return device


def _same_device(t, dev, name):
    """The kernels take raw device pointers: a buffer elsewhere (the host or
    another GPU) must be refused here, before any launch."""
    if t.device != dev:
        raise ValueError(f"{name} is on {t.device}, the octree on {dev}")


def healpix_npix(nside):
    return _abi.rt_healpix_npix(nside)


def healpix_dirs(nside):
    """HEALPix RING pixel centres as a host float64 array [12 nside^2, 3]."""
    n = _abi.rt_healpix_npix(nside)
    if n < 0:
        raise ValueError(f"nside {nside} out of range")
    out = np.empty((n, 3), dtype=np.float64)
    _abi.rt_healpix_dirs(nside, out.ctypes.data)
    return out


def healpix_dirs_nested(nside):
    """HEALPix NESTED pixel centres as a host float64 array [12 nside^2, 3]
    (nside a power of two); pixels 4p .. 4p+3 at 2 nside subdivide pixel p."""
    n = _abi.rt_healpix_npix(nside)
    if n < 0:
        raise ValueError(f"nside {nside} out of range")
    out = np.empty((n, 3), dtype=np.float64)
    _abi.rt_healpix_dirs_nested(nside, out.ctypes.data)
    return out


class Octree:
    """A validated leaf-only linear octree staged on one GPU.

    keys (uint64) and levels (uint8) are host arrays describing the leaves;
    the leaf values are not stored here: they go with every walk call.  The
    device workspace is a torch tensor owned by this object.
    """

    def __init__(self, keys, levels, depth, device="cuda"):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        levels = np.ascontiguousarray(levels, dtype=np.uint8)
        if keys.shape != levels.shape or keys.ndim != 1:
            raise ValueError("keys and levels must be 1-D arrays of equal length")
        self.n = int(keys.shape[0])
        self.depth = int(depth)
        self.device = _gpu(device)
        nbytes = _abi.rt_octree_workspace_bytes(self.n, self.depth)
        if nbytes == 0:
            raise ValueError(f"invalid octree size n={self.n} depth={self.depth}")
        # 256 extra bytes so that the workspace can start on a 256-byte boundary
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        self._handle = None
        with torch.cuda.device(self.device):
            self._handle = _abi.rt_build_octree(keys.ctypes.data, levels.ctypes.data, self.n,
                                                self.depth, base + off, nbytes,
                                                _stream(self.device))

    @classmethod
    def from_device(cls, keys, levels, depth):
        """The octree of leaf arrays already on the device (keys int64 holding
        the uint64 Morton keys, levels uint8), e.g. from grid_tree(); checked
        and staged by kernels, without a copy to the host."""
        if not (torch.is_tensor(keys) and torch.is_tensor(levels) and keys.is_cuda and levels.is_cuda):
            raise TypeError("keys and levels must be device tensors")
        if keys.dtype != torch.int64 or levels.dtype != torch.uint8 or keys.shape != levels.shape:
            raise ValueError("keys must be int64 and levels uint8, of equal length")
        _same_device(levels, keys.device, "levels")
        self = cls.__new__(cls)
        keys = keys.contiguous()
        levels = levels.contiguous()
        self.n = int(keys.numel())
        self.depth = int(depth)
        self.device = keys.device
        nbytes = _abi.rt_octree_workspace_bytes(self.n, self.depth)
        if nbytes == 0:
            raise ValueError(f"invalid octree size n={self.n} depth={self.depth}")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        self._handle = None
        with torch.cuda.device(self.device):
            self._handle = _abi.rt_build_octree_device(keys.data_ptr(), levels.data_ptr(), self.n,
                                                       self.depth, base + off, nbytes,
                                                       _stream(self.device))
        self._inputs = (keys, levels)  # kept until the queued staging has run
        return self

    @property
    def handle(self):
        return self._handle

    def __del__(self, _free=_abi.rt_octree_free):
        h = getattr(self, "_handle", None)
        if h:
            self._handle = None
            try:
                _free(h)
            except Exception:  # interpreter shutdown: the library may be gone
                pass


def grid_tree(grid, depth, density_floor, rel_uniformity=0.01):
    """The contribution grid of the density + uniformity rule, built on the
    device from a uniform grid (device float64 [8^depth], Morton order).
    Returns (keys uint64-as-int64, levels uint8, values float64) device
    tensors of the leaves in Morton order (the count is read back, which
    synchronises the stream)."""
    if not torch.is_tensor(grid) or not grid.is_cuda or grid.dtype != torch.float64:
        raise TypeError("grid must be a float64 device tensor")
    grid = grid.reshape(-1).contiguous()
    if grid.numel() != 8 ** depth:
        raise ValueError(f"grid must hold 8^{depth} values")
    dev = grid.device
    nbytes = _abi.rt_grid_tree_workspace_bytes(depth)
    if nbytes == 0:
        raise ValueError(f"depth {depth} not in 1..10")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    off = (-base) % 256
    keys = torch.empty(grid.numel(), dtype=torch.int64, device=dev)
    levels = torch.empty(grid.numel(), dtype=torch.uint8, device=dev)
    values = torch.empty(grid.numel(), dtype=torch.float64, device=dev)
    n = torch.empty(1, dtype=torch.int64, device=dev)
    _abi.rt_grid_tree(grid.data_ptr(), depth, density_floor, rel_uniformity, base + off, nbytes,
                      keys.data_ptr(), levels.data_ptr(), values.data_ptr(), n.data_ptr(),
                      _stream(dev))
    k = int(n.item())
    del ws
    return keys[:k], levels[:k], values[:k]


def _as_dev(x, dtype, device, shape_last=None):
    if not torch.is_tensor(x):
        x = torch.as_tensor(np.ascontiguousarray(x))
    x = x.to(device=device, dtype=dtype).contiguous()
    if shape_last is not None and (x.ndim != 2 or x.shape[1] != shape_last):
        raise ValueError(f"expected an [n, {shape_last}] array, got {tuple(x.shape)}")
    return x


def columns(tree, rho, src, dirs, kappa=1.0, with_A=True):
    """N (and A = exp(-kappa N)) for every (source, direction).

    rho: device tensor [n_leaves], float64 (FP64 walk) or float32 (FP32
    walk with Kahan-compensated sums); src [S, 3] and dirs [Dn, 3] float64.
    Returns (N, A) as [S, Dn] views (A is None unless with_A)."""
    if rho.dtype not in _PREC:
        raise TypeError("rho must be float64 or float32")
    if not rho.is_cuda or rho.numel() != tree.n or not rho.is_contiguous():
        raise ValueError("rho must be a contiguous device tensor with one value per leaf")
    dev = tree.device
    _same_device(rho, dev, "rho")
    src = _as_dev(src, torch.float64, dev, 3)
    dirs = _as_dev(dirs, torch.float64, dev, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    N = torch.empty((Dn, S), dtype=rho.dtype, device=dev)
    A = torch.empty((Dn, S), dtype=rho.dtype, device=dev) if with_A else None
    _abi.rt_columns(tree.handle, rho.data_ptr(), _PREC[rho.dtype], src.data_ptr(), S,
                    dirs.data_ptr(), Dn, kappa, N.data_ptr(), _ptr(A), 1, S, _stream(dev))
    return N.t(), (A.t() if A is not None else None)


def _dir_major_f32(x, S, Dn, dev):
    """x as float32 with strides (1, S) over a [Dn, S] buffer (or None)."""
    if x is None:
        return None
    x = x.to(device=dev, dtype=torch.float32)
    if x.shape != (S, Dn):
        raise ValueError(f"gradient shape {tuple(x.shape)} != {(S, Dn)}")
    if x.stride() == (1, S):
        return x
    return x.t().contiguous().t()


def columns_backward(tree, src, dirs, kappa, gN=None, gA=None, A=None, grad=None):
    """Adds dL/drho (float64, [n_leaves]) into grad (created zeroed if None)."""
    dev = tree.device
    src = _as_dev(src, torch.float64, dev, 3)
    dirs = _as_dev(dirs, torch.float64, dev, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    gN = _dir_major_f32(gN, S, Dn, dev)
    gA = _dir_major_f32(gA, S, Dn, dev)
    A = _dir_major_f32(A, S, Dn, dev) if gA is not None else None
    if grad is None:
        grad = torch.zeros(tree.n, dtype=torch.float64, device=dev)
    elif grad.dtype != torch.float64 or grad.numel() != tree.n or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous float64 tensor with one value per leaf")
    else:
        _same_device(grad, dev, "grad")
    _abi.rt_columns_backward(tree.handle, src.data_ptr(), S, dirs.data_ptr(), Dn, kappa,
                             _ptr(gN), _ptr(gA), _ptr(A), 1, S, grad.data_ptr(), _stream(dev))
    return grad


def columns_with_adjoint(tree, rho, src, dirs, kappa, wN=None, wA=None, grad=None):
    """FP32-Kahan (N, A) and, in the same pass, dL/drho for the loss
    L = sum(wN * N) + sum(wA * A) with weights known in advance.

    rho: device float32 [n_leaves]; wN, wA: [S, Dn] weights or None.
    Returns (N, A, grad): N and A [S, Dn] views with the bits of columns(),
    grad float64 [n_leaves] (added into grad when given).  The result is that
    of columns() followed by columns_backward(gN=wN, gA=wA); one kernel walks
    each ray twice, the second time with its leaves still in cache."""
    if rho.dtype != torch.float32:
        raise TypeError("rho must be float32 (the FP32-Kahan walk)")
    if not rho.is_cuda or rho.numel() != tree.n or not rho.is_contiguous():
        raise ValueError("rho must be a contiguous device tensor with one value per leaf")
    dev = tree.device
    _same_device(rho, dev, "rho")
    src = _as_dev(src, torch.float64, dev, 3)
    dirs = _as_dev(dirs, torch.float64, dev, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    wN = _dir_major_f32(wN, S, Dn, dev)
    wA = _dir_major_f32(wA, S, Dn, dev)
    if grad is None:
        grad = torch.zeros(tree.n, dtype=torch.float64, device=dev)
    elif grad.dtype != torch.float64 or grad.numel() != tree.n or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous float64 tensor with one value per leaf")
    else:
        _same_device(grad, dev, "grad")
    N = torch.empty((Dn, S), dtype=torch.float32, device=dev)
    A = torch.empty((Dn, S), dtype=torch.float32, device=dev)
    _abi.rt_columns_with_adjoint(tree.handle, rho.data_ptr(), src.data_ptr(), S, dirs.data_ptr(), Dn,
                                 kappa, _ptr(wN), _ptr(wA), N.data_ptr(), A.data_ptr(), 1, S,
                                 grad.data_ptr(), _stream(dev))
    return N.t(), A.t(), grad


def columns_trace(tree, src, dirs, sample=None, cap=0):
    """Per ray: leaves visited (int32) and the FNV hash of their indices
    (int64 holding the uint64 bits), as [S, Dn] views; plus, for the ray ids
    in sample (r = d * S + s), the first cap visited leaf indices."""
    dev = tree.device
    src = _as_dev(src, torch.float64, dev, 3)
    dirs = _as_dev(dirs, torch.float64, dev, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    steps = torch.empty((Dn, S), dtype=torch.int32, device=dev)
    h = torch.empty((Dn, S), dtype=torch.int64, device=dev)
    visited = None
    n_sample = 0
    sp = None
    if sample is not None and len(sample) > 0:
        sample = torch.as_tensor(np.asarray(sample, dtype=np.int64)).to(dev)
        n_sample = int(sample.numel())
        visited = torch.empty((n_sample, cap), dtype=torch.int32, device=dev)
        sp = sample.data_ptr()
    _abi.rt_columns_trace(tree.handle, src.data_ptr(), S, dirs.data_ptr(), Dn, steps.data_ptr(),
                          h.data_ptr(), 1, S, sp, n_sample, _ptr(visited), cap, _stream(dev))
    return steps.t(), h.t(), visited


def shielding(tree, fields, src, dirs, length, temp=None, vturb=0.0, line_A=(), line_nu=(),
              gamma=3.02, av0=6.29e-22, rays=False, av_eff=True, beta=True):
    """Line optical depths, escape probabilities and the effective visual
    extinction (sec. 2.4, sec. 3) from one walk per ray over K leaf fields.

    fields: device float64 or float32 [n_leaves, K] (field 0 = n_H, field
    f >= 1 = the population term of line f with Einstein A line_A[f-1] and
    frequency line_nu[f-1]; float32 fields go to rt_shielding_f32, which
    widens them to float64 before the same arithmetic); src [S, 3],
    dirs [Dn, 3]; length = box edge in cm;
    temp [S] source temperatures in K (needed when K > 1); vturb in cm/s.
    Returns a dict with "av_eff" [S], "beta" [S, K-1] (views over
    line-major buffers) and, if rays, "rays" [S, Dn, K] (N_H, then tau per
    line; a view over the [K, Dn, S] buffer)."""
    dev = tree.device
    if not torch.is_tensor(fields) or fields.dtype not in (torch.float64, torch.float32) \
            or not fields.is_cuda:
        raise TypeError("fields must be a float64 or float32 device tensor")
    if fields.ndim == 1:
        fields = fields[:, None]
    fields = fields.contiguous()
    if fields.shape[0] != tree.n:
        raise ValueError("fields must hold one row per leaf")
    _same_device(fields, dev, "fields")
    K = int(fields.shape[1])
    src = _as_dev(src, torch.float64, dev, 3)
    dirs = _as_dev(dirs, torch.float64, dev, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    T = None
    lA = lnu = None
    if K > 1:
        if temp is None:
            raise ValueError("lines need source temperatures")
        T = temp if torch.is_tensor(temp) else torch.as_tensor(
            np.array(np.broadcast_to(np.asarray(temp, dtype=np.float64), (S,))))
        T = T.to(device=dev, dtype=torch.float64).contiguous()
        lA = np.ascontiguousarray(line_A, dtype=np.float64)
        lnu = np.ascontiguousarray(line_nu, dtype=np.float64)
        if lA.shape != (K - 1,) or lnu.shape != (K - 1,):
            raise ValueError(f"line_A and line_nu need {K - 1} entries")
    out_rays = torch.empty((K, Dn, S), dtype=torch.float64, device=dev) if rays else None
    out_av = torch.empty(S, dtype=torch.float64, device=dev) if av_eff else None
    out_beta = torch.empty((K - 1, S), dtype=torch.float64, device=dev) if beta and K > 1 else None
    call = _abi.rt_shielding if fields.dtype == torch.float64 else _abi.rt_shielding_f32
    call(tree.handle, fields.data_ptr(), K, src.data_ptr(), S, dirs.data_ptr(), Dn, float(length),
         _ptr(T), float(vturb), None if lA is None else lA.ctypes.data,
         None if lnu is None else lnu.ctypes.data, float(gamma), float(av0), _ptr(out_rays),
         _ptr(out_av), _ptr(out_beta), _stream(dev))
    res = {}
    if out_av is not None:
        res["av_eff"] = out_av
    if out_beta is not None:
        res["beta"] = out_beta.t()
    if out_rays is not None:
        res["rays"] = out_rays.permute(2, 1, 0)
    return res


class RayColumns(torch.autograd.Function):
    """(N, A) = RayColumns.apply(rho, tree, src, dirs, kappa), differentiable
    in rho through the library's adjoint walk."""

    @staticmethod
    def forward(ctx, rho, tree, src, dirs, kappa):
        dev = tree.device
        src = _as_dev(src, torch.float64, dev, 3)
        dirs = _as_dev(dirs, torch.float64, dev, 3)
        N, A = columns(tree, rho.detach(), src, dirs, kappa, with_A=True)
        ctx.tree = tree
        ctx.kappa = kappa
        ctx.rho_dtype = rho.dtype
        ctx.save_for_backward(src, dirs, A)
        return N, A

    @staticmethod
    def backward(ctx, gN, gA):
        src, dirs, A = ctx.saved_tensors
        grad = columns_backward(ctx.tree, src, dirs, ctx.kappa, gN=gN, gA=gA, A=A)
        return grad.to(ctx.rho_dtype), None, None, None, None


def ray_columns(rho, tree, src, dirs, kappa=1.0):
    """Differentiable (N, A); see RayColumns."""
    return RayColumns.apply(rho, tree, src, dirs, kappa)
