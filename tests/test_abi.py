"""Host side of the C ABI (no GPU needed): the library loads, exports every
symbol the header declares, validates its arguments before touching the
device, and its HEALPix table matches the oracle's."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_09882_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("raytheia.h", "raytheia_calib.h")]


@pytest.fixture(scope="module")
def lib():
    return _abi.load()


def declared_functions():
    names = set()
    for h in HEADERS:
        with open(h) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_header_is_checked():
    inc = os.path.join(ROOT, "include")
    assert sorted(os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")) == sorted(HEADERS)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_abi.EXPORTS)


def test_version_and_status_strings(lib):
    assert _abi.rt_abi_version() == 1
    for st in (0, -1, -2, -3, -4, -5, -6):
        assert _abi.rt_status_string(st) not in ("", "unknown status")
    assert _abi.rt_status_string(-99) == "unknown status"


def test_healpix_npix(lib):
    assert [_abi.rt_healpix_npix(n) for n in (1, 2, 4, 8)] == [12, 48, 192, 768]
    assert _abi.rt_healpix_npix(0) == -1
    assert _abi.rt_healpix_npix(-3) == -1
    assert _abi.rt_healpix_npix((1 << 20) + 1) == -1


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 8, 16, 64])
def test_healpix_matches_oracle(orc, nside):
    import paper_2605_09882_amd as rt
    mine = rt.healpix_dirs(nside)
    ref = orc.healpix_ring(nside)
    assert mine.shape == ref.shape
    assert np.abs(mine - ref).max() <= 1e-15


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64])
def test_healpix_nested_matches_oracle(orc, nside):
    """The library's NESTED table against the oracle's, and row by row a
    permutation of its own RING table (the same bits)."""
    import paper_2605_09882_amd as rt
    mine = rt.healpix_dirs_nested(nside)
    ref = orc.healpix_nested(nside)
    assert np.abs(mine - ref).max() <= 1e-15
    ring = rt.healpix_dirs(nside)
    assert np.array_equal(mine[np.lexsort(mine.T)], ring[np.lexsort(ring.T)])


def test_healpix_errors(lib):
    out = np.empty((12, 3))
    assert lib.rt_healpix_dirs(0, out.ctypes.data) == _abi.RT_ERR_ARG
    assert b"nside" in lib.rt_last_error()
    assert lib.rt_healpix_dirs(1, None) == _abi.RT_ERR_ARG
    assert lib.rt_healpix_dirs_nested(3, out.ctypes.data) == _abi.RT_ERR_ARG
    assert b"power of two" in lib.rt_last_error()
    assert lib.rt_healpix_dirs_nested(0, out.ctypes.data) == _abi.RT_ERR_ARG
    assert lib.rt_healpix_dirs_nested(1, None) == _abi.RT_ERR_ARG


def test_workspace_bytes(lib):
    assert _abi.rt_octree_workspace_bytes(0, 5) == 0
    assert _abi.rt_octree_workspace_bytes(10, 0) == 0
    assert _abi.rt_octree_workspace_bytes(10, 22) == 0
    small = _abi.rt_octree_workspace_bytes(8, 1)
    assert small > 0 and small % 256 == 0
    # 64-bit keys beyond depth 10
    assert _abi.rt_octree_workspace_bytes(1000, 11) > _abi.rt_octree_workspace_bytes(1000, 10)


def _build(lib, keys, levels, depth, ws=None, nbytes=None):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    levels = np.ascontiguousarray(levels, dtype=np.uint8)
    h = ctypes.c_void_p()
    st = lib.rt_build_octree(keys.ctypes.data, levels.ctypes.data, len(keys), depth, ws,
                             nbytes or 0, None, ctypes.byref(h))
    return st, h


def test_build_rejects_bad_trees_before_device_work(lib):
    import workloads as W
    t = W.random_octree(4, 0.4, 11, min_level=1)
    k, L = t.keys.copy(), t.levels.copy()
    k[[3, 4]] = k[[4, 3]]
    L[[3, 4]] = L[[4, 3]]
    assert _build(lib, k, L, 4)[0] == _abi.RT_ERR_UNSORTED
    assert _build(lib, np.delete(t.keys, 5), np.delete(t.levels, 5), 4)[0] == _abi.RT_ERR_TILING
    L = t.levels.copy()
    L[int(np.nonzero(t.levels == 4)[0][1])] = 3
    assert _build(lib, t.keys, L, 4)[0] == _abi.RT_ERR_TILING
    k = t.keys.copy()
    k[int(np.nonzero(t.levels <= 3)[0][2])] += np.uint64(1)
    assert _build(lib, k, t.levels, 4)[0] in (_abi.RT_ERR_TILING, _abi.RT_ERR_UNSORTED)
    assert _build(lib, t.keys[:-1], t.levels[:-1], 4)[0] == _abi.RT_ERR_TILING
    assert _build(lib, t.keys, t.levels, 0)[0] == _abi.RT_ERR_ARG
    assert _build(lib, t.keys, t.levels, 22)[0] == _abi.RT_ERR_ARG
    # valid tree, bad workspace: rejected on the host
    assert _build(lib, t.keys, t.levels, 4, None, 0)[0] == _abi.RT_ERR_WORKSPACE
    assert _build(lib, t.keys, t.levels, 4, 0x1001, 1 << 20)[0] == _abi.RT_ERR_WORKSPACE
    assert _build(lib, t.keys, t.levels, 4, 0x100000, 16)[0] == _abi.RT_ERR_WORKSPACE
    # null arrays and output
    h = ctypes.c_void_p()
    assert lib.rt_build_octree(None, None, 5, 4, None, 0, None, ctypes.byref(h)) == _abi.RT_ERR_ARG
    assert lib.rt_build_octree(t.keys.ctypes.data, t.levels.ctypes.data, len(t.keys), 4, None, 0,
                               None, None) == _abi.RT_ERR_ARG


def test_walk_calls_reject_null_handles(lib):
    assert lib.rt_columns(None, 1, 0, 1, 1, 1, 1, 1.0, 1, None, 1, 1, None) == _abi.RT_ERR_ARG
    assert lib.rt_columns_backward(None, 1, 1, 1, 1, 1.0, 1, None, None, 1, 1, 1, None) == \
        _abi.RT_ERR_ARG
    assert lib.rt_columns_trace(None, 1, 1, 1, 1, 1, 1, 1, 1, None, 0, None, 0, None) == \
        _abi.RT_ERR_ARG
    assert lib.rt_columns_with_adjoint(None, 1, 1, 1, 1, 1, 1.0, 1, None, 1, None, 1, 1, 1, None) == \
        _abi.RT_ERR_ARG
    assert lib.rt_shielding(None, 1, 1, 1, 1, 1, 1, 1.0, None, 0.0, None, None, 3.02, 6.29e-22, None,
                            1, None, None) == _abi.RT_ERR_ARG
    assert lib.rt_octree_leaves(None) == -1
    assert lib.rt_octree_depth(None) == -1
    lib.rt_octree_free(None)


def test_new_calls_validate_before_device_work(lib):
    """The grid construction, the device octree build and the nested
    reference reject bad arguments on the host, before any device work."""
    E, W_ = _abi.RT_ERR_ARG, _abi.RT_ERR_WORKSPACE
    assert _abi.rt_grid_tree_workspace_bytes(0) == 0 and _abi.rt_grid_tree_workspace_bytes(11) == 0
    assert _abi.rt_grid_tree_workspace_bytes(9) > 8 ** 9 // 7 * 25
    p = 256  # a fake, aligned, never dereferenced address
    assert lib.rt_grid_tree(None, 3, 1.0, 0.01, p, 1 << 30, p, p, p, p, None) == E
    assert lib.rt_grid_tree(p, 0, 1.0, 0.01, p, 1 << 30, p, p, p, p, None) == E
    assert lib.rt_grid_tree(p, 3, float("inf"), 0.01, p, 1 << 30, p, p, p, p, None) == E
    assert lib.rt_grid_tree(p, 3, 1.0, 0.01, None, 1 << 30, p, p, p, p, None) == W_
    assert lib.rt_grid_tree(p, 3, 1.0, 0.01, p + 4, 1 << 30, p, p, p, p, None) == W_
    assert lib.rt_grid_tree(p, 3, 1.0, 0.01, p, 8, p, p, p, p, None) == W_
    import ctypes
    h = ctypes.c_void_p()
    assert lib.rt_build_octree_device(p, p, 0, 3, p, 1 << 30, None, ctypes.byref(h)) == E
    assert lib.rt_build_octree_device(p, p, 10, 22, p, 1 << 30, None, ctypes.byref(h)) == E
    assert lib.rt_build_octree_device(None, p, 10, 3, p, 1 << 30, None, ctypes.byref(h)) == E
    assert lib.rt_build_octree_device(p, p, 10, 3, p, 16, None, ctypes.byref(h)) == W_
    assert lib.rt_build_octree_device(p, p, 10, 3, p, 1 << 30, None, None) == E
    assert h.value is None
    assert lib.rt_nested_reference(p, 24, p, 12, 1, p, None, None) == E   # ratio 2
    assert lib.rt_nested_reference(p, 12, p, 48, 1, p, None, None) == E   # fine < coarse
    assert lib.rt_nested_reference(None, 48, p, 12, 1, p, None, None) == E
    assert lib.rt_nested_reference(p, 48, None, 12, 1, None, p, None) == E


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises; it has no fallback."""
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _abi.load(str(tmp_path / "absent.so"))


def test_product_never_touches_the_oracle():
    """No source of the package or its native code names the oracle, so no
    call of the product can route through it."""
    pkg = os.path.join(ROOT, "paper_2605_09882_amd")
    for base, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                with open(os.path.join(base, f)) as fh:
                    text = fh.read()
                assert not re.search(r"\boracle\b|\borc_", text), os.path.join(base, f)


def test_calibration_probes_validate_before_device_work(lib):
    """The measurement probes reject bad sizes, alignments and kinds on the
    host."""
    E = _abi.RT_ERR_ARG
    g = _abi.rt_calib_stream_granule()
    assert g == 16384
    p, q = 1 << 20, 1 << 30  # fake, aligned, never dereferenced addresses
    assert lib.rt_calib_copy(p, q, 0, None) == E
    assert lib.rt_calib_copy(p, q, g + 16, None) == E
    assert lib.rt_calib_copy(p + 8, q, g, None) == E
    assert lib.rt_calib_copy(p, p + g // 2, g, None) == E      # overlapping
    assert lib.rt_calib_copy(None, q, g, None) == E
    assert lib.rt_calib_read(p, g, None, None) == E
    assert lib.rt_calib_read(p, 3 * g // 2, q, None) == E
    assert lib.rt_calib_valu(3, 256, 10, p, None) == E
    assert lib.rt_calib_valu(0, 100, 10, p, None) == E
    assert lib.rt_calib_valu(0, 256, 0, p, None) == E
    assert lib.rt_calib_valu(0, 256, 10, None, None) == E
    assert lib.rt_calib_valu(1, 1 << 31, 1, p, None) == E
    assert b"n_threads" in lib.rt_last_error()


def test_static_grid_tree_refuses_on_the_host(lib):
    """rt_grid_tree_static (no caller workspace) refuses grids deeper than
    its static scratch holds, and bad arguments, before any device work."""
    E = _abi.RT_ERR_ARG
    p = 256  # a fake, aligned, never dereferenced address
    assert lib.rt_grid_tree_static(p, 8, 1.0, 0.01, p, p, p, p, None) == E
    assert b"static scratch" in lib.rt_last_error()
    assert lib.rt_grid_tree_static(p, 0, 1.0, 0.01, p, p, p, p, None) == E
    assert lib.rt_grid_tree_static(None, 3, 1.0, 0.01, p, p, p, p, None) == E
    assert lib.rt_grid_tree_static(p, 3, 1.0, 0.01, p, None, p, p, None) == E
    assert lib.rt_grid_tree_static(p, 3, float("nan"), 0.01, p, p, p, p, None) == E
    # the scratch holds exactly the workspace of the deepest accepted grid
    assert _abi.rt_grid_tree_workspace_bytes(7) == 7498752


def test_header_states_the_gradient_memory_kind():
    """Both calls that add into the FP64 gradient say it must be
    coarse-grained device memory (the hardware FP64 atomics lose updates on
    fine-grained, managed or host memory)."""
    with open(HEADERS[0]) as f:
        text = f.read()
    for call in ("int rt_columns_backward(", "int rt_columns_with_adjoint("):
        doc = text[:text.index(call)]
        doc = doc[doc.rindex("/*"):]
        assert "coarse-grained" in doc, call
