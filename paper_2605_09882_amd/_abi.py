"""ctypes binding of the C ABI declared in include/raytheia.h.

Argument marshalling only: every function here forwards to the symbol of the
same name in ``libraytheia_hip.so`` and raises RtError on a non-zero status.
The library must have been built (``paper_2605_09882_amd.build``); there is
no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraytheia_hip.so")

RT_OK = 0
RT_ERR_ARG = -1
RT_ERR_UNSORTED = -2
RT_ERR_TILING = -3
RT_ERR_RANGE = -4
RT_ERR_DEVICE = -5
RT_ERR_WORKSPACE = -6

RT_FP64 = 0
RT_FP32_KAHAN = 1

# every symbol include/raytheia.h and include/raytheia_calib.h declare
EXPORTS = (
    "rt_abi_version",
    "rt_status_string",
    "rt_last_error",
    "rt_healpix_npix",
    "rt_healpix_dirs",
    "rt_healpix_dirs_nested",
    "rt_octree_workspace_bytes",
    "rt_build_octree",
    "rt_build_octree_device",
    "rt_octree_free",
    "rt_octree_leaves",
    "rt_octree_depth",
    "rt_columns",
    "rt_columns_backward",
    "rt_columns_with_adjoint",
    "rt_columns_trace",
    "rt_shielding",
    "rt_shielding_f32",
    "rt_nested_reference",
    "rt_grid_tree_workspace_bytes",
    "rt_grid_tree",
    "rt_grid_tree_static",
    "rt_calib_stream_granule",
    "rt_calib_copy",
    "rt_calib_read",
    "rt_calib_valu",
)

RT_MAX_FIELDS = 8


class RtError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


_lib = None


def load(path=None):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library missing at {p}: run paper_2605_09882_amd.build.build() "
                           "(no CPU fallback exists)")
    lib = ctypes.CDLL(p)
    V, P, I64, I32, D = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "rt_abi_version": (I32, []),
        "rt_status_string": (ctypes.c_char_p, [I32]),
        "rt_last_error": (ctypes.c_char_p, []),
        "rt_healpix_npix": (I64, [I32]),
        "rt_healpix_dirs": (I32, [I32, P]),
        "rt_healpix_dirs_nested": (I32, [I32, P]),
        "rt_octree_workspace_bytes": (ctypes.c_size_t, [I64, I32]),
        "rt_build_octree": (I32, [P, P, I64, I32, P, ctypes.c_size_t, V, ctypes.POINTER(V)]),
        "rt_build_octree_device": (I32, [P, P, I64, I32, P, ctypes.c_size_t, V, ctypes.POINTER(V)]),
        "rt_octree_free": (None, [V]),
        "rt_octree_leaves": (I64, [V]),
        "rt_octree_depth": (I32, [V]),
        "rt_columns": (I32, [V, P, I32, P, I64, P, I64, D, P, P, I64, I64, V]),
        "rt_columns_backward": (I32, [V, P, I64, P, I64, D, P, P, P, I64, I64, P, V]),
        "rt_columns_with_adjoint": (I32, [V, P, P, I64, P, I64, D, P, P, P, P, I64, I64, P, V]),
        "rt_columns_trace": (I32, [V, P, I64, P, I64, P, P, I64, I64, P, I64, P, I64, V]),
        "rt_shielding": (I32, [V, P, I32, P, I64, P, I64, D, P, D, P, P, D, D, P, P, P, V]),
        "rt_shielding_f32": (I32, [V, P, I32, P, I64, P, I64, D, P, D, P, P, D, D, P, P, P, V]),
        "rt_nested_reference": (I32, [P, I64, P, I64, I64, P, P, V]),
        "rt_grid_tree_workspace_bytes": (ctypes.c_size_t, [I32]),
        "rt_grid_tree": (I32, [P, I32, D, D, P, ctypes.c_size_t, P, P, P, P, V]),
        "rt_grid_tree_static": (I32, [P, I32, D, D, P, P, P, P, V]),
        "rt_calib_stream_granule": (ctypes.c_size_t, []),
        "rt_calib_copy": (I32, [P, P, ctypes.c_size_t, V]),
        "rt_calib_read": (I32, [P, ctypes.c_size_t, P, V]),
        "rt_calib_valu": (I32, [I32, ctypes.c_int64, I32, P, V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status, where):
    if status != RT_OK:
        lib = load()
        raise RtError(status, where, lib.rt_last_error().decode())


def rt_abi_version():
    return load().rt_abi_version()


def rt_status_string(status):
    return load().rt_status_string(int(status)).decode()


def rt_last_error():
    return load().rt_last_error().decode()


def rt_healpix_npix(nside):
    return int(load().rt_healpix_npix(int(nside)))


def rt_healpix_dirs(nside, dirs_out_ptr):
    _check(load().rt_healpix_dirs(int(nside), dirs_out_ptr), "rt_healpix_dirs")


def rt_healpix_dirs_nested(nside, dirs_out_ptr):
    _check(load().rt_healpix_dirs_nested(int(nside), dirs_out_ptr), "rt_healpix_dirs_nested")


def rt_octree_workspace_bytes(n_leaves, max_depth):
    return int(load().rt_octree_workspace_bytes(int(n_leaves), int(max_depth)))


def rt_build_octree(keys_ptr, levels_ptr, n_leaves, max_depth, workspace_ptr, workspace_bytes,
                    stream):
    """Returns the opaque handle (an int)."""
    h = ctypes.c_void_p()
    _check(load().rt_build_octree(keys_ptr, levels_ptr, int(n_leaves), int(max_depth),
                                  workspace_ptr, int(workspace_bytes), stream, ctypes.byref(h)),
           "rt_build_octree")
    return h.value


def rt_build_octree_device(keys_ptr, levels_ptr, n_leaves, max_depth, workspace_ptr,
                           workspace_bytes, stream):
    """Returns the opaque handle (an int)."""
    h = ctypes.c_void_p()
    _check(load().rt_build_octree_device(keys_ptr, levels_ptr, int(n_leaves), int(max_depth),
                                         workspace_ptr, int(workspace_bytes), stream,
                                         ctypes.byref(h)), "rt_build_octree_device")
    return h.value


def rt_octree_free(handle):
    load().rt_octree_free(handle)


def rt_octree_leaves(handle):
    return int(load().rt_octree_leaves(handle))


def rt_octree_depth(handle):
    return int(load().rt_octree_depth(handle))


def rt_columns(handle, rho_ptr, precision, src_ptr, n_src, dirs_ptr, n_dirs, kappa, N_ptr, A_ptr,
               stride_src, stride_dir, stream):
    _check(load().rt_columns(handle, rho_ptr, int(precision), src_ptr, int(n_src), dirs_ptr,
                             int(n_dirs), float(kappa), N_ptr, A_ptr, int(stride_src),
                             int(stride_dir), stream), "rt_columns")


def rt_columns_backward(handle, src_ptr, n_src, dirs_ptr, n_dirs, kappa, gN_ptr, gA_ptr, A_ptr,
                        stride_src, stride_dir, grad_ptr, stream):
    _check(load().rt_columns_backward(handle, src_ptr, int(n_src), dirs_ptr, int(n_dirs),
                                      float(kappa), gN_ptr, gA_ptr, A_ptr, int(stride_src),
                                      int(stride_dir), grad_ptr, stream), "rt_columns_backward")


def rt_columns_with_adjoint(handle, rho_ptr, src_ptr, n_src, dirs_ptr, n_dirs, kappa, wN_ptr, wA_ptr,
                            N_ptr, A_ptr, stride_src, stride_dir, grad_ptr, stream):
    _check(load().rt_columns_with_adjoint(handle, rho_ptr, src_ptr, int(n_src), dirs_ptr, int(n_dirs),
                                          float(kappa), wN_ptr, wA_ptr, N_ptr, A_ptr, int(stride_src),
                                          int(stride_dir), grad_ptr, stream), "rt_columns_with_adjoint")


def rt_columns_trace(handle, src_ptr, n_src, dirs_ptr, n_dirs, steps_ptr, hash_ptr, stride_src,
                     stride_dir, sample_ptr, n_sample, visited_ptr, cap, stream):
    _check(load().rt_columns_trace(handle, src_ptr, int(n_src), dirs_ptr, int(n_dirs), steps_ptr,
                                   hash_ptr, int(stride_src), int(stride_dir), sample_ptr,
                                   int(n_sample), visited_ptr, int(cap), stream),
           "rt_columns_trace")


def rt_shielding(handle, fields_ptr, n_fields, src_ptr, n_src, dirs_ptr, n_dirs, length, temp_ptr,
                 vturb, line_A_ptr, line_nu_ptr, gamma, av0, rays_ptr, av_eff_ptr, beta_ptr,
                 stream):
    _check(load().rt_shielding(handle, fields_ptr, int(n_fields), src_ptr, int(n_src), dirs_ptr,
                               int(n_dirs), float(length), temp_ptr, float(vturb), line_A_ptr,
                               line_nu_ptr, float(gamma), float(av0), rays_ptr, av_eff_ptr,
                               beta_ptr, stream), "rt_shielding")


def rt_shielding_f32(handle, fields_ptr, n_fields, src_ptr, n_src, dirs_ptr, n_dirs, length,
                     temp_ptr, vturb, line_A_ptr, line_nu_ptr, gamma, av0, rays_ptr, av_eff_ptr,
                     beta_ptr, stream):
    _check(load().rt_shielding_f32(handle, fields_ptr, int(n_fields), src_ptr, int(n_src), dirs_ptr,
                                   int(n_dirs), float(length), temp_ptr, float(vturb), line_A_ptr,
                                   line_nu_ptr, float(gamma), float(av0), rays_ptr, av_eff_ptr,
                                   beta_ptr, stream), "rt_shielding_f32")


def rt_nested_reference(fine_ptr, n_fine_dirs, coarse_ptr, n_coarse_dirs, n_src, ref_ptr, err_ptr,
                        stream):
    _check(load().rt_nested_reference(fine_ptr, int(n_fine_dirs), coarse_ptr, int(n_coarse_dirs),
                                      int(n_src), ref_ptr, err_ptr, stream), "rt_nested_reference")


def rt_grid_tree_workspace_bytes(depth):
    return int(load().rt_grid_tree_workspace_bytes(int(depth)))


def rt_grid_tree(grid_ptr, depth, density_floor, rel_uniformity, workspace_ptr, workspace_bytes,
                 keys_ptr, levels_ptr, values_ptr, n_ptr, stream):
    _check(load().rt_grid_tree(grid_ptr, int(depth), float(density_floor), float(rel_uniformity),
                               workspace_ptr, int(workspace_bytes), keys_ptr, levels_ptr,
                               values_ptr, n_ptr, stream), "rt_grid_tree")


def rt_grid_tree_static(grid_ptr, depth, density_floor, rel_uniformity, keys_ptr, levels_ptr,
                        values_ptr, n_ptr, stream):
    _check(load().rt_grid_tree_static(grid_ptr, int(depth), float(density_floor),
                                      float(rel_uniformity), keys_ptr, levels_ptr, values_ptr,
                                      n_ptr, stream), "rt_grid_tree_static")


def rt_calib_stream_granule():
    return int(load().rt_calib_stream_granule())


def rt_calib_copy(src_ptr, dst_ptr, nbytes, stream):
    _check(load().rt_calib_copy(src_ptr, dst_ptr, int(nbytes), stream), "rt_calib_copy")


def rt_calib_read(src_ptr, nbytes, sink_ptr, stream):
    _check(load().rt_calib_read(src_ptr, int(nbytes), sink_ptr, stream), "rt_calib_read")


def rt_calib_valu(kind, n_threads, iters, out_ptr, stream):
    _check(load().rt_calib_valu(int(kind), int(n_threads), int(iters), out_ptr, stream),
           "rt_calib_valu")
