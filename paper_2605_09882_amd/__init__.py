"""MI355X reverse ray walk through a leaf-only linear octree.

Column densities N = sum_k rho_k r_k and attenuations exp(-kappa N) for every
(source point, HEALPix direction) pair, their adjoint, and -- from one walk
over several leaf fields -- line optical depths, escape probabilities and the
effective visual extinction, computed by hand-written HIP kernels for gfx950
behind the C ABI of include/raytheia.h (method: Zhu et al., RAYTHEIA,
sec. 2-3).  ``_abi`` is the ctypes binding of that ABI; ``raywalk``
passes torch device tensors and the current stream to it.
"""

from . import _abi
from .raywalk import (Octree, RayColumns, columns, columns_backward, columns_trace,
                      columns_with_adjoint, grid_tree,
                      healpix_dirs, healpix_dirs_nested, healpix_npix, ray_columns, shielding)

__all__ = [
    "_abi",
    "Octree",
    "RayColumns",
    "columns",
    "columns_backward",
    "columns_with_adjoint",
    "columns_trace",
    "grid_tree",
    "healpix_dirs",
    "healpix_dirs_nested",
    "healpix_npix",
    "ray_columns",
    "shielding",
]
