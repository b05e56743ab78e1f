"""Seeded synthetic inputs for the reverse ray walk.

This package builds the *inputs* of the column-density problem and nothing
else: turbulent density fields, the leaf-only linear octree that stands for the
contribution grid (paper Sec. 2.2 and Sec. 2.3.1), source points (the source
grid of Sec. 2.2), per-ray loss weights, and the per-leaf line fields and
per-source temperatures of the several-fields walk (Sec. 2.4).  It holds none of the walk's
arithmetic (no leaf search, no slab test, no accumulation, no direction set):
both the CPU oracle and the GPU library consume the arrays it returns.

The paper's own density cube (a SILCC-Zoom snapshot, Sec. 3 and Sec. 4) is not
available; seeded lognormal clouds with a power-law spectrum stand in for it.
"""

from .fields import gaussian_random_field, lognormal, iid_lognormal_morton
from .octree import (
    Octree,
    morton_encode,
    morton_decode,
    morton_coords,
    uniform_octree,
    threshold_refined_octree,
    uniformity_merged_octree,
    random_octree,
    sparse_random_octree,
    split_leaf,
)
from .sources import cell_centres, leaf_centres, density_weighted_points, random_points
from .configs import WORKLOADS, make_workload, Workload
from .lines import LINES, line_inputs

__all__ = [
    "gaussian_random_field",
    "lognormal",
    "iid_lognormal_morton",
    "Octree",
    "morton_encode",
    "morton_decode",
    "morton_coords",
    "uniform_octree",
    "threshold_refined_octree",
    "uniformity_merged_octree",
    "random_octree",
    "sparse_random_octree",
    "split_leaf",
    "cell_centres",
    "leaf_centres",
    "density_weighted_points",
    "random_points",
    "WORKLOADS",
    "make_workload",
    "Workload",
    "LINES",
    "line_inputs",
]
