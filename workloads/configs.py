"""The five named synthetic workloads (sizes of the benchmark study).

Seeds: density field 1000+i, sources 2000+i, loss weights 3000+i, finite-
difference leaf pick 4000+i (numpy PCG64 ``default_rng``).  Each workload
records the actual leaf count it produced.
"""

from dataclasses import dataclass, field

import numpy as np

from .fields import gaussian_random_field, lognormal, iid_lognormal_morton
from .octree import (uniform_octree, threshold_refined_octree, uniformity_merged_octree,
                     grid_to_morton)
from .sources import cell_centres, leaf_centres, density_weighted_points


@dataclass
class Workload:
    index: int
    name: str
    tree: object
    sources: np.ndarray        # float64 [S, 3]
    nside: int
    kappa: float
    variants: tuple
    info: dict = field(default_factory=dict)

    @property
    def n_dirs(self):
        return 12 * self.nside * self.nside

    @property
    def n_rays(self):
        return int(self.sources.shape[0]) * self.n_dirs

    def weights(self, dtype=np.float64):
        """Loss weights w ~ U(0,1), one per (source, direction), [S, Dn]."""
        rng = np.random.default_rng(3000 + self.index)
        return rng.random((self.sources.shape[0], self.n_dirs)).astype(dtype)

    def fd_leaves(self, count=64):
        """Leaves picked for finite-difference checks (sorted, distinct)."""
        rng = np.random.default_rng(4000 + self.index)
        return np.sort(rng.choice(self.tree.n, size=min(count, self.tree.n), replace=False))


def _w0_uniform32():
    rho_m, _ = iid_lognormal_morton(5, 1000)
    tree = uniform_octree(5, rho_m)
    return Workload(0, "uniform32_iid_nside1", tree, cell_centres(5), 1, 1.0, ("fp64",),
                    {"field": "iid lognormal exp(N(0,1)) per cell, Morton order"})


def _w1_amr256():
    g = gaussian_random_field(256, -4.0, 1001)
    rho = lognormal(g, 1.5)
    del g
    thr = 3.0 * rho.mean()
    tree = threshold_refined_octree(rho, 6, thr)
    src = density_weighted_points(tree, 1_000_000, 2001)
    return Workload(1, "amr64to256_k4_nside2", tree, src, 2, 1.0, ("fp64", "fp32k"),
                    {"field": "P(k)~k^-4, sigma_lnrho=1.5, 256^3", "threshold": thr})


def _w2_uniform128():
    g = gaussian_random_field(128, -4.0, 1002)
    rho = lognormal(g, 1.5)
    tree = uniform_octree(7, grid_to_morton(rho))
    return Workload(2, "uniform128_k4_nside4", tree, cell_centres(7), 4, 1.0, ("fp64", "fp32k"),
                    {"field": "P(k)~k^-4, sigma_lnrho=1.5, 128^3"})


def _w3_amr128_adjoint():
    g = gaussian_random_field(128, -4.0, 1003)
    rho = lognormal(g, 1.5)
    thr = 2.0 * rho.mean()
    tree = threshold_refined_octree(rho, 6, thr)
    return Workload(3, "amr64to128_adjoint_nside2", tree, leaf_centres(tree), 2, 1.0,
                    ("fp32k", "adjoint"),
                    {"field": "P(k)~k^-4, sigma_lnrho=1.5, 128^3", "threshold": thr})


def _w4_merged512():
    g = gaussian_random_field(512, -4.0, 1004)
    rho = lognormal(g, 2.0)
    del g
    thr = float(np.percentile(rho, 75.0))
    tree = uniformity_merged_octree(rho, thr, 0.01)
    del rho
    return Workload(4, "merged512_k4_nside1", tree, cell_centres(9), 1, 1.0,
                    ("fp32k", "adjoint", "fp64"),
                    {"field": "P(k)~k^-4, sigma_lnrho=2, 512^3", "density_floor": thr})


WORKLOADS = {0: _w0_uniform32, 1: _w1_amr256, 2: _w2_uniform128, 3: _w3_amr128_adjoint,
             4: _w4_merged512}


def make_workload(index):
    w = WORKLOADS[index]()
    w.info["n_leaves"] = w.tree.n
    w.info["n_sources"] = int(w.sources.shape[0])
    return w
