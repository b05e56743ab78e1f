"""Seeded density fields standing in for the paper's turbulent cloud.

A Gaussian random field with power spectrum P(k) proportional to k**alpha is
drawn as white noise filtered in Fourier space; its lognormal transform
rho = exp(sigma*g - sigma**2/2) has unit expectation.  The arrays are indexed
[ix, iy, iz] with cell (ix, iy, iz) covering [ix, ix+1) * h etc.
"""

import numpy as np

from .octree import morton_coords


def gaussian_random_field(n, spectral_index, seed):
    """Zero-mean, unit-variance periodic Gaussian field on an n**3 grid.

    The Fourier amplitude is |k|**(spectral_index/2), so the power spectrum is
    |k|**spectral_index; the k = 0 mode is removed.  White noise comes from
    numpy's PCG64 (``default_rng(seed)``), so the field is reproducible.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(white)
    del white
    kf = np.fft.fftfreq(n) * n
    kr = np.fft.rfftfreq(n) * n
    k2 = (kf[:, None, None] ** 2 + kf[None, :, None] ** 2) + kr[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (spectral_index / 4.0), 0.0)
    del k2
    fk *= amp
    del amp
    g = np.fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2))
    del fk
    g -= g.mean()
    g /= g.std()
    return g


def lognormal(g, sigma):
    """rho = exp(sigma*g - sigma**2/2): lognormal with sigma_ln(rho) = sigma."""
    return np.exp(sigma * g - 0.5 * sigma * sigma)


def iid_lognormal_morton(level, seed):
    """rho = exp(g), g ~ N(0,1) iid, drawn in Morton order of a uniform grid.

    Returns (rho_morton, rho_grid): the values in Morton order (leaf order of
    a single-level octree) and the same values scattered to an [ix,iy,iz]
    grid.
    """
    n = 1 << level
    rng = np.random.default_rng(seed)
    rho_m = np.exp(rng.standard_normal(n ** 3))
    c = morton_coords(level)
    grid = np.empty((n, n, n))
    grid[c[:, 0], c[:, 1], c[:, 2]] = rho_m
    return rho_m, grid
