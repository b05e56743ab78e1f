"""Seeded inputs of the several-fields walk: per-leaf hydrogen density and
level-population terms of a few cooling lines, per-source temperatures.

Field 0 is n_H = n0 * rho (cm^-3).  Field j >= 1 is a stand-in for the
population term [n_j g_i / g_j - n_i] of line j (sec. 2.4): x_j * n_H * u
with a fixed abundance-times-level-fraction x_j and u ~ U(-0.05, 1) per
leaf, so that about 5% of the leaves are inverted (negative term) and a few
are exactly zero.  Source temperatures are log-uniform in 10..300 K and the
turbulent speed is 1 km/s.  The box edge defaults to 125 pc, the domain of
the paper's cloud (sec. 4).

The line list holds measured Einstein A coefficients (s^-1) and rest
frequencies (Hz) of CO, [CII], [OI] and [CI] transitions (values as listed in
the Leiden LAMDA database); they only set realistic magnitudes here.
"""

import numpy as np

PARSEC_CM = 3.0857e18

# (name, Einstein A in s^-1, rest frequency in Hz, abundance x level fraction)
LINES = (
    ("CO 1-0", 7.203e-08, 115.2712018e9, 3e-5),
    ("[CII] 158um", 2.29e-06, 1900.5369e9, 3e-5),
    ("[OI] 63um", 8.91e-05, 4744.77749e9, 1e-4),
    ("CO 2-1", 6.910e-07, 230.538e9, 3e-5),
    ("[CI] 609um", 7.88e-08, 492.160651e9, 2e-5),
    ("CO 3-2", 2.497e-06, 345.7959899e9, 2e-5),
    ("[CI] 370um", 2.65e-07, 809.34197e9, 1e-5),
)


def line_inputs(tree, sources, n_lines, seed, n0=10.0, box_pc=125.0, vturb=1.0e5):
    """Inputs of one several-fields call for tree (its rho is the density
    field) and sources [S, 3]: dict with fields [n, 1 + n_lines] (float64),
    temp [S], vturb, line_A, line_nu, length (cm)."""
    if not 0 <= n_lines <= len(LINES):
        raise ValueError(f"n_lines must be in 0..{len(LINES)}")
    rng = np.random.default_rng(seed)
    n = tree.n
    nh = n0 * np.asarray(tree.rho, dtype=np.float64)
    fields = np.empty((n, 1 + n_lines))
    fields[:, 0] = nh
    for j in range(n_lines):
        u = rng.uniform(-0.05, 1.0, n)
        u[rng.random(n) < 0.01] = 0.0
        fields[:, 1 + j] = LINES[j][3] * nh * u
    S = sources.shape[0]
    temp = 10.0 ** rng.uniform(1.0, np.log10(300.0), S)
    return {
        "fields": fields,
        "temp": temp,
        "vturb": vturb,
        "line_A": np.array([ln[1] for ln in LINES[:n_lines]]),
        "line_nu": np.array([ln[2] for ln in LINES[:n_lines]]),
        "length": box_pc * PARSEC_CM,
    }
