"""CPU oracle for the reverse ray walk -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
never calls the GPU library: the two share no code.

The arithmetic lives in ``raywalk_oracle.c`` (plain single-threaded C, FP64,
no floating-point contraction); this module compiles it with gcc and passes
numpy arrays through ctypes.  Every function is pinned by tests under
``tests/`` against closed forms, invariants, brute force and textbook
algorithms (see the test module docstrings for which pin covers which
function).

Functions and the passages they follow:
  healpix_ring   HEALPix RING pixel centres (the direction set of sec. 2.1).
  healpix_nested the same centres in NESTED order (the sub-pixels of a pixel
                 are consecutive: the reference means of sec. 3).
  check_tiling   leaf-only linear octree invariants (sec. 2.3.1).
  walk_one       one ray: DDA + Morton lookup + slab chord (sec. 2.3.1-2.3.2),
                 I = sum_k f_k r_k (sec. 2.3).
  columns        all (source, direction) rays, N and exp(-kappa N) (sec. 2.1).
  gradient       dL/drho_k = sum over rays of dL/dN * r_k (N is linear in rho).
  grid_tree      the contribution grid from a uniform grid by the density +
                 uniformity rule (sec. 2.4): keys, levels, mean values.
  nested_reference  reference columns of a coarse NESTED direction set: the
                 mean of the finer rays inside each pixel, and the relative
                 column error (sec. 3).
  shielding      several fields per leaf: per-ray N_H and line optical depths
                 tau (sec. 2.4), per-source escape probabilities beta
                 (sec. 2.4) and effective visual extinction A_V,eff (sec. 3).
"""

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raywalk_oracle.c")
_LIB = os.path.join(_HERE, "libraywalk_oracle.so")
_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]

OK, ERR_ARG, ERR_UNSORTED, ERR_TILING, ERR_RANGE, ERR_STEPS = 0, -1, -2, -3, -4, -7

_lib = None


def build(source=None, output=None):
    """Compile the oracle with gcc (always recompiles).  source/output let a
    test compile a copy with a planted mistake somewhere else."""
    out = output or _LIB
    # a temporary name per process: parallel test workers may build at once
    tmp = f"{out}.tmp{os.getpid():x}"
    cmd = ["gcc", *_CFLAGS, source or _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _bind(lib):
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.orc_healpix_npix.restype = i64
    lib.orc_healpix_npix.argtypes = [ctypes.c_int]
    lib.orc_healpix_ring.restype = ctypes.c_int
    lib.orc_healpix_ring.argtypes = [ctypes.c_int, P]
    lib.orc_healpix_nested.restype = ctypes.c_int
    lib.orc_healpix_nested.argtypes = [ctypes.c_int, P]
    lib.orc_morton.restype = ctypes.c_uint64
    lib.orc_morton.argtypes = [i64, i64, i64, ctypes.c_int]
    lib.orc_check_tiling.restype = ctypes.c_int
    lib.orc_check_tiling.argtypes = [P, P, i64, ctypes.c_int]
    lib.orc_walk_one.restype = ctypes.c_int
    lib.orc_walk_one.argtypes = [P, P, P, P, i64, ctypes.c_int, P, P, P, P, P, P, P, P, P, P, i64]
    lib.orc_columns.restype = ctypes.c_int
    lib.orc_columns.argtypes = [P, P, P, P, i64, ctypes.c_int, P, i64, P, i64, ctypes.c_double,
                                P, P, P, P, P, P, P, P]
    lib.orc_gradient.restype = ctypes.c_int
    lib.orc_gradient.argtypes = [P, P, i64, ctypes.c_int, P, i64, P, i64, P, P]
    D = ctypes.c_double
    lib.orc_grid_tree.restype = ctypes.c_int
    lib.orc_grid_tree.argtypes = [P, ctypes.c_int, D, D, P, P, P, P]
    lib.orc_nested_reference.restype = ctypes.c_int
    lib.orc_nested_reference.argtypes = [P, i64, P, i64, i64, P, P]
    lib.orc_shielding.restype = ctypes.c_int
    lib.orc_shielding.argtypes = [P, P, i64, ctypes.c_int, P, ctypes.c_int, P, i64, P, i64, D, P,
                                  D, P, P, D, D, P, P, P]
    return lib


def load(path=None):
    """Load the compiled oracle (building it first if it is missing)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def healpix_npix(nside, lib=None):
    return int((lib or load()).orc_healpix_npix(int(nside)))


def healpix_ring(nside, lib=None):
    lib = lib or load()
    n = healpix_npix(nside, lib)
    if n < 0:
        raise ValueError("nside must be >= 1")
    out = np.empty((n, 3), dtype=np.float64)
    st = lib.orc_healpix_ring(int(nside), _p(out))
    if st != OK:
        raise ValueError(f"orc_healpix_ring failed: {st}")
    return out


def healpix_nested(nside, lib=None):
    """HEALPix NESTED pixel centres [12 nside^2, 3] (nside a power of two)."""
    lib = lib or load()
    n = healpix_npix(nside, lib)
    if n < 0:
        raise ValueError("nside must be >= 1")
    out = np.empty((n, 3), dtype=np.float64)
    st = lib.orc_healpix_nested(int(nside), _p(out))
    if st != OK:
        raise ValueError(f"orc_healpix_nested failed: {st}")
    return out


def morton(x, y, z, depth, lib=None):
    return int((lib or load()).orc_morton(int(x), int(y), int(z), int(depth)))


def check_tiling(keys, levels, depth, lib=None):
    keys = _c(keys, np.uint64)
    levels = _c(levels, np.uint8)
    return int((lib or load()).orc_check_tiling(_p(keys), _p(levels), keys.shape[0], int(depth)))


def walk_one(tree, Q, m, rho=None, rho32=None, cap=None, lib=None):
    """Walk one ray; returns a dict with N, N32, texit, steps, hash, clamps,
    visited (leaf indices) and chords."""
    lib = lib or load()
    keys = _c(tree.keys, np.uint64)
    levels = _c(tree.levels, np.uint8)
    rho = _c(tree.rho if rho is None else rho, np.float64)
    r32 = None if rho32 is None else _c(rho32, np.float32)
    Q = _c(Q, np.float64)
    m = _c(m, np.float64)
    cap = cap or 3 * (1 << tree.depth) + 3
    vis = np.empty(cap, dtype=np.int64)
    chords = np.empty(cap, dtype=np.float64)
    N = ctypes.c_double()
    N32 = ctypes.c_float()
    tx = ctypes.c_double()
    steps = ctypes.c_int64()
    h = ctypes.c_uint64()
    cl = ctypes.c_int64()
    st = lib.orc_walk_one(_p(keys), _p(levels), _p(rho), _p(r32), keys.shape[0], tree.depth,
                          _p(Q), _p(m), ctypes.byref(N), ctypes.byref(N32), ctypes.byref(tx),
                          ctypes.byref(steps), ctypes.byref(h), ctypes.byref(cl), _p(vis),
                          _p(chords), cap)
    k = min(steps.value, cap)
    return {"status": st, "N": N.value, "N32": N32.value, "texit": tx.value,
            "steps": steps.value, "hash": h.value, "clamps": cl.value,
            "visited": vis[:k].copy(), "chords": chords[:k].copy()}


def columns(tree, src, dirs, kappa=1.0, rho=None, rho32=None, threads=1, lib=None):
    """All rays (s, d).  Returns a dict of [S, Dn] arrays: N, A, N32, A32
    (only if rho32 is given), texit, steps, hash, plus status and clamps.
    threads > 1 splits the sources over threads (ctypes releases the GIL)."""
    lib = lib or load()
    keys = _c(tree.keys, np.uint64)
    levels = _c(tree.levels, np.uint8)
    rho = _c(tree.rho if rho is None else rho, np.float64)
    r32 = None if rho32 is None else _c(rho32, np.float32)
    src = _c(src, np.float64).reshape(-1, 3)
    dirs = _c(dirs, np.float64).reshape(-1, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    out = {"N": np.empty((S, Dn)), "A": np.empty((S, Dn)), "texit": np.empty((S, Dn)),
           "steps": np.empty((S, Dn), dtype=np.int64), "hash": np.empty((S, Dn), dtype=np.uint64)}
    if r32 is not None:
        out["N32"] = np.empty((S, Dn), dtype=np.float32)
        out["A32"] = np.empty((S, Dn), dtype=np.float32)

    def run(lo, hi):
        cl = ctypes.c_int64()
        sl = {k: v[lo:hi] for k, v in out.items()}
        st = lib.orc_columns(_p(keys), _p(levels), _p(rho), _p(r32), keys.shape[0], tree.depth,
                             _p(src[lo:hi]), hi - lo, _p(dirs), Dn, float(kappa),
                             _p(sl["N"]), _p(sl["A"]), _p(sl.get("N32")), _p(sl.get("A32")),
                             _p(sl["texit"]), _p(sl["steps"]), _p(sl["hash"]), ctypes.byref(cl))
        return st, cl.value

    if threads <= 1 or S < 2 * threads:
        results = [run(0, S)]
    else:
        bounds = np.linspace(0, S, threads + 1).astype(np.int64)
        with ThreadPoolExecutor(threads) as ex:
            results = list(ex.map(lambda ab: run(int(ab[0]), int(ab[1])),
                                  zip(bounds[:-1], bounds[1:])))
    out["status"] = next((st for st, _ in results if st != OK), OK)
    out["clamps"] = sum(c for _, c in results)
    return out


def gradient(tree, src, dirs, g, lib=None):
    """dL/drho for every leaf (FP64), given g = dL/dN of shape [S, Dn]."""
    lib = lib or load()
    keys = _c(tree.keys, np.uint64)
    levels = _c(tree.levels, np.uint8)
    src = _c(src, np.float64).reshape(-1, 3)
    dirs = _c(dirs, np.float64).reshape(-1, 3)
    g = _c(g, np.float64)
    assert g.shape == (src.shape[0], dirs.shape[0])
    grad = np.zeros(keys.shape[0])
    st = lib.orc_gradient(_p(keys), _p(levels), keys.shape[0], tree.depth, _p(src), src.shape[0],
                          _p(dirs), dirs.shape[0], _p(g), _p(grad))
    if st != OK:
        raise RuntimeError(f"orc_gradient failed: {st}")
    return grad


def shielding(tree, fields, src, dirs, length=1.0, temp=None, vturb=0.0, line_A=(), line_nu=(),
              gamma=3.02, av0=6.29e-22, rays=True, threads=1, lib=None):
    """Per-source A_V,eff and escape probabilities, and optionally the per-ray
    values, for leaf fields [n, K] (field 0 = n_H, fields 1.. = the
    population terms of the lines (line_A[f-1], line_nu[f-1])).  Returns a
    dict: rays [S, Dn, K] (N_H, then tau per line) if rays, av_eff [S],
    beta [S, K-1], status.  threads > 1 splits the sources over threads."""
    lib = lib or load()
    keys = _c(tree.keys, np.uint64)
    levels = _c(tree.levels, np.uint8)
    fields = _c(fields, np.float64)
    if fields.ndim == 1:
        fields = fields[:, None]
    n, K = fields.shape
    assert n == keys.shape[0]
    src = _c(src, np.float64).reshape(-1, 3)
    dirs = _c(dirs, np.float64).reshape(-1, 3)
    S, Dn = src.shape[0], dirs.shape[0]
    T = None if temp is None else _c(np.broadcast_to(temp, (S,)), np.float64)
    lA = _c(line_A, np.float64) if K > 1 else None
    lnu = _c(line_nu, np.float64) if K > 1 else None
    if K > 1:
        assert lA.shape == (K - 1,) and lnu.shape == (K - 1,)
    out = {"av_eff": np.empty(S), "beta": np.empty((S, K - 1))}
    if rays:
        out["rays"] = np.empty((S, Dn, K))

    def run(lo, hi):
        return lib.orc_shielding(_p(keys), _p(levels), n, tree.depth, _p(fields), K,
                                 _p(src[lo:hi]), hi - lo, _p(dirs), Dn, float(length),
                                 _p(None if T is None else T[lo:hi]), float(vturb), _p(lA), _p(lnu),
                                 float(gamma), float(av0),
                                 _p(out["rays"][lo:hi]) if rays else None,
                                 _p(out["av_eff"][lo:hi]), _p(out["beta"][lo:hi]))

    if threads <= 1 or S < 2 * threads:
        results = [run(0, S)]
    else:
        bounds = np.linspace(0, S, threads + 1).astype(np.int64)
        with ThreadPoolExecutor(threads) as ex:
            results = list(ex.map(lambda ab: run(int(ab[0]), int(ab[1])),
                                  zip(bounds[:-1], bounds[1:])))
    out["status"] = next((st for st in results if st != OK), OK)
    return out


def nested_reference(fine, coarse=None, lib=None):
    """fine [S, Dfine], coarse [S, Dcoarse] (Dfine = 4^k Dcoarse, NESTED
    order): returns (ref, err) [S, Dcoarse] (err None without coarse)."""
    lib = lib or load()
    fine = _c(fine, np.float64)
    S, Df = fine.shape
    if coarse is not None:
        coarse = _c(coarse, np.float64)
        Dc = coarse.shape[1]
    else:
        raise ValueError("coarse columns are needed to fix the coarse direction count")
    ref = np.empty((S, Dc))
    err = np.empty((S, Dc))
    st = lib.orc_nested_reference(_p(fine), Df, _p(coarse), Dc, S, _p(ref), _p(err))
    if st != OK:
        raise ValueError(f"orc_nested_reference failed: {st}")
    return ref, err


def grid_tree(grid_morton, depth, density_floor, rel_uniformity=0.01, lib=None):
    """Leaf keys (uint64), levels (uint8) and mean values (float64) of the
    refinement rule applied to a Morton-ordered [8^depth] grid."""
    lib = lib or load()
    g = _c(grid_morton, np.float64).reshape(-1)
    assert g.shape[0] == 8 ** depth
    keys = np.empty(g.shape[0], dtype=np.uint64)
    levels = np.empty(g.shape[0], dtype=np.uint8)
    values = np.empty(g.shape[0])
    n = ctypes.c_int64()
    st = lib.orc_grid_tree(_p(g), int(depth), float(density_floor), float(rel_uniformity), _p(keys),
                           _p(levels), _p(values), ctypes.byref(n))
    if st != OK:
        raise ValueError(f"orc_grid_tree failed: {st}")
    k = n.value
    return keys[:k].copy(), levels[:k].copy(), values[:k].copy()
