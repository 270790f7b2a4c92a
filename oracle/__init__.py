"""CPU FP64 oracle for the IFGF Helmholtz operator -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library never does.

* :func:`direct_sum` -- eq. (field1) of the paper, the O(N^2) definition.
* :func:`ifgf` -- the IFGF method (Algorithm "IFGF Method": LevelDEvaluations,
  then Interpolation(d) and Propagation(d) for d = D..3) plus the level-D
  neighbour direct sum, in plain FP64 C++ (``ifgf_oracle.cpp``).
* :func:`partition_counts`, :func:`interp_eval` -- hooks for structural pins.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build, library_path

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        c_i64, c_dbl, c_int = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        P = ctypes.c_void_p
        lib.oracle_direct_sum.argtypes = [P, c_i64, P, c_dbl, P, c_i64, P]
        lib.oracle_ifgf.argtypes = [P, c_i64, P, c_dbl, c_dbl, P, P, P, P]
        lib.oracle_partition_counts.argtypes = [P, c_i64, c_dbl, c_dbl, P, P, P]
        lib.oracle_interp_nodes.argtypes = [c_int, c_int, P, P]
        lib.oracle_interp_eval.argtypes = [c_int, c_int, P, P, c_i64, P]
        lib.oracle_cone_keys.argtypes = [P, c_i64, c_dbl, c_dbl, P, P, c_int, P, c_i64]
        lib.oracle_cone_keys.restype = c_i64
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = c_int
        for f in (lib.oracle_direct_sum, lib.oracle_ifgf,
                  lib.oracle_partition_counts, lib.oracle_interp_nodes,
                  lib.oracle_interp_eval):
            f.restype = c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pts(points):
    p = np.ascontiguousarray(points, dtype=np.float64)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("points must have shape (N, 3)")
    return p


def _dens(dens, n):
    a = np.ascontiguousarray(np.asarray(dens, dtype=np.complex128).reshape(n))
    return a.view(np.float64)


def direct_sum(points, dens, kappa, targets=None):
    """I(x_l) = sum_{m != l} a_m e^{i kappa r}/(4 pi r) at the given targets."""
    p = _pts(points)
    n = p.shape[0]
    a = _dens(dens, n)
    t = (np.arange(n, dtype=np.int64) if targets is None
         else np.ascontiguousarray(targets, dtype=np.int64))
    out = np.zeros(2 * t.shape[0], dtype=np.float64)
    rc = _load().oracle_direct_sum(_ptr(p), n, _ptr(a), float(kappa), _ptr(t),
                                   t.shape[0], _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_direct_sum failed ({rc})")
    return out.view(np.complex128)


GRID_RULES = {"auto": 0, "double": 1, "constant": 2}


def _options(p_s, p_ang, leaf_grid, levels, exact, stages, grid_rule, leaf_max,
             leaf_abs):
    """Flat option arrays of the C interface.

    Levels: ``levels`` if > 0, else D = max(3, 1 + round(log2(H_1 / s)))
    with s = leaf_abs (length units) if > 0, else leaf_size wavelengths;
    then, if leaf_max > 0 (wavelengths), one more level while the leaf side
    exceeds leaf_max wavelengths.  grid_rule: "auto" (the leaf cone grid
    doubles per level up for kappa > 0, constant for kappa = 0), "double"
    or "constant"."""
    opts = np.array([p_s, p_ang, leaf_grid[0], leaf_grid[1], leaf_grid[2],
                     levels, 1 if exact else 0, stages,
                     GRID_RULES[grid_rule]], dtype=np.int32)
    dopts = np.array([leaf_max, leaf_abs], dtype=np.float64)
    return opts, dopts


def ifgf(points, dens, kappa, p_s=3, p_ang=5, leaf_size=0.25,
         leaf_grid=(1, 2, 4), levels=0, exact=False, near=True, far=True,
         return_info=False, grid_rule="auto", leaf_max=0.0, leaf_abs=0.0):
    """Plain FP64 IFGF of eq. (field1) at every point (user order)."""
    p = _pts(points)
    n = p.shape[0]
    a = _dens(dens, n)
    opts, dopts = _options(p_s, p_ang, leaf_grid, levels, exact,
                           (1 if near else 0) | (2 if far else 0), grid_rule,
                           leaf_max, leaf_abs)
    out = np.zeros(2 * n, dtype=np.float64)
    info = np.zeros(2 + 2 * 32 + 2, dtype=np.float64)
    rc = _load().oracle_ifgf(_ptr(p), n, _ptr(a), float(kappa),
                             float(leaf_size), _ptr(opts), _ptr(dopts), _ptr(out),
                             _ptr(info))
    if rc != 0:
        raise RuntimeError(f"oracle_ifgf failed ({rc})")
    res = out.view(np.complex128)
    if not return_info:
        return res
    D = int(info[0])
    return res, {"D": D, "H1": float(info[1]),
                 "boxes": [int(info[2 * d]) for d in range(1, D + 1)],
                 "cones": [int(info[2 * d + 1]) for d in range(1, D + 1)],
                 "setup_s": float(info[66]), "eval_s": float(info[67])}


def threads():
    """OpenMP threads used by the oracle's parallel loops."""
    return int(_load().oracle_threads())


def partition_counts(points, kappa, leaf_size=0.25, levels=0, leaf_max=0.0,
                     leaf_abs=0.0):
    """Per-target number of sources covered by near field plus cousins."""
    p = _pts(points)
    n = p.shape[0]
    opts, dopts = _options(1, 1, (1, 2, 4), levels, False, 0, "auto", leaf_max, leaf_abs)
    out = np.zeros(n, dtype=np.int64)
    rc = _load().oracle_partition_counts(_ptr(p), n, float(kappa), float(leaf_size),
                                         _ptr(opts), _ptr(dopts), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_partition_counts failed ({rc})")
    return out


def interp_nodes(p_s, p_ang):
    ts = np.zeros(p_s)
    ta = np.zeros(p_ang)
    _load().oracle_interp_nodes(p_s, p_ang, _ptr(ts), _ptr(ta))
    return ts, ta


def interp_eval(p_s, p_ang, values, u):
    """Interpolate node values (s, theta, phi order, phi fastest) at u (m, 3)."""
    v = np.ascontiguousarray(np.asarray(values, dtype=np.complex128).ravel())
    assert v.shape[0] == p_s * p_ang * p_ang
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(2 * uu.shape[0])
    _load().oracle_interp_eval(p_s, p_ang, _ptr(v.view(np.float64)), _ptr(uu),
                               uu.shape[0], _ptr(out))
    return out.view(np.complex128)


def cone_keys(points, kappa, level, p_s=3, p_ang=5, leaf_size=0.25,
              leaf_grid=(1, 2, 4), levels=0, grid_rule="auto", leaf_max=0.0,
              leaf_abs=0.0):
    """Sorted relevant-cone keys box * grid + gamma of octree level `level`."""
    p = _pts(points)
    n = p.shape[0]
    opts, dopts = _options(p_s, p_ang, leaf_grid, levels, False, 0, grid_rule,
                           leaf_max, leaf_abs)
    L = _load()
    cnt = L.oracle_cone_keys(_ptr(p), n, float(kappa), float(leaf_size),
                             _ptr(opts), _ptr(dopts), int(level), None, 0)
    if cnt < 0:
        raise RuntimeError("oracle_cone_keys failed")
    out = np.zeros(cnt, dtype=np.uint64)
    L.oracle_cone_keys(_ptr(p), n, float(kappa), float(leaf_size), _ptr(opts),
                       _ptr(dopts), int(level), _ptr(out), cnt)
    return out
