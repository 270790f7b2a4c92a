"""Writes the stored expected values of tests/golden/ from the CPU oracle.

Calls only ``oracle`` (the plain FP64 IFGF, Algorithm "IFGF Method" of the
paper, and the FP64 direct sum of eq. (field1)) on seeded inputs from
``paper_2112_15198_amd.workloads`` (an input generator that holds none of the
method's arithmetic).  Every fixture is a .npz file holding the target
indices, the oracle's values there and the parameters it was made with.

    python tests/golden/make_golden.py [name ...]

Fixtures:
  ifgf_sphere_321k   oracle IFGF of the N = 321,536 unit-sphere lattice
                     (kappa = 32 pi, (P_s, P_ang) = (3, 5), leaf cone grid
                     (2, 4, 8)) at its 4,096 sampled targets, RHS 0
  ifgf_sphere_60k    oracle IFGF of an N = 60,000 unit-sphere lattice at
                     ~10 points per wavelength, 4 RHS (seed 38), at 8,192
                     sampled targets (seed 39)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2112_15198_amd import workloads as W  # noqa: E402


def sphere_321k():
    w = W.make("sphere_321k")
    t0 = time.perf_counter()
    full = oracle.ifgf(w.points, w.dens[0], w.kappa, p_s=3, p_ang=5, leaf_grid=(2, 4, 8))
    dt = time.perf_counter() - t0
    return dict(targets=w.targets, values=full[w.targets][None, :], n=w.points.shape[0],
                kappa=w.kappa, seed=1002, n_rhs=1, p_s=3, p_ang=5,
                leaf_grid=np.array([2, 4, 8]), oracle_seconds=dt)


def sphere_60k():
    n = 60000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 4, 38)
    tg = W.sample_targets(n, 8192, 39)
    vals = []
    t0 = time.perf_counter()
    for r in range(4):
        vals.append(oracle.ifgf(p, a[r], k, p_s=3, p_ang=5, leaf_grid=(2, 4, 8))[tg])
    dt = time.perf_counter() - t0
    return dict(targets=tg, values=np.stack(vals), n=n, kappa=k, seed=38, n_rhs=4,
                p_s=3, p_ang=5, leaf_grid=np.array([2, 4, 8]), oracle_seconds=dt)


FIXTURES = {"ifgf_sphere_321k": sphere_321k, "ifgf_sphere_60k": sphere_60k}


def main(names):
    for name in names or FIXTURES:
        rec = FIXTURES[name]()
        out = os.path.join(HERE, name + ".npz")
        np.savez(out, **rec)
        print(f"{name}: {rec['values'].shape} values, oracle {rec['oracle_seconds']:.1f} s -> {out}",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
