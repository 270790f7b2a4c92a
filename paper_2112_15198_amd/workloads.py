"""Seeded synthetic workloads for the IFGF Helmholtz operator.

This module only produces inputs: point sets, densities, wavenumbers and
sampled target indices.  It holds none of the IFGF arithmetic and imports
nothing from the rest of the package, so both the GPU path and the CPU
oracle can be fed from it.

Geometries stand in for the paper's sphere and spheroid test surfaces
(Section "Numerical results": sphere of radius a, oblate and prolate
spheroids).  The paper discretises them with parametrised patches that it
does not specify; here a Fibonacci lattice is used instead:

    z_i = 1 - (2i+1)/N,  rho_i = sqrt(1 - z_i^2),
    phi_i = (i * pi * (3 - sqrt 5)) mod 2 pi,
    x_i = (rho_i cos phi_i, rho_i sin phi_i, z_i),

mapped to a spheroid with semi-axes (ax, ay, az) by axis scaling.
Densities have real and imaginary parts iid U(-1, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Surface area of the spheroid with semi-axes (1, 1, 0.25) (oblate,
# eccentricity sqrt(1 - 1/16)); used to set ~10 points per wavelength.
OBLATE_025_AREA = 7.1201


def fibonacci_sphere(n: int) -> np.ndarray:
    """N points on the unit sphere as a Fibonacci lattice, shape (N, 3), FP64."""
    if n < 1:
        raise ValueError("n must be >= 1")
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ga = math.pi * (3.0 - math.sqrt(5.0))
    phi = np.mod(i * ga, 2.0 * math.pi)
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def spheroid(n: int, axes=(1.0, 1.0, 0.25)) -> np.ndarray:
    """Fibonacci lattice mapped to the spheroid with the given semi-axes."""
    p = fibonacci_sphere(n)
    return p * np.asarray(axes, dtype=np.float64)[None, :]


def densities(n: int, n_rhs: int, seed: int) -> np.ndarray:
    """Complex128 densities, shape (n_rhs, N), Re and Im iid U(-1, 1)."""
    a = np.random.default_rng(seed).uniform(-1.0, 1.0, (n_rhs, n, 2))
    return a[..., 0] + 1j * a[..., 1]


def sample_targets(n: int, m: int, seed: int) -> np.ndarray:
    """Sorted int64 indices of m distinct targets (all of them if m >= n)."""
    if m >= n:
        return np.arange(n, dtype=np.int64)
    idx = np.random.default_rng(seed).choice(n, m, replace=False)
    return np.sort(idx.astype(np.int64))


def kappa_sphere_10ppw(n: int) -> float:
    """Wavenumber giving ~10 points per wavelength on the unit sphere."""
    return math.sqrt(math.pi * n) / 10.0


def kappa_oblate_10ppw(n: int) -> float:
    """Wavenumber giving ~10 points per wavelength on the (1,1,0.25) spheroid."""
    return 2.0 * math.pi * math.sqrt(n / (100.0 * OBLATE_025_AREA))


@dataclass
class Instance:
    name: str
    points: np.ndarray          # (N, 3) float64
    kappa: float
    dens: np.ndarray            # (n_rhs, N) complex128
    targets: np.ndarray         # sampled target indices for the error estimate
    meta: dict = field(default_factory=dict)


def _instance(name, pts, kappa, n_rhs, seed, n_samples):
    n = pts.shape[0]
    return Instance(name, pts, float(kappa), densities(n, n_rhs, seed),
                    sample_targets(n, n_samples, seed + 1),
                    {"N": n, "n_rhs": n_rhs, "seed": seed})


# Plan options of each workload (keyword arguments of plan / plan_batched).
# The 48-instance batch takes a finer radial cone grid at the leaf level:
# with (2, 4, 8) its worst instance is within 8.2e-5 of the direct sum on
# its 4,096 sampled targets but beyond 1e-4 on subsets of them, the error of
# the radial interpolation setting the floor (more levels barely lower it);
# (3, 4, 8) halves that error at 1.3 times the apply time.
PLAN_OPTIONS = {"batch48": dict(leaf_grid=(3, 4, 8))}


def plan_options(name: str) -> dict:
    """Plan options with which the workload is run (leaf cone grid etc.)."""
    opts = {"leaf_grid": (2, 4, 8)}
    opts.update(PLAN_OPTIONS.get(name, {}))
    return opts

# The workloads.  Keys name what each workload is.
WORKLOADS = {
    # N=5,024 unit-sphere lattice, kappa = 4 pi (4 wavelengths across).
    "sphere_5k": dict(kind="sphere", n=5024, kappa=4.0 * math.pi, n_rhs=1,
                      seed=1001, n_samples=5024),
    # N=321,536 unit-sphere lattice, kappa = 32 pi.
    "sphere_321k": dict(kind="sphere", n=321536, kappa=32.0 * math.pi,
                        n_rhs=1, seed=1002, n_samples=4096),
    # N=1,048,576 on the (1,1,0.25) spheroid, kappa = 64 pi, 4 RHS.
    "oblate_1m": dict(kind="oblate", n=1048576, kappa=64.0 * math.pi,
                      n_rhs=4, seed=1003, n_samples=4096),
    # 48 uneven instances (sphere or spheroid by seed), 4 RHS each.
    "batch48": dict(kind="batch", n_inst=48, n_min=4000, n_max=200000,
                    n_rhs=4, seed=1004, n_samples=4096),
    # N=5,144,576 unit-sphere lattice, kappa = 128 pi.
    "sphere_5m": dict(kind="sphere", n=5144576, kappa=128.0 * math.pi,
                      n_rhs=1, seed=1005, n_samples=4096),
    # The paper's single-node test geometries (Section "Numerical results"),
    # sized by their diameter d in wavelengths, with the paper's point
    # counts: the unit sphere and the oblate spheroid
    # x^2 + y^2 + (z/0.1)^2 = 1 at d = 2 = 128 lambda (kappa = 128 pi), and
    # the prolate spheroid x^2 + y^2 + (z/10)^2 = 1 at d = 20 = 256 lambda
    # (kappa = 25.6 pi).
    "sphere_128l": dict(kind="sphere", n=1572864, kappa=128.0 * math.pi, n_rhs=1,
                        seed=1008, n_samples=4096),
    "oblate01_128l": dict(kind="spheroid", axes=(1.0, 1.0, 0.1), n=1572864,
                          kappa=128.0 * math.pi, n_rhs=1, seed=1006, n_samples=4096),
    "prolate10_256l": dict(kind="spheroid", axes=(1.0, 1.0, 10.0), n=6291456,
                           kappa=25.6 * math.pi, n_rhs=1, seed=1007, n_samples=4096),
}


def make(name: str, n_rhs: int | None = None, n_samples: int | None = None):
    """Build a workload by name; returns an Instance, or a list for batches."""
    w = dict(WORKLOADS[name])
    if n_rhs is not None:
        w["n_rhs"] = n_rhs
    if n_samples is not None:
        w["n_samples"] = n_samples
    if w["kind"] == "sphere":
        return _instance(name, fibonacci_sphere(w["n"]), w["kappa"],
                         w["n_rhs"], w["seed"], w["n_samples"])
    if w["kind"] == "oblate":
        return _instance(name, spheroid(w["n"]), w["kappa"], w["n_rhs"],
                         w["seed"], w["n_samples"])
    if w["kind"] == "spheroid":
        return _instance(name, spheroid(w["n"], w["axes"]), w["kappa"], w["n_rhs"],
                         w["seed"], w["n_samples"])
    if w["kind"] == "batch":
        return make_batch(w["n_inst"], w["n_min"], w["n_max"], w["n_rhs"],
                          w["seed"], w["n_samples"])
    raise KeyError(name)


def make_batch(n_inst, n_min, n_max, n_rhs, seed, n_samples):
    """Uneven instances: N log-uniform in [n_min, n_max], geometry by seed.

    Instance i uses seed 3000 + seed + i (seed 1004 gives 4004+i), draws
    its kind (sphere or (1,1,0.25) spheroid) and N from that seed, and sets
    kappa for ~10 points per wavelength.
    """
    out = []
    for i in range(n_inst):
        s = 3000 + seed + i
        rng = np.random.default_rng(s)
        oblate = bool(rng.integers(0, 2))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        if oblate:
            pts, kap, kind = spheroid(n), kappa_oblate_10ppw(n), "oblate"
        else:
            pts, kap, kind = fibonacci_sphere(n), kappa_sphere_10ppw(n), "sphere"
        inst = _instance(f"inst{i}_{kind}_{n}", pts, kap, n_rhs, s, n_samples)
        inst.meta["kind"] = kind
        out.append(inst)
    return out
