"""Pins of the oracle's plain FP64 IFGF against facts outside itself:

* the partition of the sources into the level-D neighbour points and the
  cousin points of levels D..3 (Section 2; the method ends at level 3),
* "exact" mode -- every interpolant evaluation replaced by the exact sum
  over relevant children weighted by G(x, x_child)/G(x, x_box) down to the
  exact leaf field of eq. (fieldperbox) -- reproduces the direct sum, which
  pins the tree, neighbour/cousin lists, the factorisation, the propagation
  ratio and the completeness of the relevant cones,
* the interpolation operator reproduces tensor polynomials exactly,
* the IFGF error against the direct sum converges as the interpolation
  order grows, and meets 1e-4 at the default (P_s, P_ang) = (3, 5).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2112_15198_amd import workloads as W


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _two_clusters(n=1200, seed=3):
    rng = np.random.default_rng(seed)
    c1 = rng.normal(size=(n // 2, 3)) * 0.05 + np.array([-1.0, 0, 0])
    c2 = rng.normal(size=(n - n // 2, 3)) * 0.05 + np.array([1.0, 0.3, 0])
    return np.vstack([c1, c2])


GEOMS = {
    "sphere": lambda: (W.fibonacci_sphere(3000), W.kappa_sphere_10ppw(3000)),
    "oblate": lambda: (W.spheroid(3000), W.kappa_oblate_10ppw(3000)),
    "clusters": lambda: (_two_clusters(), 12.0),
    # The paper's test spheroids (1,1,0.1) and (1,1,10) at 8 wavelengths
    # across their diameters d = 2 and d = 20.
    "oblate01": lambda: (W.spheroid(3000, (1.0, 1.0, 0.1)), 8.0 * math.pi),
    "prolate10": lambda: (W.spheroid(3000, (1.0, 1.0, 10.0)), 0.8 * math.pi),
}


@pytest.mark.parametrize("geom", list(GEOMS))
def test_partition_of_sources(geom):
    p, k = GEOMS[geom]()
    cnt = oracle.partition_counts(p, k)
    assert (cnt == p.shape[0]).all()


@pytest.mark.parametrize("geom", list(GEOMS))
def test_exact_mode_reproduces_direct_sum(geom):
    p, k = GEOMS[geom]()
    a = W.densities(p.shape[0], 1, 21)[0]
    ref = oracle.direct_sum(p, a, k)
    ex = oracle.ifgf(p, a, k, exact=True)
    assert relerr(ex, ref) < 1e-12


def test_exact_mode_more_levels():
    # Forcing a deeper tree exercises more propagation ratios.
    p = W.fibonacci_sphere(2000)
    a = W.densities(2000, 1, 22)[0]
    ref = oracle.direct_sum(p, a, 6.0)
    ex = oracle.ifgf(p, a, 6.0, exact=True, levels=6)
    assert relerr(ex, ref) < 1e-12


def test_near_plus_far_is_total():
    p = W.fibonacci_sphere(2500)
    k = W.kappa_sphere_10ppw(2500)
    a = W.densities(2500, 1, 23)[0]
    tot = oracle.ifgf(p, a, k)
    nf = oracle.ifgf(p, a, k, far=False)
    ff = oracle.ifgf(p, a, k, near=False)
    np.testing.assert_allclose(nf + ff, tot, rtol=0, atol=1e-13 * np.abs(tot).max())


@pytest.mark.parametrize("p_s,p_ang", [(3, 5), (2, 3), (5, 7)])
def test_interpolation_reproduces_tensor_polynomials(p_s, p_ang):
    ts, ta = oracle.interp_nodes(p_s, p_ang)
    # Nodes are the first-kind Chebyshev points cos((2j+1) pi / (2n)).
    np.testing.assert_allclose(ts, np.cos((2 * np.arange(p_s) + 1) * np.pi / (2 * p_s)))
    rng = np.random.default_rng(p_s * 10 + p_ang)
    cs = rng.normal(size=p_s) + 1j * rng.normal(size=p_s)
    ct = rng.normal(size=p_ang)
    cp = rng.normal(size=p_ang)

    def f(u):  # degree p_s-1 in u0, p_ang-1 in u1 and u2 (separable sum + product)
        return (np.polyval(cs, u[:, 0]) * np.polyval(ct, u[:, 1]) * np.polyval(cp, u[:, 2])
                + 0.5 * u[:, 0] ** (p_s - 1) * u[:, 1] ** (p_ang - 1))

    grid = np.array([[a, b, c] for a in ts for b in ta for c in ta])
    vals = f(grid)
    u = rng.uniform(-1, 1, (200, 3))
    np.testing.assert_allclose(oracle.interp_eval(p_s, p_ang, vals, u), f(u),
                               rtol=1e-12, atol=1e-12)
    # One degree more is not reproduced.
    g = lambda u: u[:, 1] ** p_ang
    err = np.abs(oracle.interp_eval(p_s, p_ang, g(grid), u) - g(u)).max()
    assert err > 1e-3


def test_convergence_in_interpolation_order():
    n = 4000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 1, 24)[0]
    ref = oracle.direct_sum(p, a, k)
    errs = [relerr(oracle.ifgf(p, a, k, p_s=ps, p_ang=pa, leaf_grid=(1, 2, 4)), ref)
            for ps, pa in [(2, 3), (3, 5), (5, 7), (7, 9)]]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 5e-6 and errs[1] / errs[3] > 100
    # Finer leaf cones at fixed order also converge.
    e2 = relerr(oracle.ifgf(p, a, k, leaf_grid=(2, 4, 8)), ref)
    assert e2 < errs[1] / 5


def test_default_accuracy_sphere_5k():
    w = W.make("sphere_5k")
    ref = oracle.direct_sum(w.points, w.dens[0], w.kappa)
    res, info = oracle.ifgf(w.points, w.dens[0], w.kappa, leaf_grid=(2, 4, 8),
                            return_info=True)
    assert info["D"] == 5
    assert relerr(res, ref) < 1e-4


def test_linearity_in_densities():
    n = 2000
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    a, b = W.densities(n, 2, 25)
    al, be = 1.5 - 0.5j, -0.25 + 2j
    lhs = oracle.ifgf(p, al * a + be * b, k)
    rhs = al * oracle.ifgf(p, a, k) + be * oracle.ifgf(p, b, k)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(rhs).max())


def test_levels_from_leaf_size():
    # D = max(3, 1 + round(log2(H_1 / (leaf_size * lambda)))).
    p = W.fibonacci_sphere(5024)
    _, info = oracle.ifgf(p, np.zeros(5024), 4 * math.pi, far=False, return_info=True)
    assert info["D"] == 5
    _, info = oracle.ifgf(p, np.zeros(5024), 0.5, far=False, return_info=True)
    assert info["D"] == 3
