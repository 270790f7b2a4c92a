"""Pins of the oracle's FP64 direct sum (eq. (field1)) against facts that do
not come from the oracle itself: closed forms of small symmetric point sets,
the analytic single-layer integral over a sphere, and the symmetry and
linearity of the discrete operator."""
import math

import numpy as np
import pytest

import oracle
from paper_2112_15198_amd import workloads as W


def test_two_points_closed_form():
    # |x1 - x2| = 1 and kappa = pi: G = e^{i pi} / (4 pi) = -1/(4 pi).
    p = np.array([[0.0, 0.0, 0.0], [0.0, 0.6, 0.8]])
    a = np.array([2.0 - 1.0j, 0.5 + 3.0j])
    out = oracle.direct_sum(p, a, math.pi)
    g = -1.0 / (4.0 * math.pi)
    assert abs(out[0] - a[1] * g) < 1e-15
    assert abs(out[1] - a[0] * g) < 1e-15


def test_laplace_tetrahedron():
    # kappa = 0: regular tetrahedron with edge L, unit densities:
    # I = 3 / (4 pi L) at every vertex.
    L = 0.7
    # (+-1, 0, -1/sqrt 2), (0, +-1, 1/sqrt 2) have edge 2.
    p = L / 2 * np.array([[1, 0, -1 / math.sqrt(2)],
                           [-1, 0, -1 / math.sqrt(2)],
                           [0, 1, 1 / math.sqrt(2)],
                           [0, -1, 1 / math.sqrt(2)]])
    out = oracle.direct_sum(p, np.ones(4), 0.0)
    np.testing.assert_allclose(out, 3.0 / (4.0 * math.pi * L), rtol=1e-14, atol=0)


def test_octahedron_helmholtz_closed_form():
    # Vertices (+-1,0,0),(0,+-1,0),(0,0,+-1): four neighbours at sqrt 2 and
    # one opposite vertex at 2.  Unit densities.
    p = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=float)
    k = 3.7
    r2 = math.sqrt(2.0)
    exact = 4 * np.exp(1j * k * r2) / (4 * math.pi * r2) + np.exp(2j * k) / (8 * math.pi)
    out = oracle.direct_sum(p, np.ones(6), k)
    np.testing.assert_allclose(out, exact, rtol=1e-14, atol=0)


def test_sign_convention_outgoing():
    # e^{+i kappa r}: a quarter wavelength apart the value is +i/(4 pi r).
    k = 2.0
    r = math.pi / (2 * k)
    p = np.array([[0.0, 0, 0], [r, 0, 0]])
    out = oracle.direct_sum(p, np.array([0.0, 1.0]), k)
    assert abs(out[0] - 1j / (4 * math.pi * r)) < 1e-15


def test_sphere_single_layer_integral():
    # For |x| = R = 1, int_S e^{i k |x-y|}/(4 pi |x-y|) dS(y) = (e^{2ik} - 1)/(2ik)
    # (dS = 2 pi r dr in the distance r).  The Fibonacci lattice is an
    # equal-area rule (weights 4 pi/N); the excluded self cell of radius
    # rho = 2/sqrt(N) carries int_{disk} 1/(4 pi r) dA = rho/2 to leading order.
    n = 20000
    p = W.fibonacci_sphere(n)
    k = 3.0
    tg = np.array([0, 5000, 10000, 15000, 19999])
    out = oracle.direct_sum(p, np.full(n, 4 * math.pi / n), k, tg)
    exact = (np.exp(2j * k) - 1) / (2j * k)
    approx = out + 1.0 / math.sqrt(n)
    rel = np.abs(approx - exact) / abs(exact)
    assert rel.max() < 2e-2, rel
    # Without the self-cell term the error is several times larger; the pin
    # therefore sees the 1/(4 pi) and the sign of the phase.
    assert (np.abs(out - exact) / abs(exact)).min() > 2 * rel.max()


def _matrix_apply(p, a, k):
    return oracle.direct_sum(p, a, k)


def test_reciprocity_and_linearity():
    rng = np.random.default_rng(5)
    p = rng.uniform(-1, 1, (300, 3))
    k = 5.5
    a = rng.normal(size=300) + 1j * rng.normal(size=300)
    b = rng.normal(size=300) + 1j * rng.normal(size=300)
    Aa, Ab = _matrix_apply(p, a, k), _matrix_apply(p, b, k)
    # Complex-symmetric operator: b^T (A a) = a^T (A b), no conjugation.
    lhs, rhs = np.dot(b, Aa), np.dot(a, Ab)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    al, be = 0.3 - 2j, -1.7 + 0.2j
    comb = _matrix_apply(p, al * a + be * b, k)
    np.testing.assert_allclose(comb, al * Aa + be * Ab, rtol=1e-12, atol=1e-13)


def test_targets_subset_matches_full():
    rng = np.random.default_rng(9)
    p = rng.uniform(-1, 1, (500, 3))
    a = rng.normal(size=500) + 1j * rng.normal(size=500)
    full = oracle.direct_sum(p, a, 4.0)
    tg = np.array([3, 77, 499, 0])
    np.testing.assert_array_equal(oracle.direct_sum(p, a, 4.0, tg), full[tg])


def test_small_brute_force_dense_matrix():
    # Dense-matrix evaluation of eq. (field1) on N = 1500 (numpy, FP64).
    rng = np.random.default_rng(11)
    n = 1500
    p = rng.uniform(-1, 1, (n, 3))
    a = rng.normal(size=n) + 1j * rng.normal(size=n)
    k = 7.0
    d = np.linalg.norm(p[:, None, :] - p[None, :, :], axis=2)
    np.fill_diagonal(d, 1.0)
    G = np.exp(1j * k * d) / (4 * np.pi * d)
    np.fill_diagonal(G, 0.0)
    np.testing.assert_allclose(oracle.direct_sum(p, a, k), G @ a, rtol=1e-11, atol=1e-12)
