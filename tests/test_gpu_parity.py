"""GPU parity of libifgf.so against the CPU oracle.

Bars (written in each test), each checked in relative l2 AND element-wise
(max_i |g_i - o_i| / max_i |o_i|, see tests/parity.py):
  * FP64 mode vs the oracle's plain FP64 IFGF (same discrete choices): 1e-10.
  * FP32-mixed and FP32 with the three-term BF16 product vs the oracle IFGF:
    2e-5 (their rounding through the levels; measured 3e-7 and 3e-6 in l2).
  * Near field alone: FP64 1e-13, FP32-mixed 1e-6.
  * Against the FP64 direct sum of eq. (field1): relative l2 <= 1e-4, the
    paper's error measure (eq. errorcomputation).
All inputs are seeded; every case prints its name before touching the GPU.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2112_15198_amd import workloads as W
from parity import assert_close, relerr

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def run_gpu(points, dens, kappa, precision="fp64", **kw):
    """dens: (n_rhs, N) complex128 numpy -> (n_rhs, N) complex128 numpy."""
    import torch
    import paper_2112_15198_amd as ifgf
    dens = np.atleast_2d(dens)
    pl = ifgf.plan(points, kappa, precision=precision, n_rhs=dens.shape[0], **kw)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    a = torch.from_numpy(np.ascontiguousarray(dens)).to(dt).cuda()
    out = pl.apply(a)
    pl.check()
    res = out.cpu().numpy().astype(np.complex128)
    info = pl.info()
    pl.close()
    return res, info


def test_fp64_matches_oracle_ifgf_sphere_5k():
    w = W.make("sphere_5k")
    say("fp64 sphere_5k N=5024")
    g, info = run_gpu(w.points, w.dens, w.kappa)
    o, oi = oracle.ifgf(w.points, w.dens[0], w.kappa, leaf_grid=(2, 4, 8), return_info=True)
    assert info["D"] == oi["D"] == 5
    # The GPU marks cones adjacent to a boundary within 1e-9 of a cone width
    # as relevant too; it never has fewer relevant cones than the oracle.
    assert all(gc >= oc for gc, oc in zip(info["cones"], oi["cones"][2:][::-1]))
    assert_close(g[0], o, 1e-10, "fp64 sphere_5k vs oracle")
    ref = oracle.direct_sum(w.points, w.dens[0], w.kappa)
    assert relerr(g[0], ref) <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_fp32_mixed_sphere_5k_vs_direct_sum(precision):
    w = W.make("sphere_5k")
    say(precision, "sphere_5k N=5024")
    g, _ = run_gpu(w.points, w.dens, w.kappa, precision=precision)
    o = oracle.ifgf(w.points, w.dens[0], w.kappa, leaf_grid=(2, 4, 8))
    assert_close(g[0], o, 2e-5, f"{precision} sphere_5k vs oracle")
    ref = oracle.direct_sum(w.points, w.dens[0], w.kappa)
    assert relerr(g[0], ref) <= 1e-4


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_near_field_alone(precision, tol):
    n = 9001  # ragged: not a multiple of any block size
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    a = W.densities(n, 1, 31)
    say("near field", precision, "N=", n)
    g, _ = run_gpu(p, a, k, precision=precision, stages=1)
    o = oracle.ifgf(p, a[0], k, far=False)
    assert_close(g[0], o, tol, f"near field {precision}")


def test_far_field_alone_fp64():
    n = 7333
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 1, 32)
    say("far field fp64 N=", n)
    g, _ = run_gpu(p, a, k, stages=2)
    o = oracle.ifgf(p, a[0], k, near=False, leaf_grid=(2, 4, 8))
    assert_close(g[0], o, 1e-10, "far field fp64")


def _paper_spheroid(geom, n):
    """The paper's (1,1,0.1) and (1,1,10) spheroids at 12 wavelengths across
    their diameters (2 and 20)."""
    if geom == "oblate01":
        return W.spheroid(n, (1.0, 1.0, 0.1)), 12.0 * math.pi
    return W.spheroid(n, (1.0, 1.0, 10.0)), 1.2 * math.pi


@pytest.mark.parametrize("geom", ["oblate", "clusters", "deep", "oblate01", "prolate10"])
def test_fp64_matches_oracle_geometries(geom):
    if geom == "oblate":
        n = 12000
        p, k, lv = W.spheroid(n), W.kappa_oblate_10ppw(n), 0
    elif geom in ("oblate01", "prolate10"):
        p, k = _paper_spheroid(geom, 8000)
        lv = 0
    elif geom == "clusters":
        rng = np.random.default_rng(3)
        p = np.vstack([rng.normal(size=(1500, 3)) * 0.05 - [1.0, 0, 0],
                       rng.normal(size=(1500, 3)) * 0.05 + [1.0, 0.3, 0]])
        k, lv = 12.0, 0
    else:  # forced deep tree on a small sphere: many propagation levels
        p, k, lv = W.fibonacci_sphere(2500), 10.0, 6
    a = W.densities(len(p), 1, 33)
    say("fp64 geometry", geom, "N=", len(p))
    g, _ = run_gpu(p, a, k, levels=lv)
    o = oracle.ifgf(p, a[0], k, leaf_grid=(2, 4, 8), levels=lv)
    assert_close(g[0], o, 1e-10, f"fp64 {geom}")


@pytest.mark.parametrize("geom", ["oblate01", "prolate10"])
def test_fp32_paper_spheroids(geom):
    """FP32-mixed on the paper's spheroids (autotuned kernels): the oracle
    IFGF to 2e-5 (FP32 rounding) and the direct sum to 1e-3 (the method's
    error on these anisotropic point sets)."""
    p, k = _paper_spheroid(geom, 8000)
    a = W.densities(len(p), 1, 36)
    say("fp32 paper spheroid", geom)
    g, _ = run_gpu(p, a, k, precision="fp32", autotune=True)
    o = oracle.ifgf(p, a[0], k, leaf_grid=(2, 4, 8))
    assert_close(g[0], o, 2e-5, f"fp32 {geom}")
    d = oracle.direct_sum(p, a[0], k)
    assert relerr(g[0], d) <= 1e-3


@pytest.mark.parametrize("prop", ["node", "small", "medium"])
@pytest.mark.parametrize("case", ["wide", "odd", "deep", "clusters", "bigleaf"])
def test_fp32_cone_selection_matches_oracle(case, prop):
    """FP32-mixed propagation picks each angle's cone from an FP32 estimate
    confirmed with FP64 side tests against the cone boundaries, and the leaf
    evaluation reduces its phase turns in FP32.  Cases that stress both: the
    widest cones (leaf grid (1,2,4): theta and phi widths pi/2), odd cone
    counts ((3,3,5)), a forced deep tree (narrow cones at the top), clustered
    points, and leaves of a wavelength (four times the default side).  The
    per-node, one-wave and four-wave forms against the oracle IFGF at the
    FP32 bar, 2e-5, element-wise and in l2."""
    grid, lv, size = (2, 4, 8), 0, 0.25
    if case == "wide":
        p, k, grid = W.fibonacci_sphere(3000), W.kappa_sphere_10ppw(3000), (1, 2, 4)
    elif case == "odd":
        p, k, grid = W.fibonacci_sphere(3000), W.kappa_sphere_10ppw(3000), (3, 3, 5)
    elif case == "deep":
        p, k, lv = W.fibonacci_sphere(2500), 10.0, 6
    elif case == "clusters":
        rng = np.random.default_rng(3)
        p = np.vstack([rng.normal(size=(1500, 3)) * 0.05 - [1.0, 0, 0],
                       rng.normal(size=(1500, 3)) * 0.05 + [1.0, 0.3, 0]])
        k = 12.0
    else:  # 2.5 points per wavelength: leaf boxes of about a wavelength, D = 5
        p, k, size = W.fibonacci_sphere(6000), 4.0 * W.kappa_sphere_10ppw(6000), 1.0
    a = W.densities(len(p), 1, 52)
    say("fp32 cone selection", case, prop, "N=", len(p), "grid", grid, "levels", lv)
    g, _ = run_gpu(p, a, k, precision="fp32", prop_kernel=prop, leaf_grid=grid, levels=lv,
                   leaf_size=size)
    o = oracle.ifgf(p, a[0], k, leaf_grid=grid, levels=lv, leaf_size=size)
    assert_close(g[0], o, 2e-5, f"fp32 {case} {prop}")


@pytest.mark.parametrize("ps,pa", [(2, 3), (5, 7)])
def test_other_orders_match_oracle(ps, pa):
    n = 3000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 1, 34)
    say("fp64 order", ps, pa)
    g, _ = run_gpu(p, a, k, p_s=ps, p_ang=pa, leaf_grid=(1, 2, 4))
    o = oracle.ifgf(p, a[0], k, p_s=ps, p_ang=pa, leaf_grid=(1, 2, 4))
    assert_close(g[0], o, 1e-10, f"fp64 order {ps},{pa}")


@pytest.mark.parametrize("prop", ["auto", "grouped", "small", "medium", "lean", "node"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_multi_rhs_equals_single_rhs(precision, prop):
    n = 6000
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    a = W.densities(n, 4, 35)
    say("multi-rhs", precision, prop)
    g4, _ = run_gpu(p, a, k, precision=precision, prop_kernel=prop)
    tol = 1e-13 if precision == "fp64" else 1e-6 if precision == "fp32" else 1e-5
    for r in range(4):
        g1, _ = run_gpu(p, a[r:r + 1], k, precision=precision, prop_kernel=prop)
        assert_close(g4[r], g1[0], tol, f"rhs {r} of 4 vs alone")
    o = oracle.ifgf(p, a[2], k, leaf_grid=(2, 4, 8))
    assert_close(g4[2], o, 1e-10 if precision == "fp64" else 2e-5, "rhs 2 vs oracle")


def test_batched_equals_separate_plans():
    import torch
    import paper_2112_15198_amd as ifgf
    pts = [W.fibonacci_sphere(3000), W.spheroid(5200), W.fibonacci_sphere(900)]
    kap = [W.kappa_sphere_10ppw(3000), W.kappa_oblate_10ppw(5200), 9.0]
    dens = [W.densities(len(q), 2, 40 + i) for i, q in enumerate(pts)]
    say("batched 3 instances")
    pl = ifgf.plan_batched(pts, kap, n_rhs=2)
    a = torch.from_numpy(np.concatenate(dens, axis=1)).cuda()
    out = pl.apply(a).cpu().numpy()
    pl.check()
    off = np.cumsum([0] + [len(q) for q in pts])
    for i in range(3):
        sep, _ = run_gpu(pts[i], dens[i], kap[i])
        assert_close(out[:, off[i]:off[i + 1]], sep, 1e-13, f"instance {i} vs own plan")
        o = oracle.ifgf(pts[i], dens[i][1], kap[i], leaf_grid=(2, 4, 8))
        assert_close(out[1, off[i]:off[i + 1]], o, 1e-10, f"instance {i} vs oracle")


def test_two_points_and_tiny():
    p = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.0]])
    a = np.array([[1.0 + 2.0j, -0.5 + 0.25j]])
    say("two points")
    g, _ = run_gpu(p, a, 2.0)
    # A single cousin interaction at the closest cousin distance is the
    # interpolation's worst case: compare with the oracle IFGF, and with the
    # direct sum at a looser bound.
    o = oracle.ifgf(p, a[0], 2.0, leaf_grid=(2, 4, 8))
    assert relerr(g[0], o) <= 1e-10
    ref = oracle.direct_sum(p, a[0], 2.0)
    assert relerr(g[0], ref) <= 1e-3
    # Near field only reproduces the pair exactly.
    g, _ = run_gpu(p, a, 2.0, stages=1)
    nf = oracle.ifgf(p, a[0], 2.0, far=False)
    np.testing.assert_allclose(g[0], nf, rtol=1e-14, atol=0)


def test_linearity_fp64():
    n = 4000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a, b = W.densities(n, 2, 36)
    al, be = 0.7 - 1.2j, 2.0 + 0.1j
    say("linearity")
    g, _ = run_gpu(p, np.stack([a, b, al * a + be * b]), k)
    assert_close(g[2], al * g[0] + be * g[1], 1e-13, "linearity")


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.fail(f"missing fixture {path}: run tests/golden/make_golden.py")
    return np.load(path, allow_pickle=False)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 2e-5)])
def test_sphere_321k_vs_oracle_fixture(precision, tol):
    """sphere_321k (N = 321,536, kappa = 32 pi, D = 8) at full size against
    the oracle's plain FP64 IFGF at its 4,096 sampled targets (a stored
    fixture written by tests/golden/make_golden.py), element by element,
    with the autotuned kernels that bench.py times; and against the FP64
    direct sum at the same targets."""
    w = W.make("sphere_321k")
    fx = _golden("ifgf_sphere_321k")
    np.testing.assert_array_equal(fx["targets"], w.targets)
    say("sphere_321k vs oracle fixture", precision)
    g, info = run_gpu(w.points, w.dens, w.kappa, precision=precision, autotune=True)
    assert info["D"] == 8
    assert_close(g[0][w.targets], fx["values"][0], tol, f"sphere_321k {precision}")
    ref = oracle.direct_sum(w.points, w.dens[0], w.kappa, w.targets)
    err = relerr(g[0][w.targets], ref)
    print(f"sphere_321k {precision} rel-err vs direct sum {err:.3e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("geom", ["sphere", "oblate"])
def test_relevant_cones_match_oracle_exactly(geom):
    """Index work, bit-exact: with no boundary margin the GPU's relevant
    cone segments (eq. relevantconesegments, point-based) are exactly the
    oracle's, key by key, at every level; with the default margin they are
    a superset."""
    import paper_2112_15198_amd as ifgf
    if geom == "sphere":
        p, k = W.fibonacci_sphere(5024), 4 * math.pi
    else:
        p, k = W.spheroid(9000), W.kappa_oblate_10ppw(9000)
    say("cone keys", geom)
    exact = ifgf.plan(p, k, cone_margin=0.0)
    loose = ifgf.plan(p, k)
    D = exact.info()["D"]
    for l in range(D - 2):
        ok = oracle.cone_keys(p, k, D - l, leaf_grid=(2, 4, 8))
        ge = exact.cone_keys(l)
        np.testing.assert_array_equal(ge, ok)
        gl = loose.cone_keys(l)
        assert np.isin(ok, gl).all()
    exact.close()
    loose.close()


@pytest.mark.parametrize("prop,lookup", [("node", "auto"), ("grouped", "auto"),
                                         ("grouped", "hash"), ("node", "hash"),
                                         ("small", "auto"), ("small", "hash"),
                                         ("medium", "auto"), ("lean", "auto")])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 2e-5)])
def test_kernel_variants_match_oracle(prop, lookup, precision, tol):
    """Per-node, matrix-core block and wave-task (one and four waves)
    propagation, dense and hashed cone look-up: all agree with the oracle
    IFGF (FP64: 1e-10; FP32-mixed: 2e-5, its rounding, measured 3e-7;
    FP32 with the three-term BF16 product: 2e-5, about 2^-16 per product
    through the levels, measured 3e-6)."""
    n = 7000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 1, 37)
    say("variant", prop, lookup, precision)
    g, _ = run_gpu(p, a, k, precision=precision, prop_kernel=prop, lookup=lookup)
    o = oracle.ifgf(p, a[0], k, leaf_grid=(2, 4, 8))
    assert_close(g[0], o, tol, f"{prop} {lookup} {precision}")


@pytest.mark.parametrize("n_rhs", [1, 4])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_kernels_match_oracle_at_60k(n_rhs, precision, tol):
    """At N = 60,000 parent cone indices are shared by tens to hundreds of
    boxes, so the task kernels' octants span several N-tiles split over
    their waves.  Every propagation kernel matches the oracle's plain IFGF
    (a stored fixture of 8,192 sampled targets per RHS, written by
    tests/golden/make_golden.py) element by element."""
    n = 60000
    fx = _golden("ifgf_sphere_60k")
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 4, 38)[:n_rhs]
    tg = fx["targets"]
    for prop, mode in (("node", 1), ("small", 3), ("medium", 4), ("lean", 5), ("auto", None)):
        say("60k vs oracle fixture", precision, prop, "rhs", n_rhs)
        g, info = run_gpu(p, a, k, precision=precision, prop_kernel=prop)
        if mode is not None:
            assert mode in info["prop_mode"], (prop, info["prop_mode"])
        for r in range(n_rhs):
            assert_close(g[r][tg], fx["values"][r], tol, f"60k {prop} {precision} rhs {r}")


@pytest.mark.parametrize("n_rhs", [1, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_prop_tables_give_identical_results(precision, n_rhs):
    """The wave-task propagation kernels read the box-independent octant
    records (node geometry and grouping by child cone) from the plan-time
    table or compute them per chunk; the records are made by the same device
    code, so both paths give bit-identical outputs.  N = 60,000 sphere, both
    task kernels forced on every level, 1 and 4 RHS; the tabled apply also
    matches the oracle fixture."""
    n = 60000
    fx = _golden("ifgf_sphere_60k")
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 4, 38)[:n_rhs]
    for prop in ("small", "medium", "lean"):
        say("prop tables", precision, prop, "rhs", n_rhs)
        g0, i0 = run_gpu(p, a, k, precision=precision, prop_kernel=prop, prop_tables="never")
        g1, i1 = run_gpu(p, a, k, precision=precision, prop_kernel=prop, prop_tables="always")
        assert i0["prop_table_bytes"] == 0 and i1["prop_table_bytes"] > 0
        assert np.array_equal(g0, g1), (prop, float(np.max(np.abs(g0 - g1))))
        tol = 1e-10 if precision == "fp64" else 2e-5
        for r in range(n_rhs):
            assert_close(g1[r][fx["targets"]], fx["values"][r], tol,
                         f"60k tables {prop} {precision} rhs {r}")


@pytest.mark.parametrize("prop", ["grouped", "small", "medium", "lean"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16x3", 1e-6)])
def test_graph_replays_match_eager(precision, tol, prop):
    """The HIP-graph apply, replayed several times with eager work and
    synchronisations in between, matches the eager apply every time."""
    import torch
    import paper_2112_15198_amd as ifgf
    n = 9000
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    say("graph replay", precision, prop)
    pl = ifgf.plan(p, k, precision=precision, n_rhs=2, prop_kernel=prop)
    a = torch.from_numpy(W.densities(n, 2, 51)).to(dt).cuda()
    b = torch.from_numpy(W.densities(n, 2, 52)).to(dt).cuda()
    ref_a = pl.apply(a).cpu().numpy()
    ref_b = pl.apply(b).cpu().numpy()
    out = torch.empty_like(a)
    for rep in range(3):
        pl.apply(a, out=out, graph=True)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert_close(got, ref_a, tol, f"replay {rep}")
        eager_b = pl.apply(b).cpu().numpy()      # eager work between replays
        assert_close(eager_b, ref_b, tol, "eager between replays")
        torch.cuda.synchronize()
    pl.check()
    o = oracle.ifgf(p, W.densities(n, 2, 51)[1], k, leaf_grid=(2, 4, 8))
    assert_close(got[1], o, 1e-10 if precision == "fp64" else 2e-5, "replay vs oracle")
    pl.close()


def test_autotune_picks_a_kernel_per_level_and_stays_exact():
    import paper_2112_15198_amd as ifgf
    n = 20000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 1, 53)
    say("autotune")
    g, info = run_gpu(p, a, k, autotune=True)
    tuned = [l for l in range(1, info["n_steps"]) if info["autotune_ms"][l][0] > 0]
    assert tuned, info["autotune_ms"]
    for l in tuned:
        t = info["autotune_ms"][l]
        assert all(x > 0 for x in t), t
        assert info["prop_mode"][l] == 1 + min(range(len(t)), key=lambda g: t[g])
    o = oracle.ifgf(p, a[0], k, leaf_grid=(2, 4, 8))
    assert_close(g[0], o, 1e-10, "autotuned")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
@pytest.mark.parametrize("geom", ["sphere", "oblate"])
def test_laplace_matches_oracle(geom, precision, tol):
    """The Laplace kernel (kappa = 0) through the same factorisation, with
    the wavelength-free level rule (absolute leaf side) and the leaf cone
    grid kept at every level: GPU vs the oracle IFGF element by element,
    and vs the direct sum at the method's 1e-4."""
    n = 6000
    p = W.fibonacci_sphere(n) if geom == "sphere" else W.spheroid(n)
    a = W.densities(n, 1, 61)
    say("laplace", geom, precision)
    g, info = run_gpu(p, a, 0.0, precision=precision, leaf_abs=0.125)
    assert not info["grid_doubling"] and len(set(info["grid"])) == 1
    o, oi = oracle.ifgf(p, a[0], 0.0, leaf_grid=(2, 4, 8), leaf_abs=0.125, return_info=True)
    assert info["D"] == oi["D"]
    assert_close(g[0], o, tol, f"laplace {geom} {precision}")
    ref = oracle.direct_sum(p, a[0], 0.0)
    assert relerr(g[0], ref) <= 1e-4


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_leaf_max_matches_oracle(precision, tol):
    """The per-instance leaf-side cap: the batch's N = 4,373 spheroid (leaves
    of 0.31 wavelengths by the rounding rule) planned with a 0.3-wavelength
    cap has one more level, matches the oracle with the same cap, and meets
    1e-4 against the direct sum."""
    n = 4373
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    a = W.densities(n, 1, 62)
    say("leaf_max", precision)
    g, info = run_gpu(p, a, k, precision=precision, leaf_max=0.3)
    o, oi = oracle.ifgf(p, a[0], k, leaf_grid=(2, 4, 8), leaf_max=0.3, return_info=True)
    assert info["D"] == oi["D"] == 6
    assert_close(g[0], o, tol, f"leaf_max {precision}")
    assert relerr(g[0], oracle.direct_sum(p, a[0], k)) <= 1e-4


def test_tuning_cache_reuses_choices(tmp_path):
    """A second autotuned plan of the same shape reads the kernels from the
    cache file instead of timing them, and gives the same result."""
    n = 20000
    p = W.fibonacci_sphere(n)
    k = W.kappa_sphere_10ppw(n)
    a = W.densities(n, 1, 63)
    cache = str(tmp_path / "tune.txt")
    say("tuning cache")
    g1, i1 = run_gpu(p, a, k, precision="fp32", autotune=True, tune_cache=cache)
    g2, i2 = run_gpu(p, a, k, precision="fp32", autotune=True, tune_cache=cache)
    assert not i1["tune_cache_hit"] and i2["tune_cache_hit"]
    assert i1["prop_mode"] == i2["prop_mode"]
    assert all(all(x == 0 for x in t) for t in i2["autotune_ms"])
    np.testing.assert_array_equal(g1, g2)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and "| modes=" in lines[0]
    # Another precision is another key: timed again, a second line.
    run_gpu(p, a, k, precision="fp64", autotune=True, tune_cache=cache)
    assert len(open(cache).read().splitlines()) == 2


def test_device_points_equal_host_points():
    """Points given as a CUDA tensor plan the same octree as host points."""
    import torch
    n = 5000
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    a = W.densities(n, 1, 64)
    say("device points")
    g1, i1 = run_gpu(p, a, k)
    g2, i2 = run_gpu(torch.from_numpy(p).cuda(), a, k)
    assert i1["cones"] == i2["cones"]
    np.testing.assert_array_equal(g1, g2)
