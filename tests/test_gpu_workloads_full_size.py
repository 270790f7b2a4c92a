"""Parity at the workloads' full sizes, in the configuration bench.py times
(autotuned plan, captured HIP-graph apply, FP32-mixed), on sampled targets
against the oracle's FP64 direct sum (eq. field1; relative l2 error, eq.
errorcomputation).  Collected after the smaller parity tests."""
import sys

import numpy as np
import pytest

import oracle
from paper_2112_15198_amd import workloads as W
from parity import assert_close, relerr

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def graph_apply(pl, dens, precision, graph=True):
    """Two applies into one output (graph replays when graph=True)."""
    import torch
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    a = torch.from_numpy(np.ascontiguousarray(dens)).to(dt).cuda()
    out = torch.empty_like(a)
    for _ in range(2):
        pl.apply(a, out=out, graph=graph)
    torch.cuda.synchronize()
    pl.check()
    return out.cpu().numpy().astype(np.complex128)




@pytest.mark.parametrize("name,precision", [("oblate_1m", "fp32"), ("sphere_5m", "fp32"),
                                            ("sphere_321k", "bf16x3"),
                                            ("oblate_1m", "bf16x3")])
def test_full_size_vs_direct_sum(name, precision):
    """oblate_1m (N = 1,048,576, kappa 64 pi, 4 RHS), sphere_5m
    (N = 5,144,576, kappa 128 pi) and sphere_321k (N = 321,536, kappa 32 pi),
    FP32-mixed and with the three-term BF16 propagation product: every RHS
    within 1e-4 of the FP64 direct sum on 512 of the workload's 4,096
    sampled targets."""
    import paper_2112_15198_amd as ifgf
    w = W.make(name)
    n_rhs = w.dens.shape[0]
    tg = w.targets[::8]
    say("full size", name, precision, "N", w.points.shape[0], "rhs", n_rhs)
    pl = ifgf.plan(w.points, w.kappa, precision=precision, n_rhs=n_rhs,
                   leaf_grid=(2, 4, 8), autotune=True)
    out = graph_apply(pl, w.dens, precision)
    pl.close()
    for r in range(n_rhs):
        ref = oracle.direct_sum(w.points, w.dens[r], w.kappa, tg)
        e = relerr(out[r][tg], ref)
        say(name, precision, "rhs", r, "rel-err", f"{e:.3e}")
        assert e <= 1e-4, (name, r, e)


def test_batch48_fp32_vs_direct_sum():
    """batch48 (48 instances, N from 4k to 200k, 4 RHS), planned as bench.py
    plans it (workloads.plan_options: leaf cone grid (3, 4, 8)).  FP32-mixed
    agrees with an FP64 apply of the same batch to 2e-5 per instance and
    RHS, element by element (its rounding), and with the FP64 direct sum to
    relative l2 <= 1e-4 on every instance and RHS (eq. errorcomputation) over
    the workload's error set: each instance's 4,096 sampled targets, or all
    of its points when it has fewer."""
    import paper_2112_15198_amd as ifgf
    insts = W.make("batch48")
    pts = [x.points for x in insts]
    kap = [x.kappa for x in insts]
    dens = np.concatenate([x.dens for x in insts], axis=1)
    popts = W.plan_options("batch48")
    say("batch48 fp32", len(insts), "instances", dens.shape[1], "points", popts)
    pl = ifgf.plan_batched(pts, kap, precision="fp32", n_rhs=4, autotune=True, **popts)
    out32 = graph_apply(pl, dens, "fp32")
    pl.close()
    say("batch48 fp64")
    pl = ifgf.plan_batched(pts, kap, precision="fp64", n_rhs=4, **popts)
    out64 = graph_apply(pl, dens, "fp64", graph=False)
    pl.close()
    off, worst = 0, 0.0
    for i, x in enumerate(insts):
        ni = x.points.shape[0]
        tg = x.targets
        for r in range(4):
            g32 = out32[r, off:off + ni][tg]
            g64 = out64[r, off:off + ni][tg]
            assert_close(g32, g64, 2e-5, f"batch48 instance {i} rhs {r} fp32 vs fp64")
            e = relerr(g32, oracle.direct_sum(x.points, x.dens[r], x.kappa, tg))
            worst = max(worst, e)
            assert e <= 1e-4, (i, r, e)
        off += ni
    say("batch48 worst rel-err", f"{worst:.3e}")
