"""Benchmark of the IFGF Helmholtz matvec on one MI355X.

A step is one complete ifgf_apply (permute in, near field, leaf
evaluations, interpolation and propagation at every level, permute out)
over one set of densities already resident in HBM.

Workload: N = 321,536 points on the unit sphere (Fibonacci lattice),
kappa = 32 pi, complex densities iid U(-1,1), (P_s, P_ang) = (3, 5), leaf
cone grid (2,4,8), one right-hand side.  The headline figure is the
FP32-mixed path; the plain FP64 path is timed on the same GPU beside it.

Prints one JSON line:
  value      = N^2 / t (FP32-mixed), t = mean apply time
  fp64       = the same for the FP64 path
  rel_err    = relative l2 error against the FP64 direct sum on 4,096
               sampled targets (eq. errorcomputation of the paper)
  roofline   = the dominant kernel (propagation): algorithmic FLOP per
               launch over its mean HIP-event launch time, against the
               MI355X vector peak of its precision
  cpu_baseline = the CPU oracle (FP64 direct sum, OpenMP) on the sampled
               targets, scaled to N^2/s
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "IFGF matvec ms & N^2/t at rel-err<=1e-4 vs FP64 direct: FP32-mixed vs FP64"

# MI355X published peaks (dense): vector FP32 157.3 TFLOP/s, FP64 78.6.
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}


def flops_per_eval(P):
    """Algorithmic FLOP of one interpolant evaluation times one complex
    factor, per right-hand side: P complex-by-real multiply-adds of the
    tensor contraction (4 FLOP each) plus one complex multiply-add (8)."""
    return 4 * P + 8


def time_applies(pl, a, steps, warmup, profile):
    import torch
    for _ in range(warmup):
        pl.apply(a)
    pl.check()
    pl.profile_read(reset=True)
    if profile:
        pl.profile(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    out = None
    for _ in range(steps):
        out = pl.apply(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    stages = pl.profile_read(reset=True) if profile else {}
    pl.profile(False)
    pl.check()
    return ms, out, stages


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere_321k")
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle (baseline and error check)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is not part of this build)", flush=True)
        sys.exit(2)

    import torch
    import paper_2112_15198_amd as ifgf
    from paper_2112_15198_amd import workloads as W

    w = W.make(args.workload)
    n = w.points.shape[0]
    n_rhs = w.dens.shape[0]
    p_s, p_ang, grid = 3, 5, (2, 4, 8)
    P = p_s * p_ang * p_ang
    precs = ["fp32", "fp64"] if args.precision == "both" else [args.precision]
    res = {}
    for prec in precs:
        t0 = time.perf_counter()
        pl = ifgf.plan(w.points, w.kappa, p_s=p_s, p_ang=p_ang, precision=prec,
                       n_rhs=n_rhs, leaf_grid=grid)
        plan_s = time.perf_counter() - t0
        dt = torch.complex64 if prec == "fp32" else torch.complex128
        a = torch.from_numpy(w.dens).to(dt).cuda()
        ms, out, stages = time_applies(pl, a, args.steps, args.warmup, profile=True)
        info = pl.info()
        res[prec] = {"ms": ms, "out": out.cpu().numpy().astype(np.complex128),
                     "stages": stages, "info": info, "plan_s": plan_s}
        print(f"# {prec}: {ms:.3f} ms/apply, plan {plan_s:.2f} s, "
              + ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms x{v[1] // args.steps}"
                          for k, v in stages.items()), file=sys.stderr, flush=True)
        pl.close()
        del a, out
        torch.cuda.empty_cache()

    head = "fp32" if "fp32" in res else "fp64"
    R = res[head]
    ms = R["ms"]
    value = n * n / (ms * 1e-3)

    # Dominant kernel: the stage with the largest summed time.
    st = R["stages"]
    dom = max(st, key=lambda k: st[k][0])
    info = R["info"]
    launches = st[dom][1] / args.steps
    avg_ms = st[dom][0] / st[dom][1]
    if dom == "propagation":
        units = sum(info["prop_pairs"])
        flop = units * n_rhs * flops_per_eval(P)
        unit_txt = "(parent-cone node, relevant child) evaluations"
    elif dom == "interpolation":
        units = sum(info["cousin_pairs"])
        flop = units * n_rhs * flops_per_eval(P)
        unit_txt = "(target, cousin box) evaluations"
    elif dom == "leaf":
        units = info["leaf_pairs"]
        flop = units * n_rhs * 30
        unit_txt = "(leaf-cone node, source) evaluations"
    else:
        units = info["near_pairs"]
        flop = units * n_rhs * 30
        unit_txt = "near-field pairs"
    per_launch = flop / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[head]
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": dom, "launches_per_step": launches,
                "avg_launch_ms": round(avg_ms, 4),
                "flop_per_launch": per_launch,
                "units_per_step": units,
                "flop_per_unit_per_rhs": flops_per_eval(P) if dom in ("propagation", "interpolation") else 30,
                "unit_desc": unit_txt}

    line = {"metric": METRIC, "value": value, "unit": "N^2/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32-mixed" if head == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": args.workload, "N": n, "kappa": w.kappa,
                       "geometry": "unit-sphere Fibonacci lattice",
                       "p_s": p_s, "p_ang": p_ang, "leaf_grid": list(grid),
                       "n_rhs": n_rhs, "D": info["D"],
                       "precision": "fp32-mixed" if head == "fp32" else "fp64"},
            "plan_s": R["plan_s"],
            "stages_ms": {k: round(v[0] / args.steps, 4) for k, v in st.items()},
            "roofline": roofline}
    if "fp64" in res and head != "fp64":
        line["fp64"] = {"ms_per_step": res["fp64"]["ms"],
                        "value": n * n / (res["fp64"]["ms"] * 1e-3),
                        "stages_ms": {k: round(v[0] / args.steps, 4)
                                      for k, v in res["fp64"]["stages"].items()}}
        line["speedup_fp32_mixed_over_fp64"] = res["fp64"]["ms"] / ms

    if not args.no_cpu:
        # CPU baseline leg: the oracle's FP64 direct sum at the sampled
        # targets, which is also the reference for the error estimate.
        import oracle
        tg = w.targets
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        t0 = time.perf_counter()
        ref = oracle.direct_sum(w.points, w.dens[0], w.kappa, tg)
        t_cpu = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": n * len(tg) / t_cpu, "unit": "N^2/s", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 direct sum (eq. field1) at {len(tg)} seeded targets x all "
                      f"{n} sources; full-matvec time extrapolated as t*N/{len(tg)}",
            "seconds": t_cpu}
        for prec in res:
            e = float(np.linalg.norm(res[prec]["out"][0][tg] - ref) / np.linalg.norm(ref))
            if prec == head:
                line["rel_err"] = e
            else:
                line["fp64"]["rel_err"] = e
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
