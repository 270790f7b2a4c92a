"""Benchmark of the IFGF Helmholtz matvec on one MI355X.

A step is one complete apply (permute in, near field, leaf evaluations,
interpolation and propagation at every level, permute out) over one set of
densities already resident in HBM, replayed as one captured HIP graph; the
eager (launch-by-launch) time is reported beside it.  The plan is built
with the autotuner on (per-level choice of propagation kernel).

Workload: N = 321,536 points on the unit sphere (Fibonacci lattice),
kappa = 32 pi, complex densities iid U(-1,1), (P_s, P_ang) = (3, 5), leaf
cone grid (2,4,8), one right-hand side.  The headline figure is the
FP32-mixed path; the plain FP64 path is timed on the same GPU beside it.

Prints one JSON line:
  value      = N^2 * n_rhs / t (FP32-mixed), t = mean apply time (sum of
               N_i^2 over the instances of a batched workload)
  fp64       = the same for the FP64 path
  bf16x3     = the same for FP32-mixed with the propagation product on BF16
               matrix cores in three-term split form (not the headline)
  rel_err    = relative l2 error against the FP64 direct sum on 4,096
               sampled targets (eq. errorcomputation of the paper)
  roofline   = the dominant kernel: algorithmic FLOP per launch over its
               mean HIP-event launch time (eager applies), against the
               MI355X peak of its precision (matrix cores for the
               matrix-core propagation, vector ALUs otherwise)
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

# MI355X published dense peaks: FP32 157.3 TFLOP/s, FP64 78.6 (vector and
# matrix cores alike); BF16 matrix cores 2,500, of which a three-term split
# product uses three per FP32-equivalent product.
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 157.3}
PEAK_BF16X3_PRODUCT = 2500.0 / 3


def flops_per_eval(P):
    """Algorithmic FLOP of one interpolant evaluation times one complex
    factor, per right-hand side: P complex-by-real multiply-adds of the
    tensor contraction (4 FLOP each) plus one complex multiply-add (8)."""
    return 4 * P + 8


def measured_traffic(stage, workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE record (copy-calibrated), or None when
    there is no record for it or the kernel source changed since."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2112_15198_amd", "csrc", "ifgf_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for f in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        rec = json.load(open(f))
        if (rec.get("stage") == stage and rec.get("workload") == workload
                and rec.get("precision") == precision
                and rec.get("kernel_source_sha256") == sha):
            return rec["traffic_bytes_per_launch"]
    return None


def time_applies(pl, a, steps, warmup, graph):
    """Mean ms per apply over `steps` applies (after `warmup`), bracketed by
    torch.cuda.synchronize; graph=True replays the captured apply."""
    import torch
    out = torch.empty_like(a)
    for _ in range(warmup):
        pl.apply(a, out=out, graph=graph)
    pl.check()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pl.apply(a, out=out, graph=graph)
    e1.record()
    torch.cuda.synchronize()
    pl.check()
    return e0.elapsed_time(e1) / steps, out


def stage_times(pl, a, steps):
    """Per-stage kernel times (HIP events around every launch), eager applies."""
    import torch
    out = torch.empty_like(a)
    pl.profile_read(reset=True)
    pl.profile(True)
    for _ in range(steps):
        pl.apply(a, out=out)
    st = pl.profile_read(reset=True)
    pl.profile(False)
    return st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere_321k")
    ap.add_argument("--precision", choices=["all", "both", "fp32", "fp64", "bf16x3"],
                    default="all",
                    help="all: FP32-mixed (headline), FP64 and FP32 with the three-term BF16 "
                         "propagation product; both: the first two")
    ap.add_argument("--samples-batch", type=int, default=256,
                    help="error-check targets per instance of a batched workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device-to-device copy three times "
                         "(known bytes, for calibrating rocprofv3 FETCH/WRITE_SIZE)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle (baseline and error check)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported",
              flush=True)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        nel = 64 * 1024 * 1024
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nel * 4, "copies": 3}), flush=True)
        return
    import paper_2112_15198_amd as ifgf
    from paper_2112_15198_amd import workloads as W

    w = W.make(args.workload)
    batch = isinstance(w, list)
    insts = w if batch else [w]
    n = sum(x.points.shape[0] for x in insts)
    n2 = float(sum(float(x.points.shape[0]) ** 2 for x in insts))
    n_rhs = insts[0].dens.shape[0]
    dens = np.concatenate([x.dens for x in insts], axis=1)
    p_s, p_ang, grid = 3, 5, (2, 4, 8)
    P = p_s * p_ang * p_ang
    precs = {"all": ["fp32", "fp64", "bf16x3"], "both": ["fp32", "fp64"]}.get(
        args.precision, [args.precision])
    res = {}
    for prec in precs:
        t0 = time.perf_counter()
        if batch:
            pl = ifgf.plan_batched([x.points for x in insts], [x.kappa for x in insts],
                                   p_s=p_s, p_ang=p_ang, precision=prec, n_rhs=n_rhs,
                                   leaf_grid=grid, autotune=True)
        else:
            pl = ifgf.plan(w.points, w.kappa, p_s=p_s, p_ang=p_ang, precision=prec,
                           n_rhs=n_rhs, leaf_grid=grid, autotune=True)
        plan_s = time.perf_counter() - t0
        print(f"# {prec}: plan {plan_s:.2f} s (N={n}, D={pl.info()['D']})",
              file=sys.stderr, flush=True)
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        a = torch.from_numpy(dens).to(dt).cuda()
        ms_eager, _ = time_applies(pl, a, args.steps, args.warmup, graph=False)
        print(f"# {prec}: eager {ms_eager:.3f} ms/apply", file=sys.stderr, flush=True)
        stages = stage_times(pl, a, args.steps)
        ms, out = time_applies(pl, a, args.steps, args.warmup, graph=True)
        info = pl.info()
        res[prec] = {"ms": ms, "ms_eager": ms_eager,
                     "out": out.cpu().numpy().astype(np.complex128),
                     "stages": stages, "info": info, "plan_s": plan_s}
        print(f"# {prec}: {ms:.3f} ms/apply (graph), {ms_eager:.3f} eager, plan {plan_s:.2f} s, "
              + ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms x{v[1] // args.steps}"
                          for k, v in stages.items())
              + f"; prop kernels {info['prop_mode']}", file=sys.stderr, flush=True)
        pl.close()
        del a, out
        torch.cuda.empty_cache()

    head = next(p for p in ("fp32", "bf16x3", "fp64") if p in res)
    R = res[head]
    ms = R["ms"]
    # Matvec-equivalents: one apply evaluates n_rhs operators.
    value = n2 * n_rhs / (ms * 1e-3)

    # Dominant kernel: the stage with the largest summed time.
    st = R["stages"]
    dom = max(st, key=lambda k: st[k][0])
    info = R["info"]
    launches = st[dom][1] / args.steps
    avg_ms = st[dom][0] / st[dom][1]
    bound = "alu"
    if dom in ("propagation", "propagation_mfma", "propagation_small"):
        modes = {"propagation": (1,), "propagation_mfma": (2,), "propagation_small": (3, 4)}[dom]
        mode = modes[0]
        units = sum(pp for pp, md in zip(info["prop_pairs"], info["prop_mode"]) if md in modes)
        flop = units * n_rhs * flops_per_eval(P)
        unit_txt = "(parent-cone node, relevant child) evaluations"
        bound = "mfma" if mode >= 2 else "alu"
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
    peak = PEAK_BF16X3_PRODUCT if (head == "bf16x3" and dom == "propagation_small") \
        else PEAK_TFLOPS[head]
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(dom, args.workload, head),
                "kernel": dom, "launches_per_step": launches,
                "avg_launch_ms": round(avg_ms, 4),
                "flop_per_launch": per_launch,
                "units_per_step": units,
                "flop_per_unit_per_rhs": flops_per_eval(P) if dom.startswith("prop") or dom == "interpolation" else 30,
                "unit_desc": unit_txt}

    if batch:
        cfg = {"workload": args.workload, "instances": len(insts), "N_total": n,
               "sum_N2": n2, "N_min": min(x.points.shape[0] for x in insts),
               "N_max": max(x.points.shape[0] for x in insts),
               "geometry": "spheres and (1,1,0.25) spheroids, Fibonacci lattices, ~10 ppw"}
    else:
        cfg = {"workload": args.workload, "N": n, "kappa": w.kappa,
               "geometry": ("unit-sphere" if "sphere" in args.workload else
                            "(1,1,0.25) spheroid") + " Fibonacci lattice"}
    cfg.update({"p_s": p_s, "p_ang": p_ang, "leaf_grid": list(grid), "n_rhs": n_rhs,
                "D": info["D"], "precision": {"fp32": "fp32-mixed", "fp64": "fp64",
                                              "bf16x3": "fp32-mixed, bf16x3 propagation"}[head],
                "apply": "captured HIP graph"})
    line = {"metric": METRIC, "value": value, "unit": "N^2/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": {"fp32": "f32-mixed", "fp64": "f64", "bf16x3": "f32-mixed+bf16x3"}[head],
            "data": "synthetic",
            "config": cfg,
            "plan_s": R["plan_s"], "ms_per_step_eager": R["ms_eager"],
            "prop_kernel_per_level": info["prop_mode"],
            "stages_ms": {k: round(v[0] / args.steps, 4) for k, v in st.items()},
            "roofline": roofline}
    for other in ("fp64", "bf16x3"):
        if other in res and head != other:
            line[other] = {"ms_per_step": res[other]["ms"],
                           "ms_per_step_eager": res[other]["ms_eager"],
                           "value": n2 * n_rhs / (res[other]["ms"] * 1e-3),
                           "prop_kernel_per_level": res[other]["info"]["prop_mode"],
                           "stages_ms": {k: round(v[0] / args.steps, 4)
                                         for k, v in res[other]["stages"].items()}}
    if "fp64" in res and head != "fp64":
        line["speedup_fp32_mixed_over_fp64"] = res["fp64"]["ms"] / ms

    if not args.no_cpu:
        # CPU baseline leg: the oracle's FP64 direct sum at the sampled
        # targets, which is also the reference for the error estimate
        # (relative l2, eq. errorcomputation; max over RHS and instances).
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        per_inst = args.samples_batch if batch else None
        t_cpu, pairs = 0.0, 0
        errs = {prec: 0.0 for prec in res}
        off = 0
        for x in insts:
            ni = x.points.shape[0]
            tg = x.targets if per_inst is None else x.targets[:per_inst]
            for r in range(n_rhs):
                t0 = time.perf_counter()
                ref = oracle.direct_sum(x.points, x.dens[r], x.kappa, tg)
                t_cpu += time.perf_counter() - t0
                pairs += ni * len(tg)
                for prec in res:
                    g = res[prec]["out"][r, off:off + ni][tg]
                    e = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
                    errs[prec] = max(errs[prec], e)
            off += ni
        line["cpu_baseline"] = {
            "value": pairs / t_cpu, "unit": "N^2/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 direct sum (eq. field1) at the sampled targets x all sources "
                       f"({pairs} pairs, {len(insts)} instance(s), {n_rhs} RHS); "
                       f"full-matvec time extrapolated pro rata"),
            "seconds": t_cpu}
        line["rel_err"] = errs[head]
        for other in ("fp64", "bf16x3"):
            if other in line:
                line[other]["rel_err"] = errs[other]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
