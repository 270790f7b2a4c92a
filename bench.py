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
               matrix-core propagation, vector ALUs otherwise).  FLOP per
               unit and RHS: 380 per (parent-cone node, relevant child) of
               the propagation (a 75-term complex-by-real tensor contraction
               in sum-factorised form, 186 FMA, plus the Lagrange basis and
               the complex ratio), 490 per (target, cousin box) of the
               interpolation, 25 per (leaf-cone node, source) and 20 per
               near-field pair (transcendentals not counted)
  cpu_baseline = the CPU oracle (FP64 direct sum, OpenMP) on the sampled
               targets, scaled to N^2/s
  cpu_baseline_ifgf = the CPU oracle's plain FP64 IFGF (OpenMP) on a
               smaller sphere, with the GPU paths timed on the same sphere
  cpu        = the host the CPU legs ran on (model, logical CPUs, OpenMP
               threads used)
  configs    = compact records of the other workloads (default kernel
               choice, fewer applies): ms, N^2/t, plan time and the error
               against the FP64 direct sum on a stated sample of targets
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


# Algorithmic FLOP per unit and right-hand side, (P_s, P_ang) = (3, 5).
FLOP_PROP = 380      # (parent-cone node, relevant child)
FLOP_INTERP = 490    # (target, cousin box): contraction, FP64 r and phase
FLOP_LEAF = 25       # (leaf-cone node, source)
FLOP_NEAR = 20       # (target, source) pair


def flop_scale(P):
    """The counts above are for P = 75 nodes; other orders scale with P."""
    return P / 75.0


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


def cpu_info():
    """The host the CPU legs run on."""
    import oracle
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_allowed": affinity,
            "omp_threads": oracle.threads()}


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def time_plan(pl, a, steps, warmup):
    """Mean ms per captured-graph apply, and the output."""
    ms, out = time_applies(pl, a, steps, warmup, graph=True)
    return ms, out.cpu().numpy().astype(np.complex128)


def cpu_ifgf_leg(n, steps, warmup):
    """The oracle's plain FP64 IFGF (OpenMP, all threads) on an N-point unit
    sphere at ~10 points per wavelength, its error against the FP64 direct
    sum on every target, and the GPU FP32-mixed and FP64 applies of the same
    sphere timed beside it."""
    import torch
    import oracle
    import paper_2112_15198_amd as ifgf
    from paper_2112_15198_amd import workloads as W
    pts = W.fibonacci_sphere(n)
    kappa = W.kappa_sphere_10ppw(n)
    dens = W.densities(n, 1, 1010)
    print(f"# cpu ifgf: oracle on sphere N={n}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    o, oi = oracle.ifgf(pts, dens[0], kappa, leaf_grid=(2, 4, 8), return_info=True)
    wall = time.perf_counter() - t0
    ref = oracle.direct_sum(pts, dens[0], kappa)
    rec = {"kind": "oracle IFGF", "N": n, "kappa": kappa, "D": oi["D"],
           "precision": "fp64", "threads": oracle.threads(),
           "apply_s": oi["eval_s"], "setup_s": oi["setup_s"], "wall_s": wall,
           "value": float(n) ** 2 / oi["eval_s"], "unit": "N^2/s",
           "rel_err_vs_direct_sum": relerr(o, ref),
           "sample": "all N targets; apply = near field, leaf evaluations, interpolation "
                     "and propagation (set-up timed apart)"}
    for prec in ("fp32", "fp64"):
        pl = ifgf.plan(pts, kappa, precision=prec, leaf_grid=(2, 4, 8))
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        a = torch.from_numpy(dens).to(dt).cuda()
        ms, g = time_plan(pl, a, steps, warmup)
        pl.close()
        rec["gpu_" + prec] = {"ms": ms, "value": float(n) ** 2 / (ms * 1e-3),
                              "rel_err_vs_direct_sum": relerr(g[0], ref),
                              "rel_err_vs_oracle_ifgf": relerr(g[0], o)}
        rec["gpu_" + prec]["speedup_vs_oracle_ifgf"] = oi["eval_s"] * 1e3 / ms
    print(f"# cpu ifgf: oracle {oi['eval_s']:.2f} s apply ({wall:.1f} s with set-up); "
          f"GPU fp32 {rec['gpu_fp32']['ms']:.3f} ms, fp64 {rec['gpu_fp64']['ms']:.3f} ms",
          file=sys.stderr, flush=True)
    return rec


# The other workloads, as compact records: (record, workload, precisions,
# sampled targets per instance for the error; None = the workload's own).
CONFIG_RUNS = [
    ("sphere_5k", ["fp64", "fp32"], None),
    ("oblate_1m", ["fp32"], 1024),
    ("batch48", ["fp32"], 512),
    ("sphere_5m", ["fp32"], 1024),
]


def run_configs(steps, warmup, names=None):
    import torch
    import oracle
    import paper_2112_15198_amd as ifgf
    from paper_2112_15198_amd import workloads as W
    recs = {}
    for name, precs, nsamp in CONFIG_RUNS:
        if names and name not in names:
            continue
        w = W.make(name)
        insts = w if isinstance(w, list) else [w]
        n_rhs = insts[0].dens.shape[0]
        dens = np.concatenate([x.dens for x in insts], axis=1)
        n2 = float(sum(float(x.points.shape[0]) ** 2 for x in insts))
        popts = W.plan_options(name)
        rec = {"N_total": int(dens.shape[1]), "instances": len(insts), "n_rhs": n_rhs,
               "plan_options": {k: (list(v) if isinstance(v, tuple) else v)
                                for k, v in popts.items()},
               "kernel_choice": "default (no autotuning)"}
        outs = {}
        for prec in precs:
            print(f"# config {name} {prec}: planning", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            if len(insts) > 1:
                pl = ifgf.plan_batched([x.points for x in insts], [x.kappa for x in insts],
                                       precision=prec, n_rhs=n_rhs, **popts)
            else:
                pl = ifgf.plan(insts[0].points, insts[0].kappa, precision=prec,
                               n_rhs=n_rhs, **popts)
            plan_s = time.perf_counter() - t0
            dt = torch.complex128 if prec == "fp64" else torch.complex64
            a = torch.from_numpy(dens).to(dt).cuda()
            ms, g = time_plan(pl, a, steps, warmup)
            info = pl.info()
            pl.close()
            del a
            torch.cuda.empty_cache()
            outs[prec] = g
            rec[prec] = {"ms": ms, "value": n2 * n_rhs / (ms * 1e-3), "unit": "N^2/s",
                         "plan_s": plan_s, "D": info["D"]}
            print(f"# config {name} {prec}: {ms:.3f} ms/apply, plan {plan_s:.1f} s",
                  file=sys.stderr, flush=True)
        # Error against the FP64 direct sum (eq. errorcomputation), max over
        # instances and RHS.
        errs = {p: 0.0 for p in precs}
        off, pairs = 0, 0
        for x in insts:
            ni = x.points.shape[0]
            tg = x.targets if nsamp is None else x.targets[:nsamp]
            for r in range(n_rhs):
                ref = oracle.direct_sum(x.points, x.dens[r], x.kappa, tg)
                pairs += ni * len(tg)
                for p in precs:
                    errs[p] = max(errs[p], relerr(outs[p][r, off:off + ni][tg], ref))
            off += ni
        for p in precs:
            rec[p]["rel_err"] = errs[p]
        rec["error_sample"] = ("all targets" if nsamp is None else
                               f"the first {nsamp} of each instance's sampled targets") + \
            ", max over instances and RHS"
        recs[name] = rec
        print(f"# config {name}: rel-err " + ", ".join(f"{p} {errs[p]:.2e}" for p in precs),
              file=sys.stderr, flush=True)
    return recs


def arg_parser():
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
    ap.add_argument("--cpu-ifgf-n", type=int, default=40000,
                    help="sphere size of the CPU oracle IFGF leg (0: skip)")
    ap.add_argument("--configs", default="all",
                    help="compact records of the other workloads: all, none, or a "
                         "comma-separated list of workload names")
    ap.add_argument("--config-steps", type=int, default=5)
    ap.add_argument("--tune-cache", default=None,
                    help="file that keeps the autotuner's per-level choices, so that "
                         "profiled runs of one workload plan the same kernels")
    return ap


def main():
    args = arg_parser().parse_args()
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
    p_s, p_ang = 3, 5
    popts = W.plan_options(args.workload)
    grid = popts["leaf_grid"]
    P = p_s * p_ang * p_ang
    precs = {"all": ["fp32", "fp64", "bf16x3"], "both": ["fp32", "fp64"]}.get(
        args.precision, [args.precision])
    res = {}
    for prec in precs:
        t0 = time.perf_counter()
        if batch:
            pl = ifgf.plan_batched([x.points for x in insts], [x.kappa for x in insts],
                                   p_s=p_s, p_ang=p_ang, precision=prec, n_rhs=n_rhs,
                                   autotune=True, tune_cache=args.tune_cache, **popts)
        else:
            pl = ifgf.plan(w.points, w.kappa, p_s=p_s, p_ang=p_ang, precision=prec,
                           n_rhs=n_rhs, autotune=True, tune_cache=args.tune_cache, **popts)
        plan_s = time.perf_counter() - t0
        pi = pl.info()
        print(f"# {prec}: plan {plan_s:.2f} s (N={n}, D={pi['D']})", file=sys.stderr, flush=True)
        # Work units per apply, by level: the algorithmic counts behind
        # per-kernel rates computed from a profiler's trace.
        print(f"# {prec}: units " + json.dumps(
            {k: pi[k] for k in ("boxes", "cones", "cousin_pairs", "prop_pairs", "prop_mode",
                                "leaf_pairs", "near_pairs", "tune_cache_hit")}),
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
        modes = {"propagation": (1,), "propagation_mfma": (2,),
                 "propagation_small": (3, 4, 5)}[dom]
        mode = modes[0]
        units = sum(pp for pp, md in zip(info["prop_pairs"], info["prop_mode"]) if md in modes)
        fpu = FLOP_PROP * flop_scale(P)
        unit_txt = "(parent-cone node, relevant child) evaluations"
        bound = "mfma" if mode >= 2 else "alu"
    elif dom == "interpolation":
        units = sum(info["cousin_pairs"])
        fpu = FLOP_INTERP * flop_scale(P)
        unit_txt = "(target, cousin box) evaluations"
    elif dom == "leaf":
        units = info["leaf_pairs"]
        fpu = FLOP_LEAF
        unit_txt = "(leaf-cone node, source) evaluations"
    else:
        units = info["near_pairs"]
        fpu = FLOP_NEAR
        unit_txt = "near-field pairs"
    flop = units * n_rhs * fpu
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
                "flop_per_unit_per_rhs": fpu,
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
        threads = oracle.threads()
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
        line["cpu"] = cpu_info()
        line["cpu_baseline"]["cores"] = line["cpu"]["omp_threads"]
        if args.cpu_ifgf_n > 0:
            line["cpu_baseline_ifgf"] = cpu_ifgf_leg(args.cpu_ifgf_n, args.steps, args.warmup)
    if args.configs != "none":
        names = None if args.configs == "all" else args.configs.split(",")
        line["configs"] = run_configs(args.config_steps, 2, names)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
