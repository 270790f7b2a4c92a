"""CPU-side checks of libifgf.so: it loads, exports every entry point that
include/ifgf.h declares, and its host planner builds the octree of Section 2
(boxes per level, the partition of sources into neighbours and cousins)
and rejects invalid input with the documented status codes.  No GPU call is
made here."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2112_15198_amd as ifgf
from paper_2112_15198_amd import ifgf as lib
from paper_2112_15198_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ifgf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ifgf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = ifgf.load_library()
    names = declared_functions()
    assert "ifgf_plan" in names and "ifgf_apply" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(lib.EXPORTED) == names


@pytest.mark.parametrize("geom", ["sphere", "oblate", "clusters"])
def test_host_tree_matches_oracle_tree(geom):
    if geom == "sphere":
        p, k = W.fibonacci_sphere(5024), 4 * np.pi
    elif geom == "oblate":
        p, k = W.spheroid(6000), W.kappa_oblate_10ppw(6000)
    else:
        rng = np.random.default_rng(3)
        p = np.vstack([rng.normal(size=(700, 3)) * 0.05 - [1.0, 0, 0],
                       rng.normal(size=(700, 3)) * 0.05 + [1.0, 0.3, 0]])
        k = 12.0
    pl = ifgf.plan(p, k, host_only=True)
    info = pl.info()
    _, oi = oracle.ifgf(p, np.zeros(len(p)), k, far=False, return_info=True)
    assert info["D"] == oi["D"]
    # Steps count from the leaf: step l is level D - l.
    assert info["boxes"] == oi["boxes"][2:][::-1]
    cnt = pl.partition_counts()
    assert (cnt == len(p)).all()
    np.testing.assert_array_equal(cnt, oracle.partition_counts(p, k))


@pytest.mark.parametrize("rule", ["leaf_max", "leaf_abs", "laplace"])
def test_host_level_rules_match_oracle(rule):
    """The level rules (leaf-side cap in wavelengths; absolute leaf side, the
    rule for kappa = 0) give the oracle's D and boxes, and the partition of
    the sources."""
    n = 4373
    p = W.spheroid(n)
    k = W.kappa_oblate_10ppw(n)
    kw = {"leaf_max": dict(leaf_max=0.3), "leaf_abs": dict(leaf_abs=0.05),
          "laplace": dict(leaf_abs=0.1)}[rule]
    if rule == "laplace":
        k = 0.0
    pl = ifgf.plan(p, k, host_only=True, **kw)
    info = pl.info()
    _, oi = oracle.ifgf(p, np.zeros(n), k, far=False, return_info=True, **kw)
    assert info["D"] == oi["D"]
    assert info["boxes"] == oi["boxes"][2:][::-1]
    np.testing.assert_array_equal(pl.partition_counts(), oracle.partition_counts(p, k, **kw))
    assert info["grid_doubling"] == (k > 0)
    if rule == "leaf_max":
        assert info["D"] == 6


def test_laplace_and_grid_rules_validated():
    p = W.fibonacci_sphere(200)
    # kappa = 0 without a wavelength-free rule, negative kappa, bad grid rule.
    assert _status(lambda: ifgf.plan(p, 0.0, host_only=True)) == 1  # no level rule
    assert _status(lambda: ifgf.plan(p, -2.0, leaf_abs=0.1, host_only=True)) == 1
    assert _status(lambda: ifgf.plan(p, 3.0, grid_rule=3, host_only=True)) == 1
    assert _status(lambda: ifgf.plan(p, 3.0, leaf_max=-1.0, host_only=True)) == 1
    # One batched plan cannot mix kappa = 0 and kappa > 0 under the automatic
    # grid rule; an explicit rule allows it.
    assert _status(lambda: ifgf.plan_batched([p, p], [0.0, 3.0], leaf_abs=0.2,
                                             host_only=True)) == 1
    ifgf.plan_batched([p, p], [0.0, 3.0], leaf_abs=0.2, grid_rule="constant",
                      host_only=True).close()
    ifgf.plan(p, 0.0, levels=4, host_only=True).close()


def test_batched_host_plan_partition():
    pts = [W.fibonacci_sphere(3000), W.spheroid(4500), W.fibonacci_sphere(800)]
    kap = [W.kappa_sphere_10ppw(3000), W.kappa_oblate_10ppw(4500), 9.0]
    pl = ifgf.plan_batched(pts, kap, host_only=True)
    cnt = pl.partition_counts()
    expect = np.concatenate([np.full(len(q), len(q)) for q in pts])
    np.testing.assert_array_equal(cnt, expect)
    assert pl.info()["n_instances"] == 3


def _status(fn):
    with pytest.raises(ifgf.IFGFError) as e:
        fn()
    return e.value.status


def test_error_codes():
    p = W.fibonacci_sphere(100)
    assert _status(lambda: ifgf.plan(p[:1], 3.0, host_only=True)) == 1
    assert _status(lambda: ifgf.plan(p, -1.0, host_only=True)) == 1
    assert _status(lambda: ifgf.plan(p, 0.0, host_only=True)) == 1  # no level rule
    q = p.copy()
    q[7, 1] = np.nan
    assert _status(lambda: ifgf.plan(q, 3.0, host_only=True)) == 1
    q = p.copy()
    q[50] = q[3]
    assert _status(lambda: ifgf.plan(q, 3.0, host_only=True)) == 3
    assert _status(lambda: ifgf.plan(p, 3.0, p_s=4, p_ang=4)) == 5
    assert _status(lambda: ifgf.plan(p, 3.0, n_rhs=9)) == 5
    assert _status(lambda: ifgf.plan(p, 3.0, leaf_grid=(0, 4, 8))) == 1
    assert _status(lambda: ifgf.plan(p, 3.0, levels=2, host_only=True)) == 1
    # Precision: the three modes plan (host only); another value is EINVAL.
    for prec in ("fp64", "fp32", "bf16x3"):
        ifgf.plan(p, 3.0, precision=prec, host_only=True).close()
    import ctypes
    o = lib._opts("fp32", 1, (2, 4, 8), 0, 3, True, None)
    o.precision = 3
    h = ctypes.c_void_p()
    pts = np.ascontiguousarray(p)
    rc = lib.load_library().ifgf_plan_ex(ctypes.byref(h), pts.ctypes.data_as(ctypes.c_void_p),
                                         pts.shape[0], 3.0, 3, 5, 0.25, ctypes.byref(o))
    assert rc == 1


def test_status_strings():
    L = ifgf.load_library()
    for s in range(7):
        assert L.ifgf_status_string(s)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without libifgf.so the binding raises; there is no CPU fallback."""
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "libifgf.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(RuntimeError, match="is missing"):
        lib.load_library()
    with pytest.raises(RuntimeError, match="is missing"):
        ifgf.plan(W.fibonacci_sphere(100), 3.0, host_only=True)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; --gpus 2 exits with a message before any
    GPU work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout


def test_bench_traffic_record_follows_the_kernel_source(tmp_path, monkeypatch):
    """bench.py reports the rocprofv3 HBM traffic of the dominant kernel only
    while the committed record's SHA-256 matches the kernel source; after any
    change to the source it reports none (null) until the counters are
    taken again."""
    import hashlib
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src_dir = tmp_path / "paper_2112_15198_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "ifgf_kernels.hip"
    src.write_text("// kernel source\n")
    rec = {"stage": "propagation_small", "workload": "sphere_321k", "precision": "fp32",
           "kernel_source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "traffic_bytes_per_launch": 123456789}
    (tmp_path / "profiles" / "k_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("propagation_small", "sphere_321k", "fp32") == 123456789
    assert bench.measured_traffic("propagation_small", "sphere_321k", "fp64") is None
    assert bench.measured_traffic("interpolation", "sphere_321k", "fp32") is None
    src.write_text("// kernel source, changed\n")
    assert bench.measured_traffic("propagation_small", "sphere_321k", "fp32") is None


def test_profile_commands_are_valid_bench_invocations():
    """Every bench.py command quoted in profiles/*.md parses with bench.py's
    own argument parser and names a known workload, so the committed
    summaries can be reproduced as written."""
    import glob
    import shlex
    import sys
    sys.path.insert(0, ROOT)
    import bench
    ap = bench.arg_parser()
    found = 0
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        text = open(f).read()
        for m in re.finditer(r'python3 \$R/bench\.py([^"`\n]*)', text):
            argv = shlex.split(m.group(1).replace("$R", "/tmp/r").replace("\\", ""))
            args = ap.parse_args(argv)
            assert args.workload in W.WORKLOADS, (f, args.workload)
            found += 1
    assert found >= 10
