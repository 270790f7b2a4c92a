"""Python binding of libifgf.so (ctypes).

Argument marshalling only: every step of the IFGF evaluation runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IFGF_LIB_PATH selects another build of the library (the host-sanitized one
# of build_sanitized.py); by default the in-tree libifgf.so.
LIB_PATH = os.environ.get("IFGF_LIB_PATH") or os.path.join(HERE, "libifgf.so")

IFGF_MAX_LEVELS = 24
FP64, FP32_MIXED, FP32_BF16X3 = 0, 1, 2

STATUS = {0: "IFGF_OK", 1: "IFGF_EINVAL", 2: "IFGF_ENOMEM", 3: "IFGF_EDUPLICATE",
          4: "IFGF_EHIP", 5: "IFGF_EUNSUPPORTED", 6: "IFGF_ELOOKUP"}

EXPORTED = ["ifgf_default_opts", "ifgf_plan", "ifgf_plan_ex", "ifgf_plan_batched",
            "ifgf_apply", "ifgf_check", "ifgf_set_stream", "ifgf_plan_info",
            "ifgf_partition_counts", "ifgf_destroy", "ifgf_status_string",
            "ifgf_profile", "ifgf_profile_read", "ifgf_cone_keys",
            "ifgf_apply_graph", "ifgf_apply_noalloc"]

STAGES = ["permute_in", "near_field", "leaf", "interpolation", "propagation",
          "permute_out", "propagation_mfma", "propagation_small"]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("n_rhs", ctypes.c_int),
                ("leaf_grid", ctypes.c_int * 3), ("levels", ctypes.c_int),
                ("stages", ctypes.c_int), ("host_only", ctypes.c_int),
                ("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("prop_kernel", ctypes.c_int), ("lookup", ctypes.c_int),
                ("autotune", ctypes.c_int), ("cone_margin", ctypes.c_double),
                ("leaf_max", ctypes.c_double), ("leaf_abs", ctypes.c_double),
                ("grid_rule", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("prop_tables", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_instances", ctypes.c_int),
                ("max_levels", ctypes.c_int), ("n_steps", ctypes.c_int),
                ("p_s", ctypes.c_int), ("p_ang", ctypes.c_int),
                ("n_rhs", ctypes.c_int), ("precision", ctypes.c_int),
                ("boxes", ctypes.c_int64 * IFGF_MAX_LEVELS),
                ("cones", ctypes.c_int64 * IFGF_MAX_LEVELS),
                ("cousin_pairs", ctypes.c_int64 * IFGF_MAX_LEVELS),
                ("grid", ctypes.c_int64 * IFGF_MAX_LEVELS),
                ("prop_pairs", ctypes.c_int64 * IFGF_MAX_LEVELS),
                ("prop_mode", ctypes.c_int * IFGF_MAX_LEVELS),
                ("autotune_ms", (ctypes.c_float * 5) * IFGF_MAX_LEVELS),
                ("leaf_pairs", ctypes.c_int64),
                ("near_pairs", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("plan_seconds", ctypes.c_double), ("tune_cache_hit", ctypes.c_int),
                ("grid_doubling", ctypes.c_int), ("prop_table_bytes", ctypes.c_int64)]


class StageTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)),
                ("launches", ctypes.c_int64 * len(STAGES))]


class IFGFError(RuntimeError):
    def __init__(self, status, text):
        super().__init__(f"{STATUS.get(status, status)}: {text}")
        self.status = status


_lib = None


def load_library():
    """Load libifgf.so (built by ``paper_2112_15198_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run "
                           "`python -m paper_2112_15198_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.ifgf_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.ifgf_plan.argtypes = [ctypes.POINTER(P), P, I64, D, I, I, D]
    lib.ifgf_plan_ex.argtypes = [ctypes.POINTER(P), P, I64, D, I, I, D, ctypes.POINTER(Opts)]
    lib.ifgf_plan_batched.argtypes = [ctypes.POINTER(P), I, P, P, P, I, I, D,
                                      ctypes.POINTER(Opts)]
    lib.ifgf_apply.argtypes = [P, P, P]
    lib.ifgf_apply_graph.argtypes = [P, P, P]
    lib.ifgf_apply_noalloc.argtypes = [P, P, P]
    lib.ifgf_check.argtypes = [P]
    lib.ifgf_set_stream.argtypes = [P, P]
    lib.ifgf_plan_info.argtypes = [P, ctypes.POINTER(Info)]
    lib.ifgf_partition_counts.argtypes = [P, P]
    lib.ifgf_cone_keys.argtypes = [P, I, P, I64]
    lib.ifgf_profile.argtypes = [P, I]
    lib.ifgf_profile_read.argtypes = [P, ctypes.POINTER(StageTimes), I]
    lib.ifgf_destroy.argtypes = [P]
    lib.ifgf_destroy.restype = None
    lib.ifgf_status_string.argtypes = [I]
    lib.ifgf_status_string.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("ifgf_destroy", "ifgf_status_string"):
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise IFGFError(rc, load_library().ifgf_status_string(rc).decode())


GRID_RULES = {"auto": 0, "double": 1, "constant": 2, 0: 0, 1: 1, 2: 2}


def _opts(precision, n_rhs, leaf_grid, levels, stages, host_only, device,
          cone_margin=None, prop_kernel=0, lookup=0, autotune=False,
          leaf_max=0.0, leaf_abs=0.0, grid_rule="auto", tune_cache=None,
          prop_tables="auto"):
    o = Opts()
    _check(load_library().ifgf_default_opts(ctypes.byref(o)))
    o.precision = {"fp64": FP64, "fp32": FP32_MIXED, "mixed": FP32_MIXED,
                   "bf16x3": FP32_BF16X3, FP64: FP64, FP32_MIXED: FP32_MIXED,
                   FP32_BF16X3: FP32_BF16X3}[precision]
    o.n_rhs = int(n_rhs)
    o.leaf_grid[0], o.leaf_grid[1], o.leaf_grid[2] = (int(v) for v in leaf_grid)
    o.levels = int(levels)
    o.stages = int(stages)
    o.host_only = 1 if host_only else 0
    o.device = -1 if device is None else int(device)
    if cone_margin is not None:
        o.cone_margin = float(cone_margin)
    o.prop_kernel = {"auto": 0, "node": 1, "grouped": 2, "small": 3, "medium": 4,
                     "lean": 5, 0: 0, 1: 1, 2: 2, 3: 3, 4: 4, 5: 5}[prop_kernel]
    o.lookup = {"auto": 0, "hash": 1, 0: 0, 1: 1}[lookup]
    o.autotune = 1 if autotune else 0
    o.leaf_max = float(leaf_max)
    o.leaf_abs = float(leaf_abs)
    o.grid_rule = GRID_RULES[grid_rule] if grid_rule in GRID_RULES else int(grid_rule)
    # The plan copies the path at plan time.
    o.tune_cache = None if not tune_cache else os.fsencode(tune_cache)
    o.prop_tables = {"auto": 0, "never": 1, "always": 2, 0: 0, 1: 1, 2: 2}[prop_tables]
    return o


class Plan:
    """An IFGF plan: octree, cone segments and device buffers for fixed points.

    ``apply(a)`` evaluates I(x_l) = sum_{m != l} a_m e^{i kappa r}/(4 pi r).
    """

    def __init__(self, handle, n, n_rhs, precision, offsets=None):
        self._h = handle
        self.n = n
        self.n_rhs = n_rhs
        self.precision = precision
        self.offsets = offsets

    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.precision == FP64 else torch.complex64

    def apply(self, dens, out=None, check=None, graph=False):
        """dens: CUDA tensor (n_rhs, N) or (N,) of the plan's complex dtype.

        graph=True replays a HIP graph of the whole apply, captured on the
        first call for this (dens, out) pair.  check (default: True for an
        eager apply, False for a graph replay) waits for the apply and
        raises IFGFError(IFGF_ELOOKUP) if a cone look-up missed; with
        check=False call check() before trusting the result."""
        if check is None:
            check = not graph
        import torch
        if self._h is None:
            raise ValueError("plan is closed")
        shape = dens.shape
        if not (dens.is_cuda and dens.dtype == self.dtype and dens.numel() == self.n * self.n_rhs):
            raise ValueError(f"densities must be a CUDA {self.dtype} tensor with "
                             f"{self.n_rhs} x {self.n} entries")
        dens = dens.contiguous()
        if out is None:
            out = torch.empty_like(dens)
        lib = load_library()
        _check(lib.ifgf_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        fn = lib.ifgf_apply_graph if graph else lib.ifgf_apply
        _check(fn(self._h, ctypes.c_void_p(dens.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        if check:
            self.check()
        return out.reshape(shape)

    def check(self):
        _check(load_library().ifgf_check(self._h))

    def info(self):
        inf = Info()
        _check(load_library().ifgf_plan_info(self._h, ctypes.byref(inf)))
        L = inf.n_steps
        return {"n_points": inf.n_points, "n_instances": inf.n_instances,
                "D": inf.max_levels, "n_steps": L, "p_s": inf.p_s, "p_ang": inf.p_ang,
                "n_rhs": inf.n_rhs, "precision": inf.precision,
                "boxes": list(inf.boxes[:L]), "cones": list(inf.cones[:L]),
                "cousin_pairs": list(inf.cousin_pairs[:L]), "grid": list(inf.grid[:L]),
                "prop_pairs": list(inf.prop_pairs[:L]), "leaf_pairs": inf.leaf_pairs,
                "prop_mode": list(inf.prop_mode[:L]),
                "autotune_ms": [tuple(inf.autotune_ms[l]) for l in range(L)],
                "near_pairs": inf.near_pairs, "device_bytes": inf.device_bytes,
                "plan_seconds": inf.plan_seconds, "tune_cache_hit": bool(inf.tune_cache_hit),
                "grid_doubling": bool(inf.grid_doubling),
                "prop_table_bytes": int(inf.prop_table_bytes)}

    def profile(self, enable=True):
        """Time every kernel launch of later applies with HIP events."""
        _check(load_library().ifgf_profile(self._h, 1 if enable else 0))

    def profile_read(self, reset=True):
        """{stage: (total ms, launches)} of the timed launches so far."""
        t = StageTimes()
        _check(load_library().ifgf_profile_read(self._h, ctypes.byref(t), 1 if reset else 0))
        return {s: (t.ms[i], t.launches[i]) for i, s in enumerate(STAGES)}

    def cone_keys(self, step):
        """Sorted relevant-cone keys box * grid + gamma of step l = D - d."""
        n = self.info()["cones"][step]
        out = np.zeros(n, dtype=np.uint64)
        _check(load_library().ifgf_cone_keys(self._h, int(step),
                                             out.ctypes.data_as(ctypes.c_void_p), n))
        return out

    def partition_counts(self):
        out = np.zeros(self.n, dtype=np.int64)
        _check(load_library().ifgf_partition_counts(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if self._h is not None:
            load_library().ifgf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _points_arg(points):
    """(pointer, N, keep-alive) of an (N, 3) float64 array: a numpy array
    (host) or a contiguous CUDA tensor (device)."""
    if hasattr(points, "is_cuda") and points.is_cuda:
        import torch
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("device points must be a float64 tensor of shape (N, 3)")
        t = points.contiguous()
        return ctypes.c_void_p(t.data_ptr()), t.shape[0], t
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
    if pts.ndim != 2 or pts.shape[1] != 3:
        raise ValueError("points must have shape (N, 3)")
    return pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0], pts


def plan(points, kappa, p_s=3, p_ang=5, leaf_size=0.25, precision="fp64",
         n_rhs=1, leaf_grid=(2, 4, 8), levels=0, stages=3, host_only=False,
         device=None, cone_margin=None, prop_kernel="auto", lookup="auto",
         autotune=False, leaf_max=0.0, leaf_abs=0.0, grid_rule="auto",
         tune_cache=None, prop_tables="auto"):
    """Plan one instance; points is an (N, 3) float64 array on the host or a
    float64 CUDA tensor.

    precision: "fp64" (IFGF_FP64, complex128 densities), "fp32"
    (IFGF_FP32_MIXED, complex64) or "bf16x3" (IFGF_FP32_BF16X3, complex64:
    FP32-mixed with the wave-task propagation product in three-term BF16
    form).  prop_kernel: "auto", "node", "grouped", "small" (one-wave),
    "medium" (four-wave) or "lean" (four-wave, smaller chunks); autotune=True
    times the five per level instead
    (tune_cache: a file that keeps the choices across plans).  kappa = 0
    (the Laplace kernel) needs leaf_abs (leaf side in length units) or
    levels; leaf_max caps the leaf side in wavelengths.  prop_tables:
    "auto", "never" or "always" keeps the box-independent propagation
    geometry in plan-time tables (identical results)."""
    ptr, n, keep = _points_arg(points)
    o = _opts(precision, n_rhs, leaf_grid, levels, stages, host_only, device,
              cone_margin, prop_kernel, lookup, autotune, leaf_max, leaf_abs,
              grid_rule, tune_cache, prop_tables)
    h = ctypes.c_void_p()
    _check(load_library().ifgf_plan_ex(ctypes.byref(h), ptr, n, float(kappa), int(p_s),
                                       int(p_ang), float(leaf_size), ctypes.byref(o)))
    del keep
    return Plan(h, n, o.n_rhs, o.precision)


def plan_batched(points_list, kappas, p_s=3, p_ang=5, leaf_size=0.25,
                 precision="fp64", n_rhs=1, leaf_grid=(2, 4, 8), levels=0,
                 stages=3, host_only=False, device=None, cone_margin=None,
                 prop_kernel="auto", lookup="auto", autotune=False, leaf_max=0.0,
                 leaf_abs=0.0, grid_rule="auto", tune_cache=None, prop_tables="auto"):
    """Plan several independent instances evaluated together by each apply.

    Densities and outputs are (n_rhs, sum N_i), instances concatenated.
    """
    pts = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64)
                                               for p in points_list], axis=0))
    offsets = np.zeros(len(points_list) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) for p in points_list])
    kap = np.ascontiguousarray(np.asarray(kappas, dtype=np.float64))
    o = _opts(precision, n_rhs, leaf_grid, levels, stages, host_only, device,
              cone_margin, prop_kernel, lookup, autotune, leaf_max, leaf_abs,
              grid_rule, tune_cache, prop_tables)
    h = ctypes.c_void_p()
    _check(load_library().ifgf_plan_batched(
        ctypes.byref(h), len(points_list), offsets.ctypes.data_as(ctypes.c_void_p),
        pts.ctypes.data_as(ctypes.c_void_p), kap.ctypes.data_as(ctypes.c_void_p),
        int(p_s), int(p_ang), float(leaf_size), ctypes.byref(o)))
    return Plan(h, int(offsets[-1]), o.n_rhs, o.precision, offsets)
