"""IFGF evaluation of the discrete Helmholtz operator on MI355X (gfx950).

    I(x_l) = sum_{m != l} a_m e^{i kappa |x_l - x_m|} / (4 pi |x_l - x_m|)

The work runs in hand-written HIP kernels of ``libifgf.so`` behind a C ABI
(``include/ifgf.h``); this package is its Python binding.
"""
from .ifgf import (FP32_MIXED, FP64, IFGFError, Plan, load_library, plan,
                   plan_batched)

__all__ = ["plan", "plan_batched", "Plan", "IFGFError", "load_library",
           "FP64", "FP32_MIXED"]
