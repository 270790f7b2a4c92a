"""The allocation-free apply (ifgf_apply_noalloc), called through the C ABI,
against ifgf_apply on the same plan: the same kernels on the same inputs, so
the outputs agree to the FP64 bar (1e-10; they are expected bit-identical).
Two calls in a row, the second on a smaller plan, so that the second reuses
the static workspace the first one filled.  FP64 and FP32-mixed."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2112_15198_amd import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _apply_both(pl, dens, precision):
    """(ifgf_apply result, ifgf_apply_noalloc result) for one plan."""
    import torch
    from paper_2112_15198_amd import ifgf
    lib = ifgf.load_library()
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    a = torch.from_numpy(np.ascontiguousarray(dens)).to(dt).cuda()
    ref = torch.empty_like(a)
    got = torch.full_like(a, complex(float("nan"), float("nan")))
    torch.cuda.synchronize()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ifgf._check(lib.ifgf_set_stream(pl._h, stream))
    ifgf._check(lib.ifgf_apply(pl._h, ctypes.c_void_p(a.data_ptr()),
                               ctypes.c_void_p(ref.data_ptr())))
    ifgf._check(lib.ifgf_check(pl._h))
    ifgf._check(lib.ifgf_apply_noalloc(pl._h, ctypes.c_void_p(a.data_ptr()),
                                       ctypes.c_void_p(got.data_ptr())))
    ifgf._check(lib.ifgf_check(pl._h))
    return (ref.cpu().numpy().astype(np.complex128),
            got.cpu().numpy().astype(np.complex128))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_apply_twice(precision):
    import paper_2112_15198_amd as ifgf
    big = W.make("sphere_5k")
    n_small = 2000
    small_pts = W.fibonacci_sphere(n_small)
    rng = np.random.default_rng(77)
    small_dens = (rng.uniform(-1, 1, (2, n_small)) + 1j * rng.uniform(-1, 1, (2, n_small)))
    cases = [("sphere N=5024, 1 RHS", big.points, big.kappa, big.dens),
             ("sphere N=2000, 2 RHS", small_pts, 2.0 * np.pi, small_dens)]
    for name, pts, kappa, dens in cases:
        say("noalloc", precision, name)
        pl = ifgf.plan(pts, kappa, precision=precision, n_rhs=dens.shape[0],
                       leaf_grid=(2, 4, 8))
        ref, got = _apply_both(pl, dens, precision)
        pl.close()
        for r in range(dens.shape[0]):
            assert_close(got[r], ref[r], 1e-10, f"noalloc {precision} {name} rhs {r}")


def test_noalloc_rejects_oversized_workspace():
    """A plan whose workspace exceeds the static array is refused with
    IFGF_EINVAL before anything is launched."""
    import torch
    import paper_2112_15198_amd as ifgf
    n = 321536
    w = W.make("sphere_321k")
    say("noalloc oversized sphere_321k fp64")
    pl = ifgf.plan(w.points, w.kappa, precision="fp64", leaf_grid=(2, 4, 8))
    a = torch.from_numpy(w.dens).to(torch.complex128).cuda()
    out = torch.empty_like(a)
    lib = ifgf.load_library()
    rc = lib.ifgf_apply_noalloc(pl._h, ctypes.c_void_p(a.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()))
    assert rc == 1, rc
    assert b"exceeds the static scratch" in lib.ifgf_status_string(rc)
    pl.close()
    assert out.shape[1] == n
