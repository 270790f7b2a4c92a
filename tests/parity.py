"""Comparison helpers shared by the parity tests.

Every comparison checks two norms of the difference at the same bar:
  * relative l2:        ||g - o||_2 / ||o||_2     (eq. errorcomputation)
  * element-wise max:   max_i |g_i - o_i| / max_i |o_i|
The second catches a single wrong cone or box, which the l2 norm dilutes by
about sqrt(N).
"""
import numpy as np


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def assert_close(g, o, tol, what=""):
    """g matches o to `tol` in relative l2 and in the element-wise max norm."""
    e2, em = relerr(g, o), maxerr(g, o)
    print(f"[parity] {what} rel-l2 {e2:.3e} max-elem {em:.3e} (bar {tol:.1e})", flush=True)
    assert e2 <= tol, (what, "rel-l2", e2, tol)
    assert em <= tol, (what, "max-elem", em, tol)
    return e2, em
