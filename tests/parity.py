"""Comparison helpers of the GPU parity tests (imported by the tests; not a
test module).

Every comparison checks two bars on each right-hand side column:
  * norm-wise:     ||x - ref||_2 / ||ref||_2                 <= tol
  * element-wise:  max_i |x_i - ref_i| / max_i |ref_i|       <= 10 tol
The norm-wise bar is the accuracy a result is claimed at; the element-wise
one makes sure no single entry carries the error (a 1% error in one entry
of a 24,576-vector passes a 1e-4 norm-wise bar).  Tolerances: FP64 path vs
oracle 1e-10 (entries 1e-9), FP32 blocks 1e-4 (entries 1e-3), refinement
vs x* 1e-8 (entries 1e-7), FP64 H-matvec 1e-12 (entries 1e-11).
"""
import numpy as np

ELEM_FACTOR = 10.0


def _cols(x, ref):
    ref = np.asarray(ref)
    x = np.asarray(x).reshape(ref.shape[0], -1)
    return x, ref.reshape(ref.shape[0], -1)


def norm_err(x, ref) -> float:
    """Max over columns of ||x - ref||_2 / ||ref||_2."""
    x, ref = _cols(x, ref)
    return float(np.max(np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def elem_err(x, ref) -> float:
    """Max over columns of max_i |x_i - ref_i| / max_i |ref_i|."""
    x, ref = _cols(x, ref)
    return float(np.max(np.max(np.abs(x - ref), axis=0) / np.max(np.abs(ref), axis=0)))


def assert_close(x, ref, tol, what=None):
    """Both bars at once; the message names the case and both errors."""
    ne, ee = norm_err(x, ref), elem_err(x, ref)
    assert ne <= tol and ee <= ELEM_FACTOR * tol, \
        f"{what}: norm-wise {ne:.3e} (bar {tol:.1e}), element-wise {ee:.3e} " \
        f"(bar {ELEM_FACTOR * tol:.1e})"
    return ne, ee
