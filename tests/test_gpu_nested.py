"""GPU nested multi-level solve (ps_solve kind PS_NESTED, eq. 14-22 with the
factors taken from the leaf level up) against the oracle's ``nested``,
through the C-ABI.

Bar: FP64 <= 1e-10, FP32 blocks <= 1e-4 (relative 2-norm per right-hand
side, max over right-hand sides), as for the flat series.
"""
import ctypes as C
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import hmatrix, series
from parity import assert_close

torch = pytest.importorskip("torch")
from paper_2307_03968_amd import hmps  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10
TOL_F32 = 1e-4


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    a = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


class Case:
    def __init__(self, name, prob, leaf, tol, nrhs):
        self.name = name
        self.prob = prob
        self.H = hmatrix.HMatrix(prob, leaf, 1.0, tol)
        _say(f"build {name} n={prob.n} leaf={leaf}")
        self.h = hmps.HMatrix(prob, leaf, 1.0, tol)
        self.b = W.plane_waves(prob.xyz, W.directions(nrhs, 3))


@pytest.fixture(scope="module")
def sphere_levels():
    return Case("sphere_1200_leaf32", W.sphere_problem(1200, math.sqrt(1200 / 1536)), 32, 1e-6, 3)


def test_nested_each_level_and_K(sphere_levels):
    c = sphere_levels
    for lev in [-1] + sorted(c.H.far_levels, reverse=True):
        for K in (0, 1, 3):
            ref = series.nested(c.H, c.b, K, lev)
            for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
                _say(f"nested {c.name} level={lev} K={K} precision={prec}")
                x = _host(c.h.solve(_dev(c.b), K=K, level=lev, precision=prec,
                                    kind=hmps.PS_NESTED))
                assert_close(x, ref, tol, (lev, K, prec))


def test_nested_leaf_level_equals_series(sphere_levels):
    """One factor: the nested solve and the flat series agree to rounding."""
    c = sphere_levels
    _say(f"nested vs series {c.name}")
    b = _dev(c.b)
    xn = _host(c.h.solve(b, K=4, kind=hmps.PS_NESTED))
    xs = _host(c.h.solve(b, K=4))
    assert_close(xn, xs, 1e-13)


def test_nested_volume():
    """The 1,000-point cube (rho > 1: the products grow, the parity bar is
    relative and still holds)."""
    c = Case("cube_1000_leaf32", W.cube_problem(10, 10 / 16), 32, 1e-5, 2)
    for lev in [-1] + sorted(c.H.far_levels, reverse=True):
        ref = series.nested(c.H, c.b, 2, lev)
        _say(f"nested {c.name} level={lev} K=2")
        x = _host(c.h.solve(_dev(c.b), K=2, level=lev, kind=hmps.PS_NESTED))
        assert_close(x, ref, TOL_F64, lev)
    c.h.close()


def test_nested_matrix_core_ragged_depths():
    """Leaves at two depths (68 and 34/35 points), 17 right-hand sides on the
    matrix-core kernels (forced from one right-hand side on), every level."""
    c = Case("sphere_2200_leaf68", W.sphere_problem(2200, math.sqrt(2200 / 1536)), 68, 1e-4, 17)
    c.h.tune(mm_min_rhs=1)
    try:
        for lev in [-1] + sorted(c.H.far_levels, reverse=True):
            ref = series.nested(c.H, c.b, 2, lev)
            for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
                _say(f"nested {c.name} nrhs=17 mfma level={lev} precision={prec}")
                x = _host(c.h.solve(_dev(c.b), K=2, level=lev, precision=prec,
                                    kind=hmps.PS_NESTED))
                assert_close(x, ref, tol, (lev, prec))
    finally:
        c.h.tune(mm_min_rhs=-1)
    c.h.close()


def test_nested_argument_errors(sphere_levels):
    c = sphere_levels
    lib = hmps._lib()
    b = _dev(c.b[:, 0])
    x = torch.empty_like(b)
    n = c.prob.n
    lo = min(c.H.far_levels)
    # (K + 1)^2 - 1 level products above the limit
    o = hmps.ps_opts(1000, lo, 0, hmps.PS_NESTED, 0, 1e-9, 0)
    assert lib.ps_solve(c.h.handle, C.byref(o), C.c_void_p(b.data_ptr()), n,
                        C.c_void_p(x.data_ptr()), n, 1, None, None) == hmps.HM_EINVAL
    probs = [W.sphere_problem(200, 0.4), W.sphere_problem(150, 0.35, seed=7)]
    _say("nested batched handle refused")
    hb = hmps.HMatrix(probs, 32, 1.0, 1e-4)
    bb = _dev(np.zeros(350, complex))
    xb = torch.empty_like(bb)
    o = hmps.ps_opts(1, -1, 0, hmps.PS_NESTED, 0, 1e-9, 0)
    assert lib.ps_solve(hb.handle, C.byref(o), C.c_void_p(bb.data_ptr()), 350,
                        C.c_void_p(xb.data_ptr()), 350, 1, None, None) == hmps.HM_EINVAL
    hb.close()
