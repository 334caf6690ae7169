"""GPU GMRES preconditioned by the power series (ps_solve kind PS_GMRES),
through the C-ABI, against the oracle's x* = Z_l^{-1} b (dense LU of the
assembled H-matrix at level l).

Bar: relative 2-norm error per right-hand side <= 1e-8 against x* for a
residual tolerance of 1e-11 (the systems here have condition numbers far
below 1e3); the reported residual is checked against the oracle's own
residual of the returned x.
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

TOL_X = 1e-8
RES_TOL = 1e-11


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
    def __init__(self, name, prob, leaf, tol, nrhs=1):
        self.name = name
        self.prob = prob
        self.H = hmatrix.HMatrix(prob, leaf, 1.0, tol)
        _say(f"build {name} n={prob.n} leaf={leaf}")
        self.h = hmps.HMatrix(prob, leaf, 1.0, tol)
        self.b = W.plane_waves(prob.xyz, W.directions(nrhs, 3)) if nrhs > 1 else \
            W.plane_waves(prob.xyz, W.Z_HAT)


@pytest.fixture(scope="module")
def sphere():
    return Case("sphere_1536", W.sphere_small().problem, 64, 1e-4)


@pytest.fixture(scope="module")
def cube():
    return Case("cube_1000_leaf32", W.cube_problem(10, 10 / 16), 32, 1e-5, 3)


@pytest.fixture(scope="module")
def ragged():
    return Case("sphere_1000_leaf40", W.sphere_problem(1000, math.sqrt(1000 / 1536)), 40, 1e-4, 7)


def _oracle_resid(H, x, b, level=-1):
    """Per-column ||b - Z_l x|| / ||b|| with the oracle's H-matvec."""
    x = x.reshape(b.shape)
    r = b - series.apply_Z(H, x, level)
    if b.ndim == 1:
        return np.array([np.linalg.norm(r) / np.linalg.norm(b)])
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


def _check(case, x, st, level=-1, b=None):
    b = case.b if b is None else b
    xs = series.solve_exact(case.H, b, level)
    assert_close(x, xs, TOL_X)
    res = _oracle_resid(case.H, x, b, level)
    for c, s in enumerate(st):
        assert s["diverged"] == 0 and s["passes"] >= 1, s
        assert s["resid_rel"] <= RES_TOL, s
        # the library's true residual and the oracle's agree to rounding
        assert abs(s["resid_rel"] - res[c]) <= 1e-13 + 1e-3 * res[c], (s, res[c])


def test_gmres_sphere_reaches_xstar(sphere):
    """Block-Jacobi (K = 0) and series (K = 4, FP64 and FP32 blocks)
    preconditioners all reach x*; the series preconditioner needs fewer
    Arnoldi steps (rho = 0.82 here)."""
    steps = {}
    for K, prec in ((0, hmps.HM_F64), (4, hmps.HM_F64), (4, hmps.HM_F32_APPLY)):
        _say(f"gmres {sphere.name} K={K} precision={prec}")
        x, st = sphere.h.solve(_dev(sphere.b), K=K, precision=prec, kind=hmps.PS_GMRES,
                               max_passes=300, refine_tol=RES_TOL, stats=True)
        _check(sphere, _host(x), st)
        steps[(K, prec)] = st[0]["passes"]
    assert steps[(4, hmps.HM_F64)] < steps[(0, hmps.HM_F64)], steps


def test_gmres_volume_where_the_series_diverges(cube):
    """rho(D^{-1} R) > 1 on the 1,000-point cube: the series and its
    refinement diverge, GMRES with D^{-1} (K = 0) or a one-term series (K = 1)
    as preconditioner reaches x* for every column, also with short cycles
    (restart 10, so several restarts)."""
    assert series.rho(cube.H) > 1
    for K, restart in ((0, 0), (0, 10), (1, 10)):
        _say(f"gmres {cube.name} K={K} restart={restart}")
        x, st = cube.h.solve(_dev(cube.b), K=K, kind=hmps.PS_GMRES, max_passes=2000,
                             refine_tol=RES_TOL, restart=restart, stats=True)
        _check(cube, _host(x), st)
        if restart:
            assert max(s["passes"] for s in st) > restart


def test_gmres_ragged_leaves_each_level(ragged):
    """Seven right-hand sides on ragged leaves (40 / 39 points), at the leaf
    level and every coarser far level, against x* of Z_l at that level."""
    for lev in [-1] + sorted(ragged.H.far_levels, reverse=True):
        _say(f"gmres {ragged.name} nrhs=7 level={lev}")
        x, st = ragged.h.solve(_dev(ragged.b), K=2, level=lev, kind=hmps.PS_GMRES,
                               max_passes=400, refine_tol=RES_TOL, stats=True)
        _check(ragged, _host(x), st, lev)


def test_gmres_matrix_core_path():
    """Sixteen right-hand sides on the matrix-core kernels (forced from one
    right-hand side on) for both the preconditioner and the products with
    Z_l."""
    case = Case("sphere_2200_leaf68", W.sphere_problem(2200, math.sqrt(2200 / 1536)), 68, 1e-4, 16)
    case.h.tune(mm_min_rhs=1)
    try:
        for prec in (hmps.HM_F64, hmps.HM_F32_APPLY):
            _say(f"gmres {case.name} nrhs=16 mfma precision={prec}")
            x, st = case.h.solve(_dev(case.b), K=3, precision=prec, kind=hmps.PS_GMRES,
                                 max_passes=300, refine_tol=RES_TOL, stats=True)
            _check(case, _host(x), st)
    finally:
        case.h.tune(mm_min_rhs=-1)
    case.h.close()


def test_gmres_budget_and_zero_column(sphere):
    """A step budget too small for the tolerance: the call returns with the
    column flagged diverged after exactly that many steps, x is the iterate
    reached (its residual as reported); a zero right-hand side gives x = 0
    with no steps."""
    b = np.stack([sphere.b.reshape(-1), np.zeros(sphere.prob.n, complex)], axis=1)
    _say(f"gmres {sphere.name} budget 3, zero column")
    x, st = sphere.h.solve(_dev(b), K=0, kind=hmps.PS_GMRES, max_passes=3,
                           refine_tol=1e-14, stats=True)
    x = _host(x)
    assert st[0]["diverged"] == 1 and st[0]["passes"] == 3
    res = _oracle_resid(sphere.H, x[:, :1], b[:, :1])
    assert abs(st[0]["resid_rel"] - res[0]) <= 1e-3 * res[0]
    assert 1e-14 < st[0]["resid_rel"] < 1.0
    assert st[1]["passes"] == 0 and st[1]["resid_rel"] == 0.0 and st[1]["diverged"] == 0
    assert np.all(x[:, 1] == 0)


def test_gmres_deterministic(sphere):
    _say(f"gmres {sphere.name} determinism")
    b = _dev(sphere.b)
    x1 = _host(sphere.h.solve(b, K=2, kind=hmps.PS_GMRES, max_passes=200, refine_tol=RES_TOL))
    x2 = _host(sphere.h.solve(b, K=2, kind=hmps.PS_GMRES, max_passes=200, refine_tol=RES_TOL))
    assert np.array_equal(x1, x2)


def test_gmres_argument_errors(sphere):
    lib = hmps._lib()
    b = _dev(sphere.b)
    x = torch.empty_like(b)
    n = sphere.prob.n

    def call(h, o, nrhs=1):
        return lib.ps_solve(h, C.byref(o), C.c_void_p(b.data_ptr()), n, C.c_void_p(x.data_ptr()),
                            n, nrhs, None, None)

    G = hmps.PS_GMRES
    assert call(sphere.h.handle, hmps.ps_opts(0, -1, 0, G, 10, 1e-9, 65)) == hmps.HM_EINVAL
    assert call(sphere.h.handle, hmps.ps_opts(0, -1, 0, G, 10, 1e-9, -1)) == hmps.HM_EINVAL
    assert call(sphere.h.handle, hmps.ps_opts(0, -1, 0, G, 0, 1e-9, 0)) == hmps.HM_EINVAL
    assert call(sphere.h.handle, hmps.ps_opts(0, -1, 0, G, 10, 0.0, 0)) == hmps.HM_EINVAL
    assert call(sphere.h.handle, hmps.ps_opts(0, -1, 0, 5, 10, 1e-9, 0)) == hmps.HM_EINVAL  # no such kind
    probs = [W.sphere_problem(200, 0.4), W.sphere_problem(150, 0.35, seed=7)]
    # a batched handle is taken (one Krylov space over both instances); with
    # b = 0 every instance norm is zero and the solution is x = 0
    _say("gmres batched handle, b = 0")
    hb = hmps.HMatrix(probs, 32, 1.0, 1e-4)
    bb = _dev(np.zeros(350, complex))
    xb = torch.full_like(bb, complex(np.nan, np.nan))
    o = hmps.ps_opts(0, -1, 0, G, 10, 1e-9, 0)
    assert lib.ps_solve(hb.handle, C.byref(o), C.c_void_p(bb.data_ptr()), 350,
                        C.c_void_p(xb.data_ptr()), 350, 1, None, None) == hmps.HM_OK
    assert not np.any(_host(xb))
    hb.close()


@pytest.mark.parametrize("restart", [1, 2, 64])
def test_gmres_restart_lengths(sphere, restart):
    """The smallest cycles (one and two basis vectors, restarted every step
    or two) and the largest basis (64) reach x* as well."""
    _say(f"gmres {sphere.name} K=4 restart={restart}")
    x, st = sphere.h.solve(_dev(sphere.b), K=4, kind=hmps.PS_GMRES, max_passes=2000,
                           refine_tol=RES_TOL, restart=restart, stats=True)
    _check(sphere, _host(x), st)
