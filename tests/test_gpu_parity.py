"""GPU parity of libhmps against the FP64 oracle, through the C-ABI.

Tolerances (relative 2-norm per right-hand side, max over right-hand sides):
  FP64 path vs oracle x_K                1e-10
  FP32 apply (before refinement) vs x_K  1e-4
  refinement vs oracle x* = Z_l^{-1} b   1e-8
  H-matvec FP64 vs oracle                1e-12
"""
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
TOL_REFINE = 1e-8


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
    def __init__(self, name, prob, leaf, tol, nrhs=1, flags=0):
        self.name = name
        self.prob = prob
        self.H = hmatrix.HMatrix(prob, leaf, 1.0, tol)
        _say(f"build {name} n={prob.n} leaf={leaf}")
        self.h = hmps.HMatrix(prob, leaf, 1.0, tol, flags=flags)
        self.b = W.plane_waves(prob.xyz, W.directions(nrhs, 3)) if nrhs > 1 else \
            W.plane_waves(prob.xyz, W.Z_HAT)


@pytest.fixture(scope="module")
def sphere():
    return Case("sphere_1536", W.sphere_small().problem, 64, 1e-4)


@pytest.fixture(scope="module")
def sphere_levels():
    return Case("sphere_1200_leaf32", W.sphere_problem(1200, math.sqrt(1200 / 1536)), 32, 1e-6, 3)


@pytest.fixture(scope="module")
def cube():
    return Case("cube_1000_leaf32", W.cube_problem(10, 10 / 16), 32, 1e-5, 3)


@pytest.fixture(scope="module")
def ragged():
    return Case("sphere_1000_leaf40", W.sphere_problem(1000, math.sqrt(1000 / 1536)), 40, 1e-4, 7)


@pytest.fixture(scope="module")
def ragged_depth():
    """Leaves at depths 5 and 6 (sizes 68 and 34/35); far blocks on levels 5
    and 6, some of them with a one-leaf row cluster at level 5."""
    return Case("sphere_2200_leaf68", W.sphere_problem(2200, math.sqrt(2200 / 1536)), 68, 1e-4, 3)


def test_series_ragged_depths_each_level(ragged_depth):
    c = ragged_depth
    for lev in [-1] + list(reversed(c.H.far_levels)):
        for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
            _say(f"series {c.name} level={lev} precision={prec}")
            x = _host(c.h.solve(_dev(c.b), K=3, level=lev, precision=prec))
            assert_close(x, series.series(c.H, c.b, 3, lev), tol, (lev, prec))
        _say(f"hmat_apply {c.name} level={lev}")
        y = _host(c.h.apply(_dev(c.b), level=lev))
        assert_close(y, series.apply_Z(c.H, c.b, lev), 1e-12)


def test_series_f64_sphere(sphere):
    _say("series f64 sphere_1536 K=4 leaf level")
    x = _host(sphere.h.solve(_dev(sphere.b), K=4))
    ref = series.series(sphere.H, sphere.b, 4)
    assert_close(x, ref, TOL_F64)


@pytest.mark.parametrize("K", [0, 1, 3])
def test_series_f64_each_level(sphere_levels, K):
    c = sphere_levels
    for lev in [-1] + list(reversed(c.H.far_levels)):
        _say(f"series f64 {c.name} K={K} level={lev}")
        x = _host(c.h.solve(_dev(c.b), K=K, level=lev))
        ref = series.series(c.H, c.b, K, lev)
        assert_close(x, ref, TOL_F64, (K, lev))


def test_series_f64_volume(cube):
    _say("series f64 cube_1000 K=5")
    x = _host(cube.h.solve(_dev(cube.b), K=5))
    ref = series.series(cube.H, cube.b, 5)
    assert_close(x, ref, TOL_F64)


@pytest.mark.parametrize("nrhs", [1, 2, 5, 7])
def test_series_ragged_leaves_many_rhs(ragged, nrhs):
    b = ragged.b[:, :nrhs]
    _say(f"series f64 {ragged.name} nrhs={nrhs}")
    x = _host(ragged.h.solve(_dev(b), K=4))
    ref = series.series(ragged.H, b, 4)
    assert_close(x, ref, TOL_F64)


@pytest.mark.parametrize("precision", [hmps.HM_F64, hmps.HM_F32_APPLY])
def test_hmatvec(sphere_levels, cube, precision):
    tol = 1e-12 if precision == hmps.HM_F64 else 1e-6
    for c in (sphere_levels, cube):
        g = np.random.default_rng(1)
        x = g.standard_normal((c.prob.n, 2)) + 1j * g.standard_normal((c.prob.n, 2))
        for lev in [-1] + list(c.H.far_levels):
            _say(f"hmat_apply {c.name} precision={precision} level={lev}")
            y = _host(c.h.apply(_dev(x), level=lev, precision=precision))
            ref = series.apply_Z(c.H, x, lev)
            assert_close(y, ref, tol, (c.name, lev))


def test_series_f32_apply(sphere, cube):
    for c, K in ((sphere, 4), (cube, 5)):
        _say(f"series f32 {c.name}")
        x = _host(c.h.solve(_dev(c.b), K=K, precision=hmps.HM_F32_APPLY))
        ref = series.series(c.H, c.b, K)
        assert_close(x, ref, TOL_F32)


@pytest.mark.parametrize("precision", [hmps.HM_F32_APPLY, hmps.HM_F64])
def test_refine_reaches_exact_solution(sphere, precision):
    """rho(D^{-1} R)^{K+1} < 1 on this sphere: refinement converges to
    x* = Z_l^{-1} b of the H-matrix (dense LU in the oracle)."""
    rho = series.rho(sphere.H)
    assert rho ** 5 < 1
    _say(f"refine sphere_1536 precision={precision}")
    x, st = sphere.h.solve(_dev(sphere.b), K=4, precision=precision, kind=hmps.PS_REFINE,
                           max_passes=200, refine_tol=1e-10, stats=True)
    x = _host(x)
    xs = series.solve_exact(sphere.H, sphere.b)
    assert_close(x, xs, TOL_REFINE)
    assert st[0]["diverged"] == 0 and 1 <= st[0]["passes"] < 200


def test_stats_growth(sphere):
    _, terms = series.series(sphere.H, sphere.b, 4, return_terms=True)
    g_ref = np.linalg.norm(terms[-1]) / np.linalg.norm(terms[0])
    _say("stats sphere_1536")
    x, st = sphere.h.solve(_dev(sphere.b), K=4, stats=True)
    assert abs(st[0]["growth"] - g_ref) <= 1e-9 * g_ref
    assert st[0]["diverged"] == (1 if g_ref > 1 else 0)
    assert st[0]["t_ms"] > 0


def test_single_leaf_is_direct_solve():
    prob = W.sphere_problem(50, 0.3)
    _say("single leaf n=50")
    h = hmps.HMatrix(prob, 64)
    b = W.plane_waves(prob.xyz, W.Z_HAT)
    from oracle import entries
    ref = np.linalg.solve(entries.dense(prob), b)
    for K in (0, 2):
        x = _host(h.solve(_dev(b), K=K))
        assert_close(x, ref, TOL_F64)


def test_deterministic(sphere):
    _say("determinism sphere_1536")
    b = _dev(sphere.b)
    x1 = _host(sphere.h.solve(b, K=4))
    x2 = _host(sphere.h.solve(b, K=4))
    assert np.array_equal(x1, x2)


def test_argument_errors(sphere):
    import ctypes as C
    lib = hmps._lib()
    b = _dev(sphere.b)
    x = torch.empty_like(b)
    n = sphere.prob.n
    o = hmps.ps_opts(4, 99, 0, 0, 0, 1e-9)  # level beyond the leaf level
    st = lib.ps_solve(sphere.h.handle, C.byref(o), C.c_void_p(b.data_ptr()), n,
                      C.c_void_p(x.data_ptr()), n, 1, None, None)
    assert st == hmps.HM_EINVAL
    o = hmps.ps_opts(-1, -1, 0, 0, 0, 1e-9)
    assert lib.ps_solve(sphere.h.handle, C.byref(o), C.c_void_p(b.data_ptr()), n,
                        C.c_void_p(x.data_ptr()), n, 1, None, None) == hmps.HM_EINVAL
    o = hmps.ps_opts(4, -1, 0, 0, 0, 1e-9)
    assert lib.ps_solve(sphere.h.handle, C.byref(o), C.c_void_p(b.data_ptr()), n - 1,
                        C.c_void_p(x.data_ptr()), n, 1, None, None) == hmps.HM_EINVAL
    assert lib.ps_solve(sphere.h.handle, C.byref(o), None, n, None, n, 0, None, None) == hmps.HM_OK


def test_export_lu_factors_reconstruct_diagonal(tmp_path):
    """The device LU (with pivots) reproduces the leaf self-blocks."""
    prob = W.sphere_problem(300, 0.5)
    _say("export lu n=300")
    h = hmps.HMatrix(prob, 40, flags=hmps.HM_BUILD_KEEP_HOST)
    p = str(tmp_path / "h.bin")
    h.export(p)
    E = hmps.read_export(p)
    lo, ls = E["leaf_off"], E["leaf_size"]
    dl = 0
    for a in range(len(ls)):
        m = ls[a]
        LU = E["diag_lu"][dl:dl + m * m].reshape(m, m).T
        piv = E["diag_piv"][lo[a]:lo[a] + m]
        dl += m * m
        blk = [row for row in E["near"] if row[0] == a and row[1] == a][0]
        D = E["near_data"][blk[2]:blk[2] + m * m].reshape(m, m).T
        L = np.tril(LU, -1) + np.eye(m)
        U = np.triu(LU)
        A = D.copy()
        for k in range(m):
            A[[k, piv[k]]] = A[[piv[k], k]]
        assert np.linalg.norm(L @ U - A) <= 1e-13 * np.linalg.norm(D)


def test_device_entry_fill_matches_host_fill():
    """Near entries computed on the device (the default build) give the
    operator of the host's entries (HM_BUILD_KEEP_HOST): H-matvec and series
    agree to rounding on a surface, a volume and a batched (surface + volume)
    handle; the device fill refuses coincident points as the host does."""
    cases = [("sphere_1200", W.sphere_problem(1200, math.sqrt(1200 / 1536)), 1e-6),
             ("cube_1000", W.cube_problem(10, 10 / 16), 1e-5),
             ("batched", [W.sphere_problem(700, math.sqrt(700 / 1536), instance=3),
                          W.cube_problem(8, 8 / 16, instance=2)], 1e-5)]
    for name, prob, tol in cases:
        _say(f"device vs host entry fill: {name}")
        parts = prob if isinstance(prob, list) else [prob]
        b = np.vstack([W.plane_waves(p.xyz, W.directions(3, 3, instance=40 + i))
                       for i, p in enumerate(parts)])
        hd = hmps.HMatrix(prob, 32, 1.0, tol)
        hh = hmps.HMatrix(prob, 32, 1.0, tol, flags=hmps.HM_BUILD_KEEP_HOST)
        assert_close(_host(hd.apply(_dev(b))), _host(hh.apply(_dev(b))), 1e-14, name)
        assert_close(_host(hd.solve(_dev(b), K=3)), _host(hh.solve(_dev(b), K=3)), 1e-13, name)
        hd.close()
        hh.close()
    p = W.sphere_problem(300, 0.5)
    p.xyz[5] = p.xyz[6]
    _say("device entry fill: coincident points")
    with pytest.raises(hmps.HmpsError) as e:
        hmps.HMatrix(p, 40)
    assert e.value.status == hmps.HM_EINVAL


@pytest.mark.timeout(900)
def test_full_size_sphere_24576():
    """The 24,576-point sphere (leaf <= 128, tol 1e-4, K = 4) at the leaf
    level in FP64, and at the coarsest level, against the oracle."""
    wl = W.sphere_large()
    _say("oracle build sphere_24576")
    H = hmatrix.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol)
    _say("library build sphere_24576")
    h = hmps.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol)
    b = wl.rhs()
    for lev in (-1, min(H.far_levels)):
        _say(f"series f64 sphere_24576 level={lev}")
        x = _host(h.solve(_dev(b), K=4, level=lev))
        assert_close(x, series.series(H, b, 4, lev), TOL_F64)
    _say("series f32 sphere_24576")
    x = _host(h.solve(_dev(b), K=4, precision=hmps.HM_F32_APPLY))
    assert_close(x, series.series(H, b, 4), TOL_F32)


@pytest.mark.timeout(900)
def test_full_size_cube_32768():
    """The 32^3 dielectric cube (leaf <= 128, tol 1e-5, K = 5, 64 plane
    waves) in the configuration the benchmark times (autotuned: matrix-core
    kernels), FP64 and FP32 blocks, against the oracle's x_K."""
    wl = W.cube_volume()
    _say("oracle build cube_32768")
    H = hmatrix.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol)
    _say("library build cube_32768")
    h = hmps.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol)
    b = wl.rhs()
    _say("autotune cube_32768 nrhs=64")
    best, _ = h.autotune(b.shape[1], K=wl.K)
    assert b.shape[1] >= best["mm_min_rhs"]  # the matrix-core kernels, as timed
    ref = series.series(H, b, wl.K)
    _say("series f64 cube_32768")
    x = _host(h.solve(_dev(b), K=wl.K))
    assert_close(x, ref, TOL_F64)
    _say("series f32 cube_32768")
    x = _host(h.solve(_dev(b), K=wl.K, precision=hmps.HM_F32_APPLY))
    assert_close(x, ref, TOL_F32)
    h.close()


def test_batched_instances_match_per_instance_oracle():
    """One batched handle (three instances: sphere, volume cube, a sphere
    without far blocks) solves every instance as its own oracle would, at the
    leaf level and one and two levels above each instance's leaf level."""
    probs = [W.sphere_problem(1200, math.sqrt(1200 / 1536)),
             W.cube_problem(10, 10 / 16),
             W.sphere_problem(450, math.sqrt(450 / 1536), seed=7)]
    leaf, tol, K, nrhs = 32, 1e-5, 3, 3
    _say("build batched sphere_1200 + cube_1000 + sphere_450 leaf=32")
    h = hmps.HMatrix(probs, leaf, 1.0, tol)
    Hs = [hmatrix.HMatrix(p, leaf, 1.0, tol) for p in probs]
    bs = [W.plane_waves(p.xyz, W.directions(nrhs, 3, instance=i)) for i, p in enumerate(probs)]
    b = np.vstack(bs)
    top = hmps.HM_MAX_LEVELS - 1
    for d in (0, 1, 2):
        for prec, tol_s in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
            _say(f"batched series level=top-{d} precision={prec}")
            x = _host(h.solve(_dev(b), K=K, level=top - d, precision=prec))
            for i, H in enumerate(Hs):
                o0, o1 = h.offsets[i], h.offsets[i + 1]
                ref = series.series(H, bs[i], K, H.L - d)
                assert_close(x[o0:o1], ref, tol_s, (i, d, prec))
        _say(f"batched hmat_apply level=top-{d}")
        y = _host(h.apply(_dev(b), level=top - d))
        for i, H in enumerate(Hs):
            o0, o1 = h.offsets[i], h.offsets[i + 1]
            assert_close(y[o0:o1], series.apply_Z(H, bs[i], H.L - d), 1e-12, (i, d))
    x1 = _host(h.solve(_dev(b), K=K))
    x0 = _host(h.solve(_dev(b), K=K, level=-1))
    assert np.array_equal(x0, x1)
    # GMRES with D^{-1} over all three instances at once reaches each one's
    # own x*; column 1 of the last instance is zero (its x stays near zero,
    # and the stopping norm is the smallest nonzero ||b_i||)
    _say("batched gmres jacobi f64")
    bs[2][:, 1] = 0
    b = np.vstack(bs)
    xg, stg = h.solve(_dev(b), K=0, precision=hmps.HM_F64, kind=hmps.PS_GMRES, max_passes=500,
                      refine_tol=1e-11, stats=True)
    assert all(s_["diverged"] == 0 for s_ in stg), stg
    xg = _host(xg)
    for i, H in enumerate(Hs):
        o0, o1 = h.offsets[i], h.offsets[i + 1]
        cols = [c for c in range(nrhs) if np.any(bs[i][:, c])]
        assert_close(xg[o0:o1, cols], series.solve_exact(H, bs[i][:, cols]), 1e-8, ("gmres", i))
    o0, o1 = h.offsets[2], h.offsets[3]
    assert np.linalg.norm(xg[o0:o1, 1]) <= 1e-8 * np.linalg.norm(xg[o0:o1, 0])
    h.close()


# ---------------------------------------------------------------- many RHS
@pytest.fixture(scope="module")
def many_rhs(ragged_depth):
    """64 plane waves on the ragged-depth sphere (leaves of 34/35 and 68)."""
    c = ragged_depth
    return c, W.plane_waves(c.prob.xyz, W.directions(64, 9))


@pytest.mark.parametrize("nrhs", [1, 16, 17, 33, 64])
def test_mfma_series_each_level(many_rhs, nrhs):
    """The matrix-core kernels (forced from one right-hand side on) against
    the oracle, at every level, FP64 (4M) and FP32 (3M)."""
    c, B = many_rhs
    b = B[:, :nrhs]
    c.h.tune(mm_min_rhs=1)
    try:
        for lev in [-1] + list(reversed(c.H.far_levels)):
            ref = series.series(c.H, b, 3, lev)
            for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
                _say(f"mfma series {c.name} nrhs={nrhs} level={lev} precision={prec}")
                x = _host(c.h.solve(_dev(b), K=3, level=lev, precision=prec))
                assert_close(x, ref, tol, (lev, prec))
            _say(f"mfma hmat_apply {c.name} nrhs={nrhs} level={lev}")
            y = _host(c.h.apply(_dev(b), level=lev))
            assert_close(y, series.apply_Z(c.H, b, lev), 1e-12)
    finally:
        c.h.tune(mm_min_rhs=-1)


def test_mfma_matches_streaming_path(many_rhs):
    """Both kernel families on the same 24 right-hand sides: FP64 results
    agree to rounding; FP32 to the FP32 bar."""
    c, B = many_rhs
    b = _dev(B[:, :24])
    c.h.tune(mm_min_rhs=1000)
    _say("streaming path nrhs=24")
    x_s = _host(c.h.solve(b, K=4))
    x_s32 = _host(c.h.solve(b, K=4, precision=hmps.HM_F32_APPLY))
    c.h.tune(mm_min_rhs=-1)
    assert c.h.tuning()["mm_min_rhs"] == 8
    _say("mfma path nrhs=24")
    x_m = _host(c.h.solve(b, K=4))
    x_m32 = _host(c.h.solve(b, K=4, precision=hmps.HM_F32_APPLY))
    assert_close(x_m, x_s, 1e-12)
    assert_close(x_m32, x_s, TOL_F32)
    assert_close(x_s32, x_s, TOL_F32)


def test_mfma_volume_and_large_leaves():
    """Volume kernel (contrast folded into W) and leaves up to 250 points
    (four 16-row tiles per wave) on the matrix-core path, 20 RHS."""
    cases = [("cube_1728_leaf40", W.cube_problem(12, 12 / 16), 40, 1e-5),
             ("sphere_6000_leaf250", W.sphere_problem(6000, math.sqrt(6000 / 1536)), 250, 1e-4)]
    for name, prob, leaf, tol in cases:
        _say(f"build {name}")
        H = hmatrix.HMatrix(prob, leaf, 1.0, tol)
        h = hmps.HMatrix(prob, leaf, 1.0, tol)
        b = W.plane_waves(prob.xyz, W.directions(20, 11))
        for lev in [-1] + list(H.far_levels):
            ref = series.series(H, b, 3, lev)
            for prec, tol_s in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
                _say(f"mfma series {name} level={lev} precision={prec}")
                x = _host(h.solve(_dev(b), K=3, level=lev, precision=prec))
                assert_close(x, ref, tol_s, (name, lev, prec))
        h.close()


def test_retuned_work_lists_same_result(many_rhs):
    """Re-splitting the term work over another workgroup count changes only
    the rounding order."""
    c, B = many_rhs
    b = _dev(B[:, :5])
    x0 = _host(c.h.solve(b, K=4))
    default = c.h.tuning()["term_wgs"]
    try:
        for wgs in (37, 3000):
            _say(f"retune term_wgs={wgs}")
            c.h.tune(term_wgs=wgs)
            assert c.h.tuning()["term_wgs"] == wgs
            x1 = _host(c.h.solve(b, K=4))
            assert_close(x1, x0, 1e-13)
    finally:
        c.h.tune(term_wgs=-1)
    assert c.h.tuning()["term_wgs"] == default
    assert np.array_equal(_host(c.h.solve(b, K=4)), x0)


# ---------------------------------------------------------------- refinement, graphs, tuning
def test_refine_fixed_matches_adaptive(sphere):
    """PS_REFINE_FIXED with the pass count adaptive refinement needed gives
    the same x, bit for bit (same kernels, same order)."""
    b = _dev(sphere.b)
    _say("adaptive refine sphere_1536 f32")
    x1, st = sphere.h.solve(b, K=4, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE,
                            max_passes=200, refine_tol=1e-10, stats=True)
    p = st[0]["passes"]
    _say(f"fixed refine passes={p}")
    x2, st2 = sphere.h.solve(b, K=4, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE_FIXED,
                             max_passes=p, refine_tol=1e-10, stats=True)
    assert np.array_equal(_host(x1), _host(x2))
    assert st2[0]["passes"] == p and st2[0]["diverged"] == 0
    assert st2[0]["resid_rel"] == st[0]["resid_rel"]


def test_batched_refine_each_instance_reaches_xstar():
    """Refinement on a batched handle stops on the per-instance criterion:
    every instance reaches its own x* = Z_l^{-1} b to 1e-8 (FP32 blocks)."""
    probs = [W.sphere_problem(n, math.sqrt(n / 1536), instance=i)
             for i, n in enumerate((700, 1100, 300))]
    h = hmps.HMatrix(probs, 64, 1.0, 1e-4)
    Hs = [hmatrix.HMatrix(p, 64, 1.0, 1e-4) for p in probs]
    bs = [W.plane_waves(p.xyz, W.directions(2, 3, instance=i)) for i, p in enumerate(probs)]
    for H in Hs:
        assert series.rho(H) ** 5 < 1
    _say("batched refine 3 instances f32")
    x, st = h.solve(_dev(np.vstack(bs)), K=4, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE,
                    max_passes=300, refine_tol=1e-11, stats=True)
    x = _host(x)
    for i, H in enumerate(Hs):
        o0, o1 = h.offsets[i], h.offsets[i + 1]
        assert_close(x[o0:o1], series.solve_exact(H, bs[i]), TOL_REFINE, i)
    assert all(s["diverged"] == 0 for s in st)
    h.close()


def test_graph_replay_matches_eager(sphere, many_rhs):
    """ps_solve recorded by stream capture (series on the streaming and the
    MFMA kernels, fixed-pass refinement) and replayed several times, with
    eager work and synchronisation between replays: every replay equals the
    eager result bit for bit."""
    c, B = many_rhs
    cases = [(sphere.h, _dev(sphere.b), dict(K=4)),
             (c.h, _dev(B[:, :16]), dict(K=3, precision=hmps.HM_F32_APPLY)),
             (sphere.h, _dev(sphere.b), dict(K=4, precision=hmps.HM_F32_APPLY,
                                            kind=hmps.PS_REFINE_FIXED, max_passes=6))]
    for h, b, kw in cases:
        _say(f"graph capture {kw}")
        ref = _host(h.solve(b, **kw))
        out = torch.empty_like(b.t().contiguous() if b.dim() == 2 else b.reshape(1, -1))
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            h.solve(b, out=out, **kw)  # sizes the workspace before capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            h.solve(b, out=out, **kw)
        for rep in range(3):
            out.zero_()
            g.replay()
            torch.cuda.synchronize()
            got = out.reshape(-1).cpu().numpy() if b.dim() == 1 else out.t().cpu().numpy()
            assert np.array_equal(got, ref), rep
            _host(h.solve(b, **kw))  # eager work between replays
        del g


def test_autotune_choice_keeps_results(many_rhs):
    c, B = many_rhs
    b = _dev(B[:, :20])
    ref = _host(c.h.solve(b, K=3, precision=hmps.HM_F32_APPLY))
    _say("autotune nrhs=20 f32")
    best, ms = c.h.autotune(20, K=3, precision=hmps.HM_F32_APPLY)
    assert ms > 0 and c.h.tuning() == best
    # tuned at 20 right-hand sides: one right-hand side keeps the streaming kernels
    assert 2 <= best["mm_min_rhs"] <= 21
    x = _host(c.h.solve(b, K=3, precision=hmps.HM_F32_APPLY))
    assert_close(x, ref, 1e-5)
    c.h.tune(mm_min_rhs=-1, term_wgs=-1, rhs_tile=-1, inrow_pct=-1)


def test_refine_stops_when_the_series_does_not_contract(cube):
    """rho(D^{-1} R) = 1.13 on the 1,000-point cube: refinement cannot reach
    x*; the corrections grow and the solve stops early, flagged diverged."""
    rho = series.rho(cube.H)
    assert rho ** 6 > 1
    _say("refine cube_1000 (divergent)")
    x, st = cube.h.solve(_dev(cube.b), K=5, precision=hmps.HM_F64, kind=hmps.PS_REFINE,
                         max_passes=200, refine_tol=1e-10, stats=True)
    for s in st:
        assert s["diverged"] == 1 and s["passes"] < 60, s


# ---------------------------------------------------------------- half storage
def test_half_storage_matches_oracle_and_panels(ragged_depth, sphere_levels, cube):
    """One right-hand side on half storage: surface problems (symmetric) and
    a volume problem (through its symmetric part A, Z = A diag(chi)): the
    scaled series (D = C C^T, each off-diagonal near block of
    S = C^{-1} R C^{-T} read once) against the oracle and against the
    premultiplied panels, at every level (levels above the leaf level add
    stage A on the scaled W and the global far columns), FP64 and FP32
    blocks, and over several workgroup counts.  The one-RHS H-matvec on
    half storage (Z x = C (I + S) C^T x) against the oracle's Z x and the
    panels' H-matvec."""
    for c in (ragged_depth, sphere_levels, cube):
        b = c.b[:, 0]
        c.h.tune(half_storage=-1)
        assert c.h.tuning()["half_storage"] == 1
        try:
            for lev in [-1] + list(reversed(c.H.far_levels)):
                ref = series.series(c.H, b, 3, lev)
                ref_z = series.apply_Z(c.H, b, lev)
                c.h.tune(half_storage=2)
                x_p = _host(c.h.solve(_dev(b), K=3, level=lev))
                y_p = _host(c.h.apply(_dev(b), level=lev))
                for wgs in (-1, 37, 1):
                    c.h.tune(half_storage=1, term_wgs=wgs)
                    for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
                        _say(f"half storage {c.name} level={lev} wgs={wgs} precision={prec}")
                        x = _host(c.h.solve(_dev(b), K=3, level=lev, precision=prec))
                        assert_close(x, ref, tol, (lev, wgs, prec))
                        if prec == hmps.HM_F64:
                            assert_close(x, x_p, 1e-12, (lev, wgs))
                        y = _host(c.h.apply(_dev(b), level=lev, precision=prec))
                        tol_y = 1e-12 if prec == hmps.HM_F64 else 1e-6
                        assert_close(y, ref_z, tol_y, (lev, wgs, prec))
                        if prec == hmps.HM_F64:
                            assert_close(y, y_p, 1e-13, (lev, wgs))
        finally:
            c.h.tune(half_storage=-1, term_wgs=-1)
        # the half-storage product reads fewer entries than the panels
        info = c.h.info()
        L = info["leaf_level"]
        assert 0 < info["half_entries"][L] < info["series_entries"][L]


def test_half_storage_deterministic_and_refine(sphere):
    """Fixed reduction order: repeated solves are bit-identical.  Refinement
    (its residual b - Z x is the H-matvec epilogue with alpha = -1, beta = 1)
    on the half path reaches x* like the panels."""
    b = _dev(sphere.b)
    x0 = _host(sphere.h.solve(b, K=4))
    for _ in range(3):
        assert np.array_equal(_host(sphere.h.solve(b, K=4)), x0)
    xs = series.solve_exact(sphere.H, sphere.b)
    kw = dict(K=4, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE, max_passes=200,
              refine_tol=1e-10)
    _say("half storage refine sphere_1536")
    x1 = _host(sphere.h.solve(b, **kw))
    sphere.h.tune(half_storage=2)
    try:
        x2 = _host(sphere.h.solve(b, **kw))
    finally:
        sphere.h.tune(half_storage=-1)
    assert_close(x1, xs, TOL_REFINE)
    assert_close(x2, xs, TOL_REFINE)
    # autotuning for many right-hand sides leaves the one-RHS setting alone
    _say("autotune nrhs=8 keeps half storage")
    try:
        best, _ = sphere.h.autotune(8, K=2)
        assert best["half_storage"] == 1 and sphere.h.tuning()["half_storage"] == 1
        assert np.array_equal(_host(sphere.h.solve(b, K=4)), x0)
    finally:
        sphere.h.tune(mm_min_rhs=-1, term_wgs=-1, rhs_tile=-1, inrow_pct=-1, half_storage=-1)


def _term_launches(h, fn):
    """Series-term launches the handle's profiler counts while fn runs."""
    lib = hmps._lib()
    assert lib.hm_profile_enable(h.handle, 1) == 0
    torch.cuda.synchronize()
    fn()
    torch.cuda.synchronize()
    kt = (hmps.hm_kernel_time * hmps.HM_K_COUNT)()
    assert lib.hm_profile_read(h.handle, kt) == 0
    lib.hm_profile_enable(h.handle, 0)
    return kt[hmps.HM_K_TERM_SERIES].launches


def test_half_multi_term_launch_matches_per_term(sphere, ragged_depth, cube):
    """Where every far block of the level lies between two leaves, the K
    terms of the scaled series run as one launch whose pieces wait for the
    leaves they read (half_storage 1); the result equals the one launch per
    term path (half_storage 3) bit for bit: series of K = 1, 2, 5 terms in
    FP64 and FP32, and fixed-pass refinement, at every level (levels with
    other far blocks take the per-term launches either way)."""
    K_all = (1, 2, 5)
    for c in (sphere, ragged_depth, cube):
        b = _dev(c.b if c.b.ndim == 1 or c.b.shape[1] == 1 else c.b[:, 0])
        for lev in [-1] + list(reversed(c.H.far_levels)):
            for prec in (hmps.HM_F64, hmps.HM_F32_APPLY):
                for K in K_all:
                    _say(f"multi-term {c.name} level={lev} precision={prec} K={K}")
                    c.h.tune(half_storage=3)
                    try:
                        x3 = _host(c.h.solve(b, K=K, level=lev, precision=prec))
                    finally:
                        c.h.tune(half_storage=-1)
                    x1 = _host(c.h.solve(b, K=K, level=lev, precision=prec))
                    assert np.array_equal(x1, x3), (c.name, lev, prec, K)
        kw = dict(K=4, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE_FIXED, max_passes=5)
        _say(f"multi-term {c.name} fixed refinement")
        c.h.tune(half_storage=3)
        try:
            x3 = _host(c.h.solve(b, **kw))
        finally:
            c.h.tune(half_storage=-1)
        assert np.array_equal(_host(c.h.solve(b, **kw)), x3)
    # the sphere's leaf level runs its four terms as one launch
    b = _dev(sphere.b)
    assert _term_launches(sphere.h, lambda: sphere.h.solve(b, K=4)) == 1
    sphere.h.tune(half_storage=3)
    try:
        assert _term_launches(sphere.h, lambda: sphere.h.solve(b, K=4)) == 4
    finally:
        sphere.h.tune(half_storage=-1)


def test_mfma_small_leaves_16rhs_tiles(ragged, cube):
    """Leaves of at most 64 rows (one 16-row tile per wave) with 16-RHS
    tiles on the matrix cores: against the oracle at every level, FP64 (4M)
    and FP32 (3M), for 1, 16 and 23 right-hand sides (one tile, a full tile,
    a ragged second tile), surface and volume, series and H-matvec."""
    for c in (ragged, cube):
        B = W.plane_waves(c.prob.xyz, W.directions(23, 13))
        c.h.tune(mm_min_rhs=1, rhs_tile=16)
        try:
            for nrhs in (1, 16, 23):
                b = B[:, :nrhs]
                for lev in [-1] + list(reversed(c.H.far_levels)):
                    ref = series.series(c.H, b, 3, lev)
                    for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
                        _say(f"small-leaf mfma {c.name} nrhs={nrhs} level={lev} precision={prec}")
                        x = _host(c.h.solve(_dev(b), K=3, level=lev, precision=prec))
                        assert_close(x, ref, tol, (c.name, nrhs, lev, prec))
                    y = _host(c.h.apply(_dev(b), level=lev))
                    assert_close(y, series.apply_Z(c.H, b, lev), 1e-12)
        finally:
            c.h.tune(mm_min_rhs=-1, rhs_tile=-1)


def test_build_without_half_storage(sphere):
    """HM_BUILD_NO_HALF: a surface handle without the half-storage data (for
    many right-hand sides) takes less device memory and solves one
    right-hand side on the premultiplied panels, as a handle with the data
    does when told to use the panels."""
    _say("build without half storage")
    h = hmps.HMatrix(sphere.prob, 64, 1.0, 1e-4, flags=hmps.HM_BUILD_NO_HALF)
    try:
        assert max(h.info()["half_entries"]) == 0
        assert h.info()["device_bytes"] < sphere.h.info()["device_bytes"]
        b = _dev(sphere.b)
        x = _host(h.solve(b, K=4))
        assert_close(x, series.series(sphere.H, sphere.b, 4, -1), TOL_F64)
        sphere.h.tune(half_storage=2)
        try:
            assert_close(x, _host(sphere.h.solve(b, K=4)), 1e-13)
        finally:
            sphere.h.tune(half_storage=-1)
    finally:
        h.close()


def test_half_storage_batched_surfaces_one_rhs():
    """A batched handle of surface instances (one without far blocks) with
    one right-hand side runs the scaled half-storage series: every instance
    matches its own oracle at the leaf level and above, and refinement in
    the scaled basis reaches each instance's x*."""
    probs = [W.sphere_problem(n, math.sqrt(n / 1536), instance=i)
             for i, n in enumerate((900, 1400, 300))]
    h = hmps.HMatrix(probs, 48, 1.0, 1e-5)
    Hs = [hmatrix.HMatrix(p, 48, 1.0, 1e-5) for p in probs]
    bs = [W.plane_waves(p.xyz, W.directions(1, 3, instance=i))[:, 0] for i, p in enumerate(probs)]
    b = np.concatenate(bs)
    assert h.tuning()["half_storage"] == 1 and max(h.info()["half_entries"]) > 0
    top = hmps.HM_MAX_LEVELS - 1
    for d in (0, 1):
        for prec, tol_s in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
            _say(f"half storage batched level=top-{d} precision={prec}")
            x = _host(h.solve(_dev(b), K=3, level=top - d, precision=prec))
            for i, H in enumerate(Hs):
                o0, o1 = h.offsets[i], h.offsets[i + 1]
                ref = series.series(H, bs[i], 3, H.L - d)
                assert_close(x[o0:o1], ref, tol_s, (i, d, prec))
    for H in Hs:
        assert series.rho(H) ** 4 < 1
    _say("half storage batched refine")
    x, st = h.solve(_dev(b), K=3, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE,
                    max_passes=300, refine_tol=1e-11, stats=True)
    x = _host(x)
    for i, H in enumerate(Hs):
        o0, o1 = h.offsets[i], h.offsets[i + 1]
        assert_close(x[o0:o1], series.solve_exact(H, bs[i]), TOL_REFINE, i)
    assert st[0]["diverged"] == 0
    h.close()


# ---------------------------------------------------------------- the batched configuration
def _c4_sizes():
    """16 ragged surface instances: 14 seeded sizes of the 256-instance
    batch (those up to 3,000 points, so the oracle's dense x* stays cheap),
    one fully dense instance (512 points, no far block) and one of 8,192."""
    s = [int(n) for n in W.batched_sizes(256) if n <= 3000][:14]
    return s + [512, 8192]


@pytest.mark.timeout(900)
def test_batched_16_instances_mfma_graph_replay():
    """The batched configuration on its own path: one handle of 16 ragged
    instances, 16 plane waves each, the matrix-core term and stage-A kernels
    (the default from 8 right-hand sides on), FP64 (4M) and FP32 (3M) blocks,
    eager and replayed from captured HIP graphs; every instance against its
    own oracle x_K, and refinement (FP32 blocks, FP64 residual) captured with
    its pass count and replayed, every instance against its own x*.  Then
    the autotuner's choice (what the benchmark times) once more."""
    sizes = _c4_sizes()
    wls = [W.batched_instance(i, n) for i, n in enumerate(sizes)]
    K, nrhs = wls[0].K, wls[0].nrhs
    _say(f"build batched c4 sizes={sizes}")
    h = hmps.HMatrix([w.problem for w in wls], 64, 1.0, 1e-4)
    assert h.tuning()["mm_min_rhs"] <= nrhs
    Hs, bs, refs, xss = [], [], [], []
    for i, w in enumerate(wls):
        _say(f"oracle instance {i} n={sizes[i]}")
        H = hmatrix.HMatrix(w.problem, 64, 1.0, 1e-4)
        if sizes[i] in (512, 8192):
            assert (len(H.far) == 0) == (sizes[i] == 512)
        b = w.rhs()
        Hs.append(H)
        bs.append(b)
        refs.append(series.series(H, b, K))
        xss.append(series.solve_exact(H, b))
        if sizes[i] <= 3000:  # refinement contracts (rho^(K+1) < 1)
            assert series.rho(H) ** (K + 1) < 1
    b = _dev(np.vstack(bs))

    def per_instance(x, want, tol, what):
        for i in range(len(sizes)):
            o0, o1 = h.offsets[i], h.offsets[i + 1]
            assert_close(x[o0:o1], want[i], tol, (what, i, sizes[i]))

    def graph_of(**kw):
        out = torch.empty((nrhs, h.n), dtype=torch.complex128, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            h.solve(b, out=out, **kw)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            h.solve(b, out=out, **kw)
        return g, out

    def replay_equal(g, out, ref, reps=3):
        for rep in range(reps):
            out.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out.t().cpu().numpy(), ref), rep
            _host(h.solve(b, K=K))  # eager work between replays

    assert h.tuning()["mm_multi"] == 2
    for prec, tol in ((hmps.HM_F64, TOL_F64), (hmps.HM_F32_APPLY, TOL_F32)):
        _say(f"batched c4 series precision={prec}")
        x = _host(h.solve(b, K=K, precision=prec))
        per_instance(x, refs, tol, f"series p{prec}")
        # the K terms (stage A included) in one launch, bit for bit the
        # result of one launch per stage A and per term
        assert _term_launches(h, lambda: h.solve(b, K=K, precision=prec)) == K
        h.tune(mm_multi=1)
        assert _term_launches(h, lambda: h.solve(b, K=K, precision=prec)) == 1
        x1 = _host(h.solve(b, K=K, precision=prec))
        assert np.array_equal(x, x1), f"multi-term launch differs from per-term launches p{prec}"
        # replays of the one launch: each starts from the counters and queue
        # the previous launch's last wave cleared
        _say(f"batched c4 multi-term graph precision={prec}")
        g, out = graph_of(K=K, precision=prec)
        replay_equal(g, out, x)
        del g
        h.tune(mm_multi=2)
        _say(f"batched c4 graph precision={prec}")
        g, out = graph_of(K=K, precision=prec)
        replay_equal(g, out, x)
        del g
    _say("batched c4 adaptive refinement f32")
    x, st = h.solve(b, K=K, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE, max_passes=400,
                    refine_tol=1e-10, stats=True)
    x = _host(x)
    passes = max(s_["passes"] for s_ in st)
    assert all(s_["diverged"] == 0 for s_ in st) and passes < 400
    per_instance(x, xss, TOL_REFINE, "refine")
    # GMRES over all instances at once, preconditioned by the FP32 series:
    # stopped against the smallest instance's ||b_i||, so every instance
    # reaches its own x*
    _say("batched c4 gmres series f32")
    xg, stg = h.solve(b, K=K, precision=hmps.HM_F32_APPLY, kind=hmps.PS_GMRES, max_passes=1000,
                      refine_tol=1e-10, stats=True)
    assert all(s_["diverged"] == 0 and s_["resid_rel"] <= 1e-10 for s_ in stg), stg
    per_instance(_host(xg), xss, TOL_REFINE, "gmres")
    _say(f"batched c4 fixed refinement graph passes={passes}")
    g, out = graph_of(K=K, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE_FIXED,
                      max_passes=passes, refine_tol=1e-10)
    out.zero_()
    g.replay()
    torch.cuda.synchronize()
    xg = out.t().cpu().numpy()
    per_instance(xg, xss, TOL_REFINE, "refine graph")
    replay_equal(g, out, xg, reps=2)
    del g
    _say("batched c4 autotune f32")
    best, _ = h.autotune(nrhs, K=K, precision=hmps.HM_F32_APPLY)
    g, out = graph_of(K=K, precision=hmps.HM_F32_APPLY)
    out.zero_()
    g.replay()
    torch.cuda.synchronize()
    per_instance(out.t().cpu().numpy(), refs, TOL_F32, ("autotuned", best))
    del g
    h.close()
