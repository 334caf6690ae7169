"""Pins of the oracle's power series, exact solve, spectral radius and
refinement (Sec. IV, eq. 9-22; convergence condition of Sec. V).

The series is checked against closed forms built from dense matrices with
numpy/scipy routines (solve, matrix powers, eigenvalues), never by re-typing
its own recurrence.
"""
import math

import numpy as np
import scipy.linalg
import pytest

import workloads as W
from oracle import entries, hmatrix, series


@pytest.fixture(scope="module")
def small():
    """N = 1200 sphere (leaf 32): 64 leaves, far blocks on levels 5 and 6."""
    prob = W.sphere_problem(1200, math.sqrt(1200 / 1536.0))
    H = hmatrix.HMatrix(prob, 32, 1.0, 1e-6)
    assert len(H.far_levels) == 2
    g = np.random.default_rng(11)
    b = np.asfortranarray(W.plane_waves(prob.xyz, W.directions(3, 3)))
    return prob, H, b, g


@pytest.fixture(scope="module")
def small_volume():
    prob = W.cube_problem(10, 10 / 16)
    H = hmatrix.HMatrix(prob, 32, 1.0, 1e-6)
    assert H.far
    b = W.plane_waves(prob.xyz, W.directions(2, 3))
    return prob, H, b


def _dense_parts(H, level):
    D = H.dense(level, "D")
    R = H.dense(level, "R")
    return D, R


def test_single_leaf_is_direct_solve():
    """N <= leaf size: R is empty and x_K = D^{-1} b = Z^{-1} b for any K."""
    prob = W.sphere_problem(50, 0.3)
    H = hmatrix.HMatrix(prob, 64)
    b = W.plane_waves(prob.xyz, W.Z_HAT)
    Z = entries.dense(prob)
    ref = np.linalg.solve(Z, b)
    for K in (0, 3):
        assert series.rel_err(series.series(H, b, K), ref) < 1e-13


def test_zero_terms_is_block_jacobi(small):
    """K = 0 gives D x = b with D the leaf self-blocks of the exact Z."""
    prob, H, b, _ = small
    x0 = series.series(H, b, 0)
    Zt = entries.dense(prob)[np.ix_(H.perm, H.perm)]
    D = np.zeros_like(Zt)
    for c in H.leaves:
        sl = slice(c.off, c.off + c.size)
        D[sl, sl] = Zt[sl, sl]
    r = D @ H.to_tree(x0) - H.to_tree(b)
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b)


@pytest.mark.parametrize("level_pick", ["leaf", "coarsest"])
@pytest.mark.parametrize("K", [1, 4])
def test_truncation_identity(small, level_pick, K):
    """x* - x_K = (-M)^{K+1} x*, M = D^{-1} R_l, with x* = Z_l^{-1} b by a
    dense solve: holds for any spectral radius."""
    prob, H, b, _ = small
    level = -1 if level_pick == "leaf" else min(H.far_levels)
    D, R = _dense_parts(H, level)
    M = np.linalg.solve(D, R)
    xs = np.linalg.solve(D + R, H.to_tree(b))
    xK = H.to_tree(series.series(H, b, K, level))
    lhs = xs - xK
    rhs = np.linalg.matrix_power(-M, K + 1) @ xs
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(xs)


def test_truncation_identity_volume(small_volume):
    prob, H, b = small_volume
    D, R = _dense_parts(H, -1)
    M = np.linalg.solve(D, R)
    xs = np.linalg.solve(D + R, H.to_tree(b))
    xK = H.to_tree(series.series(H, b, 5))
    rhs = np.linalg.matrix_power(-M, 6) @ xs
    assert np.linalg.norm(xs - xK - rhs) <= 1e-11 * np.linalg.norm(xs)


def test_series_is_jacobi_iterate(small):
    """x_K is the K-th block-Jacobi iterate x_k = D^{-1}(b - R x_{k-1}) from
    x_0 = D^{-1} b (dense LU solves)."""
    prob, H, b, _ = small
    D, R = _dense_parts(H, -1)
    bt = H.to_tree(b)
    x = np.linalg.solve(D, bt)
    for _ in range(4):
        x = np.linalg.solve(D, bt - R @ x)
    assert np.linalg.norm(x - H.to_tree(series.series(H, b, 4))) <= 1e-12 * np.linalg.norm(x)


def test_refinement_passes_extend_the_series(small):
    """p passes of x += P_K (b - Z_l x) equal the series with (p+1)(K+1) terms."""
    prob, H, b, _ = small
    for K, p in ((2, 1), (1, 3)):
        xr = series.refine(H, b, K, -1, p)
        xl = series.series(H, b, (p + 1) * (K + 1) - 1, -1)
        assert series.rel_err(xr, xl) < 1e-12


def test_rho_matches_eigenvalues(small):
    """Power iteration agrees with the largest |eigenvalue| of dense D^{-1} R_l."""
    prob, H, b, _ = small
    for level in (-1, min(H.far_levels)):
        D, R = _dense_parts(H, level)
        ev = np.max(np.abs(np.linalg.eigvals(np.linalg.solve(D, R))))
        assert abs(series.rho(H, level, iters=300) - ev) <= 0.03 * ev


def test_convergence_when_rho_below_one():
    """rho < 1: ||x_K - x*|| decays geometrically at rate rho."""
    prob = W.sphere_problem(512, math.sqrt(512 / 1536.0))
    H = hmatrix.HMatrix(prob, 64, 1.0, 1e-6)
    rho = series.rho(H, -1, iters=300)
    assert rho < 1.0
    b = W.plane_waves(prob.xyz, W.Z_HAT)
    xs = series.solve_exact(H, b)
    errs = [series.rel_err(series.series(H, b, K), xs) for K in range(0, 60, 5)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6
    rate = (errs[-1] / errs[-3]) ** (1.0 / 10)
    assert abs(rate - rho) <= 0.05


def test_alpha_cancels(small):
    """A random invertible block-diagonal scaling alpha (eq. 9-11) leaves x_K
    unchanged."""
    prob, H, b, g = small
    alpha = {a: g.standard_normal((c.size, c.size)) + 1j * g.standard_normal((c.size, c.size))
             + 3 * np.eye(c.size) for a, c in enumerate(H.leaves)}
    x1 = series.series(H, b, 3, -1)
    x2 = series.series(H, b, 3, -1, alpha=alpha)
    assert series.rel_err(x2, x1) < 1e-11


def test_gmres_matches_dense_solve(small):
    prob, H, b, _ = small
    xd = series.solve_exact(H, b[:, :1], min(H.far_levels))
    xg = series.solve_gmres(H, b[:, :1], min(H.far_levels))
    assert series.rel_err(xg, xd) < 1e-11


def test_multi_rhs_columns_independent(small):
    prob, H, b, _ = small
    X = series.series(H, b, 3)
    for c in range(b.shape[1]):
        assert series.rel_err(series.series(H, b[:, c], 3), X[:, c]) < 1e-15


def _csym_factor(D):
    """D = C C^T for a complex symmetric block, C lower triangular, no
    pivoting (plain column-by-column recurrence)."""
    m = D.shape[0]
    C = np.zeros_like(D)
    for j in range(m):
        C[j, j] = np.sqrt(D[j, j] - np.sum(C[j, :j] ** 2))
        C[j + 1:, j] = (D[j + 1:, j] - C[j + 1:, :j] @ C[j, :j]) / C[j, j]
    return C


def test_scaled_series_on_symmetric_operator(small):
    """The scaled basis the half-storage path uses on symmetric problems:
    with D_a = C_a C_a^T, S = C^{-1} R_l C^{-T} is symmetric and
    yhat_{k+1} = -S yhat_k, yhat_0 = C^{-1} b, x = C^{-T} sum yhat_k gives
    the same x_K as the series (S is similar to D^{-1} R_l)."""
    prob, H, b, _ = small
    for level in (-1, H.far_levels[0]):
        D, R = _dense_parts(H, level)
        assert np.abs(D - D.T).max() <= 1e-14 * np.abs(D).max()
        assert np.abs(R - R.T).max() <= 1e-12 * np.abs(R).max()
        C = np.zeros_like(D)
        for c in H.leaves:
            sl = slice(c.off, c.off + c.size)
            C[sl, sl] = _csym_factor(D[sl, sl])
        assert np.abs(C @ C.T - D).max() <= 1e-13 * np.abs(D).max()
        Ci = scipy.linalg.solve_triangular(C, np.eye(len(C)), lower=True)
        S = Ci @ R @ Ci.T
        assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
        bt = H.to_tree(b)
        for K in (0, 3):
            y = Ci @ bt
            xh = y.copy()
            for _ in range(K):
                y = -S @ y
                xh = xh + y
            x = H.from_tree(Ci.T @ xh)
            assert series.rel_err(x, series.series(H, b, K, level)) <= 1e-12, (level, K)


# ---------------------------------------------------------------- nested form
def test_level_parts_partition_R(small):
    """The nested form's level parts (near off-diagonal + leaf-level far,
    then one coarser level each) add up to R_l exactly: no block is dropped
    or counted twice."""
    prob, H, b, g = small
    y = g.standard_normal((H.n, 2)) + 1j * g.standard_normal((H.n, 2))
    for level in H.far_levels:
        parts = sum(series.level_part(H, y, j) for j in range(H.L - level + 1))
        ref = H.apply_R(y, level)
        assert np.linalg.norm(parts - ref) <= 1e-14 * np.linalg.norm(ref)


def test_nested_at_leaf_level_is_the_flat_series(small):
    """One factor (leaf level only): the nested form is the flat series."""
    prob, H, b, _ = small
    for K in (0, 2, 4):
        assert series.rel_err(series.nested(H, b, K, -1), series.series(H, b, K, -1)) <= 1e-14


def test_nested_matches_dense_factor_products(small):
    """Two factors (levels 6 and 5) evaluated with dense matrices built from
    the assembled H-matrix: U_1 = D^{-1} R_6, U_2 = D^{-1}(R_5 - R_6),
    S_1 = sum_k (-U_1)^k, X_2 = S_1 U_2, x = S_2 S_1 D^{-1} b."""
    prob, H, b, _ = small
    lo = min(H.far_levels)
    D = H.dense(-1, "D")
    R6, R5 = H.dense(-1, "R"), H.dense(lo, "R")
    U1 = np.linalg.solve(D, R6)
    U2 = np.linalg.solve(D, R5 - R6)
    bt = H.to_tree(b)
    for K in (1, 3):
        S1 = sum(np.linalg.matrix_power(-U1, k) for k in range(K + 1))
        X2 = S1 @ U2
        S2 = sum(np.linalg.matrix_power(-X2, k) for k in range(K + 1))
        x = S2 @ (S1 @ np.linalg.solve(D, bt))
        xn = H.to_tree(series.nested(H, b, K, lo))
        assert np.linalg.norm(xn - x) <= 1e-12 * np.linalg.norm(x), K


def test_nested_factorisation_identity(small):
    """Eq. 14-19 with exact inverses: (I + U_1)(I + V_2) = I + U_1 + U_2 for
    V_2 = (I + U_1)^{-1} U_2, so the product of the exact factor inverses
    applied to D^{-1} b is x* = Z_l^{-1} b."""
    prob, H, b, _ = small
    lo = min(H.far_levels)
    D = H.dense(-1, "D")
    R6, R5 = H.dense(-1, "R"), H.dense(lo, "R")
    U1 = np.linalg.solve(D, R6)
    U2 = np.linalg.solve(D, R5 - R6)
    I = np.eye(H.n)
    V2 = np.linalg.solve(I + U1, U2)
    lhs = (I + U1) @ (I + V2)
    assert np.linalg.norm(lhs - (I + U1 + U2)) <= 1e-12 * np.linalg.norm(I + U1 + U2)
    x = np.linalg.solve(I + V2, np.linalg.solve(I + U1, np.linalg.solve(D, H.to_tree(b))))
    xs = H.to_tree(series.solve_exact(H, b, lo))
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_nested_converges_to_the_exact_solution(small):
    """Both factor series contract on this sphere: the nested solution at the
    coarsest level approaches x* = Z_l^{-1} b as K grows, and faster per K
    than the flat series (which uses K level-l products against the nested
    form's (K + 1)^2 - 1)."""
    prob, H, b, _ = small
    lo = min(H.far_levels)
    xs = series.solve_exact(H, b, lo)
    errs = [series.rel_err(series.nested(H, b, K, lo), xs) for K in (2, 5, 10)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05
    assert errs[2] < series.rel_err(series.series(H, b, 10, lo), xs)
