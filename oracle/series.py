"""Power-series solution of the H-matrix system (Sec. IV, eq. 9-22).

With the near field reduced to its block diagonal D (the leaf
self-interaction blocks; the scaling alpha of eq. 9-11 cancels, see
``series``) and R_l the rest of the H-matrix up to level l, eq. 12-13 read
(I + D^{-1} R_l) x = D^{-1} b, and the power expansion of the inverse
(eq. 20-22, truncated after a fixed number of terms as in the fast power
series the paper uses) gives

    x_K = sum_{k=0..K} (-D^{-1} R_l)^k D^{-1} b,

evaluated as y_0 = D^{-1} b, y_k = -D^{-1} (R_l y_{k-1}), x_K = sum y_k.
K is the highest power (K + 1 terms).

Also here: the nested multi-level form of eq. 14-22 (``nested``), the exact
solution x* = Z_l^{-1} b of the same H-matrix (dense LU,
or GMRES for large N), the spectral radius of D^{-1} R_l by power iteration
(the convergence condition of the expansion, Sec. V), and residual-driven
refinement x <- x + P_K (b - Z_l x).

All vectors are in original point order, shape (n,) or (n, nrhs).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg


def series(H, b: np.ndarray, K: int, level: int = -1, alpha=None, return_terms: bool = False):
    """x_K of the power series on Z_l = D + R_l.

    ``alpha``: optional dict leaf -> invertible matrix, the block-diagonal
    scaling of eq. 9-11.  Then Z~_N = alpha D, b~ = alpha b and each term is
    y_k = -Z~_N^{-1} alpha R_l y_{k-1} (eq. 12-13); the result does not
    depend on alpha."""
    squeeze = np.ndim(b) == 1
    bt = H.to_tree(b)
    if alpha is None:
        solve = H.solve_D
        scale = lambda v: v  # noqa: E731
    else:
        lus = {a: scipy.linalg.lu_factor(alpha[a] @ H.diag[a]) for a in H.diag}

        def scale(v):
            out = np.empty_like(v)
            for a in H.diag:
                sl = H.leaf_range(a)
                out[sl] = alpha[a] @ v[sl]
            return out

        def solve(v):
            out = np.empty_like(v)
            for a, f in lus.items():
                sl = H.leaf_range(a)
                out[sl] = scipy.linalg.lu_solve(f, v[sl])
            return out

    y = solve(scale(bt))
    x = y.copy()
    terms = [y]
    for _ in range(K):
        y = -solve(scale(H.apply_R(y, level)))
        x = x + y
        terms.append(y)
    out = H.from_tree(x)
    out = out[:, 0] if squeeze else out
    if return_terms:
        return out, [H.from_tree(t) for t in terms]
    return out


def level_part(H, y: np.ndarray, j: int) -> np.ndarray:
    """F_j y in tree order for factor j of the nested form: j = 0 holds the
    off-diagonal near blocks and the far blocks of the leaf level L; j >= 1
    the far blocks of level L - j exactly.  Summed over j = 0 .. L - l these
    make R_l."""
    lev = H.L - j
    y = y.reshape(H.n, -1)
    z = np.zeros_like(y, dtype=np.complex128)
    if j == 0:
        for blk in H.near:
            if blk.t != blk.s:
                z[H.leaf_range(blk.t)] += blk.Z @ y[H.leaf_range(blk.s)]
    for b in H.far:
        if b.level == lev:
            z[b.t_off:b.t_off + b.m] += H._far_apply(b, y)
    return z


def nested(H, b: np.ndarray, K: int, level: int = -1) -> np.ndarray:
    """The nested multi-level form of eq. 14-22:

        x = (I + X_n)^{-1} ... (I + X_2)^{-1} (I + X_1)^{-1} D^{-1} b,

    X_1 = U_1, X_j = (I + X_{j-1})^{-1} ... (I + X_1)^{-1} U_j (the paper's
    V_2 and W_3), U_j = D^{-1} F_j for the level parts F_j of ``level_part``,
    taken from the leaf level up to ``level``, so that the leaf level alone
    is the flat series.  Each inverse is its power series with K + 1 terms,
    (I + X)^{-1} v ~ sum_{k=0..K} (-X)^k v, and applying X_j applies the
    truncated inverses of the factors before it (nested, not premultiplied:
    (K + 1)^n - 1 level products in all for n factors)."""
    squeeze = np.ndim(b) == 1
    n = H.L - H.level(level) + 1

    def U(j, y):
        return H.solve_D(level_part(H, y, j))

    def Q(j, v):  # the first j truncated inverses, innermost first
        for i in range(j):
            v = S(i, v)
        return v

    def S(i, u):  # sum_{k=0..K} (-X_i)^k u, X_i w = Q(i, U_i w)
        acc = u.copy()
        y = u
        for _ in range(K):
            y = -Q(i, U(i, y))
            acc = acc + y
        return acc

    x = Q(n, H.solve_D(H.to_tree(b)))
    out = H.from_tree(x)
    return out[:, 0] if squeeze else out


def apply_Z(H, x: np.ndarray, level: int = -1) -> np.ndarray:
    """Z_l x in original order."""
    squeeze = np.ndim(x) == 1
    z = H.from_tree(H.apply_Z(H.to_tree(x), level))
    return z[:, 0] if squeeze else z


def solve_exact(H, b: np.ndarray, level: int = -1) -> np.ndarray:
    """x* = Z_l^{-1} b by dense LU of the assembled H-matrix (small N)."""
    squeeze = np.ndim(b) == 1
    x = scipy.linalg.solve(H.dense(level), H.to_tree(b))
    x = H.from_tree(x)
    return x[:, 0] if squeeze else x


def solve_gmres(H, b: np.ndarray, level: int = -1, tol: float = 1e-13, maxiter: int = 2000):
    """x* = Z_l^{-1} b by GMRES on the H-matvec with D^{-1} as left
    preconditioner, one right-hand side at a time (large N)."""
    bt = H.to_tree(b)
    n = H.n
    A = scipy.sparse.linalg.LinearOperator(
        (n, n), matvec=lambda v: (H.solve_D(H.apply_Z(v.reshape(n, 1), level)))[:, 0],
        dtype=np.complex128)
    out = np.empty_like(bt)
    for c in range(bt.shape[1]):
        rhs = H.solve_D(bt[:, c:c + 1])[:, 0]
        x, info = scipy.sparse.linalg.gmres(A, rhs, rtol=tol, atol=0.0, restart=200,
                                            maxiter=maxiter)
        if info != 0:
            raise RuntimeError(f"GMRES did not converge (info={info})")
        out[:, c] = x
    out = H.from_tree(out)
    return out[:, 0] if np.ndim(b) == 1 else out


def rho(H, level: int = -1, iters: int = 80, seed: int = 0) -> float:
    """Spectral radius of M_l = D^{-1} R_l by power iteration (geometric mean
    of the growth factors over the last quarter of the iterations)."""
    g = np.random.default_rng(seed)
    v = g.standard_normal((H.n, 1)) + 1j * g.standard_normal((H.n, 1))
    v /= np.linalg.norm(v)
    logs = []
    for _ in range(iters):
        w = H.solve_D(H.apply_R(v, level))
        nw = np.linalg.norm(w)
        if nw == 0.0:
            return 0.0
        logs.append(np.log(nw))
        v = w / nw
    tail = logs[-max(1, iters // 4):]
    return float(np.exp(np.mean(tail)))


def refine(H, b: np.ndarray, K: int, level: int = -1, passes: int = 1) -> np.ndarray:
    """x <- P_K b, then ``passes`` times x <- x + P_K (b - Z_l x)."""
    x = series(H, b, K, level)
    for _ in range(passes):
        r = b - apply_Z(H, x, level)
        x = x + series(H, r, K, level)
    return x


def rel_err(x: np.ndarray, ref: np.ndarray) -> float:
    """Max over right-hand sides of ||x - ref||_2 / ||ref||_2."""
    x = np.asarray(x).reshape(ref.shape[0], -1)
    ref = np.asarray(ref).reshape(ref.shape[0], -1)
    return float(np.max(np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)))
