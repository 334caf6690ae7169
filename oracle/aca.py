"""Adaptive cross approximation with partial pivoting, then recompression
(Sec. III: far blocks are compressed by a recompressed ACA into U (m x k)
and V (k x n) factors).

The paper names the method and cites it but prints no procedure; the rules
below are the ones both implementations in this repository follow, so that
their approximants agree to rounding:

ACA on A (m x n), tolerance eps, rank cap r_max = min(m, n):
  * start with row 0; the residual row is A[i,:] - sum_k u_k[i] v_k;
  * if max |row| <= 1e-300 the row is marked used and the next unused row
    in index order is taken (stop when none is left);
  * pivot column j = first index of max |row|; v = row / row[j];
    u = A[:,j] - sum_k v_k[j] u_k;
  * ||S||_F^2 of S = sum_k u_k v_k^T is updated incrementally;
  * stop after the step where ||u|| ||v|| <= eps ||S||_F, or at rank r_max;
  * next row = first index of max |u| over unused rows.
Recompression: U = Qu Ru, V = Qv Rv (thin QR), Ru Rv^T = Phi Sigma Psi^H;
keep the smallest r >= 1 with sqrt(sum_{i>=r} sigma_i^2) <= eps ||sigma||_2;
A ~ (Qu Phi_r Sigma_r) (Qv conj(Psi_r))^T.
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np

ZERO_ROW = 1e-300


def aca(row: Callable[[int], np.ndarray], col: Callable[[int], np.ndarray], m: int, n: int,
        eps: float, max_rank: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Partially pivoted ACA.  ``row(i)`` returns A[i, :], ``col(j)`` A[:, j].
    Returns U (m x r), V (n x r) with A ~ U V^T."""
    r_max = min(m, n) if max_rank <= 0 else min(max_rank, m, n)
    us, vs = [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    s2 = 0.0
    while True:
        rr = np.array(row(i), dtype=np.complex128)
        for u, v in zip(us, vs):
            rr -= u[i] * v
        used[i] = True
        mag = np.abs(rr)
        j = int(np.argmax(mag))
        if mag[j] <= ZERO_ROW:
            free = np.flatnonzero(~used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v_new = rr / rr[j]
        u_new = np.array(col(j), dtype=np.complex128)
        for u, v in zip(us, vs):
            u_new -= v[j] * u
        cross = 0.0 + 0.0j
        for u, v in zip(us, vs):
            cross += np.vdot(u, u_new) * np.vdot(v, v_new)
        nu = np.linalg.norm(u_new)
        nv = np.linalg.norm(v_new)
        s2 += 2.0 * cross.real + (nu * nv) ** 2
        us.append(u_new)
        vs.append(v_new)
        if nu * nv <= eps * np.sqrt(s2) or len(us) >= r_max:
            break
        cand = np.abs(u_new)
        cand[used] = -1.0
        if np.all(used):
            break
        i = int(np.argmax(cand))
    if not us:
        return np.zeros((m, 1), np.complex128), np.zeros((n, 1), np.complex128)
    return np.stack(us, axis=1), np.stack(vs, axis=1)


def recompress(U: np.ndarray, V: np.ndarray, eps: float) -> Tuple[np.ndarray, np.ndarray]:
    """Truncate A ~ U V^T to the smallest rank whose discarded singular
    values have 2-norm <= eps times the 2-norm of all of them."""
    qu, ru = np.linalg.qr(U)
    qv, rv = np.linalg.qr(V)
    phi, sig, psih = np.linalg.svd(ru @ rv.T)
    total = np.sqrt(np.sum(sig * sig))
    r = len(sig)
    for cand in range(1, len(sig) + 1):
        if np.sqrt(np.sum(sig[cand:] ** 2)) <= eps * total:
            r = cand
            break
    return qu @ (phi[:, :r] * sig[:r]), qv @ psih[:r, :].T


def compress(A_row, A_col, m, n, eps, max_rank=0):
    """ACA followed by recompression."""
    U, V = aca(A_row, A_col, m, n, eps, max_rank)
    return recompress(U, V, eps)
