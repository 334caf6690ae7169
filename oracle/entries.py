"""Matrix entries of the dense system [Z] x = b (Sec. II, eq. 5).

The paper fills Z by Galerkin testing of RWG (surface, eq. 3) or SWG
(volume, eq. 4) basis functions.  Those meshes are not available, so a
point-kernel stand-in with the same free-space Green's function is used,
one unknown per point, e^{-jkR} phase convention:

  surface   Z_ij = h^2 e^{-jkR_ij} / (4 pi R_ij)            (i != j)
            Z_ii = 2 h (1 + 0.1 j)
  volume    Z_ij = k^2 chi_j h^3 e^{-jkR_ij} / (4 pi R_ij)  (i != j)
            Z_ii = 1/chi_i + 0.5

For the volume case Z = Delta + G diag(chi) with the symmetric kernel part
G_ij = k^2 h^3 e^{-jkR}/(4 pi R); G is what gets compressed (the half
H-matrix of Sec. III needs a symmetric operator).
"""
from __future__ import annotations

import numpy as np

SURFACE = 0
VOLUME = 1


def distances(xyz: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """|r_i - r_j| for i in rows, j in cols, as a (len(rows), len(cols)) array."""
    d = xyz[rows][:, None, :] - xyz[cols][None, :, :]
    return np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])


def green(k: float, r: np.ndarray) -> np.ndarray:
    """Free-space Green's function e^{-jkR} / (4 pi R)."""
    return np.exp(-1j * k * r) / (4.0 * np.pi * r)


def kernel_block(prob, rows, cols) -> np.ndarray:
    """Symmetric kernel part of Z[rows, cols] for index sets that do not
    share an index: Z itself (surface) or G (volume)."""
    r = distances(prob.xyz, np.asarray(rows), np.asarray(cols))
    if np.any(r < 1e-12):
        raise ValueError("coincident points off the diagonal")
    if prob.kind == SURFACE:
        return prob.h * prob.h * green(prob.k, r)
    return (prob.k * prob.k * prob.h ** 3) * green(prob.k, r)


def block(prob, rows, cols) -> np.ndarray:
    """Exact dense Z[rows, cols], diagonal entries included where rows and
    cols share an index."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    same = rows[:, None] == cols[None, :]
    r = distances(prob.xyz, rows, cols)
    r_safe = np.where(same, 1.0, r)
    if np.any(r_safe < 1e-12):
        raise ValueError("coincident points off the diagonal")
    g = green(prob.k, r_safe)
    if prob.kind == SURFACE:
        z = prob.h * prob.h * g
        z[same] = 2.0 * prob.h * (1.0 + 0.1j)
        return z
    chi = prob.chi
    z = (prob.k * prob.k * prob.h ** 3) * g * chi[cols][None, :]
    ii, _ = np.nonzero(same)
    z[same] = 1.0 / chi[rows[ii]] + 0.5
    return z


def dense(prob) -> np.ndarray:
    """The whole dense Z in original point order (small N only)."""
    idx = np.arange(prob.n)
    return block(prob, idx, idx)
