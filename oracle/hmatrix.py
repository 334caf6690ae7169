"""H-matrix of the system: dense near blocks plus ACA-compressed far blocks
grouped by level (Sec. III, eq. 6 and Sec. IV, eq. 8).

Z = Z_N + Z_F, Z_F = sum over levels of Z_F(level).  The near part is split
into its block diagonal D (leaf self-interaction blocks) and the off-diagonal
near blocks.  For a chosen level l (the paper's "solution at each level"),
R_l = off-diagonal near blocks + far blocks of level >= l, and Z_l = D + R_l.
The leaf level L keeps only the finest far blocks, as in the paper's runs.

Half computation (Sec. III): the far block (t, s) is compressed once for
t before s and the block (s, t) is its transpose.  For the volume case the
compressed operator is the symmetric kernel part G and the contrast chi of
the source points scales the input vector.

Everything is stored and applied in tree order; ``perm`` maps tree positions
to original point indices.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.linalg

from . import aca as _aca
from . import cluster as _cl
from . import entries as _en


@dataclasses.dataclass
class FarBlock:
    t_off: int
    m: int
    s_off: int
    n: int
    level: int
    U: np.ndarray     # (m, r)
    V: np.ndarray     # (n, r): kernel block ~ U V^T


@dataclasses.dataclass
class NearBlock:
    t: int            # leaf index (row)
    s: int            # leaf index (column)
    Z: np.ndarray     # exact dense Z[t, s]


class HMatrix:
    def __init__(self, prob, leaf_max: int, eta: float = 1.0, aca_tol: float = 1e-4,
                 max_rank: int = 0, progress=None):
        """``progress`` (optional callable taking a string) is told how the
        build advances (long builds); it does not change the result."""
        self.prob = prob
        self.n = prob.n
        self.tree = _cl.build_tree(prob.xyz, leaf_max)
        self.part = _cl.partition(self.tree, eta)
        self.perm = self.tree.perm
        self.leaves = self.tree.leaves
        self.L = self.tree.depth
        leaf_id = {id(c): a for a, c in enumerate(self.leaves)}
        self.chi_tree = None if prob.chi is None else prob.chi[self.perm]

        self.near: List[NearBlock] = []
        for t, s in self.part.near:
            rows = self.perm[t.off:t.off + t.size]
            cols = self.perm[s.off:s.off + s.size]
            self.near.append(NearBlock(leaf_id[id(t)], leaf_id[id(s)], _en.block(prob, rows, cols)))
        self.diag = {b.t: b.Z for b in self.near if b.t == b.s}
        self.lu = {a: scipy.linalg.lu_factor(Z) for a, Z in self.diag.items()}

        self.far: List[FarBlock] = []
        done = {}
        if progress:
            progress(f"oracle: {len(self.near)} near blocks filled, "
                     f"{len(self.part.far) // 2} far blocks to compress")
        for q, (t, s, lev) in enumerate(self.part.far):
            if progress and q % 4000 == 0 and q:
                progress(f"oracle: far block pair {q} of {len(self.part.far)}")
            if t.off < s.off:
                rows = self.perm[t.off:t.off + t.size]
                cols = self.perm[s.off:s.off + s.size]
                U, V = _aca.compress(
                    lambda i: _en.kernel_block(prob, rows[i:i + 1], cols)[0],
                    lambda j: _en.kernel_block(prob, rows, cols[j:j + 1])[:, 0],
                    t.size, s.size, aca_tol, max_rank)
                done[(t.off, s.off)] = (U, V)
        for t, s, lev in self.part.far:
            if t.off < s.off:
                U, V = done[(t.off, s.off)]
            else:
                V, U = done[(s.off, t.off)]
            self.far.append(FarBlock(t.off, t.size, s.off, s.size, lev, U, V))
        self.far_levels = sorted({b.level for b in self.far})

    # ---- level handling ---------------------------------------------------
    def level(self, level: int) -> int:
        """-1 means the leaf level L."""
        return self.L if level < 0 else level

    def leaf_range(self, a: int):
        c = self.leaves[a]
        return slice(c.off, c.off + c.size)

    # ---- products, all in tree order -------------------------------------
    def _far_apply(self, b: FarBlock, x: np.ndarray) -> np.ndarray:
        xs = x[b.s_off:b.s_off + b.n]
        if self.chi_tree is not None:
            xs = self.chi_tree[b.s_off:b.s_off + b.n, None] * xs
        return b.U @ (b.V.T @ xs)

    def apply_R(self, x: np.ndarray, level: int) -> np.ndarray:
        """R_l x: off-diagonal near blocks plus far blocks of level >= l."""
        lev = self.level(level)
        x = x.reshape(self.n, -1)
        z = np.zeros_like(x, dtype=np.complex128)
        for blk in self.near:
            if blk.t != blk.s:
                z[self.leaf_range(blk.t)] += blk.Z @ x[self.leaf_range(blk.s)]
        for b in self.far:
            if b.level >= lev:
                z[b.t_off:b.t_off + b.m] += self._far_apply(b, x)
        return z

    def apply_D(self, x: np.ndarray) -> np.ndarray:
        x = x.reshape(self.n, -1)
        z = np.zeros_like(x, dtype=np.complex128)
        for a, Z in self.diag.items():
            z[self.leaf_range(a)] = Z @ x[self.leaf_range(a)]
        return z

    def solve_D(self, x: np.ndarray) -> np.ndarray:
        """D^{-1} x by the LU factors of each leaf self-block."""
        x = x.reshape(self.n, -1)
        z = np.zeros_like(x, dtype=np.complex128)
        for a, f in self.lu.items():
            z[self.leaf_range(a)] = scipy.linalg.lu_solve(f, x[self.leaf_range(a)])
        return z

    def apply_Z(self, x: np.ndarray, level: int) -> np.ndarray:
        return self.apply_D(x) + self.apply_R(x, level)

    # ---- dense assembly (small N) ----------------------------------------
    def dense(self, level: int, part: str = "Z") -> np.ndarray:
        """Dense Z_l, D or R_l in tree order."""
        lev = self.level(level)
        A = np.zeros((self.n, self.n), dtype=np.complex128)
        for blk in self.near:
            is_diag = blk.t == blk.s
            if (part == "D" and not is_diag) or (part == "R" and is_diag):
                continue
            A[self.leaf_range(blk.t), self.leaf_range(blk.s)] = blk.Z
        if part != "D":
            for b in self.far:
                if b.level >= lev:
                    blkv = b.V.T
                    if self.chi_tree is not None:
                        blkv = blkv * self.chi_tree[b.s_off:b.s_off + b.n][None, :]
                    A[b.t_off:b.t_off + b.m, b.s_off:b.s_off + b.n] = b.U @ blkv
        return A

    # ---- original-order helpers ------------------------------------------
    def to_tree(self, v: np.ndarray) -> np.ndarray:
        return np.asarray(v).reshape(self.n, -1)[self.perm]

    def from_tree(self, v: np.ndarray) -> np.ndarray:
        out = np.empty_like(v)
        out[self.perm] = v
        return out

    # ---- statistics --------------------------------------------------------
    def stats(self):
        near_off = [b for b in self.near if b.t != b.s]
        per_level = {}
        for b in self.far:
            d = per_level.setdefault(b.level, {"blocks": 0, "rank_sum": 0, "entries": 0})
            d["blocks"] += 1
            d["rank_sum"] += b.U.shape[1]
            d["entries"] += b.U.shape[1] * (b.m + b.n)
        return {
            "n": self.n, "leaf_level": self.L, "leaves": len(self.leaves),
            "near_blocks": len(self.near), "near_offdiag_entries": sum(b.Z.size for b in near_off),
            "diag_entries": sum(Z.size for Z in self.diag.values()), "far": per_level,
        }
