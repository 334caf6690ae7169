"""Binary cluster tree, admissibility and block partition (Sec. III, eq. 6-7).

Readings where the paper is silent:
  * split rule: a cluster with more than ``leaf_max`` points is split along
    the longest axis of its bounding box (lowest axis index on equal
    extents); its points are ordered by that coordinate, ties by original
    index, and the left child takes the first floor(n/2);
  * diam(.) is the bounding-box diagonal and dist(.,.) the Euclidean gap
    between the two boxes (0 when they overlap); eq. 7 is inclusive;
  * the partition descends from (root, root); an admissible pair becomes a
    far block at the coarsest level where it is admissible (its parent pair
    is not), a pair of two leaves that is not admissible becomes a dense
    near block, anything else recurses into all child pairs (a leaf side
    stays whole);
  * the level of a block is max(depth(t), depth(s)), root depth 0;
  * a cluster paired with itself is never admissible (it holds the diagonal).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Cluster:
    off: int                 # first position in tree order
    size: int
    depth: int
    lo: np.ndarray           # bounding box
    hi: np.ndarray
    children: List["Cluster"] = dataclasses.field(default_factory=list)

    @property
    def is_leaf(self) -> bool:
        return not self.children


@dataclasses.dataclass
class Tree:
    root: Cluster
    perm: np.ndarray         # perm[p] = original index of tree position p
    leaves: List[Cluster]    # in tree order
    depth: int               # deepest leaf depth (the leaf level L)


def build_tree(xyz: np.ndarray, leaf_max: int) -> Tree:
    perm = np.empty(xyz.shape[0], dtype=np.int64)
    leaves: List[Cluster] = []

    def split(idx: np.ndarray, off: int, depth: int) -> Cluster:
        pts = xyz[idx]
        c = Cluster(off, len(idx), depth, pts.min(axis=0), pts.max(axis=0))
        if len(idx) > leaf_max:
            ext = c.hi - c.lo
            ax = int(np.argmax(ext))            # first maximum: lowest axis on ties
            order = np.lexsort((idx, pts[:, ax]))  # key: coordinate, then original index
            s = idx[order]
            h = len(idx) // 2
            c.children = [split(s[:h], off, depth + 1), split(s[h:], off + h, depth + 1)]
        else:
            perm[off:off + len(idx)] = idx
            leaves.append(c)
        return c

    root = split(np.arange(xyz.shape[0], dtype=np.int64), 0, 0)
    return Tree(root, perm, leaves, max(l.depth for l in leaves))


def diam(c: Cluster) -> float:
    return float(np.linalg.norm(c.hi - c.lo))


def dist(t: Cluster, s: Cluster) -> float:
    gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
    return float(np.linalg.norm(gap))


def admissible(t: Cluster, s: Cluster, eta: float) -> bool:
    """eq. 7: eta * dist(t, s) >= min(diam(t), diam(s))."""
    return eta * dist(t, s) >= min(diam(t), diam(s))


@dataclasses.dataclass
class Partition:
    near: list   # (t, s) leaf pairs, diagonal included
    far: list    # (t, s, level)


def partition(tree: Tree, eta: float) -> Partition:
    near, far = [], []

    def rec(t: Cluster, s: Cluster):
        # a cluster's interaction with itself holds the diagonal and is never
        # far, even when eq. 7 holds trivially (one point: diam = dist = 0)
        if t is not s and admissible(t, s, eta):
            far.append((t, s, max(t.depth, s.depth)))
            return
        if t.is_leaf and s.is_leaf:
            near.append((t, s))
            return
        for a in (t.children or [t]):
            for b in (s.children or [s]):
                rec(a, b)

    rec(tree.root, tree.root)
    return Partition(near, far)
