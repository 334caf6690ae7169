"""Seeded synthetic problem generators shared by the solver library's callers
and by the FP64 oracle.

This module only draws inputs: point clouds, contrasts, incidence directions,
plane-wave right-hand sides, instance sizes and request streams.  It holds
none of the solver's arithmetic (no matrix entries, no tree, no compression,
no series).  Both sides receive the same arrays from here and compute
everything else on their own.

The paper's experiments (Section V) use RWG/SWG meshes of a plate, a slab
and a hollow cylinder, which are not available.  Synthetic point-kernel
problems with the same structure stand in for them: a sphere surface (the
surface-EFIE stand-in) and a dielectric cube (the volume-EFIE stand-in),
with one unknown per point.

Seeds (numpy ``Generator(PCG64(seed))``):
  1  points and jitter,  2  contrast chi,  3  incidence directions,
  4  batched instance sizes,  5  served request stream.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SURFACE = 0
VOLUME = 1

WAVELENGTH = 1.0
WAVENUMBER = 2.0 * math.pi / WAVELENGTH
JITTER = 0.01  # lambda, uniform in [-JITTER, JITTER] per coordinate


def _rng(seed, *sub) -> np.random.Generator:
    if sub:
        return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *sub])))
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Problem:
    """One scattering problem: points, wavenumber, cell size and (volume only)
    the contrast at each point.  ``kind`` is SURFACE or VOLUME."""

    kind: int
    xyz: np.ndarray          # (n, 3) float64, row-major, in wavelengths
    k: float                 # wavenumber
    h: float                 # mean spacing (surface) or cell edge (volume)
    chi: Optional[np.ndarray] = None  # (n,) float64 for VOLUME

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


def sphere_points(n: int, radius: float, seed: int = 1, instance: Optional[int] = None) -> np.ndarray:
    """Fibonacci lattice on a sphere of the given radius, jittered by
    U[-0.01, 0.01]^3 wavelengths and projected back onto the sphere."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    p = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1) * radius
    g = _rng(seed) if instance is None else _rng(seed, instance)
    p = p + g.uniform(-JITTER, JITTER, size=(n, 3))
    p *= (radius / np.linalg.norm(p, axis=1))[:, None]
    return np.ascontiguousarray(p)


def sphere_spacing(n: int, radius: float) -> float:
    """Mean spacing h of n points on a sphere: h^2 * n = 4 pi a^2."""
    return math.sqrt(4.0 * math.pi * radius * radius / n)


def cube_points(n_side: int, side: float, seed: int = 1, instance: Optional[int] = None) -> np.ndarray:
    """Cell-centred n_side^3 grid filling a cube of the given side, jittered by
    U[-0.01, 0.01]^3 wavelengths.  Point order: x fastest, then y, then z."""
    h = side / n_side
    c = (np.arange(n_side, dtype=np.float64) + 0.5) * h
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    p = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    g = _rng(seed) if instance is None else _rng(seed, instance)
    p = p + g.uniform(-JITTER, JITTER, size=p.shape)
    return np.ascontiguousarray(p)


def contrast(n: int, seed: int = 2, instance: Optional[int] = None) -> np.ndarray:
    """Contrast chi ~ U[0.5, 2.0] per volume cell."""
    g = _rng(seed) if instance is None else _rng(seed, instance)
    return g.uniform(0.5, 2.0, size=n)


def directions(nrhs: int, seed: int = 3, instance: Optional[int] = None) -> np.ndarray:
    """Incidence directions uniform on the unit sphere: theta = arccos(1 - 2u),
    phi = 2 pi v.  Returns (nrhs, 3)."""
    g = _rng(seed) if instance is None else _rng(seed, instance)
    u = g.uniform(0.0, 1.0, size=nrhs)
    v = g.uniform(0.0, 1.0, size=nrhs)
    th = np.arccos(1.0 - 2.0 * u)
    ph = 2.0 * math.pi * v
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def plane_waves(xyz: np.ndarray, dirs: np.ndarray, k: float = WAVENUMBER) -> np.ndarray:
    """Right-hand sides b[:, c] = exp(-j k d_c . r): the known incident plane
    wave of the system [Z] x = b.  Returns an (n, nrhs) complex128 array in
    column-major (Fortran) order, the layout the solver library takes."""
    ph = xyz @ np.asarray(dirs, dtype=np.float64).T
    return np.asfortranarray(np.exp(-1j * k * ph))


def sphere_problem(n: int, radius: float, seed: int = 1, instance: Optional[int] = None) -> Problem:
    return Problem(SURFACE, sphere_points(n, radius, seed, instance), WAVENUMBER,
                   sphere_spacing(n, radius))


def cube_problem(n_side: int, side: float, seed: int = 1, instance: Optional[int] = None) -> Problem:
    xyz = cube_points(n_side, side, seed, instance)
    return Problem(VOLUME, xyz, WAVENUMBER, side / n_side,
                   contrast(xyz.shape[0], 2, instance))


# --------------------------------------------------------------------------
# Named workloads.  Each gives the problem plus the build and solve settings.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    problem: Problem
    leaf_max: int
    eta: float
    aca_tol: float
    K: int
    level: int          # -1: leaf level only
    nrhs: int
    dirs: np.ndarray    # (nrhs, 3)

    def rhs(self) -> np.ndarray:
        return plane_waves(self.problem.xyz, self.dirs, self.problem.k)


Z_HAT = np.array([[0.0, 0.0, 1.0]])


def sphere_small(n: int = 1536) -> Workload:
    """Sphere surface, N=1536, radius 1 lambda, leaf <= 64, ACA tol 1e-4, K=4,
    one plane wave along z, leaf level only."""
    return Workload(f"sphere_{n}", sphere_problem(n, math.sqrt(n / 1536.0)), 64, 1.0, 1e-4,
                    4, -1, 1, Z_HAT.copy())


def sphere_large(n: int = 24576) -> Workload:
    """Sphere surface, N=24,576, radius 4 lambda (same density), leaf <= 128,
    ACA tol 1e-4, K=4, one plane wave along z."""
    return Workload(f"sphere_{n}", sphere_problem(n, 4.0 * math.sqrt(n / 24576.0)), 128, 1.0,
                    1e-4, 4, -1, 1, Z_HAT.copy())


def cube_volume(n_side: int = 32, nrhs: int = 64) -> Workload:
    """Dielectric cube, (n_side)^3 cells of edge lambda/16, chi ~ U[0.5, 2],
    leaf <= 128, ACA tol 1e-5, K=5, nrhs plane waves at seeded directions."""
    side = n_side / 16.0
    return Workload(f"cube_{n_side ** 3}", cube_problem(n_side, side), 128, 1.0, 1e-5, 5, -1,
                    nrhs, directions(nrhs, 3))


def batched_sizes(count: int = 256, lo: int = 512, hi: int = 8192, seed: int = 4) -> np.ndarray:
    """Instance sizes N_i = round(exp(U[ln lo, ln hi]))."""
    g = _rng(seed)
    return np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def batched_instance(i: int, n: int, nrhs: int = 16) -> Workload:
    """One instance of the batched surface workload: sphere radius scaled so
    the point density matches the N=1536 sphere of radius 1 lambda."""
    prob = sphere_problem(int(n), math.sqrt(n / 1536.0), 1, instance=i)
    return Workload(f"batched_{i}_{n}", prob, 64, 1.0, 1e-4, 4, -1, nrhs,
                    directions(nrhs, 3, instance=i))


@dataclasses.dataclass
class Request:
    t_arrive: float   # seconds from stream start
    kind: int         # SURFACE or VOLUME
    geom: int         # index into the geometry pool of that kind
    nrhs: int


def served_pool(count: int = 16, lo: int = 1024, hi: int = 65536, seed: int = 5):
    """Geometry pool of the served stream: ``count`` sphere sizes and
    ``count`` cube sides (volume N rounded to a cube number at the cube
    workload's density)."""
    g = _rng(seed, 0)
    ns = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    nv = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=count)))
    sides = np.maximum(2, np.rint(np.cbrt(nv))).astype(np.int64)
    return ns, sides


def served_workload(kind: int, geom: int, nrhs: int, request_seed: int) -> Workload:
    ns, sides = served_pool()
    dirs = directions(nrhs, 3, instance=request_seed)
    if kind == SURFACE:
        n = int(ns[geom])
        prob = sphere_problem(n, math.sqrt(n / 1536.0), 1, instance=1000 + geom)
        leaf = 64 if n <= 8192 else 128
        return Workload(f"served_s{geom}", prob, leaf, 1.0, 1e-4, 4, -1, nrhs, dirs)
    s = int(sides[geom])
    prob = cube_problem(s, s / 16.0, 1, instance=2000 + geom)
    return Workload(f"served_v{geom}", prob, 128, 1.0, 1e-5, 5, -1, nrhs, dirs)


def request_stream(count: int, rate: float, surface_share: float = 0.6, seed: int = 5):
    """Poisson arrivals at ``rate`` requests/s; kind surface with probability
    ``surface_share``; geometry uniform in its pool; nrhs ~ U{1..64}."""
    g = _rng(seed, 1)
    t = np.cumsum(g.exponential(1.0 / rate, size=count))
    kinds = np.where(g.uniform(size=count) < surface_share, SURFACE, VOLUME)
    geoms = g.integers(0, 16, size=count)
    nrhs = g.integers(1, 65, size=count)
    return [Request(float(t[i]), int(kinds[i]), int(geoms[i]), int(nrhs[i])) for i in range(count)]
