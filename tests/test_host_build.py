"""CPU tests of libhmps: the C-ABI loads and exports what include/hmps.h
declares, argument errors are reported, and the library's host build of the
H-matrix (tree, partition, near fill, ACA + recompression, half H-matrix)
agrees with the independent FP64 oracle (no device is used).
"""
import ctypes as C
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import hmatrix
from paper_2307_03968_amd import hmps

HOST = hmps.HM_BUILD_HOST_ONLY


def test_library_exports_header_symbols():
    lib = hmps._lib()
    names = hmps.header_functions()
    assert {"hmat_build", "hmat_apply", "ps_solve", "hmat_export", "hmat_free"} <= set(names)
    for f in names:
        assert hasattr(lib, f), f


def _lib_dense(E, n):
    """Dense H (tree order) from an export, every far level included."""
    A = np.zeros((n, n), np.complex128)
    lo, ls = E["leaf_off"], E["leaf_size"]
    for t, s, off in E["near"]:
        m, k = ls[t], ls[s]
        A[lo[t]:lo[t] + m, lo[s]:lo[s] + k] = E["near_data"][off:off + m * k].reshape(k, m).T
    chi = E.get("chi_tree")
    for t_off, m, s_off, k, lev, r, off in E["far"]:
        U = E["far_uv"][off:off + m * r].reshape(r, m).T
        V = E["far_uv"][off + m * r:off + m * r + k * r].reshape(r, k).T
        B = U @ V.T
        if chi is not None:
            B = B * chi[s_off:s_off + k][None, :]
        A[t_off:t_off + m, s_off:s_off + k] = B
    return A


CASES = {
    "sphere_1536": lambda: (W.sphere_small().problem, 64, 1e-4),
    "sphere_1000_leaf40": lambda: (W.sphere_problem(1000, math.sqrt(1000 / 1536)), 40, 1e-4),
    "cube_1000_leaf32": lambda: (W.cube_problem(10, 10 / 16), 32, 1e-5),
    "cube_1728_leaf40": lambda: (W.cube_problem(12, 12 / 16), 40, 1e-5),
    # leaves at depths 5 and 6 (sizes 68 and 34/35), far blocks on levels 5, 6
    "sphere_2200_leaf68_ragged": lambda: (W.sphere_problem(2200, math.sqrt(2200 / 1536)), 68, 1e-4),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_build_matches_oracle(case, tmp_path):
    """Same permutation, same block partition, near blocks to rounding of the
    entries, far approximants and the whole H-matvec to 1e-12 relative."""
    prob, leaf, tol = CASES[case]()
    h = hmps.HMatrix(prob, leaf, 1.0, tol, flags=HOST)
    path = str(tmp_path / "h.bin")
    h.export(path)
    E = hmps.read_export(path)
    H = hmatrix.HMatrix(prob, leaf, 1.0, tol)
    assert np.array_equal(E["perm"], H.perm)
    assert np.array_equal(E["leaf_size"], [c.size for c in H.leaves])
    lib_near = {(int(t), int(s)) for t, s, _ in E["near"]}
    assert lib_near == {(b.t, b.s) for b in H.near}
    lib_far = {tuple(int(v) for v in row[:5]): int(row[5]) for row in E["far"]}
    or_far = {(b.t_off, b.m, b.s_off, b.n, b.level): b.U.shape[1] for b in H.far}
    assert set(lib_far) == set(or_far)
    # ranks: the truncation rule decides the same rank unless a singular
    # value sits at the threshold to rounding
    same_rank = sum(lib_far[k] == or_far[k] for k in lib_far)
    assert same_rank >= len(lib_far) - max(1, len(lib_far) // 500)
    A_lib = _lib_dense(E, prob.n)
    lev = min(H.far_levels) if H.far_levels else -1
    A_or = H.dense(lev)
    assert np.linalg.norm(A_lib - A_or) <= 1e-12 * np.linalg.norm(A_or)
    g = np.random.default_rng(5)
    x = g.standard_normal(prob.n) + 1j * g.standard_normal(prob.n)
    assert np.linalg.norm(A_lib @ x - A_or @ x) <= 1e-12 * np.linalg.norm(A_or @ x)
    info = h.info()
    assert info["num_leaves"] == len(H.leaves) and info["leaf_level"] == H.L
    assert info["near_blocks"] == len(H.near)
    h.close()


def test_info_counts_match_oracle_stats():
    prob = W.sphere_small().problem
    h = hmps.HMatrix(prob, 64, 1.0, 1e-4, flags=HOST)
    st = hmatrix.HMatrix(prob, 64, 1.0, 1e-4).stats()
    info = h.info()
    assert info["near_offdiag_entries"] == st["near_offdiag_entries"]
    assert info["diag_entries"] == st["diag_entries"]
    for lev, d in st["far"].items():
        assert info["far"][lev]["blocks"] == d["blocks"]


def _raw_build(n=10, xyz=None, kind=0, chi=None, leaf=8, eta=1.0, tol=1e-4, k=2 * math.pi, hh=0.1):
    lib = hmps._lib()
    xyz = np.ascontiguousarray(W.sphere_points(max(n, 1), 0.5) if xyz is None else xyz)
    p = hmps.hm_problem(n, xyz.ctypes.data_as(C.POINTER(C.c_double)), kind, k, hh,
                        None if chi is None else chi.ctypes.data_as(C.POINTER(C.c_double)))
    o = hmps.hm_build_opts(leaf, eta, tol, 0, HOST, 0)
    h = C.c_void_p()
    st = lib.hmat_build(C.byref(p), C.byref(o), None, C.byref(h))
    if st == hmps.HM_OK:
        lib.hmat_free(h)
    return st


def test_invalid_arguments_rejected():
    assert _raw_build(n=0) == hmps.HM_EINVAL
    assert _raw_build(leaf=0) == hmps.HM_EINVAL
    assert _raw_build(leaf=300) == hmps.HM_EINVAL
    assert _raw_build(kind=1) == hmps.HM_EINVAL          # volume without chi
    assert _raw_build(kind=7) == hmps.HM_EINVAL
    assert _raw_build(tol=0.0) == hmps.HM_EINVAL
    assert _raw_build(eta=-1.0) == hmps.HM_EINVAL
    xyz = W.sphere_points(10, 0.5)
    xyz[3] = xyz[4]
    assert _raw_build(xyz=xyz) == hmps.HM_EINVAL         # coincident points
    xyz = W.sphere_points(10, 0.5)
    xyz[2, 1] = np.nan
    assert _raw_build(xyz=xyz) == hmps.HM_EINVAL
    assert _raw_build() == hmps.HM_OK
    assert b"coincident" not in hmps._lib().hm_strerror(hmps.HM_EINVAL)


def test_device_calls_on_host_only_handle():
    """A host-only handle refuses device work with HM_ESTATE (no device touched)."""
    h = hmps.HMatrix(W.sphere_problem(100, 0.5), 32, flags=HOST)
    lib = hmps._lib()
    o = hmps.ps_opts(2, -1, 0, 0, 0, 1e-9)
    assert lib.ps_solve(h.handle, C.byref(o), None, 100, None, 100, 1, None, None) == hmps.HM_ESTATE
    assert lib.hmat_apply(h.handle, -1, 0, None, 100, None, 100, 1, None) == hmps.HM_ESTATE
    t = hmps.hm_tuning(4, 0)
    assert lib.hmat_tune(h.handle, C.byref(t), None) == hmps.HM_ESTATE
    assert lib.hmat_tune(h.handle, None, None) == hmps.HM_EINVAL
    assert h.tuning()["mm_min_rhs"] == 8
    h.close()


def test_single_point_and_single_leaf():
    for n in (1, 5, 64):
        h = hmps.HMatrix(W.sphere_problem(n, 0.5), 64, flags=HOST)
        info = h.info()
        assert info["num_leaves"] == 1 and info["min_far_level"] == -1
        h.close()


def test_batched_build_is_block_diagonal(tmp_path):
    """hmat_build_batched merges independent instances (different sizes and
    kinds) into one block-diagonal H-matrix: each diagonal block equals that
    instance's oracle H-matrix, nothing couples two instances, and far
    levels count down from the top so that HM_MAX_LEVELS - 1 is every
    instance's leaf level.  The last instance has no far block at all."""
    probs = [W.sphere_problem(1200, math.sqrt(1200 / 1536)),
             W.cube_problem(10, 10 / 16),
             W.sphere_problem(450, math.sqrt(450 / 1536), seed=7)]
    leaf, tol = 32, 1e-5
    h = hmps.HMatrix(probs, leaf, 1.0, tol, flags=HOST)
    assert h.sizes == [1200, 1000, 450]
    path = str(tmp_path / "hb.bin")
    h.export(path)
    E = hmps.read_export(path)
    n = h.n
    A_lib = _lib_dense(E, n)
    top = hmps.HM_MAX_LEVELS - 1
    perm = []
    for i, p in enumerate(probs):
        o0, o1 = h.offsets[i], h.offsets[i + 1]
        H = hmatrix.HMatrix(p, leaf, 1.0, tol)
        perm.append(H.perm + o0)
        A_or = H.dense(min(H.far_levels) if H.far_levels else -1)
        blk = A_lib[o0:o1, o0:o1]
        assert np.linalg.norm(blk - A_or) <= 1e-12 * np.linalg.norm(A_or), i
        assert not A_lib[o0:o1, :o0].any() and not A_lib[o0:o1, o1:].any()
        rows = [r for r in E["far"] if o0 <= r[0] < o1]
        assert sorted({int(r[4]) for r in rows}) == sorted(top - (H.L - lv) for lv in H.far_levels)
        assert len(rows) == len(H.far)
    assert np.array_equal(E["perm"], np.concatenate(perm))
    info = h.info()
    assert info["num_instances"] == 3 and info["leaf_level"] == top
    h.close()


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets of
    its C declaration in include/hmps.h (compiled here with gcc)."""
    import ctypes as C
    import subprocess
    names = ["hm_problem", "hm_build_opts", "ps_opts", "ps_stats", "hm_info", "hm_kernel_time",
             "hm_tuning", "ps_server_stats"]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hmps.h"', "int main(void) {"]
    for nm in names:
        py = getattr(hmps, nm)
        lines.append(f'  printf("{nm} size %zu\\n", sizeof({nm}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{nm} {f} %zu\\n", offsetof({nm}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        nm, what, val = line.split()
        py = getattr(hmps, nm)
        got = C.sizeof(py) if what == "size" else getattr(py, what).offset
        assert got == int(val), (nm, what, got, val)


@pytest.mark.parametrize("case", [
    "min_not_max", "inclusive", "eta_below", "eta_equal", "diag_near", "diag_far", "gap_near",
    "gap_far"])
def test_library_partition_eq7_hand_worked(case, tmp_path):
    """The library's host build partitions the hand-worked eq. 7 cases of
    the oracle pins exactly as worked out by hand."""
    from test_oracle_build import EQ7_CASES, eq7_expected
    _, pts, eta, adm = [c for c in EQ7_CASES if c[0] == case][0]
    xyz = np.array(pts, dtype=np.float64)
    prob = W.Problem(W.SURFACE, xyz, W.WAVENUMBER, 0.1)
    h = hmps.HMatrix(prob, 2, eta, 1e-6, flags=HOST)
    path = str(tmp_path / "e.bin")
    h.export(path)
    E = hmps.read_export(path)
    lo, ls = E["leaf_off"], E["leaf_size"]
    assert list(zip(lo, ls)) == [(0, 2), (2, 2)]
    near = {(int(lo[t]), int(ls[t]), int(lo[s]), int(ls[s])) for t, s, _ in E["near"]}
    far = {((int(r[0]), int(r[1]), int(r[2]), int(r[3])), int(r[4])) for r in E["far"]}
    exp_near, exp_far = eq7_expected(adm)
    assert near == exp_near and far == exp_far
    h.close()


@pytest.mark.parametrize("key", [(1536, 1.0, 64), (24576, 4.0, 128)])
def test_library_partition_counts_match_independent_probe(key):
    """Near and per-level far block counts of the library's build of the
    1,536- and 24,576-point spheres equal those of an independent
    implementation."""
    from test_oracle_build import PROBE_COUNTS
    near, far = PROBE_COUNTS[key]
    n, radius, leaf = key
    prob = W.Problem(W.SURFACE, W.sphere_points(n, radius), W.WAVENUMBER,
                     W.sphere_spacing(n, radius))
    h = hmps.HMatrix(prob, leaf, 1.0, 1e-4, flags=HOST)
    info = h.info()
    assert info["near_blocks"] == near
    assert {lev: d["blocks"] for lev, d in info["far"].items()} == far
    h.close()
