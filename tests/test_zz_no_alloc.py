"""The allocation-free solve entry point (ps_solve_noalloc) against
ps_solve, through the C-ABI: the same kernels on a static device workspace
give the same result bit for bit, call after call, with later calls smaller
than earlier ones (the static array keeps the previous contents), and a
workspace larger than the array is refused before any device work."""
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


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _cols(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.complex128).T)).to("cuda")


def _noalloc(h, bc, K, precision=hmps.HM_F64, kind=hmps.PS_SERIES, passes=0):
    """ps_solve_noalloc on (nrhs, n) column tensor bc; returns (status, x)."""
    lib = hmps._lib()
    xc = torch.full_like(bc, complex(np.nan, np.nan))
    o = hmps.ps_opts(int(K), -1, int(precision), int(kind), int(passes), 1e-9, 0)
    st = lib.ps_solve_noalloc(h.handle, C.byref(o), C.c_void_p(bc.data_ptr()), h.n,
                              C.c_void_p(xc.data_ptr()), h.n, bc.shape[0],
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, xc.t().cpu().numpy()


def _ref(h, bc, K, precision=hmps.HM_F64, kind=hmps.PS_SERIES, passes=0):
    x = h.solve(bc.t(), K=K, precision=precision, kind=kind, max_passes=passes)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def test_noalloc_matches_ps_solve_two_calls_second_smaller():
    big = W.sphere_problem(2200, math.sqrt(2200 / 1536))   # ragged depths, far levels 5-6
    small = W.sphere_problem(700, math.sqrt(700 / 1536), instance=3)
    _say("noalloc: build sphere_2200 leaf 68 and sphere_700 leaf 64")
    hb = hmps.HMatrix(big, 68, 1.0, 1e-4)
    hs = hmps.HMatrix(small, 64, 1.0, 1e-4)
    Bb = W.plane_waves(big.xyz, W.directions(16, 3))
    Bs = W.plane_waves(small.xyz, W.directions(3, 5))
    Hb = hmatrix.HMatrix(big, 68, 1.0, 1e-4)
    Hs = hmatrix.HMatrix(small, 64, 1.0, 1e-4)
    # call 1: 16 RHS on the matrix cores (FP32 blocks), call 2: fewer RHS on
    # the streaming kernels, call 3: a smaller geometry, call 4: one RHS of a
    # symmetric problem (half storage), call 5: fixed-pass refinement
    cases = [(hb, Bb, Hb, hmps.HM_F32_APPLY, hmps.PS_SERIES, 0, 1e-4),
             (hb, Bb[:, :5], Hb, hmps.HM_F64, hmps.PS_SERIES, 0, 1e-10),
             (hs, Bs, Hs, hmps.HM_F64, hmps.PS_SERIES, 0, 1e-10),
             (hs, Bs[:, :1], Hs, hmps.HM_F64, hmps.PS_SERIES, 0, 1e-10),
             (hs, Bs[:, :2], Hs, hmps.HM_F32_APPLY, hmps.PS_REFINE_FIXED, 30, None)]
    for rep in range(2):
        for i, (h, B, H, prec, kind, passes, tol) in enumerate(cases):
            _say(f"noalloc rep {rep} case {i}: n={h.n} nrhs={B.shape[1]} precision={prec} kind={kind}")
            bc = _cols(B)
            st, x = _noalloc(h, bc, 4, prec, kind, passes)
            assert st == hmps.HM_OK, hmps._lib().hm_last_error()
            ref = _ref(h, bc, 4, prec, kind, passes)
            assert np.array_equal(x, ref), (rep, i)
            if tol is not None:
                assert_close(x, series.series(H, B, 4), tol, (rep, i))
            else:  # 30 passes at rho^5 ~ 0.2 each: x* to rounding
                assert series.rho(H) ** 5 < 0.5
                assert_close(x, series.solve_exact(H, B), 1e-8, (rep, i))
    hb.close()
    hs.close()


def test_noalloc_refuses_oversize_and_other_kinds():
    prob = W.sphere_problem(1536, 1.0)
    h = hmps.HMatrix(prob, 64, 1.0, 1e-4)
    lib = hmps._lib()
    nrhs = 4096   # workspace far above the static array
    b = torch.zeros((nrhs, h.n), dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(b)
    o = hmps.ps_opts(4, -1, hmps.HM_F64, hmps.PS_SERIES, 0, 1e-9, 0)
    _say("noalloc: oversize refused")
    st = lib.ps_solve_noalloc(h.handle, C.byref(o), C.c_void_p(b.data_ptr()), h.n,
                              C.c_void_p(x.data_ptr()), h.n, nrhs, None)
    assert st == hmps.HM_EINVAL and b"static scratch" in lib.hm_last_error()
    for kind in (hmps.PS_REFINE, hmps.PS_GMRES, hmps.PS_NESTED):
        o = hmps.ps_opts(4, -1, hmps.HM_F64, kind, 5, 1e-9, 0)
        assert lib.ps_solve_noalloc(h.handle, C.byref(o), C.c_void_p(b.data_ptr()), h.n,
                                    C.c_void_p(x.data_ptr()), h.n, 1, None) == hmps.HM_EINVAL
    torch.cuda.synchronize()
    assert not torch.any(x != 0).item()   # nothing ran
    h.close()
