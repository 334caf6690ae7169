"""ctypes binding of libhmps (include/hmps.h).

Argument marshalling only: every step of the build's device part and of the
solve runs in the library.  Device vectors are torch complex128 CUDA tensors;
the binding passes their data pointers and the current torch stream.

Layout: the C-ABI takes column-major n x nrhs arrays.  A torch tensor of
shape (nrhs, n), contiguous, is exactly that; the helpers below accept
(n,) or (n, nrhs) tensors and return (n,) or (n, nrhs) views.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmps.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hmps.h")

HM_OK, HM_ENOTREADY, HM_EDIVERGED = 0, 1, 2
HM_EINVAL, HM_ENOMEM, HM_EHIP, HM_EBUSY, HM_ESTATE = -1, -2, -3, -4, -5
HM_SURFACE, HM_VOLUME = 0, 1
HM_F64, HM_F32_APPLY = 0, 1
PS_SERIES, PS_REFINE, PS_REFINE_FIXED, PS_GMRES, PS_NESTED = 0, 1, 2, 3, 4
HM_BUILD_HOST_ONLY, HM_BUILD_NO_F32, HM_BUILD_KEEP_HOST, HM_BUILD_NO_HALF = 0x1, 0x2, 0x4, 0x8
HM_MAX_LEVELS = 32
HM_NOALLOC_SCRATCH_BYTES = 64 << 20


class hm_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", C.POINTER(C.c_double)), ("kind", C.c_int32),
                ("k", C.c_double), ("h", C.c_double), ("chi", C.POINTER(C.c_double))]


PROGRESS_FN = C.CFUNCTYPE(None, C.c_char_p, C.c_void_p)


class hm_build_opts(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("eta", C.c_double), ("aca_tol", C.c_double),
                ("max_rank", C.c_int32), ("flags", C.c_uint32), ("num_threads", C.c_int32),
                ("progress", PROGRESS_FN), ("progress_user", C.c_void_p)]


class ps_opts(C.Structure):
    _fields_ = [("K", C.c_int32), ("level", C.c_int32), ("precision", C.c_int32),
                ("kind", C.c_int32), ("max_passes", C.c_int32), ("refine_tol", C.c_double),
                ("restart", C.c_int32)]


class ps_stats(C.Structure):
    _fields_ = [("passes", C.c_int32), ("diverged", C.c_int32), ("resid_rel", C.c_double),
                ("growth", C.c_double), ("t_ms", C.c_double), ("built", C.c_int32),
                ("reserved_", C.c_int32)]


PS_QUEUED, PS_RUNNING, PS_DONE, PS_FAILED = 0, 1, 2, 3


class ps_server_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "budget_bytes", "resident_bytes", "resident_geometries", "builds", "evictions", "batches",
        "batch_rhs", "requests_submitted", "requests_done", "requests_failed", "rhs_done",
        "queued", "split_batches")]


class hm_tuning(C.Structure):
    _fields_ = [("mm_min_rhs", C.c_int32), ("term_wgs", C.c_int32), ("rhs_tile", C.c_int32),
                ("inrow_pct", C.c_int32), ("half_storage", C.c_int32), ("mm_multi", C.c_int32)]


class hm_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaf_level", C.c_int32), ("num_leaves", C.c_int32),
                ("max_leaf", C.c_int32), ("min_far_level", C.c_int32),
                ("near_blocks", C.c_int64), ("near_offdiag_entries", C.c_int64),
                ("diag_entries", C.c_int64),
                ("far_blocks", C.c_int64 * HM_MAX_LEVELS),
                ("far_rank_sum", C.c_int64 * HM_MAX_LEVELS),
                ("far_entries", C.c_int64 * HM_MAX_LEVELS),
                ("device_bytes", C.c_int64), ("build_ms", C.c_double),
                ("series_entries", C.c_int64 * HM_MAX_LEVELS),
                ("apply_entries", C.c_int64 * HM_MAX_LEVELS),
                ("stageA_entries", C.c_int64 * HM_MAX_LEVELS),
                ("coeffs", C.c_int64 * HM_MAX_LEVELS),
                ("num_instances", C.c_int32),
                ("half_entries", C.c_int64 * HM_MAX_LEVELS)]


HM_K_STAGEA, HM_K_TERM_SERIES, HM_K_TERM_APPLY, HM_K_TERM_DINV, HM_K_COUNT = range(5)


class hm_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double)]


class HmpsError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_lib().hm_strerror(status).decode()} ({status}): "
                         f"{_lib().hm_last_error().decode()}")
        self.status = status


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libhmps is not built ({LIB_PATH} missing); run "
                              "`python -m paper_2307_03968_amd.build`")
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        lib.hmat_build.argtypes = [C.POINTER(hm_problem), C.POINTER(hm_build_opts), vp, C.POINTER(vp)]
        lib.hmat_build_batched.argtypes = [C.POINTER(hm_problem), i32, C.POINTER(hm_build_opts), vp,
                                           C.POINTER(vp)]
        lib.hmat_info.argtypes = [vp, C.POINTER(hm_info)]
        lib.hmat_apply.argtypes = [vp, i32, i32, vp, i64, vp, i64, i32, vp]
        lib.ps_solve.argtypes = [vp, C.POINTER(ps_opts), vp, i64, vp, i64, i32, C.POINTER(ps_stats), vp]
        lib.ps_solve_noalloc.argtypes = [vp, C.POINTER(ps_opts), vp, i64, vp, i64, i32, vp]
        lib.hmat_export.argtypes = [vp, C.c_char_p]
        lib.hmat_free.argtypes = [vp]
        lib.hm_profile_enable.argtypes = [vp, i32]
        lib.hm_profile_read.argtypes = [vp, C.POINTER(hm_kernel_time)]
        lib.hmat_tune.argtypes = [vp, C.POINTER(hm_tuning), vp]
        lib.hmat_get_tuning.argtypes = [vp, C.POINTER(hm_tuning)]
        lib.hmat_autotune.argtypes = [vp, C.POINTER(ps_opts), i32, vp, C.POINTER(hm_tuning),
                                      C.POINTER(C.c_double)]
        lib.ps_server_create.argtypes = [C.c_size_t, i32, C.POINTER(vp)]
        lib.ps_submit.argtypes = [vp, C.c_uint64, C.POINTER(hm_problem), C.POINTER(hm_build_opts),
                                  C.POINTER(ps_opts), vp, i32, C.POINTER(C.c_uint64)]
        lib.ps_poll.argtypes = [vp, C.c_uint64, vp, C.POINTER(ps_stats), C.POINTER(i32)]
        lib.ps_server_info.argtypes = [vp, C.POINTER(ps_server_stats)]
        lib.ps_server_destroy.argtypes = [vp]
        lib.hm_strerror.argtypes = [C.c_int]
        lib.hm_strerror.restype = C.c_char_p
        lib.hm_last_error.restype = C.c_char_p
        for f in ("hmat_build", "hmat_build_batched", "hmat_info", "hmat_apply", "ps_solve",
                  "ps_solve_noalloc", "hmat_export", "hmat_free", "hm_profile_enable", "hm_profile_read", "hmat_tune",
                  "hmat_get_tuning", "hmat_autotune", "ps_server_create", "ps_submit", "ps_poll",
                  "ps_server_info", "ps_server_destroy"):
            getattr(lib, f).restype = C.c_int
        _LIB = lib
    return _LIB


def header_functions():
    """Names of the functions include/hmps.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+(?:\s+|\s*\*+\s*)(\w+)\s*\(", txt, flags=re.M)))


def _check(status: int, what: str, allow=(HM_OK,)):
    if status not in allow:
        raise HmpsError(status, what)
    return status


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _on_stream(stream, *tensors):
    """Order a call on `stream` after the work of torch's current stream
    (which produced the inputs and allocated the temporaries) and keep the
    caching allocator from reusing the tensors before `stream` is done."""
    import torch
    if stream is None or stream == torch.cuda.current_stream():
        return
    stream.wait_stream(torch.cuda.current_stream())
    for t in tensors:
        t.record_stream(stream)


def _as_cols(t):
    """(n,) or (n, nrhs) complex128 CUDA tensor -> (nrhs, n) contiguous."""
    import torch
    if t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError("expected a complex128 CUDA tensor")
    if t.dim() == 1:
        return t.reshape(1, -1).contiguous()
    return t.t().contiguous()


class HMatrix:
    """Owning wrapper of an hm_matrix_t."""

    def __init__(self, prob, leaf_max: int, eta: float = 1.0, aca_tol: float = 1e-4,
                 max_rank: int = 0, flags: int = 0, num_threads: int = 0, stream=None,
                 progress=None):
        """``prob``: one problem, or a list of problems for a batched handle
        (hmat_build_batched).  ``progress``: optional callable taking the
        build's progress messages (str)."""
        lib = _lib()
        probs = list(prob) if isinstance(prob, (list, tuple)) else [prob]
        keep = []
        arr = (hm_problem * len(probs))()
        for i, p in enumerate(probs):
            xyz = np.ascontiguousarray(p.xyz, dtype=np.float64)
            chi = None if p.chi is None else np.ascontiguousarray(p.chi, dtype=np.float64)
            keep += [xyz, chi]
            arr[i] = hm_problem(xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)), int(p.kind),
                                float(p.k), float(p.h),
                                chi.ctypes.data_as(C.POINTER(C.c_double)) if chi is not None else None)
        cb = PROGRESS_FN(lambda msg, _u: progress(msg.decode())) if progress else PROGRESS_FN()
        o = hm_build_opts(int(leaf_max), float(eta), float(aca_tol), int(max_rank), int(flags),
                          int(num_threads), cb, None)
        self.host_only = bool(flags & HM_BUILD_HOST_ONLY)
        st = C.c_void_p(None) if self.host_only else _stream(stream)
        h = C.c_void_p()
        if isinstance(prob, (list, tuple)):
            _check(lib.hmat_build_batched(arr, len(probs), C.byref(o), st, C.byref(h)),
                   "hmat_build_batched")
        else:
            _check(lib.hmat_build(C.byref(arr[0]), C.byref(o), st, C.byref(h)), "hmat_build")
        self._h = h
        self.sizes = [int(p.xyz.shape[0]) for p in probs]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            _lib().hmat_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = hm_info()
        _check(_lib().hmat_info(self._h, C.byref(i)), "hmat_info")
        per_level = ("far_", "series_entries", "apply_entries", "stageA_entries", "coeffs",
                     "half_entries")
        d = {k: getattr(i, k) for k, _ in hm_info._fields_ if not k.startswith(per_level)}
        for k in per_level[1:]:
            d[k] = list(getattr(i, k))
        d["far"] = {lev: {"blocks": i.far_blocks[lev], "rank_sum": i.far_rank_sum[lev],
                          "entries": i.far_entries[lev]}
                    for lev in range(HM_MAX_LEVELS) if i.far_blocks[lev]}
        return d

    def tune(self, mm_min_rhs: int = 0, term_wgs: int = 0, rhs_tile: int = 0, inrow_pct: int = 0,
             half_storage: int = 0, mm_multi: int = 0, stream=None) -> None:
        """hmat_tune: 0 keeps a value, -1 restores its default."""
        t = hm_tuning(int(mm_min_rhs), int(term_wgs), int(rhs_tile), int(inrow_pct),
                      int(half_storage), int(mm_multi))
        _check(_lib().hmat_tune(self._h, C.byref(t), _stream(stream)), "hmat_tune")

    def tuning(self) -> dict:
        t = hm_tuning()
        _check(_lib().hmat_get_tuning(self._h, C.byref(t)), "hmat_get_tuning")
        return {"mm_min_rhs": t.mm_min_rhs, "term_wgs": t.term_wgs, "rhs_tile": t.rhs_tile,
                "inrow_pct": t.inrow_pct, "half_storage": t.half_storage, "mm_multi": t.mm_multi}

    def autotune(self, nrhs: int, K: int, level: int = -1, precision: int = HM_F64,
                 stream=None):
        """hmat_autotune: returns (tuning dict, ms per solve of the choice)."""
        o = ps_opts(int(K), int(level), int(precision), PS_SERIES, 0, 1e-9)
        t = hm_tuning()
        ms = C.c_double()
        _check(_lib().hmat_autotune(self._h, C.byref(o), int(nrhs), _stream(stream), C.byref(t),
                                    C.byref(ms)), "hmat_autotune")
        return {"mm_min_rhs": t.mm_min_rhs, "term_wgs": t.term_wgs, "rhs_tile": t.rhs_tile,
                "inrow_pct": t.inrow_pct, "half_storage": t.half_storage, "mm_multi": t.mm_multi}, ms.value

    def export(self, path: str) -> None:
        _check(_lib().hmat_export(self._h, path.encode()), "hmat_export")

    def apply(self, x, level: int = -1, precision: int = HM_F64, out=None, stream=None):
        """y = Z_level x on the device (original point order)."""
        import torch
        xc = _as_cols(x)
        nrhs = xc.shape[0]
        yc = torch.empty_like(xc) if out is None else out
        _on_stream(stream, xc, yc)
        _check(_lib().hmat_apply(self._h, level, precision, C.c_void_p(xc.data_ptr()), self.n,
                                 C.c_void_p(yc.data_ptr()), self.n, nrhs, _stream(stream)),
               "hmat_apply")
        return yc.reshape(-1) if x.dim() == 1 else yc.t()

    def solve(self, b, K: int, level: int = -1, precision: int = HM_F64, kind: int = PS_SERIES,
              max_passes: int = 0, refine_tol: float = 1e-9, stats: bool = False, out=None,
              stream=None, restart: int = 0):
        """Power-series solve (or GMRES preconditioned by the series, kind =
        PS_GMRES); returns x (and per-RHS stats when asked)."""
        import torch
        bc = _as_cols(b)
        nrhs = bc.shape[0]
        xc = torch.empty_like(bc) if out is None else out
        _on_stream(stream, bc, xc)
        o = ps_opts(int(K), int(level), int(precision), int(kind), int(max_passes), float(refine_tol),
                    int(restart))
        st_arr = (ps_stats * nrhs)() if stats else None
        status = _lib().ps_solve(self._h, C.byref(o), C.c_void_p(bc.data_ptr()), self.n,
                                 C.c_void_p(xc.data_ptr()), self.n, nrhs,
                                 st_arr if stats else None, _stream(stream))
        _check(status, "ps_solve", allow=(HM_OK, HM_EDIVERGED))
        x = xc.reshape(-1) if b.dim() == 1 else xc.t()
        if stats:
            return x, [{k: getattr(s, k) for k, _ in ps_stats._fields_} for s in st_arr]
        return x


_DT = {1: np.int32, 2: np.int64, 3: np.float64, 4: np.complex128}


def read_export(path: str) -> Dict[str, np.ndarray]:
    """Read the named-array file written by hmat_export."""
    out = {}
    with open(path, "rb") as f:
        while True:
            hdr = f.read(4)
            if not hdr:
                break
            nl = int(np.frombuffer(hdr, np.uint32)[0])
            name = f.read(nl).decode()
            dt, nd = np.frombuffer(f.read(8), np.uint32)
            shape = tuple(int(s) for s in np.frombuffer(f.read(8 * int(nd)), np.uint64)) if nd else ()
            dtype = np.dtype(_DT[int(dt)])
            cnt = int(np.prod(shape)) if shape else 1
            out[name] = np.frombuffer(f.read(cnt * dtype.itemsize), dtype).reshape(shape)
    return out


def _problem_struct(p):
    """hm_problem for a workloads.Problem; returns (struct, arrays to keep alive)."""
    xyz = np.ascontiguousarray(p.xyz, dtype=np.float64)
    chi = None if p.chi is None else np.ascontiguousarray(p.chi, dtype=np.float64)
    st = hm_problem(xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)), int(p.kind),
                    float(p.k), float(p.h),
                    chi.ctypes.data_as(C.POINTER(C.c_double)) if chi is not None else None)
    return st, (xyz, chi)


class Server:
    """Owning wrapper of an hm_server_t (ps_server_create ... ps_server_destroy)."""

    def __init__(self, budget_bytes: int = 0, slots: int = 2):
        s = C.c_void_p()
        _check(_lib().ps_server_create(int(budget_bytes), int(slots), C.byref(s)), "ps_server_create")
        self._s = s
        self._shape = {}
        self._n = {}

    def submit(self, key: int, b: np.ndarray, K: int, level: int = -1, precision: int = HM_F64,
               kind: int = PS_SERIES, max_passes: int = 0, refine_tol: float = 1e-9, prob=None,
               leaf_max: int = 64, eta: float = 1.0, aca_tol: float = 1e-4,
               restart: int = 0) -> int:
        """Queue a solve of b (n x nrhs or n, complex128, original order) on
        geometry `key`; `prob` is required the first time a key is used."""
        b = np.asarray(b, dtype=np.complex128)
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        bc = np.asfortranarray(b.reshape(b.shape[0], nrhs))
        o = ps_opts(int(K), int(level), int(precision), int(kind), int(max_passes), float(refine_tol),
                    int(restart))
        pp = bo = None
        if prob is not None:
            pst, keep = _problem_struct(prob)
            pp = C.byref(pst)
            bo = C.byref(hm_build_opts(int(leaf_max), float(eta), float(aca_tol), 0, 0, 0,
                                       PROGRESS_FN(), None))
            self._n[key] = bc.shape[0]
        t = C.c_uint64()
        _check(_lib().ps_submit(self._s, C.c_uint64(key), pp, bo, C.byref(o),
                                bc.ctypes.data_as(C.c_void_p), nrhs, C.byref(t)), "ps_submit")
        self._shape[t.value] = (bc.shape[0], nrhs, b.ndim)
        return t.value

    def poll(self, ticket: int, want_x: bool = True):
        """(state, x or None, stats list or None) once done (x None when
        want_x is false); (state, None, None) while queued or running.
        Raises on a failed ticket."""
        n, nrhs, nd = self._shape[ticket]
        state = C.c_int32()
        status = _lib().ps_poll(self._s, C.c_uint64(ticket), None, None, C.byref(state))
        if status == HM_ENOTREADY:
            return state.value, None, None
        x = np.empty((nrhs, n), np.complex128) if want_x else None
        st = (ps_stats * nrhs)()
        status = _lib().ps_poll(self._s, C.c_uint64(ticket),
                                x.ctypes.data_as(C.c_void_p) if want_x else None, st,
                                C.byref(state))
        del self._shape[ticket]
        _check(status, "ps_poll (ticket %d)" % ticket, allow=(HM_OK, HM_EDIVERGED))
        xs = None if x is None else (x.T if nd == 2 else x[0])
        return state.value, xs, [{k: getattr(s, k) for k, _ in ps_stats._fields_} for s in st]

    def wait(self, ticket: int, timeout_s: float = 600.0, sleep_s: float = 0.0005):
        import time
        t0 = time.perf_counter()
        while True:
            state, x, st = self.poll(ticket)
            if st is not None:
                return x, st
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")
            time.sleep(sleep_s)

    def info(self) -> dict:
        i = ps_server_stats()
        _check(_lib().ps_server_info(self._s, C.byref(i)), "ps_server_info")
        return {k: getattr(i, k) for k, _ in ps_server_stats._fields_}

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value is not None:
            _lib().ps_server_destroy(self._s)
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
