"""Benchmark of the power-series H-matrix solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere_24576]
                    [--precision f64|f32] [--no-oracle] [--no-extras]

A step is one power-series solve (Sec. IV): permute in, y_0 = D^{-1} b,
K terms of stage A + D^{-1}-premultiplied near/far panel product + term
update, permute out, for the workload's right-hand sides, with the H-matrix
(blocks, leaf LU and inverse) already resident in HBM.  The result is checked
against the FP64 oracle; only a result within 1e-8 counts as solved.

Prints one JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
SOLVED_TOL = 1e-8


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import workloads as W
    if name == "sphere_1536":
        return W.sphere_small()
    if name == "sphere_24576":
        return W.sphere_large()
    if name.startswith("cube_"):
        n = round(int(name.split("_")[1]) ** (1 / 3))
        return W.cube_volume(n, 64)
    raise SystemExit(f"unknown workload {name}")


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere_24576")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the oracle check and CPU baseline (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the H-matvec, FP32 and refinement side measurements")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed region, copy a MIB-MiB device buffer 3 times (a plain "
                         "copy kernel of known size to scale HBM byte counters)")
    a = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design in DESIGN.md); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2307_03968_amd import hmps

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = workload(a.workload)
    prec = hmps.HM_F64 if a.precision == "f64" else hmps.HM_F32_APPLY
    log(f"library build {wl.name} n={wl.problem.n} leaf={wl.leaf_max} tol={wl.aca_tol}")
    t0 = time.perf_counter()
    h = hmps.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol)
    build_s = time.perf_counter() - t0
    info = h.info()
    L = info["leaf_level"]
    level = L if wl.level < 0 else wl.level
    b_np = wl.rhs()
    nrhs = b_np.shape[1]
    b = torch.from_numpy(np.ascontiguousarray(b_np)).to("cuda")
    x = None
    stream = torch.cuda.current_stream()

    for _ in range(a.warmup):
        x = h.solve(b, K=wl.K, level=wl.level, precision=prec)
    torch.cuda.synchronize()

    log(f"timed region: {a.steps} solves")
    # per-kernel HIP events (timing-only, no system fence) are recorded by the
    # library around every launch inside the timed region
    h_prof = hmps._lib().hm_profile_enable(h.handle, 1)
    assert h_prof == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        x = h.solve(b, K=wl.K, level=wl.level, precision=prec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = (hmps.hm_kernel_time * hmps.HM_K_COUNT)()
    assert hmps._lib().hm_profile_read(h.handle, kt) == 0
    hmps._lib().hm_profile_enable(h.handle, 0)
    # single-request latency: each solve issued and waited for on its own
    lat = []
    for i in range(a.steps):
        t1 = time.perf_counter()
        h.solve(b, K=wl.K, level=wl.level, precision=prec)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t1))
    step_ms = np.array(lat)
    if a.copy_calibration > 0:
        nbytes = a.copy_calibration << 20
        src_buf = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst_buf = torch.empty_like(src_buf)
        for _ in range(3):
            dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nbytes} bytes")
        del src_buf, dst_buf
    ms_per_step = wall * 1e3 / a.steps
    x_np = x.cpu().numpy()

    # ---- dominant kernel: one power-series term (k_term), algorithmic bytes:
    # series panel entries D^{-1}[near | U] + W entries of the level's far
    # blocks (all in-row at the leaf level, no separate stage-A pass), the
    # input y_{k-1}, the output y_k and x read + written.
    elem = 16 if prec == hmps.HM_F64 else 8
    n = wl.problem.n
    ent = info["series_entries"][level]
    went = info["stageA_entries"][level]
    kt_names = ["stageA", "term_series", "term_apply", "term_dinv"]
    kernels = {name: {"launches": kt[i].launches,
                      "avg_us": 1e3 * kt[i].total_ms / max(1, kt[i].launches)}
               for i, name in enumerate(kt_names)}
    assert kt[hmps.HM_K_STAGEA].launches == 0, "roofline bytes below assume no separate stage A"
    term_bytes = elem * (ent + went) + 16 * (4 * n)
    term = kt[hmps.HM_K_TERM_SERIES]
    term_ms = term.total_ms / max(1, term.launches)
    achieved = term_bytes / (term_ms * 1e-3) / 1e9
    per_solve_bytes = wl.K * (elem * (ent + went)) + 16 * info["diag_entries"]

    # ---- oracle check and CPU baseline
    rel = None
    cpu = None
    extras = {}
    H = None
    if not a.no_oracle:
        from oracle import hmatrix, series
        log("oracle build (host, FP64)")
        t1 = time.perf_counter()
        H = hmatrix.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol)
        oracle_build_s = time.perf_counter() - t1
        log("oracle series")
        ref = series.series(H, b_np, wl.K, wl.level)
        rel = series.rel_err(x_np, ref)
        log(f"rel.err vs oracle x_K = {rel:.3e}")
        # bounded sample: repeat the oracle's solve of the same workload
        t1 = time.perf_counter()
        reps = 0
        while reps < 1 or time.perf_counter() - t1 < a.cpu_seconds:
            series.series(H, b_np, wl.K, wl.level)
            reps += 1
        cpu_s = time.perf_counter() - t1
        cpu = {"value": reps * nrhs / cpu_s, "unit": "RHS/s", "cores": blas_threads(),
               "kind": "oracle",
               "sample": f"{reps} sequential numpy/scipy FP64 series solves of the same "
                         f"workload ({nrhs} RHS each) in {cpu_s:.1f} s; oracle H build "
                         f"{oracle_build_s:.1f} s not included"}
    solved = rel is not None and rel <= SOLVED_TOL
    value = (a.steps * nrhs / wall) if solved else 0.0

    # ---- side measurements: H-matvec GB/s, FP32 apply, refinement
    if not a.no_extras:
        xr = torch.randn(n, dtype=torch.complex128, device="cuda")
        for _ in range(3):
            h.apply(xr, level=wl.level)
        torch.cuda.synchronize()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            h.apply(xr, level=wl.level)
        e1.record(stream)
        torch.cuda.synchronize()
        mv_ms = e0.elapsed_time(e1) / reps
        mv_bytes = 16 * (info["apply_entries"][level] + info["stageA_entries"][level]) + 32 * n
        extras["hmatvec"] = {"ms": mv_ms, "bytes": mv_bytes,
                             "GBps": mv_bytes / (mv_ms * 1e-3) / 1e9,
                             "frac_hbm_peak": mv_bytes / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
        # FP32 apply series
        for _ in range(3):
            x32 = h.solve(b, K=wl.K, level=wl.level, precision=hmps.HM_F32_APPLY)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            x32 = h.solve(b, K=wl.K, level=wl.level, precision=hmps.HM_F32_APPLY)
        e1.record(stream)
        torch.cuda.synchronize()
        f32_ms = e0.elapsed_time(e1) / reps
        extras["series_f32_apply"] = {"ms_per_solve": f32_ms, "RHS_per_s": nrhs * 1e3 / f32_ms}
        if H is not None:
            extras["series_f32_apply"]["rel_err_vs_oracle_xK"] = series.rel_err(x32.cpu().numpy(), ref)
            extras["series_f64"] = {"rel_err_vs_oracle_xK": rel}
            rho = series.rho(H, wl.level, iters=60)
            extras["rho"] = rho
            if rho ** (wl.K + 1) < 0.9:
                log("oracle x* by GMRES for the refinement check")
                xs = series.solve_gmres(H, b_np, wl.level, tol=1e-13)
                for pname, p in (("f32_apply", hmps.HM_F32_APPLY), ("f64", hmps.HM_F64)):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    xr_, st = h.solve(b, K=wl.K, level=wl.level, precision=p,
                                      kind=hmps.PS_REFINE, max_passes=400, refine_tol=1e-10,
                                      stats=True)
                    torch.cuda.synchronize()
                    ref_s = time.perf_counter() - t1
                    err = series.rel_err(xr_.cpu().numpy(), xs)
                    extras[f"refine_{pname}"] = {
                        "ms_per_solve": 1e3 * ref_s, "passes": st[0]["passes"],
                        "rel_err_vs_oracle_xstar": err,
                        "solved_RHS_per_s": (nrhs / ref_s) if err <= SOLVED_TOL else 0.0}
            else:
                extras["refine"] = (f"not attainable by the method: rho^(K+1) = "
                                    f"{rho ** (wl.K + 1):.3f}")

    out = {
        "metric": "solved RHS/s at rel.err<=1e-8 vs FP64 oracle",
        "value": value,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == hmps.HM_F64 else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "N": n, "kind": "surface" if wl.problem.kind == 0 else "volume",
                   "leaf_max": wl.leaf_max, "eta": wl.eta, "aca_tol": wl.aca_tol, "K": wl.K,
                   "level": level, "nrhs": nrhs,
                   "precision": "complex128" if prec == hmps.HM_F64 else "complex64 blocks, complex128 vectors"},
        "rel_err_vs_oracle": rel,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                       "p99": float(np.percentile(step_ms, 99))},
        "roofline": {"bound": "hbm", "kernel": "k_term (one series term)", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": None, "bytes_per_launch": term_bytes,
                     "avg_launch_us": term_ms * 1e3},
        "per_solve_algorithmic_bytes": per_solve_bytes,
        "kernels": kernels,
        "build_s": build_s,
        "device_bytes": info["device_bytes"],
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    h.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
