"""Benchmark of the power-series H-matrix solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision f64|f32] [--no-oracle] [--no-extras]

Workloads:
  sphere_24576  (default) surface, N = 24,576, leaf <= 128, tol 1e-4, K = 4,
                one plane wave, FP64; side runs: H-matvec, FP32 blocks,
                refinement, GMRES preconditioned by the series
  cube_32768    volume, N = 32^3, leaf <= 128, tol 1e-5, K = 5, 64 plane
                waves; FP64 (4M) and FP32 (3M) matrix-core kernels; side run:
                GMRES preconditioned by D^{-1} (the series diverges there)
  batched_256   256 surface instances, N log-uniform in [512, 8192], leaf <= 64,
                tol 1e-4, K = 4, 16 plane waves each, one batched handle,
                autotuned, solves replayed from a captured HIP graph; FP32
                blocks with FP64 refinement against the plain FP64 path
  served        Poisson request stream over 16 surface + 16 volume
                geometries (N in [1024, 65536], 1..64 RHS) through the request
                server; mixed precision and plain FP64
  sphere_1536   the small surface case

A step is one power-series solve (Sec. IV): permute in, y_0 = D^{-1} b,
K terms of stage A + D^{-1}-premultiplied near/far panel product + term
update, permute out, for the workload's right-hand sides, with the H-matrix
(blocks, leaf LU and inverse) already resident in HBM.  The result is checked
against the FP64 oracle; only a result within 1e-8 of its reference counts as
solved.

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # dense MFMA (= vector) peaks
SOLVED_TOL = 1e-8
METRIC = "solved RHS/s at rel.err<=1e-8 vs FP64 oracle"


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


def cpu_model():
    """The host CPU's model name (as lscpu prints it) and its logical CPUs."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs on the host, "\
           f"{len(os.sched_getaffinity(0))} available to this process)"


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def timed(fn, reps, stream):
    """Average ms of fn() over reps calls, HIP events on `stream`."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def profiled(h, fn, reps):
    """Per-kernel-class launches and average duration (library HIP events
    around every launch, recorded on the launch stream) over reps calls."""
    import torch
    from paper_2307_03968_amd import hmps
    lib = hmps._lib()
    assert lib.hm_profile_enable(h.handle, 1) == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = (hmps.hm_kernel_time * hmps.HM_K_COUNT)()
    assert lib.hm_profile_read(h.handle, kt) == 0
    lib.hm_profile_enable(h.handle, 0)
    names = ["stageA", "term_series", "term_apply", "term_dinv"]
    return wall, {nm: {"launches": kt[i].launches,
                       "avg_us": 1e3 * kt[i].total_ms / max(1, kt[i].launches)}
                  for i, nm in enumerate(names)}


def copy_calibration(a):
    """With --copy-calibration MIB: three device copies of a MIB-MiB buffer
    (a plain copy kernel of known size that scales the HBM byte counters)."""
    import torch
    if a.copy_calibration <= 0:
        return
    nbytes = a.copy_calibration << 20
    src_buf = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst_buf = torch.empty_like(src_buf)
    for _ in range(3):
        dst_buf.copy_(src_buf)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {nbytes} bytes")
    del src_buf, dst_buf


def latency(fn, reps):
    """Per-request latency: each call issued and waited for on its own."""
    import torch
    lat = []
    for _ in range(reps):
        t1 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t1))
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}


def recorded_traffic(workload_name, prec, kernel):
    """HBM bytes per launch of `kernel` from the FETCH_SIZE / WRITE_SIZE
    runs summarised under profiles/ (calibrated against a device copy), or
    None when there is none or any source listed with it (the kernel, its
    shared headers) changed since."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-record:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
            if (kv.get("workload"), kv.get("precision"), kv.get("kernel")) != (workload_name, prec, kernel):
                continue
            # sha256 over the listed sources, concatenated in the order given
            digest = hashlib.sha256()
            for rel in kv["source"].split(","):
                src = os.path.join(ROOT, rel)
                if not os.path.exists(src):
                    return None
                digest.update(open(src, "rb").read())
            if digest.hexdigest() != kv["sha256"]:
                return None
            return float(kv["bytes_per_launch"])
    return None


def terms_per_launch(K, reps, kern):
    """Series terms one term-kernel launch ran: 1, or K where the K terms
    run as one launch (half storage, far blocks all between two leaves)."""
    n = kern["term_series"]["launches"]
    return max(1, round(K * reps / n)) if n else 1


def term_roofline(info, level, n, nrhs, prec, mm, avg_us, T, workload_name=None, half=False,
                  terms=1):
    """Roofline of one series-term launch.  Algorithmic bytes: the level's
    series panel entries (D^{-1}[near | U]) plus, on the one-RHS kernels,
    the W rows of the far blocks read in the same launch; or with half
    storage the entries of the scaled operator S it reads (near blocks
    s > t once, far blocks between two leaves once as U' and W', U' and W'
    of the other far blocks per orientation); plus the vectors (y_{k-1} with its t part
    read, y_k written, x read and written), times the terms one launch
    runs.  Flops (matrix-core kernels):
    executed real flops, 6 per complex multiply-add in FP32 (3M), 8 in
    FP64 (4M)."""
    elem = 16 if prec == "f64" else 8
    ent = info["half_entries" if half else "series_entries"][level]
    went = 0 if (mm or half) else info["stageA_entries"][level]
    vec = 16 * nrhs * ((n + (T if mm else 0)) + 3 * n)
    nbytes = terms * (elem * (ent + went) + vec)
    gbps = nbytes / (avg_us * 1e-6) / 1e9
    kname = "k_term_mm" if mm else ("k_half" if half else "k_term")
    traffic = recorded_traffic(workload_name, prec, kname)
    label = {"k_term_mm": "k_term_mm (one series term)", "k_term": "k_term (one series term)",
             "k_half": "k_half (one scaled series term, half storage)"}[kname]
    if terms > 1:
        label = f"k_half (the {terms} scaled series terms in one launch, half storage)"
    out = {"bound": "hbm", "kernel": label,
           "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
           "traffic": traffic, "bytes_per_launch": nbytes, "avg_launch_us": avg_us,
           "traffic_note": "L2-to-memory bytes per launch, 2 x FETCH_SIZE + WRITE_SIZE (profiles/)"
                           if traffic else "no counter run for this kernel source"}
    if mm:
        flops = (6 if prec == "f32" else 8) * ent * nrhs
        tf = flops / (avg_us * 1e-6) / 1e12
        fl = {"bound": "mfma", "achieved": tf, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
              "frac": tf / PEAK_TFLOPS[prec], "flops_per_launch": flops,
              "effective_TFLOPs_8_per_cmac": 8 * ent * nrhs / (avg_us * 1e-6) / 1e12}
        if fl["frac"] >= out["frac"]:
            hb = {k: out[k] for k in ("achieved", "frac")}
            out.update(fl)
            out["hbm_side"] = hb
        else:
            out["mfma_side"] = {k: fl[k] for k in ("achieved", "frac", "peak")}
    return out


# --------------------------------------------------------------------------
GMRES_TOL = 1e-10  # relative residual the GMRES legs stop at


def gmres_run(h, b, K, level, precision):
    """One untimed GMRES solve, then one timed: (x, stats, ms)."""
    import torch
    from paper_2307_03968_amd import hmps
    kw = dict(K=K, level=level, precision=precision, kind=hmps.PS_GMRES, max_passes=1000,
              refine_tol=GMRES_TOL)
    h.solve(b, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, st = h.solve(b, stats=True, **kw)
    torch.cuda.synchronize()
    return x, st, 1e3 * (time.perf_counter() - t1)


def bench_single(a):
    import torch
    from paper_2307_03968_amd import hmps

    wl = workload(a.workload)
    cube = wl.problem.kind == 1
    pname = a.precision or "f64"
    prec = hmps.HM_F64 if pname == "f64" else hmps.HM_F32_APPLY
    log(f"library build {wl.name} n={wl.problem.n} leaf={wl.leaf_max} tol={wl.aca_tol}")
    t0 = time.perf_counter()
    marks = []

    def progress(msg):
        marks.append((time.perf_counter() - t0, msg))
        log(msg)
    h = hmps.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol, progress=progress)
    build_s = time.perf_counter() - t0
    # seconds of each build phase, ending at its progress message
    build_phases = [[msg, round(t - (marks[i - 1][0] if i else 0.0), 4)] for i, (t, msg) in enumerate(marks)]
    info = h.info()
    L = info["leaf_level"]
    level = L if wl.level < 0 else wl.level
    b_np = wl.rhs()
    nrhs = b_np.shape[1]
    n = wl.problem.n
    b = torch.from_numpy(np.ascontiguousarray(b_np)).to("cuda")
    stream = torch.cuda.current_stream()
    log("autotune")
    tune = h.autotune(nrhs, K=wl.K, level=wl.level, precision=prec)
    log(f"autotune: {tune}")
    mm = nrhs >= h.tuning()["mm_min_rhs"]
    # one right-hand side of a symmetric problem: the scaled series on half
    # storage when the tuning keeps it
    # one right-hand side runs on half storage where the handle has it
    # (surface problems, and volume ones through their symmetric part)
    half1 = h.tuning()["half_storage"] in (1, 3) and info["half_entries"][level] > 0
    half = half1 and not mm and nrhs == 1
    solve = lambda p=prec: h.solve(b, K=wl.K, level=wl.level, precision=p)  # noqa: E731

    for _ in range(a.warmup):
        x = solve()
    torch.cuda.synchronize()
    log(f"timed region: {a.steps} solves")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        x = solve()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same solve captured into a HIP graph and replayed: the solve only
    # enqueues device work, so a replay saves the host's per-launch cost
    # (what bounds the small problems); kept only if bit-equal to the eager one
    xg = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        h.solve(b, K=wl.K, level=wl.level, precision=prec, out=xg)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        h.solve(b, K=wl.K, level=wl.level, precision=prec, out=xg)
    for _ in range(a.warmup):
        graph.replay()
    torch.cuda.synchronize()
    log(f"timed region: {a.steps} graph replays")
    t0 = time.perf_counter()
    for _ in range(a.steps):
        graph.replay()
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    # the same solves again with HIP events around every launch (on the
    # launch stream) for the per-kernel durations of the roofline
    _, kernels = profiled(h, solve, a.steps)
    x = solve()
    torch.cuda.synchronize()
    graph_equal = bool(torch.equal(xg.t(), x.reshape(n, nrhs)))
    use_graph = graph_equal and wall_graph < wall
    log(f"eager {1e3 * wall / a.steps:.3f} ms/solve, graph replay "
        f"{1e3 * wall_graph / a.steps:.3f} ms/solve, equal: {graph_equal}")
    wall_eager = wall
    if use_graph:
        wall = wall_graph
    lat = latency(solve, a.steps)
    copy_calibration(a)
    ms_per_step = wall * 1e3 / a.steps
    x_np = x.cpu().numpy()
    T = info["coeffs"][level]
    roof = term_roofline(info, level, n, nrhs, pname, mm, kernels["term_series"]["avg_us"], T,
                         wl.name, half, terms_per_launch(wl.K, a.steps, kernels))
    if not mm:
        assert kernels["stageA"]["launches"] == 0, "the leaf-level one-RHS path has no stage A"
    elem = 16 if prec == hmps.HM_F64 else 8
    # K terms, then the block-diagonal steps: D^{-1} b, or C^{-1} b and
    # C^{-T} x on the scaled series
    per_solve_bytes = (wl.K * elem * (info["half_entries"][level] if half else
                                      info["series_entries"][level] + info["stageA_entries"][level])
                       + (2 if half else 1) * 16 * info["diag_entries"])

    rel = cpu = None
    extras = {"timing_modes": {"eager_ms_per_solve": 1e3 * wall_eager / a.steps,
                               "graph_replay_ms_per_solve": 1e3 * wall_graph / a.steps,
                               "graph_result_bit_equal": graph_equal}}
    H = ref = None
    if not a.no_oracle:
        from oracle import hmatrix, series
        log("oracle build (host, FP64)")
        t1 = time.perf_counter()
        H = hmatrix.HMatrix(wl.problem, wl.leaf_max, wl.eta, wl.aca_tol, progress=log)
        oracle_build_s = time.perf_counter() - t1
        log("oracle series")
        t1 = time.perf_counter()
        ref = series.series(H, b_np, wl.K, wl.level)
        first_s = time.perf_counter() - t1
        rel = series.rel_err(x_np, ref)
        log(f"rel.err vs oracle x_K = {rel:.3e}")
        # bounded sample: repeat the oracle's solve of the same workload
        reps, cpu_s = 1, first_s
        t1 = time.perf_counter()
        while time.perf_counter() - t1 + first_s < a.cpu_seconds:
            series.series(H, b_np, wl.K, wl.level)
            reps += 1
        cpu_s = first_s + (time.perf_counter() - t1)
        cpu = {"value": reps * nrhs / cpu_s, "unit": "RHS/s", "cores": blas_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{reps} sequential numpy/scipy FP64 series solves of the same "
                         f"workload ({nrhs} RHS each) in {cpu_s:.1f} s; oracle H build "
                         f"{oracle_build_s:.1f} s not included"}
    tol = 1e-10 if prec == hmps.HM_F64 else 1e-4
    solved = rel is not None and rel <= min(tol, SOLVED_TOL)
    value = (a.steps * nrhs / wall) if solved else 0.0

    if not a.no_extras:
        reps = 20
        xr = torch.randn(n, dtype=torch.complex128, device="cuda")
        for _ in range(3):
            h.apply(xr, level=wl.level)
        mv_ms = timed(lambda: h.apply(xr, level=wl.level), reps, stream)
        if half1:
            # Z x = C (xhat + S xhat) with xhat = C^T x: the entries of S the
            # half storage reads, the two triangular factors C and C^T, and
            # the vectors (x, xhat written and read twice, (I + S) xhat
            # written and read, y)
            mv_bytes = 16 * (info["half_entries"][level] + info["diag_entries"] + n) + 16 * 7 * n
        else:
            mv_bytes = 16 * (info["apply_entries"][level] + info["stageA_entries"][level]) + 32 * n
        extras["hmatvec_1rhs_f64"] = {"ms": mv_ms, "bytes": mv_bytes,
                                      "GBps": mv_bytes / (mv_ms * 1e-3) / 1e9,
                                      "frac_hbm_peak": mv_bytes / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
        if nrhs > 1:
            # the same geometry with one right-hand side: the streaming term
            # kernel (a GEMV), bound by HBM bandwidth
            b1 = b[:, :1].contiguous()
            s1 = lambda: h.solve(b1, K=wl.K, level=wl.level, precision=hmps.HM_F64)  # noqa: E731
            for _ in range(3):
                x1 = s1()
            ms1 = timed(s1, reps, stream)
            _, k1 = profiled(h, s1, reps)
            x1 = s1()
            extras["series_1rhs_f64"] = {
                "ms_per_solve": ms1, "RHS_per_s": 1e3 / ms1,
                "roofline": term_roofline(info, level, n, 1, "f64", False,
                                          k1["term_series"]["avg_us"], T, wl.name, half1,
                                          terms_per_launch(wl.K, reps, k1))}
            if ref is not None:
                extras["series_1rhs_f64"]["rel_err_vs_oracle_xK"] = series.rel_err(
                    x1.cpu().numpy(), ref[:, :1])
            log(f"one RHS: {ms1:.3f} ms/solve, term "
                f"{extras['series_1rhs_f64']['roofline']['frac']:.2f} of HBM peak")
        other = hmps.HM_F32_APPLY if prec == hmps.HM_F64 else hmps.HM_F64
        oname = "f32" if other == hmps.HM_F32_APPLY else "f64"
        for _ in range(3):
            xo = solve(other)
        o_ms = timed(lambda: solve(other), reps, stream)
        xo = solve(other)
        extras[f"series_{oname}"] = {"ms_per_solve": o_ms, "RHS_per_s": nrhs * 1e3 / o_ms}
        _, ko = profiled(h, lambda: solve(other), 5)
        extras[f"series_{oname}"]["roofline"] = term_roofline(
            info, level, n, nrhs, oname, mm, ko["term_series"]["avg_us"], T, wl.name, half,
            terms_per_launch(wl.K, 5, ko))
        extras[f"series_{oname}"]["kernels"] = ko
        if H is not None:
            from oracle import series
            extras[f"series_{oname}"]["rel_err_vs_oracle_xK"] = series.rel_err(xo.cpu().numpy(), ref)
            extras[f"series_{pname}"] = {"rel_err_vs_oracle_xK": rel}
            rho = series.rho(H, wl.level, iters=60)
            extras["rho"] = rho
            if not cube and nrhs == 1:
                # the series at every coarser level (R_l with the far blocks of
                # level >= l): FP64 solves against the oracle's x_K there
                per_level = {}
                for lev in sorted(H.far_levels)[:-1]:
                    tl = timed(lambda: h.solve(b, K=wl.K, level=lev), reps, stream)
                    xl = h.solve(b, K=wl.K, level=lev).cpu().numpy()
                    el = series.rel_err(xl, series.series(H, b_np, wl.K, lev))
                    per_level[str(lev)] = {"ms_per_solve": tl, "RHS_per_s": nrhs * 1e3 / tl,
                                           "rel_err_vs_oracle_xK": el}
                    # one series term = stage A (the far-block coefficients
                    # of the coarser levels) + the term kernel: their bytes
                    # over their summed average durations
                    _, kl = profiled(h, lambda: h.solve(b, K=wl.K, level=lev), 5)
                    nt = max(1, kl["term_series"]["launches"])
                    us = (kl["term_series"]["avg_us"] * nt
                          + kl["stageA"]["avg_us"] * kl["stageA"]["launches"]) / nt
                    ent = (info["half_entries"][lev] if half else
                           info["series_entries"][lev] + info["stageA_entries"][lev])
                    nb = 16 * ent + 16 * (
                        n + info["coeffs"][lev] + 3 * n)
                    per_level[str(lev)]["term_and_stageA"] = {
                        "us": us, "bytes": nb, "GBps": nb / (us * 1e-6) / 1e9,
                        "frac_hbm_peak": nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS}
                    log(f"level {lev}: {tl:.3f} ms/solve, rel.err {el:.2e}")
                extras["series_f64_coarser_levels"] = per_level
                # the nested multi-level form (eq. 14-22) one level above the
                # leaf: two factors, (K + 1)^2 - 1 level products
                lev = H.L - 1
                if lev in H.far_levels:
                    kw = dict(K=wl.K, level=lev, kind=hmps.PS_NESTED)
                    xn = h.solve(b, **kw).cpu().numpy()  # also sizes its workspace
                    tn = timed(lambda: h.solve(b, **kw), 3, stream)
                    log(f"oracle nested form at level {lev}")
                    ref_n = series.nested(H, b_np, wl.K, lev)
                    extras["nested_f64"] = {
                        "level": lev, "K": wl.K, "level_products": (wl.K + 1) ** 2 - 1,
                        "ms_per_solve": tn, "RHS_per_s": nrhs * 1e3 / tn,
                        "rel_err_vs_oracle_nested": series.rel_err(xn, ref_n),
                        "rel_diff_vs_flat_series_same_level": series.rel_err(
                            xn, series.series(H, b_np, wl.K, lev))}
                    # both are truncations of Z_l^{-1} b: their distance to it
                    xs_l = series.solve_gmres(H, b_np, lev, tol=1e-12)
                    extras["nested_f64"]["rel_err_vs_xstar_level"] = series.rel_err(xn, xs_l)
                    extras["nested_f64"]["flat_series_rel_err_vs_xstar_level"] = series.rel_err(
                        series.series(H, b_np, wl.K, lev), xs_l)
                    log(f"nested level {lev}: {tn:.2f} ms/solve, rel.err "
                        f"{extras['nested_f64']['rel_err_vs_oracle_nested']:.2e}")
            if rho ** (wl.K + 1) < 0.9:
                log("oracle x* by GMRES for the refinement check")
                xs = series.solve_gmres(H, b_np, wl.level, tol=1e-13)
                for rname, p in (("f32_apply", hmps.HM_F32_APPLY), ("f64", hmps.HM_F64)):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    xr_, st = h.solve(b, K=wl.K, level=wl.level, precision=p,
                                      kind=hmps.PS_REFINE, max_passes=400, refine_tol=1e-10,
                                      stats=True)
                    torch.cuda.synchronize()
                    ref_s = time.perf_counter() - t1
                    err = series.rel_err(xr_.cpu().numpy(), xs)
                    extras[f"refine_{rname}"] = {
                        "ms_per_solve": 1e3 * ref_s, "passes": max(s["passes"] for s in st),
                        "rel_err_vs_oracle_xstar": err,
                        "solved_RHS_per_s": (nrhs / ref_s) if err <= SOLVED_TOL else 0.0}
                # GMRES with the FP32-block series as preconditioner
                for gname, Kg, p in (("gmres_series_f32_apply", wl.K, hmps.HM_F32_APPLY),):
                    xg, st, g_ms = gmres_run(h, b, Kg, wl.level, p)
                    err = series.rel_err(xg.cpu().numpy(), xs)
                    extras[gname] = {
                        "K": Kg, "ms_per_solve": g_ms, "steps": max(s["passes"] for s in st),
                        "resid_rel_max": max(s["resid_rel"] for s in st),
                        "rel_err_vs_oracle_xstar": err,
                        "solved_RHS_per_s": (nrhs * 1e3 / g_ms) if err <= SOLVED_TOL else 0.0}
                    log(f"{gname}: {g_ms:.2f} ms, {extras[gname]['steps']} steps, rel.err {err:.2e}")
            else:
                extras["refine"] = (f"not attainable by the method: rho = {rho:.3f}, "
                                    f"rho^(K+1) = {rho ** (wl.K + 1):.3f} >= 1 per pass")
                # GMRES preconditioned by D^{-1} (the K = 0 series) reaches x*
                # where the series diverges; checked by the oracle's residual of
                # sampled columns (an oracle x* at this size is out of reach)
                cols = sorted({0, nrhs - 1})
                # (with K = 0 the preconditioner is the FP64 D^{-1} alone, so
                # the block precision does not enter)
                for gname, p in (("gmres_jacobi_f64", hmps.HM_F64),):
                    xg, st, g_ms = gmres_run(h, b, 0, wl.level, p)
                    xgn = xg.cpu().numpy()
                    bs = b_np[:, cols] if b_np.ndim == 2 else b_np
                    xs_ = xgn[:, cols] if xgn.ndim == 2 else xgn
                    r = bs - series.apply_Z(H, xs_, wl.level)
                    ores = float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(bs, axis=0)))
                    ok = all(s["diverged"] == 0 for s in st) and ores <= GMRES_TOL * 1.01
                    extras[gname] = {
                        "K": 0, "ms_per_solve": g_ms, "steps": max(s["passes"] for s in st),
                        "resid_rel_max": max(s["resid_rel"] for s in st),
                        "oracle_resid_rel_sampled_columns": ores, "sampled_columns": cols,
                        "converged_RHS_per_s": (nrhs * 1e3 / g_ms) if ok else 0.0}
                    log(f"{gname}: {g_ms:.2f} ms, {extras[gname]['steps']} steps, "
                        f"oracle residual {ores:.2e}")

    out = {
        "metric": METRIC, "value": value, "unit": "RHS/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": pname, "data": "synthetic",
        "config": {"workload": wl.name, "N": n, "kind": "volume" if cube else "surface",
                   "leaf_max": wl.leaf_max, "eta": wl.eta, "aca_tol": wl.aca_tol, "K": wl.K,
                   "level": level, "nrhs": nrhs,
                   "timing": "HIP graph replay" if use_graph else "eager solves",
                   "kernels": "matrix-core (MFMA)" if mm else (
                       "scaled series, half storage (k_half)" if half else "streaming one-RHS tiles"),
                   "precision": "complex128" if prec == hmps.HM_F64
                   else "complex64 blocks, complex128 vectors"},
        "rel_err_vs_oracle": rel, "latency_ms": lat, "roofline": roof,
        "per_solve_algorithmic_bytes": per_solve_bytes, "kernels": kernels, "build_s": build_s,
        "build_phases_s": build_phases,
        "device_bytes": info["device_bytes"], "cpu_baseline": cpu, "extras": extras,
        "autotune": None if tune is None else {"choice": tune[0], "ms": tune[1]},
    }
    h.close()
    return out


# --------------------------------------------------------------------------
def bench_batched(a):
    """256 instances in one batched handle, 16 RHS each (one column block
    of 16 per instance), mixed precision: FP32 blocks, FP64 LU / residual /
    refinement; replayed from captured HIP graphs."""
    import torch
    import workloads as W
    from paper_2307_03968_amd import hmps

    count = a.instances
    sizes = W.batched_sizes(count)
    wls = [W.batched_instance(i, int(nn)) for i, nn in enumerate(sizes)]
    K, nrhs = wls[0].K, wls[0].nrhs
    log(f"library build of {count} instances, total N = {int(sizes.sum())}")
    t0 = time.perf_counter()
    # 16 right-hand sides per instance: the one-RHS half-storage data is not built
    h = hmps.HMatrix([w.problem for w in wls], 64, 1.0, 1e-4, progress=log,
                     flags=hmps.HM_BUILD_NO_HALF)
    build_s = time.perf_counter() - t0
    info = h.info()
    n = h.n
    level = info["leaf_level"]
    bs = [w.rhs() for w in wls]
    b = torch.from_numpy(np.ascontiguousarray(np.vstack(bs))).to("cuda")
    stream = torch.cuda.current_stream()
    F32, F64 = hmps.HM_F32_APPLY, hmps.HM_F64

    log("autotune (FP32 series, 16 RHS)")
    best, best_ms = h.autotune(nrhs, K=K, precision=F32)
    log(f"autotune: {best} {best_ms:.3f} ms")
    mm = nrhs >= best["mm_min_rhs"]
    # the FP32 series with its K terms in one persistent launch and with one
    # launch per stage A and term (eager, median of 5), then the choice again
    modes = {}
    if mm:
        for mode, name in ((1, "multi_term_launch_ms"), (2, "per_term_launches_ms")):
            h.tune(mm_multi=mode)
            ts = []
            for _ in range(7):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                h.solve(b, K=K, precision=F32)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            modes[name] = float(np.median(ts[2:]))
        h.tune(mm_multi=best["mm_multi"])
        log(f"FP32 series launch modes: {modes}")

    def graph_of(**kw):
        out = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            h.solve(b, out=out, **kw)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            h.solve(b, out=out, **kw)
        return g, out

    # ---- FP32 series (the batched launch path), graph replay
    g32, out32 = graph_of(K=K, precision=F32)
    for _ in range(a.warmup):
        g32.replay()
    torch.cuda.synchronize()
    log(f"timed region: {a.steps} graph replays of the FP32 series")
    t0 = time.perf_counter()
    for _ in range(a.steps):
        g32.replay()
    torch.cuda.synchronize()
    wall32 = time.perf_counter() - t0
    x32 = out32.t().cpu().numpy()
    lat32 = latency(g32.replay, a.steps)
    copy_calibration(a)
    # kernel durations from eager solves (same kernels as in the graph)
    _, kernels = profiled(h, lambda: h.solve(b, K=K, precision=F32), 5)
    T = info["coeffs"][level]
    wname = f"batched_{a.instances}"
    roof = term_roofline(info, level, n, nrhs, "f32", mm, kernels["term_series"]["avg_us"], T,
                         wname)

    # ---- plain FP64 series on the same handle (same tuning), graph replay
    g64, out64 = graph_of(K=K, precision=F64)
    g64.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        g64.replay()
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t0
    x64 = out64.t().cpu().numpy()
    lat64 = latency(g64.replay, a.steps)
    _, k64 = profiled(h, lambda: h.solve(b, K=K, precision=F64), 3)

    # ---- refinement to x*: adaptive once for the pass count, then the
    # fixed-pass solve captured and replayed
    log("adaptive FP32 refinement (pass count)")
    # stop when the correction is 1e-9 of x: the error left is about
    # rho^(K+1) / (1 - rho^(K+1)) times that (< 2e-9 here, rho^(K+1) <= 0.56)
    _, st = h.solve(b, K=K, precision=F32, kind=hmps.PS_REFINE, max_passes=400, refine_tol=1e-9,
                    stats=True)
    passes = max(s["passes"] for s in st)
    log(f"refinement: {passes} passes")
    gr, outr = graph_of(K=K, precision=F32, kind=hmps.PS_REFINE_FIXED, max_passes=passes,
                        refine_tol=1e-9)
    gr.replay()
    torch.cuda.synchronize()
    rsteps = max(2, a.steps // 10)
    t0 = time.perf_counter()
    for _ in range(rsteps):
        gr.replay()
    torch.cuda.synchronize()
    wallr = time.perf_counter() - t0
    xr = outr.t().cpu().numpy()
    latr = latency(gr.replay, rsteps)

    # ---- GMRES to x* over all instances at once, preconditioned by the
    # FP32-block series (stopped against each column's smallest ||b_i||)
    log("GMRES with the FP32 series as preconditioner")
    xg_, stg, g_ms = gmres_run(h, b, K, -1, F32)
    xg = xg_.cpu().numpy()
    if xg.shape != xr.shape:
        xg = xg.T
    g_steps = int(max(s["passes"] for s in stg))
    g_conv = all(s["diverged"] == 0 for s in stg)
    log(f"GMRES: {g_steps} steps, {g_ms:.1f} ms")

    # ---- oracle on a sample of instances (smallest, largest, 4 seeded)
    rel = {"series_f32": 0.0, "series_f64": 0.0, "refine_f32_vs_xstar": 0.0,
           "gmres_f32_vs_xstar": 0.0}
    cpu = None
    sample = []
    if not a.no_oracle:
        from oracle import hmatrix, series
        g = np.random.default_rng(7)
        sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                         *g.choice(count, size=min(4, count), replace=False).tolist()})
        cpu_t, cpu_rhs = 0.0, 0
        for i in sample:
            o0, o1 = h.offsets[i], h.offsets[i + 1]
            log(f"oracle instance {i} n={sizes[i]}")
            H = hmatrix.HMatrix(wls[i].problem, 64, 1.0, 1e-4)
            t1 = time.perf_counter()
            ref = series.series(H, bs[i], K)
            cpu_t += time.perf_counter() - t1
            cpu_rhs += nrhs
            rel["series_f32"] = max(rel["series_f32"], series.rel_err(x32[o0:o1], ref))
            rel["series_f64"] = max(rel["series_f64"], series.rel_err(x64[o0:o1], ref))
            xs = (series.solve_exact(H, bs[i]) if sizes[i] <= 4096
                  else series.solve_gmres(H, bs[i], tol=1e-13))
            rel["refine_f32_vs_xstar"] = max(rel["refine_f32_vs_xstar"],
                                             series.rel_err(xr[o0:o1], xs))
            rel["gmres_f32_vs_xstar"] = max(rel["gmres_f32_vs_xstar"],
                                            series.rel_err(xg[o0:o1], xs))
        cpu = {"value": cpu_rhs / cpu_t, "unit": "RHS/s", "cores": blas_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"numpy/scipy FP64 series of {len(sample)} sampled instances "
                         f"(N = {[int(sizes[i]) for i in sample]}, {nrhs} RHS each) in "
                         f"{cpu_t:.1f} s; oracle builds not included"}
        log(f"rel.err on the sample: {rel}")
    tot = count * nrhs
    ok = lambda key, tol: (not a.no_oracle) and rel[key] <= tol  # noqa: E731
    value = tot * rsteps / wallr if ok("refine_f32_vs_xstar", SOLVED_TOL) else 0.0
    extras = {
        "series_f32_graph": {"RHS_per_s": tot * a.steps / wall32, "ms_per_solve": 1e3 * wall32 / a.steps,
                             "rel_err_vs_oracle_xK_sample": rel["series_f32"], "tolerance": 1e-4,
                             "latency_ms": lat32},
        "series_f64_graph": {"RHS_per_s": tot * a.steps / wall64, "ms_per_solve": 1e3 * wall64 / a.steps,
                             "rel_err_vs_oracle_xK_sample": rel["series_f64"], "tolerance": 1e-10,
                             "solved_RHS_per_s": (tot * a.steps / wall64) if ok("series_f64", 1e-10) else 0.0,
                             "latency_ms": lat64, "kernels": k64,
                             "roofline": term_roofline(info, level, n, nrhs, "f64", mm,
                                                       k64["term_series"]["avg_us"], T, wname)},
        "refine_f32_graph": {"passes": passes, "ms_per_solve": 1e3 * wallr / rsteps,
                             "rel_err_vs_oracle_xstar_sample": rel["refine_f32_vs_xstar"]},
        "gmres_series_f32": {"steps": g_steps, "ms_per_solve": g_ms, "converged": g_conv,
                             "rel_err_vs_oracle_xstar_sample": rel["gmres_f32_vs_xstar"],
                             "solved_RHS_per_s": (tot * 1e3 / g_ms)
                             if g_conv and ok("gmres_f32_vs_xstar", SOLVED_TOL) else 0.0,
                             "note": "eager (one solve, after an untimed one); GMRES synchronises "
                                     "once per step, so it is not graph-replayed"},
        "autotune": {"choice": best, "ms": best_ms},
        "series_f32_launch_modes": modes,
        "oracle_sample_instances": sample,
    }
    out = {
        "metric": METRIC, "value": value, "unit": "RHS/s", "n_gpus": 1, "steps": rsteps,
        "warmup": a.warmup, "ms_per_step": 1e3 * wallr / rsteps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched_{count}", "instances": count, "N_total": n,
                   "N_range": [int(sizes.min()), int(sizes.max())], "kind": "surface",
                   "leaf_max": 64, "eta": 1.0, "aca_tol": 1e-4, "K": K, "level": "leaf",
                   "nrhs_per_instance": nrhs,
                   "precision": "complex64 blocks, complex128 LU/residual/refinement",
                   "path": "refinement to x* (fixed pass count), HIP graph replay"},
        "rel_err_vs_oracle": rel["refine_f32_vs_xstar"] if not a.no_oracle else None,
        "latency_ms": latr, "roofline": roof, "kernels": kernels, "build_s": build_s,
        "device_bytes": info["device_bytes"], "cpu_baseline": cpu, "extras": extras,
    }
    h.close()
    return out


def bench_served(a):
    """Poisson request stream through the request server (continuous
    batching over resident geometries under the HBM budget).  Every request
    is solved to x* by GMRES: surface requests preconditioned by the K = 4
    series on FP32 blocks, volume requests by D^{-1} (the series diverges
    there, rho > 1).  The same stream is then served with FP64 blocks in the
    surface preconditioner.  Latency = submit to done (server
    clock), with and without requests whose batch built a geometry."""
    import workloads as W
    from paper_2307_03968_amd import hmps

    ns, sides = W.served_pool()
    pool = {}
    for kind in (W.SURFACE, W.VOLUME):
        for gi in range(16):
            wl = W.served_workload(kind, gi, 64, 0)
            pool[(kind, gi)] = wl
    # per geometry a bank of 64 seeded plane waves; request r takes nrhs
    # consecutive columns from a seeded offset
    log("plane-wave banks")
    bank = {k: np.asfortranarray(wl.rhs()) for k, wl in pool.items()}
    key_of = {k: i + 1 for i, k in enumerate(sorted(pool))}

    def opts_for(kind, mixed):
        # GMRES to x* for every request (restart 20 bounds the basis each
        # geometry keeps): surface preconditioned by the K = 4 series (FP32
        # blocks in the mixed run), volume by D^{-1} (the series diverges)
        p = hmps.HM_F32_APPLY if mixed else hmps.HM_F64
        if kind == W.SURFACE:
            return dict(K=4, precision=p, kind=hmps.PS_GMRES, max_passes=1000,
                        refine_tol=GMRES_TOL, restart=20)
        return dict(K=0, precision=hmps.HM_F64, kind=hmps.PS_GMRES, max_passes=1000,
                    refine_tol=GMRES_TOL, restart=20)

    def run(srv, stream, mixed, seen, rate=None, keep=()):
        """Submit the stream (open loop at its arrival times, or all at once
        when rate is None); returns per-request records and the wall time."""
        g = np.random.default_rng(13)
        recs = {}
        out = {}
        t0 = time.perf_counter()
        i = 0
        pending = {}
        last_log = 0.0
        while i < len(stream) or pending:
            now = time.perf_counter() - t0
            if now - last_log > 20.0:
                log(f"  {len(recs)} of {len(stream)} requests done, {len(pending)} pending")
                last_log = now
            while i < len(stream) and (rate is None or stream[i].t_arrive <= now):
                rq = stream[i]
                k = (rq.kind, rq.geom)
                wl = pool[k]
                c0 = int(g.integers(0, 64 - rq.nrhs + 1))
                b = bank[k][:, c0:c0 + rq.nrhs]
                first = key_of[k] not in seen
                seen.add(key_of[k])
                t = srv.submit(key_of[k], b, prob=wl.problem if first else None,
                               leaf_max=wl.leaf_max, aca_tol=wl.aca_tol, **opts_for(rq.kind, mixed))
                pending[t] = (i, c0)
                i += 1
            done = []
            for t, (ri, c0) in list(pending.items())[:256]:
                state, x, st = srv.poll(t, want_x=ri in keep)
                if st is not None:
                    recs[ri] = {"ms": st[0]["t_ms"], "built": st[0]["built"],
                                "diverged": max(s_["diverged"] for s_ in st),
                                "passes": max(s_["passes"] for s_ in st), "c0": c0}
                    if x is not None:
                        out[ri] = x
                    done.append(t)
            for t in done:
                del pending[t]
            if not done:
                nxt = stream[i].t_arrive - (time.perf_counter() - t0) if (rate and i < len(stream)) else 0.0005
                time.sleep(min(max(nxt, 0.0), 0.0005) if pending else max(nxt, 0.0))
        return recs, out, time.perf_counter() - t0

    def split(stream, recs, sel):
        """p50 / p99 (ms) and count of the requests with sel(request, record)."""
        v = np.array([recs[i]["ms"] for i, rq in enumerate(stream) if sel(rq, recs[i])])
        if not len(v):
            return None
        return {"requests": int(len(v)), "p50": float(np.percentile(v, 50)),
                "p99": float(np.percentile(v, 99))}

    def summary(stream, recs, wall):
        lat = np.array([recs[i]["ms"] for i in range(len(stream))])
        nof = lambda rq: pool[(rq.kind, rq.geom)].problem.n  # noqa: E731
        by = {}
        for kname, kind in (("surface", W.SURFACE), ("volume", W.VOLUME)):
            by[kname] = split(stream, recs, lambda rq, r: rq.kind == kind)
            for lo, hi in ((0, 4096), (4096, 16384), (16384, 1 << 30)):
                by[f"{kname}_N_{lo}_{hi}" if hi < (1 << 30) else f"{kname}_N_above_{lo}"] = split(
                    stream, recs, lambda rq, r: rq.kind == kind and lo < nof(rq) <= hi)
        for lo, hi in ((0, 16), (16, 64)):
            by[f"nrhs_{lo + 1}_{hi}"] = split(stream, recs, lambda rq, r: lo < rq.nrhs <= hi)
        by["cold_build"] = split(stream, recs, lambda rq, r: bool(r["built"]))
        warm = np.array([recs[i]["ms"] for i in range(len(stream)) if not recs[i]["built"]])
        rhs = sum(rq.nrhs for rq in stream)
        surf_ok = sum(rq.nrhs for i, rq in enumerate(stream)
                      if rq.kind == W.SURFACE and not recs[i]["diverged"])
        vol_ok = sum(rq.nrhs for i, rq in enumerate(stream)
                     if rq.kind == W.VOLUME and not recs[i]["diverged"])
        return {"requests": len(stream), "rhs": rhs, "wall_s": wall, "RHS_per_s": rhs / wall,
                "solved_surface_RHS_per_s": surf_ok / wall,
                "gmres_volume_RHS_per_s": vol_ok / wall,
                "solved_RHS_per_s": (surf_ok + vol_ok) / wall,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "latency_ms_without_cold_builds": (
                    {"p50": float(np.percentile(warm, 50)), "p99": float(np.percentile(warm, 99))}
                    if len(warm) else None),
                "cold_build_requests": int(sum(recs[i]["built"] for i in range(len(stream)))),
                "unconverged_surface_requests": int(sum(1 for i, rq in enumerate(stream)
                                                     if rq.kind == W.SURFACE and recs[i]["diverged"])),
                "unconverged_volume_requests": int(sum(1 for i, rq in enumerate(stream)
                                                       if rq.kind == W.VOLUME and recs[i]["diverged"])),
                "max_gmres_steps": int(max(recs[i]["passes"] for i in range(len(stream)))),
                "unconverged": [{"kind": "surface" if rq.kind == W.SURFACE else "volume",
                                 "N": int(nof(rq)), "nrhs": int(rq.nrhs),
                                 "built": int(recs[i]["built"]), "steps": int(recs[i]["passes"])}
                                for i, rq in enumerate(stream) if recs[i]["diverged"]][:20],
                "latency_ms_by": by}

    results = {}
    srv_info = {}
    resident_all = 0
    runs = [("mixed", True), ("f64", False)]
    if a.evict_frac > 0:
        runs.append(("mixed_evicting", True))
    if a.served_runs:
        want = a.served_runs.split(",")
        runs = [r for r in runs if r[0] in want]
    if any(t == "mixed_evicting" for t, _ in runs) and runs[0][0] != "mixed":
        # the evicting budget is a fraction of what the pool keeps resident
        srv = hmps.Server(budget_bytes=a.budget_gb << 30 if a.budget_gb else 0, slots=a.slots)
        seen = set()
        run(srv, [W.Request(0.0, kind, gi, 8) for (kind, gi) in sorted(pool)], True, seen)
        resident_all = srv.info()["resident_bytes"]
        srv.close()
        log(f"pool resident bytes {resident_all}")
    for tag, mixed in runs:
        budget = a.budget_gb << 30 if a.budget_gb else 0
        if tag == "mixed_evicting":
            # a budget below what the pool keeps resident: the timed stream
            # evicts and rebuilds geometries
            budget = int(a.evict_frac * resident_all)
        srv = hmps.Server(budget_bytes=budget, slots=a.slots)
        seen = set()
        log(f"[{tag}] cold pass: one request per geometry")
        cold_stream = [W.Request(0.0, kind, gi, 8) for (kind, gi) in sorted(pool)]
        cold, _, cold_wall = run(srv, cold_stream, mixed, seen)
        log(f"[{tag}] cold pass {cold_wall:.1f} s; {srv.info()}")
        if tag == "mixed":
            resident_all = srv.info()["resident_bytes"]
        log(f"[{tag}] closed-loop burst for the saturated rate")
        burst = W.request_stream(a.calib_requests, 1.0, seed=6)
        brec, _, bwall = run(srv, burst, mixed, seen)
        sat = len(burst) / bwall
        rate = 0.7 * sat
        log(f"[{tag}] saturated {sat:.2f} req/s; open loop at {rate:.2f} req/s")
        stream = W.request_stream(a.requests, rate)
        small = [i for i, rq in enumerate(stream) if pool[(rq.kind, rq.geom)].problem.n <= 6000]
        keep = set(small[:40]) if tag == "mixed" else set()
        before = srv.info()
        recs, xs, wall = run(srv, stream, mixed, seen, rate=rate, keep=keep)
        after = srv.info()
        results[tag] = summary(stream, recs, wall)
        results[tag]["timed_stream_builds"] = after["builds"] - before["builds"]
        results[tag]["timed_stream_evictions"] = after["evictions"] - before["evictions"]
        results[tag]["saturated_req_per_s"] = sat
        results[tag]["offered_req_per_s"] = rate
        results[tag]["cold_pass"] = {"wall_s": cold_wall,
                                     "latency_ms_p50": float(np.median([r["ms"] for r in cold.values()]))}
        srv_info[tag] = srv.info()
        results[tag]["server"] = srv_info[tag]
        log(f"[{tag}] {results[tag]}")
        if tag == "mixed":
            mixed_stream, mixed_x, mixed_recs = stream, xs, recs
        srv.close()

    if "mixed" not in results:
        # a partial set of runs (--served-runs): their records only, no value
        return {"metric": METRIC + " (served stream, GMRES to x*)", "value": None, "unit": "RHS/s",
                "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                "config": {"workload": "served", "runs": sorted(results)}, "extras": results}
    # ---- oracle on a sample of the mixed-stream requests (small geometries)
    rel = {"surface_gmres_vs_xstar": 0.0, "volume_gmres_vs_xstar": 0.0}
    cpu = None
    checked = []
    if not a.no_oracle:
        from oracle import hmatrix, series
        cand = [i for i in sorted(mixed_x) if pool[(mixed_stream[i].kind, mixed_stream[i].geom)].problem.n <= 6000]
        pick = {}
        for i in cand:  # one request per small geometry, at most 4
            k = (mixed_stream[i].kind, mixed_stream[i].geom)
            if k not in pick and len(pick) < 4:
                pick[k] = i
        cpu_t, cpu_rhs = 0.0, 0
        for k, i in sorted(pick.items()):
            rq, wl = mixed_stream[i], pool[k]
            c0 = mixed_recs[i]["c0"]
            b = bank[k][:, c0:c0 + rq.nrhs]
            log(f"oracle request {i}: kind {rq.kind} N {wl.problem.n} nrhs {rq.nrhs}")
            H = hmatrix.HMatrix(wl.problem, wl.leaf_max, 1.0, wl.aca_tol)
            # the CPU baseline solves the same request to x* as the server
            # does: the oracle's GMRES (D^{-1}-preconditioned) to the same
            # relative residual
            t1 = time.perf_counter()
            series.solve_gmres(H, b, tol=GMRES_TOL)
            cpu_t += time.perf_counter() - t1
            cpu_rhs += rq.nrhs
            if rq.kind == W.SURFACE:
                if not mixed_recs[i]["diverged"]:
                    xs_ = series.solve_exact(H, b)
                    rel["surface_gmres_vs_xstar"] = max(rel["surface_gmres_vs_xstar"],
                                                         series.rel_err(mixed_x[i], xs_))
            elif not mixed_recs[i]["diverged"]:
                xs_ = series.solve_exact(H, b)
                rel["volume_gmres_vs_xstar"] = max(rel["volume_gmres_vs_xstar"],
                                                   series.rel_err(mixed_x[i], xs_))
            checked.append({"request": i, "kind": int(rq.kind), "N": int(wl.problem.n), "nrhs": rq.nrhs})
        if cpu_rhs:
            cpu = {"value": cpu_rhs / cpu_t, "unit": "RHS/s", "cores": blas_threads(), "kind": "oracle", "cpu_model": cpu_model(),
                   "sample": f"numpy/scipy FP64 GMRES to x* (relative residual {GMRES_TOL:g}) of "
                             f"{len(checked)} sampled requests ({cpu_rhs} RHS, N <= 6000) in "
                             f"{cpu_t:.1f} s; oracle builds not included"}
        log(f"rel.err on the sample: {rel}")
    ok = (not a.no_oracle) and rel["surface_gmres_vs_xstar"] <= SOLVED_TOL and \
        rel["volume_gmres_vs_xstar"] <= SOLVED_TOL
    m = results["mixed"]
    out = {
        "metric": METRIC + " (served stream, GMRES to x*)",
        "value": m["solved_RHS_per_s"] if ok else 0.0, "unit": "RHS/s", "n_gpus": 1,
        "steps": m["requests"], "warmup": a.calib_requests,
        "ms_per_step": 1e3 * m["wall_s"] / m["requests"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served", "pool": "16 surface + 16 volume geometries, N log-uniform "
                   "[1024, 65536]", "surface": "leaf<=64 (N<=8192) else 128, tol 1e-4, K=4, "
                   "GMRES preconditioned by the FP32-block series", "volume": "leaf<=128, tol 1e-5, "
                   "GMRES with the D^{-1} preconditioner", "gmres": "restart 20, relative "
                   "residual 1e-10",
                   "nrhs": "U{1..64}", "slots": a.slots,
                   "offered_rate": "0.7 x closed-loop saturated rate of the path",
                   "budget_bytes": srv_info["mixed"]["budget_bytes"]},
        "rel_err_vs_oracle": rel if not a.no_oracle else None,
        "latency_ms": m["latency_ms"], "roofline": None, "cpu_baseline": cpu,
        "extras": {"mixed": results["mixed"], "plain_f64": results.get("f64"),
                   "mixed_evicting": results.get("mixed_evicting"),
                   "oracle_checked_requests": checked},
    }
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere_24576")
    ap.add_argument("--precision", default=None, choices=["f64", "f32"])
    ap.add_argument("--instances", type=int, default=256, help="batched_*: instance count")
    ap.add_argument("--requests", type=int, default=600, help="served: open-loop requests")
    ap.add_argument("--calib-requests", type=int, default=100,
                    help="served: closed-loop burst for the saturated rate")
    ap.add_argument("--slots", type=int, default=4, help="served: server workers")
    ap.add_argument("--budget-gb", type=int, default=0, help="served: HBM budget (0: 90%% free)")
    ap.add_argument("--evict-frac", type=float, default=0.0,
                    help="served: also serve the mixed stream under a budget of this fraction of "
                         "the bytes the pool keeps resident (evictions in the timed stream)")
    ap.add_argument("--served-runs", default="",
                    help="served: comma list of the runs to make (mixed, f64, mixed_evicting)")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the oracle check and CPU baseline (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (H-matvec, other precision, refinement)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload only: skip the 32^3 cube and 256-instance legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed region, copy a MIB-MiB device buffer 3 times (a plain "
                         "copy kernel of known size to scale HBM byte counters)")
    a = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.workload == "served":
        out = bench_served(a)
    elif a.workload.startswith("batched"):
        if "_" in a.workload:
            a.instances = int(a.workload.split("_")[1])
        out = bench_batched(a)
    else:
        out = bench_single(a)
        if a.workload == "sphere_24576" and not (a.no_legs or a.no_extras):
            # the volume (64 RHS, matrix cores) and batched configurations,
            # each with its own oracle check, roofline and CPU baseline
            legs = {}
            for name, steps in (("cube_32768", 10), ("batched_256", 10)):
                la = argparse.Namespace(**vars(a))
                la.workload, la.steps, la.warmup = name, min(a.steps, steps), 2
                la.cpu_seconds = min(a.cpu_seconds, 10.0)
                la.instances = 256
                log(f"leg {name}")
                t0 = time.perf_counter()
                legs[name] = bench_batched(la) if name.startswith("batched") else bench_single(la)
                legs[name]["leg_wall_s"] = time.perf_counter() - t0
                torch.cuda.empty_cache()
            out["extras"]["legs"] = legs
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
