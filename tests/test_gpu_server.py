"""The request server (ps_server_create / ps_submit / ps_poll) on the GPU:
results equal the one-request-at-a-time results and the oracle, requests
are batched, the HBM budget evicts idle geometries and refuses geometries
that cannot fit."""
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


GEOMS = {
    1: (W.sphere_problem(1200, math.sqrt(1200 / 1536)), 32, 1e-6),
    2: (W.cube_problem(10, 10 / 16), 32, 1e-5),
    3: (W.sphere_problem(700, math.sqrt(700 / 1536), instance=3), 64, 1e-4),
}


@pytest.fixture(scope="module")
def oracles():
    return {k: hmatrix.HMatrix(p, leaf, 1.0, tol) for k, (p, leaf, tol) in GEOMS.items()}


def _requests():
    """(key, b) pairs: 14 requests over the three geometries, 1..9 RHS."""
    g = np.random.default_rng(11)
    out = []
    for i in range(14):
        key = [1, 2, 3, 1, 1, 2, 3, 3, 1, 2, 2, 1, 3, 1][i]
        p = GEOMS[key][0]
        nrhs = int(g.integers(1, 10))
        out.append((key, W.plane_waves(p.xyz, W.directions(nrhs, 3, instance=100 + i))))
    return out


def _submit(srv, key, b, seen, **kw):
    p, leaf, tol = GEOMS[key]
    first = key not in seen
    seen.add(key)
    return srv.submit(key, b, prob=p if first else None, leaf_max=leaf, aca_tol=tol, **kw)


def test_server_mix_equals_alone_and_oracle(oracles):
    reqs = _requests()
    K = 3
    _say("server alone: one request at a time")
    srv = hmps.Server(slots=1)
    seen = set()
    alone = []
    for key, b in reqs:
        x, st = srv.wait(_submit(srv, key, b, seen, K=K))
        alone.append(x)
    assert srv.info()["batches"] == len(reqs)
    srv.close()
    _say("server mix: all requests at once, three workers")
    srv = hmps.Server(slots=3)
    seen = set()
    tickets = [_submit(srv, key, b, seen, K=K) for key, b in reqs[:8]]
    first = srv.wait(tickets[0])  # later requests arrive while others run
    tickets += [_submit(srv, key, b, seen, K=K) for key, b in reqs[8:]]
    mix = [first[0]] + [srv.wait(t)[0] for t in tickets[1:]]
    info = srv.info()
    _say(f"server info {info}")
    assert info["builds"] == 3 and info["requests_done"] == len(reqs)
    assert info["batches"] < len(reqs), "queued requests of one geometry were not batched"
    for (key, b), xa, xm in zip(reqs, alone, mix):
        assert_close(xm, xa, 1e-12)
        assert_close(xm, series.series(oracles[key], b, K), 1e-10)
    srv.close()


def test_server_budget_evicts_idle_geometries(oracles):
    """A budget that holds one geometry at a time: alternating requests
    rebuild geometries after evicting the idle one; results stay right."""
    probe = hmps.Server(slots=1)
    sizes = {}
    seen = set()
    for key in (1, 3):
        b = W.plane_waves(GEOMS[key][0].xyz, W.Z_HAT)
        probe.wait(_submit(probe, key, b, seen, K=2))
        sizes[key] = probe.info()["resident_bytes"] - sum(sizes.values())
    probe.close()
    budget = int(max(sizes.values()) + 0.5 * min(sizes.values()))
    _say(f"server budget {budget} bytes, geometry bytes {sizes}")
    srv = hmps.Server(budget_bytes=budget, slots=1)
    seen = set()
    for rep in range(2):
        for key in (1, 3):
            b = W.plane_waves(GEOMS[key][0].xyz, W.directions(2, 3, instance=rep))
            x, st = srv.wait(_submit(srv, key, b, seen, K=2))
            assert_close(x, series.series(oracles[key], b, 2), 1e-10)
            assert st[0]["built"] == 1  # the other geometry had to go
    info = srv.info()
    assert info["evictions"] >= 3 and info["builds"] == 4
    assert info["resident_bytes"] <= budget
    srv.close()


def test_server_rebuilds_under_load_stay_exact(oracles):
    """Four workers, a budget for about two of the three geometries and a
    rotating stream of series and GMRES requests kept four deep: geometries
    are evicted and rebuilt while other workers solve, and every result
    still equals the oracle (the series) or x* (GMRES, with the FP32 series
    preconditioner on the spheres and D^{-1} on the cube)."""
    probe = hmps.Server(slots=1)
    seen = set()
    for key in (1, 2, 3):
        b = W.plane_waves(GEOMS[key][0].xyz, W.Z_HAT)
        probe.wait(_submit(probe, key, b, seen, K=0 if key == 2 else 4, kind=hmps.PS_GMRES,
                           max_passes=300, refine_tol=1e-10))
    total = probe.info()["resident_bytes"]
    probe.close()
    budget = int(0.7 * total)
    _say(f"server under load: budget {budget} of {total} bytes, four workers")
    srv = hmps.Server(budget_bytes=budget, slots=4)
    seen = set()
    g = np.random.default_rng(5)
    inflight, checks = [], []

    def drain(n):
        while len(inflight) > n:
            t, key, b, gm = inflight.pop(0)
            x, st = srv.wait(t)
            if gm:
                assert all(s["diverged"] == 0 and s["resid_rel"] <= 1e-10 and s["passes"] < 300
                           for s in st), (key, st)
                assert_close(x, series.solve_exact(oracles[key], b), 1e-8)
            else:
                assert_close(x, series.series(oracles[key], b, 3), 1e-10)
            checks.append(key)

    for i in range(36):
        key = (1, 2, 3)[i % 3]
        p = GEOMS[key][0]
        b = W.plane_waves(p.xyz, W.directions(int(g.integers(1, 6)), 3, instance=300 + i))
        gm = i % 2 == 1
        if gm:
            kw = dict(K=0, kind=hmps.PS_GMRES) if key == 2 else dict(
                K=4, kind=hmps.PS_GMRES, precision=hmps.HM_F32_APPLY)
            t = _submit(srv, key, b, seen, max_passes=300, refine_tol=1e-10, **kw)
        else:
            t = _submit(srv, key, b, seen, K=3)
        inflight.append((t, key, b, gm))
        drain(4)
    drain(0)
    info = srv.info()
    _say(f"server info {info}")
    assert len(checks) == 36 and info["requests_failed"] == 0
    assert info["evictions"] >= 3 and info["builds"] >= 6
    assert info["resident_bytes"] <= budget
    srv.close()


def test_server_splits_batch_without_room(oracles):
    """A budget that holds geometry 3 with the workspace of a narrow request:
    a 64-column request finds no room to widen the workspace (nothing else
    is resident or running), so it is solved in pieces of the width the
    workspace holds; every column equals the oracle."""
    p = GEOMS[3][0]
    probe = hmps.Server(slots=1)
    seen = set()
    probe.wait(_submit(probe, 3, W.plane_waves(p.xyz, W.Z_HAT), seen, K=2))
    one = probe.info()["resident_bytes"]
    probe.close()
    srv = hmps.Server(budget_bytes=int(1.03 * one), slots=1)
    seen = set()
    srv.wait(_submit(srv, 3, W.plane_waves(p.xyz, W.Z_HAT), seen, K=2))
    b = W.plane_waves(p.xyz, W.directions(64, 3, instance=77))
    _say("server: 64 columns without room for their workspace")
    x, st = srv.wait(_submit(srv, 3, b, seen, K=2))
    assert_close(x, series.series(oracles[3], b, 2), 1e-10)
    info = srv.info()
    _say(f"server info {info}")
    assert info["split_batches"] >= 1 and info["requests_failed"] == 0
    srv.close()


def test_server_rejects_geometry_over_budget():
    srv = hmps.Server(budget_bytes=1 << 20, slots=1)
    p, leaf, tol = GEOMS[1]
    t = srv.submit(1, W.plane_waves(p.xyz, W.Z_HAT), K=2, prob=p, leaf_max=leaf, aca_tol=tol)
    with pytest.raises(hmps.HmpsError) as e:
        srv.wait(t)
    assert e.value.status == hmps.HM_ENOMEM
    assert srv.info()["requests_failed"] == 1
    srv.close()


def test_server_refine_to_exact_solution():
    """Mixed precision with FP64 refinement through the server reaches
    x* = Z_l^{-1} b to 1e-8 (sphere of 1536 points, rho^5 < 1)."""
    wl = W.sphere_small()
    H = hmatrix.HMatrix(wl.problem, 64, 1.0, 1e-4)
    b = W.plane_waves(wl.problem.xyz, W.directions(3, 3))
    srv = hmps.Server(slots=2)
    t = srv.submit(7, b, K=4, precision=hmps.HM_F32_APPLY, kind=hmps.PS_REFINE, max_passes=300,
                   refine_tol=1e-11, prob=wl.problem, leaf_max=64, aca_tol=1e-4)
    x, st = srv.wait(t)
    assert_close(x, series.solve_exact(H, b), 1e-8)
    assert all(s["diverged"] == 0 and s["passes"] > 0 and s["t_ms"] > 0 for s in st)
    srv.close()


def test_server_argument_errors():
    import ctypes as C
    lib = hmps._lib()
    srv = hmps.Server(slots=1)
    p, leaf, tol = GEOMS[3]
    b = W.plane_waves(p.xyz, W.Z_HAT)
    with pytest.raises(hmps.HmpsError):        # unknown key without a problem
        srv.submit(99, b, K=2)
    with pytest.raises(hmps.HmpsError):        # more than 64 right-hand sides
        srv.submit(3, np.zeros((p.n, 65), np.complex128), K=2, prob=p, leaf_max=leaf)
    state = C.c_int32()
    assert lib.ps_poll(srv._s, C.c_uint64(12345), None, None, C.byref(state)) == hmps.HM_EINVAL
    t = srv.submit(3, b, K=2, prob=p, leaf_max=leaf, aca_tol=tol)
    while lib.ps_poll(srv._s, C.c_uint64(t), None, None, C.byref(state)) == hmps.HM_ENOTREADY:
        pass
    assert state.value == hmps.PS_DONE  # a state-only poll keeps the result
    assert lib.ps_poll(srv._s, C.c_uint64(t), None, None, C.byref(state)) == hmps.HM_OK
    x, st = srv.wait(t)
    assert x.shape == b.shape and st[0]["t_ms"] > 0
    assert lib.ps_poll(srv._s, C.c_uint64(t), None, None, C.byref(state)) == hmps.HM_EINVAL
    srv.close()


def test_server_gmres_where_the_series_diverges(oracles):
    """GMRES requests (D^{-1} preconditioner) on the cube, where the series
    diverges (rho > 1), reach x* = Z_l^{-1} b through the server; requests of
    the same geometry and options are batched; the GMRES basis kept on the
    geometry counts in the resident bytes.  The nested kind and a restart
    beyond 64 are refused."""
    srv = hmps.Server(slots=2)
    seen = set()
    H = oracles[2]
    p = GEOMS[2][0]
    _say("server series request on the cube")
    t0 = _submit(srv, 2, W.plane_waves(p.xyz, W.directions(2, 3, instance=200)), seen, K=2)
    srv.wait(t0)
    before = srv.info()["resident_bytes"]
    bs = [W.plane_waves(p.xyz, W.directions(n, 3, instance=210 + i)) for i, n in enumerate((3, 1, 5))]
    _say("server GMRES requests on the cube")
    ts = [_submit(srv, 2, b, seen, K=0, kind=hmps.PS_GMRES, max_passes=500, refine_tol=1e-11)
          for b in bs]
    for t, b in zip(ts, bs):
        x, st = srv.wait(t)
        assert_close(x, series.solve_exact(H, b), 1e-8)
        assert all(s["diverged"] == 0 and s["resid_rel"] <= 1e-11 and s["passes"] > 0 for s in st)
    assert srv.info()["resident_bytes"] > before
    with pytest.raises(hmps.HmpsError):
        _submit(srv, 2, bs[0], seen, K=1, kind=hmps.PS_NESTED)
    with pytest.raises(hmps.HmpsError):
        _submit(srv, 2, bs[0], seen, K=0, kind=hmps.PS_GMRES, max_passes=10, refine_tol=1e-9,
                restart=65)
    srv.close()


def test_server_cold_build_steps_aside_for_queued_resident_work(oracles):
    """One slot and a budget for one geometry: a cold request (geometry 3)
    followed at once by a request for the resident geometry 1.  Geometry 1
    cannot be evicted while its request is queued, so the cold build steps
    aside, the worker serves geometry 1 first, then evicts it and builds
    geometry 3; both requests finish and match the oracle."""
    probe = hmps.Server(slots=1)
    sizes = {}
    seen = set()
    for key in (1, 3):
        b = W.plane_waves(GEOMS[key][0].xyz, W.Z_HAT)
        probe.wait(_submit(probe, key, b, seen, K=2))
        sizes[key] = probe.info()["resident_bytes"] - sum(sizes.values())
    probe.close()
    budget = int(max(sizes.values()) + 0.5 * min(sizes.values()))
    srv = hmps.Server(budget_bytes=budget, slots=1)
    seen = set()
    b1 = W.plane_waves(GEOMS[1][0].xyz, W.directions(2, 3, instance=40))
    srv.wait(_submit(srv, 1, b1, seen, K=2))           # geometry 1 resident
    b3 = W.plane_waves(GEOMS[3][0].xyz, W.directions(3, 3, instance=41))
    b1b = W.plane_waves(GEOMS[1][0].xyz, W.directions(1, 3, instance=42))
    _say("server cold request then a resident one, one slot")
    t3 = _submit(srv, 3, b3, seen, K=2)
    t1 = _submit(srv, 1, b1b, seen, K=2)
    x1, _ = srv.wait(t1)
    x3, st3 = srv.wait(t3)
    assert_close(x1, series.series(oracles[1], b1b, 2), 1e-10)
    assert_close(x3, series.series(oracles[3], b3, 2), 1e-10)
    assert st3[0]["built"] == 1
    info = srv.info()
    assert info["requests_failed"] == 0 and info["evictions"] >= 1
    assert info["resident_bytes"] <= budget
    srv.close()


def test_non_finite_rhs_reported():
    """A right-hand side with a NaN entry: the series and refinement report
    the column as diverged (HM_EDIVERGED with statistics) and leave the
    other columns exact; through the server, the request with the NaN is
    reported diverged and a clean request of the same batch is not."""
    wl = W.sphere_small()
    H = hmatrix.HMatrix(wl.problem, 64, 1.0, 1e-4)
    b = W.plane_waves(wl.problem.xyz, W.directions(3, 3))
    bad = b.copy()
    bad[17, 1] = np.nan
    h = hmps.HMatrix(wl.problem, 64, 1.0, 1e-4)
    for kw in (dict(kind=hmps.PS_SERIES), dict(kind=hmps.PS_REFINE, max_passes=50, refine_tol=1e-10),
               dict(kind=hmps.PS_GMRES, max_passes=40, refine_tol=1e-10)):
        for cols in ([1], [0, 1, 2]):
            _say(f"NaN right-hand side {kw} columns {cols}")
            x, st = h.solve(torch.from_numpy(np.ascontiguousarray(bad[:, cols])).to("cuda"), K=4,
                            stats=True, **kw)
            x = x.cpu().numpy().reshape(wl.problem.n, -1)
            for j, c in enumerate(cols):
                if c == 1:
                    assert st[j]["diverged"] == 1, (kw, st[j])
                else:
                    assert st[j]["diverged"] == 0, (kw, st[j])
                    assert np.all(np.isfinite(x[:, j]))
    h.close()
    srv = hmps.Server(slots=1)
    ok = b[:, [0, 2]]
    t_bad = srv.submit(5, bad[:, [1]], K=4, prob=wl.problem, leaf_max=64, aca_tol=1e-4)
    t_ok = srv.submit(5, ok, K=4)
    _, st_ok = srv.wait(t_ok)
    assert all(s_["diverged"] == 0 for s_ in st_ok)
    state, x_bad, st_bad = srv.poll(t_bad)
    while st_bad is None:
        state, x_bad, st_bad = srv.poll(t_bad)
    assert state == hmps.PS_DONE and st_bad[0]["diverged"] == 1
    srv.close()
