"""Batched stepping and serving on the GPU, through the C ABI.

gdc_batch_step advances several resident suspensions with overlapped work;
each suspension must end where gdc_step takes it alone (same kernels, same
order, same Philox noise: the results are compared exactly where no
pair-force cell list is built, and to the FP32 step tolerance 1e-5 of the
increment otherwise).  The served run must give each request the result it
gets alone.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from tests._common import rel_l2

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2106_00449_amd as g
    return g


def _mix():
    return [
        wl.small_case("b_rods", n_bodies=12, n=32, L=24.0, shapes=[wl.rod(5)], precision="fp32", seed=21,
                      dt=0.005),
        wl.small_case("b_mixed", n_bodies=9, n=(24, 32, 48), L=(20.0, 24.0, 36.0),
                      shapes=[wl.rod(4), wl.boomerang(), wl.tetrahedron()], precision="fp32", seed=22,
                      dt=0.005, const_force=(0.0, 0.0, 1.0, 0.0, 0.0, 0.0)),
        wl.small_case("b_fp64", n_bodies=6, n=24, L=20.0, shapes=[wl.rod(3)], precision="fp64", seed=23,
                      dt=0.005),
        wl.small_case("b_steric", n_bodies=16, n=48, L=32.0, shapes=[wl.rod(5)], precision="fp32", seed=24,
                      dt=0.005, steric_k=40.0 / 2.2, steric_cutoff=2.2),
    ]


def _alone(lib, w, n_steps):
    Y, q = wl.initial_state(w)
    Y0 = Y.copy()
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-6))
    s.step(Y, q, n_steps)
    s.close()
    return Y0, Y, q


def _close(a, b, Y0, exact):
    if exact:
        return np.array_equal(a, b)
    return rel_l2(a - Y0, b - Y0) < 1e-5


def test_footprint_matches_allocation(lib):
    for w in _mix():
        kw = wl.library_kwargs(w)
        s = lib.Suspension(**kw)
        assert s.device_bytes == lib.footprint(**kw)
        s.close()


@pytest.mark.parametrize("until", ["all", "any"])
def test_batch_step_equals_each_alone(lib, until):
    ws = _mix()
    n_steps = [3, 2, 4, 3]
    ref = [_alone(lib, w, k) for w, k in zip(ws, n_steps)]
    _say("batch", until)
    ss = []
    for w in ws:
        s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-6))
        Y, q = wl.initial_state(w)
        s.set_state(Y, q)
        ss.append(s)
    left = list(n_steps)
    calls = 0
    while any(left):
        left, stats, rc = lib.batch_step(ss, left, until=until)
        assert rc == 0
        calls += 1
        assert calls <= sum(n_steps)
    for s, w, (Y0, Yr, qr), k in zip(ss, ws, ref, n_steps):
        Y, q = s.get_state()
        exact = w.steric_k == 0.0
        assert _close(Y, Yr, Y0, exact), w.name
        assert _close(q, qr, 0.0 * qr, exact), w.name
        assert s.step_counter == k
        log = s.step_log()
        assert len(log) == k + 1 and np.all(np.diff(log) > 0)
        s.close()


@pytest.mark.parametrize("k", [0, 2])
def test_pipelined_steps_equal_single_steps(lib, k):
    # one call of 5 steps queues each step behind the previous one's update
    # and reads nu and the flags back later: the result, the means and the
    # step log must be those of 5 calls of one step
    w = _mix()[k]
    Y0, q0 = wl.initial_state(w)
    _say("pipeline", w.name)
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-6))
    Y1, q1 = Y0.copy(), q0.copy()
    singles = [s.step(Y1, q1, 1) for _ in range(5)]
    s.step_counter = 0
    s.step_log()
    Y5, q5 = Y0.copy(), q0.copy()
    st = s.step(Y5, q5, 5)
    log = s.step_log()
    s.close()
    assert np.array_equal(Y5, Y1) and np.array_equal(q5, q1)
    assert st["steps_done"] == 5 and len(log) == 6 and np.all(np.diff(log) > 0)
    assert st["gmres_iterations"] == singles[-1]["gmres_iterations"]
    assert st["nu"] == singles[-1]["nu"]
    assert st["gmres_iterations_mean"] == pytest.approx(np.mean([x["gmres_iterations"] for x in singles]))
    nus = np.array([x["nu"] for x in singles])
    assert st["nu_mean"] == pytest.approx(nus.mean())
    assert st["nu_min"] == nus.min() and st["nu_max"] == nus.max()
    assert st["nu_std"] == pytest.approx(nus.std(), rel=1e-9, abs=1e-12)


def test_batch_step_resumes_a_step_left_in_flight(lib):
    ws = _mix()[:3]
    ref = [_alone(lib, w, 2) for w in ws]
    _say("resume")
    ss = []
    for w in ws:
        s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-6))
        s.set_state(*wl.initial_state(w))
        ss.append(s)
    # a wall-clock limit far below one step returns with steps in flight
    left, _, rc = lib.batch_step(ss, [2, 2, 2], until="all", max_ms=0.001)
    assert rc == 0
    with pytest.raises(lib.GdcError):
        ss[0].get_state()
    while any(left):
        left, _, rc = lib.batch_step(ss, left, until="all")
        assert rc == 0
    for s, (Y0, Yr, qr) in zip(ss, ref):
        Y, q = s.get_state()
        assert np.array_equal(Y, Yr) and np.array_equal(q, qr)
        s.close()


# fusion: none, every suspension, or the server's default (32^3 grids only:
# fused and unfused handles in the same batch calls)
@pytest.mark.parametrize("fusion", [False, True, 32])
def test_served_results_equal_alone(lib, fusion):
    from paper_2106_00449_amd.serving import LibraryExecutor, Request, Server, summarise
    ws = _mix() + (_fuse_mix()[:3] if fusion else [])
    n_steps = [6, 4, 5, 6] + ([5, 3, 4] if fusion else [])
    reqs = []
    for i, (w, k) in enumerate(zip(ws, n_steps)):
        Y, q = wl.initial_state(w)
        reqs.append(Request(i, wl.library_kwargs(w, gmres_tol=1e-6), Y, q, k, arrival=0.002 * i, blobs=w.M))
    _say("serve mix", {False: "streams", True: "fused"}.get(fusion, f"fused up to {fusion}^3"))
    # a budget that holds all but the smallest at once, so admission binds
    fps = sorted(lib.footprint(**r.kwargs) for r in reqs)
    srv = Server(hbm_budget=sum(fps[1:]), max_slots=8, executor=LibraryExecutor(fusion=fusion))
    res = srv.run(reqs)
    summ = summarise(res)
    assert summ["completed"] == len(ws), summ
    assert srv.peak_bytes <= srv.budget
    for r, w in zip(reqs, ws):
        Y0, Yr, qr = _alone(lib, w, r.n_steps)
        out = res[r.rid]
        exact = w.steric_k == 0.0
        assert _close(out.Y, Yr, Y0, exact), w.name
        assert _close(out.q, qr, 0.0 * qr, exact), w.name
        assert len(out.step_times) == r.n_steps + 1
    assert summ["step_latency_p99_ms"] >= summ["step_latency_p50_ms"] > 0


@pytest.mark.parametrize("prec,n,L", [("fp32", 32, 24.0), ("fp32", (24, 32, 48), (20.0, 24.0, 36.0)),
                                      ("fp64", 32, 24.0),
                                      # five-pass, every pass moving whole-wave runs
                                      ("fp32", (128, 128, 256), (96.0, 96.0, 192.0)),
                                      # ragged lines along axis 1 in the projection pass
                                      ("fp32", (128, 12, 24), (96.0, 12.0, 19.0))])
def test_every_fft_launch_shape_gives_identical_results(lib, prec, n, L):
    # the autotuner only chooses among workgroup sizes that distribute the
    # same arithmetic: forcing each size must give the same mobility bit for bit
    w = wl.small_case("shapes", n_bodies=6, n=n, L=L, shapes=[wl.rod(4), wl.boomerang()], precision=prec, seed=17)
    Y, q = wl.initial_state(w)
    lam = np.random.default_rng(5).standard_normal((w.M, 3))
    s = lib.Suspension(**wl.library_kwargs(w))
    tuned = s.launch_config
    _say("shapes", prec, n, tuned)
    ref = s.mobility_apply("blob", Y, q, lam)
    for t in [256, 512, 1024]:
        cfg = {k: (t if k in ("plane_fwd", "plane_inv") else min(t, 512)) for k in s.FFT_PASSES}
        s.launch_config = cfg
        assert s.launch_config == cfg
        v = s.mobility_apply("blob", Y, q, lam)
        assert np.array_equal(v, ref), t
    with pytest.raises(lib.GdcError):
        s.launch_config = {"r2c": 1024}
    s.close()


@pytest.mark.parametrize("k", [0, 1, 2])
def test_graph_replay_equals_eager_launches(lib, k):
    # GMRES iterations and step set-ups replayed from captured HIP graphs
    # against every kernel launched on its own: the same results bit for bit
    # over several steps with restart cycles (restart 4, so every column's
    # graph is replayed across cycles), eager work between the replays (a body
    # solve at another configuration re-keys the graphs), a jump of the step
    # counter (the set-up graph reads it from the device), and batched
    # stepping
    w = _mix()[k]
    Y0, q0 = wl.initial_state(w)
    F = np.random.default_rng(3).standard_normal((w.N, 6))
    out = {}
    for graphs in (False, True):
        _say("graphs", w.name, graphs)
        s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-6, gmres_restart=4, gmres_maxit=400))
        s.graphs = graphs
        assert s.graphs == graphs
        Y, q = Y0.copy(), q0.copy()
        st1 = s.step(Y, q, 3)
        assert st1["gmres_iterations"] > 4          # more than one restart cycle
        V = s.mobility_apply("body", Y, q, F, allow_notconv=True)
        s.step_counter = s.step_counter + 7
        st2 = s.step(Y, q, 2)
        s.set_state(Y, q)
        left = [2]
        while any(left):
            left, _, rc = lib.batch_step([s], left)
            assert rc == 0
        Yb, qb = s.get_state()
        out[graphs] = (Y, q, V, Yb, qb, st1["gmres_iterations"], st2["nu"], st2["gmres_iterations_mean"])
        s.close()
    for a, b in zip(out[False], out[True]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def _fuse_mix():
    # four fusable suspensions (FP32, plane-path grids, matrix-core
    # preconditioner) in two groups by grid size, and an FP64 one that runs
    # unfused beside them
    return [
        wl.small_case("f_rods", n_bodies=12, n=32, L=24.0, shapes=[wl.rod(5)], precision="fp32", seed=31,
                      dt=0.005),
        wl.small_case("f_mixed", n_bodies=20, n=32, L=28.0, shapes=[wl.rod(3), wl.tetrahedron()],
                      precision="fp32", seed=32, dt=0.005, const_force=(0.0, 0.0, 1.0, 0.0, 0.0, 0.0)),
        wl.small_case("f_boom", n_bodies=7, n=32, L=20.0, shapes=[wl.boomerang()], precision="fp32", seed=33,
                      dt=0.005),
        wl.small_case("f_48", n_bodies=16, n=48, L=32.0, shapes=[wl.rod(5)], precision="fp32", seed=34,
                      dt=0.005),
        wl.small_case("f_64", n_bodies=6, n=32, L=20.0, shapes=[wl.rod(3)], precision="fp64", seed=35,
                      dt=0.005),
    ]


@pytest.mark.parametrize("until,graphs", [("all", True), ("any", True), ("all", False)])
def test_fused_batch_equals_each_alone(lib, until, graphs):
    # GMRES iterations launched once per kernel for all ready suspensions
    # (each at its own Krylov column: restart 4 makes cycles end at
    # different times) give every suspension the result of stepping it
    # alone, bit for bit; with graphs off the rest of each step is launched
    # kernel by kernel beside the fused iterations
    ws = _fuse_mix()
    n_steps = [3, 2, 4, 3, 2]
    kw = dict(gmres_tol=1e-6, gmres_restart=4, gmres_maxit=400)
    ref = []
    for w, k in zip(ws, n_steps):
        Y, q = wl.initial_state(w)
        s = lib.Suspension(**wl.library_kwargs(w, **kw))
        s.step(Y, q, k)
        s.close()
        ref.append((Y, q))
    _say("fused batch", until, "graphs" if graphs else "eager")
    ss = []
    for w in ws:
        s = lib.Suspension(**wl.library_kwargs(w, **kw))
        s.graphs = graphs
        Y, q = wl.initial_state(w)
        s.set_state(Y, q)
        s.fusion = True
        assert s.fusion
        ss.append(s)
    left = list(n_steps)
    fused = [0] * len(ws)
    while any(left):
        left, stats, _ = lib.batch_step(ss, left, until=until)
        for i, x in enumerate(stats):
            assert x["status"] in (lib.GDC_OK,), (ws[i].name, x)
            fused[i] += x["fused_iterations"]
    for i, (s, w) in enumerate(zip(ss, ws)):
        Y, q = s.get_state()
        assert np.array_equal(Y, ref[i][0]), w.name
        assert np.array_equal(q, ref[i][1]), w.name
        s.close()
    # every FP32 suspension had its iterations fused; the FP64 one none
    assert all(f > 0 for f in fused[:4]), fused
    assert fused[4] == 0, fused
