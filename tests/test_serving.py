"""Host logic of the continuous-batching server (no GPU): admission by
footprint and slots, FIFO order, rejection of oversize requests, admission of
arrivals while other suspensions are in flight, and the latency bookkeeping.
A simulated executor stands in for the library: each suspension's step takes
a fixed simulated time, and suspensions in flight run concurrently."""
import numpy as np

from paper_2106_00449_amd.serving import Request, Server, summarise


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class SimExecutor:
    """Suspension state = Y0 + (steps taken); step time per suspension =
    kwargs["step_s"]; footprint = kwargs["bytes"]."""

    def __init__(self, clock):
        self.clock = clock
        self.calls = []
        self.live = set()

    def footprint(self, req):
        return req.kwargs["bytes"]

    def open(self, req):
        h = {"req": req, "done": 0, "next": self.clock() + req.kwargs["step_s"], "log": [self.clock() * 1e3]}
        self.live.add(id(h))
        return h

    def step(self, handles, steps, until, max_ms):
        """Like the library: each handle's outcome counts only the steps
        completed in this call; kwargs["fail_at"] = (step, code) makes that
        step of the suspension report the code."""
        assert until == "any"
        self.calls.append(len(handles))
        left = list(steps)
        status = [0] * len(handles)
        deadline = self.clock() + max_ms / 1e3 if max_ms > 0 else float("inf")
        while True:
            i = min(range(len(handles)), key=lambda k: handles[k]["next"] if left[k] > 0 else float("inf"))
            t_next = handles[i]["next"]
            if t_next > deadline:
                self.clock.t = deadline
                return left, status
            self.clock.t = t_next
            h = handles[i]
            h["done"] += 1
            h["log"].append(t_next * 1e3)
            left[i] -= 1
            h["next"] = t_next + h["req"].kwargs["step_s"]
            fail = h["req"].kwargs.get("fail_at")
            if fail and fail[0] == h["done"]:
                status[i] = fail[1]
                if fail[1] == -4:     # a failed handle counts as done
                    return left, status
            if left[i] == 0:
                return left, status

    def close(self, h):
        self.live.discard(id(h))
        r = h["req"]
        return r.Y0 + h["done"], r.q0.copy(), h["log"]

    def discard(self, h):
        self.live.discard(id(h))


def _req(rid, arrival, n_steps, step_s, nbytes):
    return Request(rid, {"step_s": step_s, "bytes": nbytes}, np.full((2, 3), float(rid)),
                   np.tile([1.0, 0, 0, 0], (2, 1)), n_steps, arrival, blobs=20)


def _serve(reqs, budget, slots):
    clk = SimClock()
    ex = SimExecutor(clk)
    srv = Server(hbm_budget=budget, max_slots=slots, executor=ex, clock=clk, sleep=clk.sleep)
    return srv, ex, srv.run(reqs)


def test_every_request_completes_with_its_own_result():
    reqs = [_req(i, 0.01 * i, 5 + i % 3, 0.001 * (1 + i % 4), 100) for i in range(20)]
    srv, ex, res = _serve(reqs, budget=1000, slots=4)
    assert len(res) == 20 and not ex.live
    for r in reqs:
        out = res[r.rid]
        assert not out.error
        assert np.array_equal(out.Y, r.Y0 + r.n_steps)
        assert len(out.step_times) == r.n_steps + 1
        assert np.all(out.latencies > 0)
        assert out.admitted >= r.arrival and out.finished >= out.admitted


def test_budget_and_slots_bind():
    reqs = [_req(i, 0.0, 4, 0.002, 300) for i in range(10)]
    srv, _, res = _serve(reqs, budget=1000, slots=8)
    assert srv.peak_bytes <= 1000 and srv.peak_slots == 3   # 3 x 300 fit, 4 do not
    srv, _, res = _serve(reqs, budget=10_000, slots=2)
    assert srv.peak_slots == 2


def test_fifo_admission_and_oversize_rejection():
    reqs = [_req(0, 0.0, 3, 0.001, 600), _req(1, 0.0001, 3, 0.001, 5000), _req(2, 0.0002, 3, 0.001, 600),
            _req(3, 0.0003, 3, 0.001, 300)]
    _, _, res = _serve(reqs, budget=1000, slots=8)
    assert res[1].error and not res[0].error and not res[2].error
    # request 3 fits beside 0 but must not overtake 2, which does not
    assert res[3].admitted >= res[2].admitted
    order = sorted([r for r in res.values() if not r.error], key=lambda r: r.arrival)
    assert all(a.admitted <= b.admitted for a, b in zip(order, order[1:]))


def test_arrivals_are_admitted_while_others_run():
    # a long suspension is in flight when a short one arrives: the short one
    # must be admitted at its arrival and finish long before the long one
    reqs = [_req(0, 0.0, 100, 0.01, 100), _req(1, 0.05, 5, 0.001, 100)]
    _, ex, res = _serve(reqs, budget=1000, slots=4)
    assert abs(res[1].admitted - 0.05) < 1e-9
    assert res[1].finished < res[0].finished
    assert max(ex.calls) == 2


def test_summary_figures():
    reqs = [_req(i, 0.0, 4, 0.001, 100) for i in range(4)]
    _, _, res = _serve(reqs, budget=1000, slots=4)
    s = summarise(res)
    assert s["completed"] == 4 and s["rejected"] == 0
    assert abs(s["step_latency_p50_ms"] - 1.0) < 1e-9
    assert abs(s["blob_steps_per_s"] - 4 * 20 * 4 / 0.004) < 1e-6


def test_step_errors_are_attributed_to_their_own_suspension():
    # request 1's third step goes non-finite while request 0 finishes and
    # request 2 misses a solve tolerance: 1 is stopped at once and its
    # memory released, 0 completes untouched, 2 runs to its end and is
    # reported; requests admitted later (3) still run
    reqs = [_req(0, 0.0, 4, 0.001, 300), _req(1, 0.0, 50, 0.0015, 300), _req(2, 0.0, 6, 0.002, 300),
            _req(3, 0.0, 3, 0.001, 300)]
    reqs[1].kwargs["fail_at"] = (3, -4)
    reqs[2].kwargs["fail_at"] = (2, -3)
    srv, ex, res = _serve(reqs, budget=900, slots=3)
    assert not ex.live
    assert not res[0].error and np.array_equal(res[0].Y, reqs[0].Y0 + 4)
    assert "code -4" in res[1].error and res[1].Y is None
    assert res[1].finished < 0.005     # stopped at its third step, not after 50
    assert "tolerance" in res[2].error and res[2].Y is not None
    assert not res[3].error and np.array_equal(res[3].Y, reqs[3].Y0 + 3)
    s = summarise(res)
    assert s["completed"] == 2 and s["rejected"] == 2


def test_library_executor_fusion_policy():
    # the executor fuses every suspension, none, or those whose grid edge is
    # at most the given size (the default: 32^3 grids)
    from paper_2106_00449_amd.serving import FUSE_MAX_GRID, LibraryExecutor

    def req(n):
        return Request(0, {"n": n}, np.zeros((1, 3)), np.zeros((1, 4)), 1)

    assert LibraryExecutor().fusion == FUSE_MAX_GRID == 32
    small, cubic48, mixed = req(32), req((48, 48, 48)), req((24, 32, 48))
    assert LibraryExecutor()._fused(small) and not LibraryExecutor()._fused(cubic48)
    assert not LibraryExecutor()._fused(mixed)
    assert LibraryExecutor(fusion=48)._fused(cubic48)
    assert all(LibraryExecutor(fusion=True)._fused(r) for r in (small, cubic48, mixed))
    assert not any(LibraryExecutor(fusion=False)._fused(r) for r in (small, cubic48, mixed))
