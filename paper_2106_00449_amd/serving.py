"""Continuous batching of independent suspensions on one GPU.

A request is one suspension (its library arguments, an initial state and a
number of gDC steps) with an arrival time.  The server admits requests in
arrival order as slots and device memory free up (admission by the HBM
footprint the library reports for the request, against a budget), keeps
every admitted suspension's state resident on the device, and advances all
of them together with gdc_batch_step: each suspension's kernels run on its
own stream, so their work overlaps on the GPU, and the call returns as soon
as one suspension finishes (or the next arrival is due) so that the freed
memory is handed on at once.  A suspension's result does not depend on what
else is in the mix: its kernels, their order and its noise are its own.

Reported per request: admission, finish and step completion times; per-step
latency is the time between consecutive step completions of the same
suspension (the first from its admission).  Step errors are the
suspension's own (the library reports an outcome per handle): a suspension
whose state became non-finite (or whose pair-force cell list overflowed) is
stopped and reported at once without disturbing the others; one whose
solve missed the tolerance runs to the end and is reported as failed.

The executor is pluggable (footprint / open / step / close / discard) so
that the admission logic can be exercised without a GPU.
"""

import collections
import time
from dataclasses import dataclass, field

import numpy as np

# per-suspension outcomes of a batched step (include/gdc.h)
GDC_OK, GDC_ENOTCONV, GDC_ENUMERIC = 0, -3, -4


@dataclass
class Request:
    rid: int
    kwargs: dict          # paper_2106_00449_amd.Suspension arguments
    Y0: np.ndarray
    q0: np.ndarray
    n_steps: int
    arrival: float = 0.0  # seconds after the start of the run
    blobs: int = 0


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    Y: np.ndarray = None
    q: np.ndarray = None
    step_times: np.ndarray = None   # completion times (s, run clock), first = admission
    error: str = ""
    blobs: int = 0
    n_steps: int = 0

    @property
    def latencies(self):
        if self.step_times is None or len(self.step_times) < 2:
            return np.zeros(0)
        return np.diff(self.step_times)


# Largest grid edge whose suspensions the default executor fuses: on one
# MI355X the fused GMRES iterations serve 32^3 suspensions faster than
# concurrent streams, tie at 48^3 and lose from 64^3 up.
FUSE_MAX_GRID = 32


class LibraryExecutor:
    """Runs requests on the HIP library (one handle and stream each).  With
    fusion, the suspensions' GMRES iterations are launched fused: one launch
    per kernel for all the ready suspensions of a grid size.  fusion is a
    bool, or an int: the largest grid edge whose suspensions are fused
    (smaller grids gain from fusion, larger ones from concurrent streams)."""

    def __init__(self, fusion=FUSE_MAX_GRID):
        import paper_2106_00449_amd as g
        self.g = g
        self.fusion = fusion if isinstance(fusion, int) and not isinstance(fusion, bool) else bool(fusion)

    def _fused(self, req):
        if isinstance(self.fusion, bool):
            return self.fusion
        return max(int(x) for x in np.atleast_1d(req.kwargs["n"])) <= self.fusion

    def footprint(self, req):
        return self.g.footprint(**req.kwargs)

    def open(self, req):
        s = self.g.Suspension(**req.kwargs)
        s.set_state(req.Y0, req.q0)
        if self._fused(req):
            s.fusion = True
        return s

    def step(self, handles, steps, until, max_ms):
        """Returns (steps left, each handle's outcome for this call)."""
        left, stats, _ = self.g.batch_step(handles, steps, until=until, max_ms=max_ms)
        return left, [x["status"] for x in stats]

    def step_log(self, h):
        return h.step_log()

    def close(self, h):
        Y, q = h.get_state()
        log = h.step_log()
        h.close()
        return Y, q, log

    def discard(self, h):
        """Release a failed suspension (steps may still be queued; freeing
        waits for them)."""
        h.close()


@dataclass
class _Active:
    req: Request
    handle: object
    fp: int
    left: int
    notconv: int = 0      # calls in which one of its solves missed the tolerance
    times: list = field(default_factory=list)


class Server:
    """Admission by HBM footprint and a slot cap, FIFO (a request that does
    not fit waits, and so do the ones behind it: no overtaking, no
    starvation); a request larger than the whole budget is rejected."""

    def __init__(self, hbm_budget=32 << 30, max_slots=32, executor=None, clock=time.monotonic,
                 sleep=time.sleep):
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.ex = executor if executor is not None else LibraryExecutor()
        self.clock = clock
        self.sleep = sleep
        self.peak_bytes = 0
        self.peak_slots = 0

    def run(self, requests):
        """Serve every request; returns {rid: Result}."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        fps = {r.rid: int(self.ex.footprint(r)) for r in reqs}
        results = {r.rid: Result(r.rid, r.arrival, blobs=r.blobs, n_steps=r.n_steps) for r in reqs}
        pending = collections.deque(reqs)
        queue = collections.deque()
        active = []
        used = 0
        t0 = self.clock()
        ms0 = t0 * 1e3   # the library's step log uses the same monotonic clock, in ms

        def now():
            return self.clock() - t0

        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            while queue:
                r = queue[0]
                if fps[r.rid] > self.budget:
                    queue.popleft()
                    results[r.rid].error = "footprint exceeds the HBM budget"
                    continue
                if len(active) >= self.max_slots or used + fps[r.rid] > self.budget:
                    break
                queue.popleft()
                res = results[r.rid]
                res.admitted = now()
                if r.n_steps == 0:
                    res.Y, res.q = r.Y0.copy(), r.q0.copy()
                    res.finished = res.admitted
                    res.step_times = np.array([res.admitted])
                    continue
                try:
                    h = self.ex.open(r)
                except Exception as e:   # noqa: BLE001 -- reported per request
                    res.error = f"admission failed: {e}"
                    continue
                used += fps[r.rid]
                active.append(_Active(r, h, fps[r.rid], r.n_steps))
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_slots = max(self.peak_slots, len(active))
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            # wake for the next arrival only if it could be admitted
            max_ms = 0.0
            if pending and not queue:
                max_ms = max((pending[0].arrival - now()) * 1e3, 1e-3)
            left, status = self.ex.step([a.handle for a in active], [a.left for a in active], "any", max_ms)
            still = []
            for a, lft, code in zip(active, left, status):
                a.left = lft
                res = results[a.req.rid]
                if code not in (GDC_OK, GDC_ENOTCONV):
                    # this suspension's state is unusable: stop it now
                    res.error = f"step failed with code {code} after {a.req.n_steps - lft} steps"
                    res.finished = now()
                    try:
                        self.ex.discard(a.handle)
                    except Exception as e:   # noqa: BLE001
                        res.error += f"; release failed: {e}"
                    used -= a.fp
                    continue
                if code == GDC_ENOTCONV:
                    a.notconv += 1
                if lft > 0:
                    still.append(a)
                    continue
                try:
                    Y, q, log = self.ex.close(a.handle)
                    res.Y, res.q = Y, q
                    res.step_times = np.asarray(log, dtype=np.float64) / 1e3 - (ms0 / 1e3)
                    res.finished = float(res.step_times[-1]) if len(res.step_times) else now()
                except Exception as e:   # noqa: BLE001
                    res.error = f"readback failed: {e}"
                    res.finished = now()
                if a.notconv and not res.error:
                    res.error = f"GMRES missed the tolerance in {a.notconv} batched calls"
                used -= a.fp
            active = still
        return results


def summarise(results, makespan=None):
    """Throughput and latency figures of a served run."""
    ok = [r for r in results.values() if not r.error]
    lat = np.concatenate([r.latencies for r in ok]) if ok else np.zeros(0)
    start = min((r.arrival for r in results.values()), default=0.0)
    end = max((r.finished for r in ok), default=0.0)
    span = makespan if makespan is not None else end - start
    blob_steps = sum(r.blobs * r.n_steps for r in ok)
    resp = np.array([r.finished - r.arrival for r in ok]) if ok else np.zeros(0)
    wait = np.array([r.admitted - r.arrival for r in ok]) if ok else np.zeros(0)
    pct = (lambda a, p: float(np.percentile(a, p)) * 1e3 if a.size else float("nan"))
    return {
        "requests": len(results), "completed": len(ok),
        "rejected": len(results) - len(ok),
        "makespan_s": span,
        "blob_steps_per_s": blob_steps / span if span > 0 else float("nan"),
        "step_latency_p50_ms": pct(lat, 50), "step_latency_p99_ms": pct(lat, 99),
        "queue_wait_p50_ms": pct(wait, 50), "queue_wait_p99_ms": pct(wait, 99),
        "response_p50_ms": pct(resp, 50), "response_p99_ms": pct(resp, 99),
    }
