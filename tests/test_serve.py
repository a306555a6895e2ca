"""Server logic on the CPU: admission by slots and HBM budget, batching, failure
handling, and results that are the same for an event alone and in the mix.

A simulated clock drives the server; the executor runs the CPU oracle and takes a
simulated time per batch, so every property is checked without a GPU.
"""

import numpy as np
import pytest

from oracle import oracle
from paper_2202_06929_amd import serve

R, K, D = 0.15, 32, 6


class SimClock:
    def __init__(self):
        self.now = 0.0

    def __call__(self):
        self.now += 1e-6  # every look at the clock costs a microsecond
        return self.now

    def idle(self, until):
        self.now = max(self.now, until)


class FakeExecutor:
    """Runs the oracle per event; a batch takes 50 us + 10 ns per point."""

    def __init__(self, clock, n_streams=2, fail_batches=(), fail_finish=(), fail_poll=(), bytes_per_point=100):
        self.clock = clock
        self.n_streams = n_streams
        self.busy = 0
        self.fail_batches = set(fail_batches)
        self.fail_finish = set(fail_finish)
        self.fail_poll = set(fail_poll)
        self.aborted = []
        self.bpp = bytes_per_point
        self.batches = 0
        self.admitted = []
        self.live = set()
        self.peak_live_bytes = 0

    def footprint(self, req):
        return self.bpp * max(req.n, 1)

    def admit(self, req):
        self.admitted.append(req.rid)
        self.live.add(req.rid)

    def free_streams(self):
        return self.n_streams - self.busy

    def start(self, batch):
        b = self.batches
        self.batches += 1
        if b in self.fail_batches:
            raise RuntimeError("injected start failure")
        self.busy += 1
        cost = 50e-6 + 10e-9 * sum(r.n for r in batch)
        return {"b": b, "ready": self.clock.now + cost, "batch": batch}

    def poll(self, h):
        if h["b"] in self.fail_poll and self.clock.now >= h["ready"]:
            raise RuntimeError("injected poll failure")
        return self.clock.now >= h["ready"]

    def _free(self, h):
        if not h.get("freed"):
            h["freed"] = True
            self.busy -= 1

    def finish(self, h):
        self._free(h)
        if h["b"] in self.fail_finish:
            raise RuntimeError("injected finish failure")
        return [(serve.OK, oracle.frnn_grid(r.points, R, K)) for r in h["batch"]]

    def abort(self, h):
        self.aborted.append(h["b"])
        self._free(h)

    def release(self, req):
        self.live.discard(req.rid)


def make_trace(n_events=40, rate=20000.0, seed=3, lo=20, hi=400):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_events))
    out = []
    for k in range(n_events):
        n = int(rng.integers(lo, hi))
        c = rng.uniform(-1, 1, size=(max(1, n // 8), D))
        pts = (c[rng.integers(0, len(c), size=n)] + rng.normal(0, 0.05, size=(n, D))).astype(np.float32)
        out.append(serve.Request(rid=k, arrival=float(t[k]), points=pts))
    return out


def run(trace, budget=10**9, **kw):
    clock = SimClock()
    ex = FakeExecutor(clock, **{k: v for k, v in kw.items()
                                if k in ("n_streams", "fail_batches", "fail_finish", "fail_poll")})
    srv = serve.Server(ex, hbm_budget=budget, max_slots=kw.get("max_slots", 64), max_batch=kw.get("max_batch", 8),
                       clock=clock, idle=clock.idle)
    stats = srv.run(trace)
    return srv, ex, stats


def test_each_result_is_the_same_alone_and_in_the_mix():
    trace = make_trace()
    srv, ex, stats = run(trace)
    assert stats.completed == len(trace) and stats.failed == 0
    assert stats.batches < len(trace)  # requests were batched
    for req in trace:
        assert np.array_equal(req.edges, oracle.frnn_grid(req.points, R, K))
    assert srv.used == 0 and srv.slots == 0 and not ex.live


def test_admission_respects_budget_and_order():
    trace = make_trace(n_events=30, rate=1e6)  # all arrive at once
    budget = 100 * 1200
    clock = SimClock()
    ex = FakeExecutor(clock)
    srv = serve.Server(ex, hbm_budget=budget, max_slots=64, max_batch=4, clock=clock, idle=clock.idle)
    peak = {"used": 0}
    orig_admit = ex.admit

    def admit(req):
        orig_admit(req)
        peak["used"] = max(peak["used"], srv.used)

    ex.admit = admit
    stats = srv.run(trace)
    assert stats.completed == len(trace)
    assert peak["used"] <= budget
    order = [r.rid for r in sorted(trace, key=lambda r: r.arrival)]
    assert ex.admitted == order  # first come, first admitted
    assert srv.used == 0


def test_event_larger_than_budget_is_rejected_and_others_finish():
    trace = make_trace(n_events=12)
    big = serve.Request(rid=99, arrival=trace[3].arrival, points=np.zeros((5000, D), np.float32))
    srv, ex, stats = run(trace + [big], budget=100 * 2000)
    assert big.status == serve.REJECTED
    assert stats.rejected == 1 and stats.completed == len(trace)
    assert srv.used == 0


def test_slot_limit_bounds_requests_in_flight():
    trace = make_trace(n_events=25, rate=1e6)
    srv, ex, stats = run(trace, max_slots=3)
    assert stats.max_in_flight <= 3
    assert stats.completed == len(trace)


@pytest.mark.parametrize("where", ["start", "finish", "poll"])
def test_injected_executor_failure_fails_only_that_batch(where):
    trace = make_trace(n_events=30)
    kw = {"start": {"fail_batches": {2}}, "finish": {"fail_finish": {1}}, "poll": {"fail_poll": {1}}}[where]
    srv, ex, stats = run(trace, **kw)
    failed = [r for r in trace if r.status == serve.FAILED]
    assert failed and len({r.batch for r in failed}) == 1
    assert stats.completed == len(trace) - len(failed)
    for r in trace:
        if r.status == serve.OK:
            assert np.array_equal(r.edges, oracle.frnn_grid(r.points, R, K))
    assert srv.used == 0 and srv.slots == 0 and not ex.live  # memory returned after the failure


def test_plain_loop_baseline():
    trace = make_trace(n_events=10)
    clock = SimClock()

    def build(req):
        clock.now += 50e-6 + 10e-9 * req.n
        return oracle.frnn_grid(req.points, R, K)

    stats = serve.plain_loop(trace, build, clock=clock, idle=clock.idle)
    assert stats.completed == 10 and stats.p50_ms > 0.05
    for req in trace:
        assert req.latency >= 50e-6


def test_poll_failures_give_every_stream_back():
    """A batch whose completion check raises is aborted, so its stream is free
    again: with every batch failing that way the server still drains the trace
    (it would spin forever if the streams stayed taken)."""
    trace = make_trace(n_events=20, rate=1e6)
    srv, ex, stats = run(trace, n_streams=2, fail_poll=set(range(100)))
    assert stats.failed == len(trace) and stats.completed == 0
    assert ex.busy == 0 and sorted(ex.aborted) == list(range(stats.batches))
    assert srv.used == 0 and srv.slots == 0 and not ex.live


def test_cancelled_requests_never_run_and_return_their_admission():
    """Requests cancelled while queued (waiting for admission, or admitted but not
    yet started) complete as CANCELLED without reaching the executor; the others
    finish with the oracle's edges; slots and budget return to zero."""
    trace = make_trace(n_events=30, rate=1e6)  # all arrive at once; one stream, batches of 2
    clock = SimClock()
    ex = FakeExecutor(clock, n_streams=1)
    srv = serve.Server(ex, hbm_budget=10 ** 9, max_slots=64, max_batch=2, clock=clock, idle=clock.idle)
    started = []
    orig_start = ex.start

    def start(batch):
        started.extend(r.rid for r in batch)
        if len(started) == 2:   # while the first batch runs, cancel three queued requests
            for rid in (5, 11, 29):
                srv.cancel(rid)
        return orig_start(batch)

    ex.start = start
    srv.cancel(17)  # cancelled before it arrives
    stats = srv.run(trace)
    cancelled = sorted(r.rid for r in trace if r.status == serve.CANCELLED)
    assert cancelled == [5, 11, 17, 29] and stats.cancelled == 4
    assert not set(cancelled) & set(started)
    assert stats.completed == len(trace) - 4
    for r in trace:
        if r.status == serve.OK:
            assert np.array_equal(r.edges, oracle.frnn_grid(r.points, R, K))
    assert srv.used == 0 and srv.slots == 0 and not ex.live


def test_requests_that_wait_past_their_timeout_time_out():
    """With one stream and a burst of arrivals, requests whose timeout passes
    before they can start complete as TIMED_OUT; a generous timeout never fires."""
    trace = make_trace(n_events=24, rate=1e6)
    for k, r in enumerate(trace):
        r.timeout = 1.0 if k % 2 else 150e-6
    srv, ex, stats = run(trace, n_streams=1, max_batch=2)
    late = [r for r in trace if r.status == serve.TIMED_OUT]
    assert late and stats.timed_out == len(late)
    assert all(r.timeout == 150e-6 for r in late)
    for r in trace:
        if r.status == serve.OK:
            assert r.started - r.arrival <= r.timeout + 1e-5
    assert stats.completed + stats.timed_out == len(trace)
    assert srv.used == 0 and srv.slots == 0 and not ex.live
