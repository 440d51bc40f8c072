"""Scheduler logic of the serving loop on the host: a fake executor stands in for the device
(tests only), so admission, continuous batching and latency accounting run without a GPU."""
import threading

import pytest

from paper_1910_13247_amd import _lib
from paper_1910_13247_amd.serve import Request, Server, percentile, run_stream


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor:
    """Footprint = 100 * degree bytes; a request finishes after `n` steps; each step costs 1 ms."""

    def __init__(self, clock):
        self.clock = clock
        self.started = []
        self.live = {}
        self.max_live_bytes = 0
        self.prepared = 0
        self.gates = {}            # request id -> threading.Event its set-up waits for
        self.lock = threading.Lock()
        self.scheduler_thread = threading.get_ident()

    def prepare(self, req):
        self.prepared += 1
        return {"bytes": 100 * req.degree, "req": req}

    def setup(self, req, h):
        gate = self.gates.get(req.id)
        if gate is not None:
            assert gate.wait(10.0), "set-up gate never opened"
        with self.lock:
            self.started.append(req.id)
            self.live[req.id] = h["bytes"]
            self.max_live_bytes = max(self.max_live_bytes, sum(self.live.values()))
        h["setup_thread"] = threading.get_ident()

    def begin(self, req, h):
        # the solve itself starts on the scheduler thread
        assert threading.get_ident() == self.scheduler_thread
        h["left"] = req.n

    def step(self, handles, iters):
        self.clock.t += 1e-3
        out = []
        for h in handles:
            h["left"] -= 1
            out.append(h["left"] <= 0)
        return out

    # asynchronous protocol: a submitted step is ready after `lag` polls
    def submit(self, h, iters):
        assert not h.get("pending"), "submit while a step is in flight"
        h["pending"] = h["req"].seed % 3 + 1

    def poll(self, h):
        self.clock.t += 1e-4
        h["pending"] -= 1
        if h["pending"] > 0:
            return False, False
        h["left"] -= 1
        return True, h["left"] <= 0

    def finish(self, req, h):
        req.status = _lib.MFQ_OK
        req.iterations = req.n * 2
        req.rel_residual = 1e-11

    def release(self, h):
        if "req" in h:
            with self.lock:
                self.live.pop(h["req"].id, None)


def make(budget, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock)
    return Server(ex, budget, clock=clock, **kw), ex, clock


def test_fifo_admission_within_budget():
    srv, ex, clock = make(budget=500)
    reqs = [Request(degree=d, n=n, alpha=0.1, seed=i) for i, (d, n) in enumerate([(3, 5), (2, 2), (4, 1), (1, 1)])]
    for r in reqs:
        srv.submit(r)
    srv.step()
    # 300 + 200 fit, the 400-byte request waits (FIFO: the 100-byte one behind it waits too)
    assert ex.started == [0, 1]
    assert srv.used == 500 and len(srv.queue) == 2
    srv.drain()
    assert ex.started == [0, 1, 2, 3]
    assert ex.max_live_bytes <= 500 and srv.peak_used <= 500
    assert all(r.status == _lib.MFQ_OK for r in reqs)
    assert srv.used == 0


def test_oversized_request_rejected_without_blocking():
    srv, ex, clock = make(budget=250)
    big = Request(degree=6, n=1, alpha=0.0, seed=0)     # 600 bytes: can never fit
    small = Request(degree=2, n=1, alpha=0.0, seed=1)
    srv.submit(big)
    srv.submit(small)
    srv.drain()
    assert big.status == _lib.MFQ_ENOMEM and srv.rejected == [big]
    assert small.status == _lib.MFQ_OK


def test_continuous_batching_joins_mid_run():
    """A request that arrives while a long one runs is admitted at the next step and finishes first."""
    srv, ex, clock = make(budget=10_000)
    long = Request(degree=1, n=50, alpha=0.0, seed=0)
    short = Request(degree=1, n=3, alpha=0.0, seed=1)
    srv.submit(long)
    for _ in range(5):
        srv.step()
    srv.submit(short)
    finished_order = []
    while not srv.idle:
        finished_order += [r.id for r in srv.step()]
    assert finished_order == [short.id, long.id]
    assert short.admitted - short.arrival < 2e-3     # admitted at the next step


def test_max_active_limit():
    srv, ex, clock = make(budget=10**9, max_active=3)
    for i in range(10):
        srv.submit(Request(degree=1, n=4, alpha=0.0, seed=i))
    srv.step()
    assert len(srv.active) == 3
    srv.drain()
    assert srv.peak_active == 3 and len(srv.done) == 10


def test_latency_accounting_and_stream_replay():
    srv, ex, clock = make(budget=10**6)
    reqs = [Request(degree=1 + i % 3, n=2 + i % 4, alpha=0.0, seed=i) for i in range(20)]
    arrivals = [0.01 * i for i in range(20)]
    st = run_stream(srv, reqs, arrivals, sleep=clock.sleep)
    assert st["requests"] == 20 and st["converged"] == 20
    for r, a in zip(reqs, arrivals):
        assert r.arrival == pytest.approx(a)
        assert r.finished >= r.admitted >= r.arrival
        # n steps of 1 ms each after admission (admitted at the first step after arrival)
        assert r.finished - r.admitted == pytest.approx(r.n * 1e-3, abs=1.5e-3)
    lat = sorted(r.latency for r in reqs)
    assert st["p50_s"] == percentile(lat, 50) and st["p99_s"] == lat[-1]


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([7.0], 99) == 7.0


@pytest.mark.parametrize("budget", [500, 10**6])
def test_async_mode_completes_everything_within_budget(budget):
    """Asynchronous stepping: every request finishes, the budget is never exceeded, each request's
    steps are submitted only after the previous one was polled complete (asserted by the fake)."""
    srv, ex, clock = make(budget=budget, mode="async", idle_sleep=0)
    reqs = [Request(degree=1 + i % 4, n=1 + i % 5, alpha=0.0, seed=i) for i in range(30)]
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert all(r.status == _lib.MFQ_OK for r in reqs) and len(srv.done) == 30
    assert ex.max_live_bytes <= budget and srv.peak_used <= budget and srv.used == 0
    assert all(r.finished >= r.admitted >= r.arrival for r in reqs)


def test_async_mode_short_request_overtakes_long_one():
    srv, ex, clock = make(budget=10**6, mode="async", idle_sleep=0)
    long = Request(degree=1, n=60, alpha=0.0, seed=0)
    short = Request(degree=1, n=2, alpha=0.0, seed=3)
    srv.submit(long)
    srv.submit(short)
    order = []
    while not srv.idle:
        order += [r.id for r in srv.step()]
    assert order == [short.id, long.id]


def test_mode_is_validated():
    with pytest.raises(ValueError):
        make(budget=1, mode="parallel")


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_setup_thread_overlaps_stepping(mode):
    """With a set-up worker, a running request keeps stepping (and finishes) while a later
    request's set-up is still blocked; the later one joins once its set-up is done."""
    srv, ex, clock = make(budget=10**6, mode=mode, idle_sleep=0, setup_threads=1)
    a = Request(degree=1, n=4, alpha=0.0, seed=0)
    b = Request(degree=1, n=2, alpha=0.0, seed=1)
    gate = threading.Event()
    ex.gates[1] = gate
    srv.submit(a)
    finished = []
    for _ in range(3):
        finished += srv.step()
    srv.submit(b)
    for _ in range(200):
        finished += srv.step()
        if a in finished:
            break
    assert a in finished and a.status == _lib.MFQ_OK
    assert b.status is None and len(srv.starting) == 1 and not srv.idle
    assert srv.used == 100          # b's memory is held from admission on
    gate.set()
    while not srv.idle:
        finished += srv.step()
    srv.close()
    assert finished == [a, b] and b.status == _lib.MFQ_OK and srv.used == 0
    assert srv.peak_active == 2
    # set-up ran on the worker, the solves began on the scheduler thread (asserted in begin)
    assert all(r.id in ex.started for r in (a, b))


def test_setup_errors_reach_the_scheduler():
    srv, ex, clock = make(budget=10**6, setup_threads=1)

    def broken(req, h):
        raise RuntimeError("set-up failed")

    ex.setup = broken
    srv.submit(Request(degree=1, n=1, alpha=0.0, seed=0))
    with pytest.raises(RuntimeError, match="set-up failed"):
        for _ in range(10):
            srv.step()
    srv.close()
