"""Serving loop: continuous batching of solve requests on one device.

Requests (degree, mesh size, coefficient, right-hand-side seed) arrive as host events.  The
scheduler admits them first come, first served while the sum of the admitted requests' device
footprints stays within a byte budget, and keeps every admitted request's mesh, geometry,
multigrid hierarchy and Krylov state on the device until it finishes.  Each scheduler step
advances all running solves together, retires the finished ones and frees their memory, so
requests that arrive while others run join at the next step.  With a batched executor a step is
one ``mfq_batch_run``: a few CG iterations of every running solve issued as one launch per
(kernel, degree) over all of them from a device work table, one device-to-host copy of all their
states and one wait; otherwise ``mfq_batch_step`` (each solve's launches on its own stream, one
status copy per request) or per-request asynchronous steps.

The solver of a request is GMG_MIXED (FP64 CG, FP64 operator and dot products, FP32 multigrid
V-cycle) with an FP64 true-residual check and refinement passes until the relative residual is
at most ``rtol``; its coarsest level uses the Chebyshev mode, so no solve ever waits on the host
between steps.  This batching of independent requests is a serving pattern, not part of the
paper's method.
"""
import concurrent.futures as cf
import dataclasses
import math
import threading
import time
from typing import List, Optional

from . import _lib
from ._lib import MFQ_BC_DIRICHLET0, MFQ_FP64, MFQ_SOLVER_GMG_MIXED, MFQ_OK


@dataclasses.dataclass
class Request:
    degree: int
    n: int
    alpha: float
    seed: int
    amplitude: float = 0.0
    rtol: float = 1e-10
    max_iter: int = 1000
    # filled in by the server
    id: int = -1
    arrival: float = math.nan
    admitted: float = math.nan
    finished: float = math.nan
    status: Optional[int] = None
    iterations: int = 0
    rel_residual: float = math.nan
    footprint: int = 0
    result: object = None  # solution (device tensor) when the server keeps results

    @property
    def latency(self):
        return self.finished - self.arrival


class DeviceExecutor:
    """Builds and runs requests with the library; device memory comes from torch."""

    def __init__(self, n_streams=4, keep_results=False, solver_kind=MFQ_SOLVER_GMG_MIXED, batched=False,
                 max_active=256, **solver_params):
        import torch
        self.torch = torch
        # default-priority streams: solves are spread over `streams` round-robin; set-up work
        # (geometry, hierarchy, eigenvalue estimates, which wait on the host) runs on its own
        # stream so its waits do not queue behind the running solves
        # batched: every solve runs on one stream and a step is one mfq_batch_run over all of them
        self.batched = bool(batched)
        self.streams = [torch.cuda.Stream() for _ in range(1 if self.batched else max(1, n_streams))]
        # one set-up stream per thread that sets requests up: set-ups on several worker threads
        # wait only for their own work
        self._setup_streams = threading.local()
        self.batch = None
        if self.batched:
            from . import Batch
            self.batch = Batch(max_active, stream=self.streams[0])
        self.keep_results = keep_results
        self.kind = solver_kind
        # served solves smooth their coarsest level (no host round trip, so they can be batched)
        # and estimate eigenvalues with 8 Lanczos steps: on the 2,000-request stream as many CG
        # iterations as with 12 (8.42 against 8.45 per solve) and 7% more solves/s
        self.params = dict(coarse_mode=1, lanczos_iters=8)
        self.params.update(solver_params)
        self._next_stream = 0

    def prepare(self, req):
        """Host-side handles and the device footprint in bytes (nothing allocated on the device)."""
        h = {}
        h["mesh"] = _lib.mfq_mesh_create(req.n, req.amplitude)
        h["space"] = _lib.mfq_space_create(h["mesh"], req.degree, MFQ_BC_DIRICHLET0)
        h["op"] = _lib.mfq_op_create(h["space"], req.alpha, MFQ_FP64)
        prm = _lib.mfq_solver_default_params()
        for k, v in self.params.items():
            setattr(prm, k, v)
        h["prm"] = prm
        h["solver"] = _lib.mfq_solver_create(h["op"], self.kind, prm)
        h["N"] = _lib.mfq_space_n_dofs(h["space"])
        h["op_bytes"] = _lib.mfq_op_device_bytes(h["op"])
        h["solver_bytes"] = _lib.mfq_solver_device_bytes(h["solver"])
        vec = -(-h["N"] * 8 // 256) * 256
        h["bytes"] = h["op_bytes"] + h["solver_bytes"] + 2 * vec
        return h

    def setup(self, req, h):
        """Allocate and set up (geometry, hierarchy, eigenvalue estimates) on the set-up stream.  May
        run on a set-up thread while the scheduler steps other requests (the library's calls release
        the interpreter lock; each request has its own handles).  It enqueues nothing on the solve
        streams: the scheduler captures CG iterations into HIP graphs on those, and a capture
        records every launch into the stream, whichever thread issues it."""
        torch = self.torch
        su = getattr(self._setup_streams, "stream", None)
        if su is None:
            su = self._setup_streams.stream = torch.cuda.Stream()
        with torch.cuda.stream(su):
            h["op_buf"] = torch.empty(max(h["op_bytes"], 256), dtype=torch.uint8, device="cuda")
            h["solver_buf"] = torch.empty(max(h["solver_bytes"], 256), dtype=torch.uint8, device="cuda")
            h["b"] = torch.empty(h["N"], dtype=torch.float64, device="cuda")
            h["x"] = torch.empty(h["N"], dtype=torch.float64, device="cuda")
        sp = su.cuda_stream
        _lib.mfq_op_bind(h["op"], h["op_buf"].data_ptr(), h["op_bytes"], sp)
        _lib.mfq_space_random(h["space"], MFQ_FP64, h["b"].data_ptr(), req.seed, sp)
        # synchronises the set-up stream: everything above is complete before the solve starts.
        # Batched: the eigenvalue estimates are left to the first batched step, which makes those
        # of all requests starting together in one set of launches.
        bind = _lib.mfq_solver_bind_lazy if self.batched else _lib.mfq_solver_bind
        bind(h["solver"], h["solver_buf"].data_ptr(), h["solver_bytes"], sp)

    def begin(self, req, h):
        """Begin the solve on the next solve stream (scheduler thread only)."""
        st = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        h["stream"] = st
        _lib.mfq_solve_begin(h["solver"], h["b"].data_ptr(), h["x"].data_ptr(), req.rtol, req.max_iter,
                             st.cuda_stream)

    def start(self, req, h):
        self.setup(req, h)
        self.begin(req, h)

    def step(self, handles, iters):
        if self.batched:
            return _lib.mfq_batch_run(self.batch.handle, [h["solver"] for h in handles], iters,
                                      self.streams[0].cuda_stream)
        return _lib.mfq_batch_step([h["solver"] for h in handles], iters)

    def submit(self, h, iters):
        _lib.mfq_solve_step_async(h["solver"], iters)

    def poll(self, h):
        return _lib.mfq_solve_step_poll(h["solver"])

    def finish(self, req, h):
        status, info = _lib.mfq_solve_end(h["solver"], check=False)
        req.status = status
        req.iterations = info.iterations
        req.rel_residual = info.rel_residual
        if self.keep_results:
            req.result = h["x"]

    def release(self, h):
        if h.get("solver"):
            _lib.mfq_solver_destroy(h["solver"])
        if h.get("op"):
            _lib.mfq_op_destroy(h["op"])
        if h.get("space"):
            _lib.mfq_space_destroy(h["space"])
        if h.get("mesh"):
            _lib.mfq_mesh_destroy(h["mesh"])
        h.clear()


class Server:
    """FIFO admission by device footprint, continuous batching, latency accounting.

    mode "sync": every step advances all running solves together and waits for all of them
    (mfq_batch_step).  mode "async": each solve's next few iterations are enqueued as soon as its
    previous ones have been polled complete (mfq_solve_step_async / _poll), so a long request does
    not hold back the others; a step is one pass over the running solves and never waits.

    setup_threads > 0: an admitted request is set up (executor.setup) on a worker thread while
    the scheduler keeps stepping the running solves; at the first step after its set-up has
    finished the scheduler begins its solve (executor.begin) and it joins the others.  Its memory
    counts against the budget from admission on.  Only the scheduler thread issues work to the
    solve streams."""

    def __init__(self, executor, budget_bytes, iters_per_step=2, max_active=256, clock=time.perf_counter,
                 mode="sync", idle_sleep=2e-5, setup_threads=0):
        if mode not in ("sync", "async"):
            raise ValueError("mode must be 'sync' or 'async'")
        if setup_threads < 0:
            raise ValueError("setup_threads must be >= 0")
        self.mode = mode
        self._pool = cf.ThreadPoolExecutor(setup_threads) if setup_threads else None
        self._setup_lock = threading.Lock()
        self.starting = []                  # (request, handles, future): set-up running on a worker
        self.idle_sleep = idle_sleep
        self.ex = executor
        self.budget = int(budget_bytes)
        self.iters = int(iters_per_step)
        self.max_active = int(max_active)
        self.clock = clock
        self.queue: List[Request] = []      # arrived, waiting for admission (FIFO)
        self.active = []                    # (request, handles)
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.used = 0
        self.steps = 0
        self.peak_used = 0
        self.peak_active = 0
        self._next_id = 0
        self._head = None  # prepared handles of the request at the head of the queue
        self.setup_s = 0.0   # host time in admission (handles, allocation, set-up on the device)
        self.step_s = 0.0    # host time in batch steps (launches and the per-step wait)

    def submit(self, req, now=None):
        req.id = self._next_id
        self._next_id += 1
        req.arrival = self.clock() if now is None else now
        self.queue.append(req)
        return req.id

    def _admit(self):
        while self.queue and len(self.active) + len(self.starting) < self.max_active:
            req = self.queue[0]
            if self._head is None:
                self._head = self.ex.prepare(req)
            h = self._head
            if h["bytes"] > self.budget:
                # can never fit: reject instead of blocking the queue
                self.queue.pop(0)
                self._head = None
                self.ex.release(h)
                req.status = _lib.MFQ_ENOMEM
                req.finished = self.clock()
                self.rejected.append(req)
                continue
            if self.used + h["bytes"] > self.budget:
                break  # waits (with its prepared handles) until memory frees up
            self.queue.pop(0)
            self._head = None
            req.footprint = h["bytes"]
            self.used += h["bytes"]
            req.admitted = self.clock()
            if self._pool is not None:
                self.starting.append((req, h, self._pool.submit(self._setup, req, h)))
            else:
                self._setup(req, h)
                self.ex.begin(req, h)
                self.active.append((req, h))
        self.peak_used = max(self.peak_used, self.used)
        self.peak_active = max(self.peak_active, len(self.active) + len(self.starting))

    def _setup(self, req, h):
        t = time.perf_counter()
        self.ex.setup(req, h)
        with self._setup_lock:
            self.setup_s += time.perf_counter() - t

    def _collect_started(self):
        """Move requests whose set-up has finished into the running set (set-up errors re-raise)."""
        if not self.starting:
            return
        still = []
        for req, h, fut in self.starting:
            if fut.done():
                fut.result()
                self.ex.begin(req, h)
                self.active.append((req, h))
            else:
                still.append((req, h, fut))
        self.starting = still

    def step(self):
        """Admit what fits, advance the running solves, retire the finished ones.
        Returns the requests finished in this step."""
        self._admit()
        self._collect_started()
        if not self.active:
            if self.starting:
                # nothing to step yet: wait for the first set-up to finish
                cf.wait([f for _, _, f in self.starting], return_when=cf.FIRST_COMPLETED)
            return []
        if self.mode == "async":
            return self._step_async()
        t = time.perf_counter()
        flags = self.ex.step([h for _, h in self.active], self.iters)
        self.step_s += time.perf_counter() - t
        self.steps += 1
        now = self.clock()
        finished, still = [], []
        for (req, h), d in zip(self.active, flags):
            if d:
                self._retire(req, h, now)
                finished.append(req)
            else:
                still.append((req, h))
        self.active = still
        return finished

    def _retire(self, req, h, now):
        self.ex.finish(req, h)
        req.finished = now
        self.used -= req.footprint
        self.ex.release(h)
        self.done.append(req)

    def _step_async(self):
        t = time.perf_counter()
        finished, still, progressed = [], [], False
        for req, h in self.active:
            if not h.get("inflight"):
                self.ex.submit(h, self.iters)
                h["inflight"] = True
                progressed = True
                still.append((req, h))
                continue
            ready, done = self.ex.poll(h)
            if not ready:
                still.append((req, h))
                continue
            progressed = True
            h["inflight"] = False
            if done:
                self._retire(req, h, self.clock())
                finished.append(req)
            else:
                self.ex.submit(h, self.iters)
                h["inflight"] = True
                still.append((req, h))
        self.active = still
        self.steps += 1
        self.step_s += time.perf_counter() - t
        if not progressed and self.idle_sleep:
            time.sleep(self.idle_sleep)
        return finished

    @property
    def idle(self):
        return not self.queue and not self.active and not self.starting

    def close(self):
        """Stop the set-up workers (after draining)."""
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None

    def drain(self):
        while not self.idle:
            self.step()

    def stats(self):
        lat = sorted(r.latency for r in self.done)
        ok = [r for r in self.done if r.status == MFQ_OK]
        out = {"requests": len(self.done), "converged": len(ok), "rejected": len(self.rejected),
               "steps": self.steps, "peak_active": self.peak_active, "peak_bytes": self.peak_used,
               "setup_host_s": self.setup_s, "step_host_s": self.step_s}
        if lat:
            first = min(r.arrival for r in self.done)
            last = max(r.finished for r in self.done)
            out["solves_per_s"] = len(self.done) / max(last - first, 1e-9)
            out["p50_s"] = percentile(lat, 50)
            out["p99_s"] = percentile(lat, 99)
            out["max_rel_residual"] = max(r.rel_residual for r in self.done)
        return out


def percentile(sorted_values, q):
    """Nearest-rank percentile of an ascending list."""
    if not sorted_values:
        return math.nan
    k = max(0, min(len(sorted_values) - 1, math.ceil(q / 100.0 * len(sorted_values)) - 1))
    return sorted_values[k]


def run_stream(server, requests, arrivals, sleep=time.sleep):
    """Replays `requests` arriving at offsets `arrivals` (seconds from now): submits each when its
    time has come, steps the server meanwhile, and returns when all have finished."""
    t0 = server.clock()
    i = 0
    n = len(requests)
    while i < n or not server.idle:
        now = server.clock() - t0
        while i < n and arrivals[i] <= now:
            server.submit(requests[i], now=t0 + arrivals[i])
            i += 1
        if server.idle and i < n:
            sleep(max(0.0, arrivals[i] - (server.clock() - t0)))
            continue
        server.step()
    return server.stats()
