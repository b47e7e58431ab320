"""Serving loop for completion requests: admission by HBM footprint, iterates
resident on the device, iteration-level continuous batching.

Every tick advances each running request by one PGA iteration (Alg. 5) through
one batch of the engine (`lt.Batch`): all frontal slices of all running
requests go through one Jacobi launch.  Requests that arrive while others run
are admitted at the next tick boundary when their footprint fits the HBM
budget; finished requests leave and free their memory, and the batch is rebuilt
from the running set (each request's state lives in its own workspace, so its
iteration continues unchanged in the new batch).

The scheduler talks to an executor (make / rebuild / step / poll / result /
release), so its policy can be exercised without a GPU.
"""
import heapq
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float              # seconds on the server clock
    M: np.ndarray               # observed tensor (host, float32/float64)
    mask: np.ndarray            # bool / uint8
    params: dict                # mu0, nu, mu_bar, tol, max_iter (+ optional precision)
    kinds: tuple = None
    footprint: int = 0          # device bytes while resident
    admitted: float = None
    finished: float = None
    iters: int = 0
    converged: bool = False
    result: np.ndarray = None
    handle: object = None

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class GpuExecutor:
    """Executor on the HIP engine (paper_2202_02870_amd.lt)."""

    def __init__(self, use_graph=True, precision="f32"):
        import torch  # noqa: F401
        from . import lt
        self.lt = lt
        self.use_graph = use_graph
        self.precision = precision
        self.batch = None

    def _params(self, req):
        p = req.params
        return self.lt.pga_params(mu0=p["mu0"], nu=p.get("nu", 0.9), mu_bar=p["mu_bar"], tol=p.get("tol", 0.0),
                                  max_iter=p["max_iter"], precision=p.get("precision", self.precision))

    def footprint(self, req):
        lt = self.lt
        d = lt.make_desc(req.M.shape, req.kinds)
        prm = self._params(req)
        ws = lt._lib.lt_problem_workspace_bytes(lt.ctypes.byref(d), lt.ctypes.byref(prm))
        n = int(np.prod(req.M.shape))
        return int(ws) + 9 * n          # + M (4 B), mask (1 B), X (4 B) per entry

    def make(self, req):
        import torch
        lt = self.lt
        M = lt.to_device(req.M)
        mask = lt.to_device(np.asarray(req.mask, dtype=np.uint8), dtype=torch.uint8)
        return lt.Problem(M, mask, self._params(req), req.kinds)

    def rebuild(self, handles):
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        if handles:
            self.batch = self.lt.Batch(handles, use_graph=self.use_graph)

    def step(self, ticks):
        if self.batch is not None:
            self.batch.step(ticks)

    def poll(self, handle):
        rep, done = handle.status()
        return rep["iters"], done, rep["converged"]

    def result(self, handle):
        return self.lt.to_host(handle.X)

    def release(self, handle):
        pass    # the tensors go when the last reference does


class CompletionServer:
    """Continuous-batching completion server.

    hbm_budget: device bytes the resident requests may hold together.
    ticks_per_round: PGA iterations enqueued between two polls of the running
    requests (a request may overrun its stopping point by up to this many
    ticks' worth of idle work, never by iterations: finished problems are
    skipped on the device).
    """

    def __init__(self, executor, hbm_budget, ticks_per_round=1, clock=None):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.ticks = int(ticks_per_round)
        self.clock = clock or time.perf_counter
        self.t0 = None
        self.waiting = []           # heap of (arrival, rid)
        self.requests = {}
        self.running = []
        self.done = []
        self.used = 0
        self.peak_used = 0
        self.rejected = []
        self.ticks_run = 0
        self.rebuilds = 0

    def now(self):
        if self.t0 is None:
            self.t0 = self.clock()
        return self.clock() - self.t0

    def submit(self, req):
        req.footprint = self.ex.footprint(req)
        if req.footprint > self.budget:
            self.rejected.append(req)     # could never fit: refused, not queued forever
            return False
        self.requests[req.rid] = req
        heapq.heappush(self.waiting, (req.arrival, req.rid))
        return True

    def _admit(self, now):
        """Admit arrived requests in arrival order; a request that does not fit
        lets later, smaller ones in (backfill)."""
        admitted = []
        skipped = []
        while self.waiting and self.waiting[0][0] <= now:
            arr, rid = heapq.heappop(self.waiting)
            req = self.requests[rid]
            if self.used + req.footprint <= self.budget:
                req.handle = self.ex.make(req)
                req.admitted = now
                self.used += req.footprint
                self.peak_used = max(self.peak_used, self.used)
                self.running.append(req)
                admitted.append(req)
            else:
                skipped.append((arr, rid))
        for item in skipped:
            heapq.heappush(self.waiting, item)
        return admitted

    def step(self):
        """One scheduling round: admit, (re)batch, run ticks, retire."""
        now = self.now()
        changed = bool(self._admit(now))
        if changed:
            self.ex.rebuild([r.handle for r in self.running])
            self.rebuilds += 1
        if not self.running:
            return False
        self.ex.step(self.ticks)
        self.ticks_run += self.ticks
        finished = []
        for r in self.running:
            iters, done, conv = self.ex.poll(r.handle)
            r.iters = iters
            if done:
                r.converged = conv
                r.finished = self.now()
                r.result = self.ex.result(r.handle)
                finished.append(r)
        if finished:
            for r in finished:
                self.running.remove(r)
                self.used -= r.footprint
                self.ex.release(r.handle)
                r.handle = None
                self.done.append(r)
            self.ex.rebuild([r.handle for r in self.running])
            self.rebuilds += 1
        return True

    def idle(self):
        return not self.running and not self.waiting

    def run(self, max_rounds=10 ** 9, sleep=0.0):
        rounds = 0
        while not self.idle() and rounds < max_rounds:
            if not self.step() and self.waiting:
                # nothing resident: wait for the next arrival
                nxt = self.waiting[0][0]
                delay = nxt - self.now()
                if delay > 0 and sleep:
                    time.sleep(min(delay, sleep))
            rounds += 1
        return self.stats()

    def stats(self):
        lat = np.array([r.latency for r in self.done], dtype=np.float64)
        out = dict(completed=len(self.done), rejected=len(self.rejected), ticks=self.ticks_run,
                   rebuilds=self.rebuilds, peak_bytes=self.peak_used)
        if lat.size:
            out.update(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                       mean=float(lat.mean()), max=float(lat.max()))
        return out


def poisson_arrivals(n, rate, seed):
    """n arrival times of a Poisson process of the given rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
