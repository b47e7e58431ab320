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
    lane: int = 0               # executor lane (see GpuExecutor)
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
    """Executor on the HIP engine (paper_2202_02870_amd.lt).

    Lanes: requests whose slices take the blocked Jacobi kernel (slices wider
    than 256 columns: a tick of tens of milliseconds) run in lane 1, a batch of
    their own on a second stream, and the others in lane 0, so the long ticks do
    not set the tick length of the short requests; the two streams' kernels
    share the GPU.  lanes=False puts every request in lane 0."""

    def __init__(self, use_graph=True, precision="f32", lanes=True):
        import torch
        from . import lt
        self.torch = torch
        self.lt = lt
        self.use_graph = use_graph
        self.precision = precision
        self.lanes = lanes
        self.batches = {}
        self.streams = {}

    def _params(self, req):
        p = req.params
        return self.lt.pga_params(mu0=p["mu0"], nu=p.get("nu", 0.9), mu_bar=p["mu_bar"], tol=p.get("tol", 0.0),
                                  max_iter=p["max_iter"], precision=p.get("precision", self.precision))

    def _stream(self, lane):
        s = self.streams.get(lane)
        if s is None:
            s = self.torch.cuda.Stream()   # default priority
            self.streams[lane] = s
        return s

    def lane(self, req):
        if not self.lanes:
            return 0
        return 1 if "blocked" in self.lt.svt_path(req.M.shape, req.kinds) else 0

    def footprint(self, req):
        lt = self.lt
        d = lt.make_desc(req.M.shape, req.kinds)
        prm = self._params(req)
        ws = lt._lib.lt_problem_workspace_bytes(lt.ctypes.byref(d), lt.ctypes.byref(prm))
        if ws == 0:
            raise ValueError("the batch engine does not take this problem")
        n = int(np.prod(req.M.shape))
        return int(ws) + 9 * n          # + M (4 B), mask (1 B), X (4 B) per entry

    def make(self, req):
        lt = self.lt
        M = lt.to_device(req.M)
        mask = lt.to_device(np.asarray(req.mask, dtype=np.uint8), dtype=self.torch.uint8)
        h = lt.Problem(M, mask, self._params(req), req.kinds)
        h.lane = self.lane(req)
        return h

    def rebuild(self, handles, lane=0):
        """New batch of the lane's running problems (the lane's stream is idle)."""
        b = self.batches.pop(lane, None)
        if b is not None:
            b.close()
        if handles:
            with self.torch.cuda.stream(self._stream(lane)):
                self.batches[lane] = self.lt.Batch(handles, use_graph=self.use_graph)

    def step(self, ticks, lane=0):
        """Enqueue ticks on the lane's stream (returns without waiting)."""
        b = self.batches.get(lane)
        if b is not None:
            with self.torch.cuda.stream(self._stream(lane)):
                b.step(ticks)

    def busy(self, lane):
        s = self.streams.get(lane)
        return s is not None and not s.query()

    def poll(self, handle):
        """(iterations, done, converged); waits for the handle's lane."""
        with self.torch.cuda.stream(self._stream(getattr(handle, "lane", 0))):
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

    Admission: the arrived requests are admitted in order of HBM footprint,
    smallest first, while they fit the budget (the most requests resident, the
    small ones not held behind large ones); a request that has waited max_wait
    seconds goes ahead of the others in arrival order, and while such a request
    does not fit nothing behind it is admitted, so memory frees up for it
    (large requests are not starved).

    Lanes (when the executor has `lane`, `busy`): lane 0 is stepped and polled
    every round; every other lane runs asynchronously: it is polled, rebuilt
    and given new ticks (lane_ticks per enqueue) only when its previous ticks
    have finished, so its long ticks overlap lane 0's rounds instead of
    lengthening them.
    """

    def __init__(self, executor, hbm_budget, ticks_per_round=1, clock=None, on_finish=None,
                 lane_ticks=1, max_wait=2.0):
        self.ex = executor
        self.max_wait = float(max_wait)
        self.on_finish = on_finish      # called with each finished request
        self.budget = int(hbm_budget)
        self.ticks = int(ticks_per_round)
        self.lane_ticks = int(lane_ticks)
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
        self.dirty = set()          # lanes whose running set changed since their last batch

    def now(self):
        if self.t0 is None:
            self.t0 = self.clock()
        return self.clock() - self.t0

    def _lane(self, req):
        f = getattr(self.ex, "lane", None)
        return f(req) if f is not None else 0

    def _busy(self, lane):
        f = getattr(self.ex, "busy", None)
        return f(lane) if f is not None else False

    def submit(self, req):
        try:
            req.footprint = self.ex.footprint(req)
            req.lane = self._lane(req)
        except Exception:                 # a shape no kernel takes: refused
            self.rejected.append(req)
            return False
        if req.footprint <= 0 or req.footprint > self.budget:
            self.rejected.append(req)     # could never fit: refused, not queued forever
            return False
        self.requests[req.rid] = req
        heapq.heappush(self.waiting, (req.arrival, req.rid))
        return True

    def _admit(self, now):
        """Admit arrived requests by footprint, smallest first; requests that
        waited max_wait seconds first, in arrival order (see the class)."""
        arrived = []
        while self.waiting and self.waiting[0][0] <= now:
            arrived.append(heapq.heappop(self.waiting))

        def order(item):
            arr, rid = item
            aged = now - arr >= self.max_wait
            return (0, arr, rid) if aged else (1, self.requests[rid].footprint, rid)

        arrived.sort(key=order)
        admitted = []
        skipped = []
        blocked = False   # an aged request does not fit: hold the rest back
        for arr, rid in arrived:
            req = self.requests[rid]
            if not blocked and self.used + req.footprint <= self.budget:
                req.handle = self.ex.make(req)
                req.admitted = now
                self.used += req.footprint
                self.peak_used = max(self.peak_used, self.used)
                self.running.append(req)
                admitted.append(req)
                self.dirty.add(req.lane)
            else:
                skipped.append((arr, rid))
                if now - arr >= self.max_wait:
                    blocked = True
        for item in skipped:
            heapq.heappush(self.waiting, item)
        return admitted

    def _in_lane(self, lane):
        return [r for r in self.running if r.lane == lane]

    def _rebuild(self, lane):
        if lane == 0 and not hasattr(self.ex, "lane"):
            self.ex.rebuild([r.handle for r in self._in_lane(0)])
        else:
            self.ex.rebuild([r.handle for r in self._in_lane(lane)], lane=lane)
        self.rebuilds += 1
        self.dirty.discard(lane)

    def _step_lane(self, lane, ticks):
        if lane == 0 and not hasattr(self.ex, "lane"):
            self.ex.step(ticks)
        else:
            self.ex.step(ticks, lane=lane)

    def _retire(self, lane):
        """Poll the lane's running requests and retire the finished ones."""
        finished = []
        for r in self._in_lane(lane):
            iters, done, conv = self.ex.poll(r.handle)
            r.iters = iters
            if done:
                r.converged = conv
                r.finished = self.now()
                r.result = self.ex.result(r.handle)
                finished.append(r)
        for r in finished:
            self.running.remove(r)
            self.used -= r.footprint
            self.ex.release(r.handle)
            r.handle = None
            self.done.append(r)
            self.dirty.add(lane)
            if self.on_finish is not None:
                self.on_finish(r)

    def step(self):
        """One scheduling round: admit, (re)batch, run ticks, retire.  Returns
        False when nothing is resident."""
        now = self.now()
        self._admit(now)
        if not self.running:
            return False
        lanes = sorted({r.lane for r in self.running} | {l for l in self.dirty})
        for lane in lanes:
            if lane == 0 or self._busy(lane):
                continue
            # an idle asynchronous lane: retire, rebatch, enqueue its next ticks
            self._retire(lane)
            if lane in self.dirty:
                self._rebuild(lane)
            if self._in_lane(lane):
                self._step_lane(lane, self.lane_ticks)
                self.ticks_run += self.lane_ticks
        if 0 in self.dirty:
            self._rebuild(0)
        if self._in_lane(0):
            self._step_lane(0, self.ticks)
            self.ticks_run += self.ticks
            self._retire(0)
            if 0 in self.dirty:
                self._rebuild(0)
        elif self.running:
            time.sleep(0.0005)      # only asynchronous lanes are running: wait for them
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
