"""Scheduler tests of the serving loop on the CPU: a fake executor advances each
request by one oracle PGA iteration per tick, so admission, backfill, late
arrivals, budget accounting and per-request results can be checked without a
GPU."""
import numpy as np

import oracle as o
from paper_2202_02870_amd import serving, workloads as wl


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """One oracle PGA iteration per tick for every request of the current batch."""

    def __init__(self, clock, tick_seconds=1.0, bytes_per_entry=16):
        self.clock = clock
        self.dt = tick_seconds
        self.bpe = bytes_per_entry
        self.batch = []
        self.sizes = []

    def footprint(self, req):
        return self.bpe * req.M.size

    def make(self, req):
        p = req.params
        betas, mus = o.pga_schedule(p["max_iter"], p["mu0"], p.get("nu", 0.9), p["mu_bar"])
        return dict(req=req, X=np.zeros(req.M.shape), Xp=np.zeros(req.M.shape), k=0, done=0,
                    betas=betas, mus=mus, mats=o.mats_for(req.M.shape, list(req.kinds)))

    def rebuild(self, handles):
        self.batch = list(handles)
        self.sizes.append(len(handles))

    def step(self, ticks):
        for _ in range(ticks):
            for h in self.batch:
                if h["done"]:
                    continue
                k = h["k"]
                Xn, Y = o.pga_step(h["X"], h["Xp"], h["req"].M, h["req"].mask, h["betas"][k], h["mus"][k], h["mats"])
                h["Xp"], h["X"] = h["X"], Xn
                h["k"] = k + 1
                if h["k"] >= len(h["betas"]):
                    h["done"] = 2
            self.clock.t += self.dt

    def poll(self, h):
        return h["k"], h["done"], False

    def result(self, h):
        return h["X"]

    def release(self, h):
        pass


def _req(rid, arrival, shape, iters, seed):
    p = wl.make_problem(shape, 2, 0.5, seed=seed)
    prm = dict(wl.pga_schedule_params(p.M, p.mask), max_iter=iters, tol=0.0)
    return serving.Request(rid=rid, arrival=arrival, M=p.M, mask=p.mask, params=prm, kinds=p.kinds)


def test_continuous_batching_admits_late_arrivals():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = serving.CompletionServer(ex, hbm_budget=10 ** 9, clock=clock)
    reqs = [_req(0, 0.0, (8, 6, 3), 10, 1), _req(1, 3.0, (6, 8, 4), 10, 2), _req(2, 4.5, (7, 7, 2, 2), 6, 3)]
    for r in reqs:
        assert srv.submit(r)
    srv.run()
    done = {r.rid: r for r in srv.done}
    assert sorted(done) == [0, 1, 2]
    # request 1 joined while request 0 was running, and 2 while 1 was
    assert done[1].admitted < done[0].finished
    assert done[2].admitted < done[1].finished
    assert max(ex.sizes) == 3
    # every result equals the request's own oracle run
    for r in reqs:
        X, _ = o.complete_pga(r.M, r.mask, o.mats_for(r.M.shape, list(r.kinds)), mu0=r.params["mu0"],
                              nu=r.params["nu"], mu_bar=r.params["mu_bar"], max_iter=r.params["max_iter"])
        assert np.array_equal(done[r.rid].result, X)
    st = srv.stats()
    assert st["completed"] == 3 and st["p99"] >= st["p50"] > 0


def test_admission_respects_budget_and_backfills():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    big, small = (16, 16, 4), (4, 4, 2)
    budget = 16 * (16 * 16 * 4) + 16 * (4 * 4 * 2)        # one big + one small fit, not two big
    srv = serving.CompletionServer(ex, hbm_budget=budget, clock=clock)
    reqs = [_req(0, 0.0, big, 8, 4), _req(1, 0.0, big, 8, 5), _req(2, 0.0, small, 3, 6)]
    for r in reqs:
        srv.submit(r)
    srv.run()
    done = {r.rid: r for r in srv.done}
    assert srv.peak_used <= budget
    assert done[2].admitted == 0.0                 # backfilled next to request 0
    assert done[1].admitted >= done[0].finished    # waited for memory
    assert len(srv.done) == 3


def test_admission_orders_by_footprint_and_ages():
    """Arrived requests go in smallest footprint first; one that waited
    max_wait seconds goes first and holds smaller ones back until it fits."""
    clock = FakeClock()
    ex = FakeExecutor(clock)
    big, mid, small = (16, 16, 4), (8, 8, 4), (4, 4, 2)
    budget = 16 * (16 * 16 * 4) + 16 * (8 * 8 * 4)        # the big one and the mid one fit together
    srv = serving.CompletionServer(ex, hbm_budget=budget, clock=clock, max_wait=1e9)
    reqs = [_req(0, 0.0, big, 6, 10), _req(1, 0.0, mid, 6, 11), _req(2, 0.0, small, 6, 12)]
    for r in reqs:
        srv.submit(r)
    srv.step()
    # smallest first: small and mid are admitted, big does not fit beside them
    assert [r.rid for r in srv.running] == [2, 1]
    srv.run()
    assert len(srv.done) == 3 and srv.peak_used <= budget
    # aging: the big request has waited, so it goes first and the later small
    # ones wait for memory instead of overtaking it again
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = serving.CompletionServer(ex, hbm_budget=budget, clock=clock, max_wait=2.0)
    first = [_req(0, 0.0, mid, 8, 13), _req(1, 0.0, mid, 8, 14)]
    later = [_req(2, 0.0, big, 6, 15), _req(3, 3.0, small, 4, 16), _req(4, 3.0, small, 4, 17)]
    for r in first + later:
        srv.submit(r)
    srv.run()
    done = {r.rid: r for r in srv.done}
    assert len(done) == 5 and srv.peak_used <= budget
    assert done[2].admitted <= done[3].admitted and done[2].admitted <= done[4].admitted


def test_oversized_request_is_rejected():
    clock = FakeClock()
    srv = serving.CompletionServer(FakeExecutor(clock), hbm_budget=1000, clock=clock)
    assert not srv.submit(_req(0, 0.0, (16, 16, 4), 3, 7))
    assert srv.stats()["rejected"] == 1 and srv.idle()


def test_poisson_arrivals():
    t = serving.poisson_arrivals(2000, rate=5.0, seed=0)
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.2) < 0.02


class LanedFakeExecutor(FakeExecutor):
    """Two lanes: requests with more than 100 entries per slice in lane 1.
    Lane 1's enqueued ticks stay 'in flight' for `lag` polls of busy()."""

    def __init__(self, clock, lag=2):
        super().__init__(clock)
        self.batches = {0: [], 1: []}
        self.lane_sizes = {0: [], 1: []}
        self.inflight = {0: 0, 1: 0}
        self.lag = lag
        self.steps = {0: 0, 1: 0}

    def lane(self, req):
        return 1 if req.M.shape[0] * req.M.shape[1] > 100 else 0

    def rebuild(self, handles, lane=0):
        assert not self.busy(lane)
        self.batches[lane] = list(handles)
        self.lane_sizes[lane].append(len(handles))

    def step(self, ticks, lane=0):
        self.batch = self.batches[lane]
        super().step(ticks)
        self.steps[lane] += ticks
        if lane:
            self.inflight[lane] = self.lag

    def busy(self, lane):
        if self.inflight[lane] > 0:
            self.inflight[lane] -= 1
            return True
        return False


def test_lanes_keep_long_requests_apart():
    clock = FakeClock()
    ex = LanedFakeExecutor(clock)
    srv = serving.CompletionServer(ex, hbm_budget=10 ** 9, clock=clock)
    reqs = [_req(0, 0.0, (12, 12, 2), 6, 11), _req(1, 0.0, (4, 5, 3), 9, 12), _req(2, 1.0, (5, 4, 2), 7, 13),
            _req(3, 2.0, (11, 13, 2), 5, 14)]
    for r in reqs:
        assert srv.submit(r)
    assert [r.lane for r in reqs] == [1, 0, 0, 1]
    srv.run()
    done = {r.rid: r for r in srv.done}
    assert sorted(done) == [0, 1, 2, 3]
    # batches of each lane hold only that lane's requests; both lanes ran
    assert max(ex.lane_sizes[1]) == 2 and max(ex.lane_sizes[0]) == 2
    assert ex.steps[0] > 0 and ex.steps[1] > 0
    for r in reqs:
        X, _ = o.complete_pga(r.M, r.mask, o.mats_for(r.M.shape, list(r.kinds)), mu0=r.params["mu0"],
                              nu=r.params["nu"], mu_bar=r.params["mu_bar"], max_iter=r.params["max_iter"])
        assert np.array_equal(done[r.rid].result, X), r.rid
        assert done[r.rid].iters == r.params["max_iter"]


def test_request_no_kernel_takes_is_rejected():
    class Picky(FakeExecutor):
        def lane(self, req):
            raise RuntimeError("no Jacobi kernel takes this shape")

    clock = FakeClock()
    srv = serving.CompletionServer(Picky(clock), hbm_budget=10 ** 9, clock=clock)
    assert not srv.submit(_req(0, 0.0, (6, 5, 2), 3, 31))
    assert srv.stats()["rejected"] == 1 and srv.idle()
