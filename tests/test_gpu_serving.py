"""GPU serving: a small stream of requests with staggered arrivals runs through
the continuous-batching server; every result equals the request run alone
(bitwise) and matches the FP64 oracle."""
import numpy as np
import pytest

import oracle as o
from paper_2202_02870_amd import serving, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_02870_amd import lt as _lt
    return _lt


class TickClock:
    """Server clock advanced by the executor: one unit per tick, so arrivals
    land at deterministic tick boundaries."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class TickedGpu(serving.GpuExecutor):
    def __init__(self, clock):
        super().__init__(use_graph=True)
        self.clock = clock

    def step(self, ticks, lane=0):
        super().step(ticks, lane)
        self.clock.t += ticks


def _stream(n=6, iters=25):
    shapes = [(32, 48, 3), (64, 40, 3, 2), (96, 64, 8), (33, 17, 5), (20, 20, 16), (128, 96, 3)]
    reqs = []
    for i in range(n):
        p = wl.make_problem(shapes[i % len(shapes)], 3, 0.4, seed=800 + i)
        prm = dict(wl.pga_schedule_params(p.M, p.mask), max_iter=iters, tol=0.0)
        reqs.append(serving.Request(rid=i, arrival=4.0 * i, M=p.M.astype(np.float32), mask=p.mask,
                                    params=prm, kinds=p.kinds))
    return reqs


def test_served_results_equal_alone(lt):
    clock = TickClock()
    srv = serving.CompletionServer(TickedGpu(clock), hbm_budget=1 << 34, clock=clock)
    reqs = _stream()
    for r in reqs:
        assert srv.submit(r)
    st = srv.run()
    print("serving stats", st, flush=True)
    assert st["completed"] == len(reqs)
    done = {r.rid: r for r in srv.done}
    # overlap: later requests were admitted before earlier ones finished
    assert any(done[i + 1].admitted < done[i].finished for i in range(len(reqs) - 1))
    ex = serving.GpuExecutor(use_graph=False)
    for r in reqs:
        h = ex.make(r)
        ex.rebuild([h])
        ex.step(r.params["max_iter"])
        alone = ex.result(h) if ex.poll(h)[1] else None
        assert alone is not None and np.array_equal(alone, done[r.rid].result), r.rid
        X, _ = o.complete_pga(r.M.astype(np.float64), r.mask, o.mats_for(r.M.shape, list(r.kinds)),
                              mu0=r.params["mu0"], nu=r.params["nu"], mu_bar=r.params["mu_bar"],
                              max_iter=r.params["max_iter"])
        if np.linalg.norm(X) > 0:
            assert np.linalg.norm(done[r.rid].result - X) / np.linalg.norm(X) < 1e-4
    ex.rebuild([])


def test_budget_limits_residency(lt):
    clock = TickClock()
    ex = TickedGpu(clock)
    reqs = _stream(4, iters=10)
    for r in reqs:
        r.arrival = 0.0
    one = max(ex.footprint(r) for r in reqs)
    srv = serving.CompletionServer(ex, hbm_budget=2 * one, clock=clock)
    for r in reqs:
        srv.submit(r)
    st = srv.run()
    assert st["completed"] == 4 and srv.peak_used <= 2 * one


def test_blocked_requests_run_in_their_own_lane(lt):
    """A request whose slices take the blocked Jacobi kernel runs in lane 1 (its
    own batch and stream) beside small requests in lane 0; every result equals
    the request run alone (bitwise) and matches the oracle."""
    specs = [((300, 280, 2), 4, 0.4, 25), ((32, 48, 3), 3, 0.5, 30), ((64, 40, 3, 2), 3, 0.4, 20),
             ((96, 64, 8), 3, 0.4, 25)]
    reqs = []
    for i, (shape, r, f, iters) in enumerate(specs):
        p = wl.make_problem(shape, r, f, seed=820 + i)
        prm = dict(wl.pga_schedule_params(p.M, p.mask), max_iter=iters, tol=0.0)
        reqs.append(serving.Request(rid=i, arrival=0.0, M=p.M.astype(np.float32), mask=p.mask,
                                    params=prm, kinds=p.kinds))
    ex = serving.GpuExecutor(use_graph=True)
    srv = serving.CompletionServer(ex, hbm_budget=1 << 34, ticks_per_round=2)
    for r in reqs:
        assert srv.submit(r)
    assert [r.lane for r in reqs] == [1, 0, 0, 0]
    st = srv.run()
    print("laned serving stats", st, flush=True)
    assert st["completed"] == len(reqs)
    done = {r.rid: r for r in srv.done}
    alone_ex = serving.GpuExecutor(use_graph=False, lanes=False)
    for r in reqs:
        assert done[r.rid].iters == r.params["max_iter"]
        h = alone_ex.make(r)
        alone_ex.rebuild([h])
        alone_ex.step(r.params["max_iter"])
        assert alone_ex.poll(h)[1]
        assert np.array_equal(alone_ex.result(h), done[r.rid].result), r.rid
        X, _ = o.complete_pga(r.M.astype(np.float64), r.mask, o.mats_for(r.M.shape, list(r.kinds)),
                              mu0=r.params["mu0"], nu=r.params["nu"], mu_bar=r.params["mu_bar"],
                              max_iter=r.params["max_iter"])
        if np.linalg.norm(X) > 0:
            assert np.linalg.norm(done[r.rid].result - X) / np.linalg.norm(X) < 1e-4
    alone_ex.rebuild([])
