"""GPU tests of the batched completion engine: every problem of a mixed batch
against the FP64 oracle, the same result alone and in a mix (bitwise), graph
replay equal to eager launches, a problem joining a running batch, and the
device-side stopping rule per problem."""
import numpy as np
import pytest

import oracle as o
from paper_2202_02870_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_02870_amd import lt as _lt
    return _lt


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


# shapes: transposed and not, odd n, order 3 and 4, slices packed several per workgroup
MIX = [((32, 48, 3), 3, 0.5), ((64, 40, 3, 2), 4, 0.4), ((96, 64, 8), 4, 0.35),
       ((33, 17, 5), 2, 0.6), ((128, 128, 3, 2), 6, 0.3), ((20, 20, 16), 2, 0.5)]


def _problems(iters, tol=0.0, seed0=300):
    out = []
    for i, (shape, r, f) in enumerate(MIX):
        p = wl.make_problem(shape, r, f, seed=seed0 + i, name="mix%d" % i)
        p.schedule = dict(wl.pga_schedule_params(p.M, p.mask), max_iter=iters, tol=tol)
        out.append(p)
    return out


def _gpu_problem(lt, p, precision="f32", check_every=1, precondition=True):
    import torch
    s = p.schedule
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=s["tol"],
                           max_iter=s["max_iter"], check_every=check_every, precision=precision,
                           precondition=precondition)
    return lt.Problem(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)


def _run(lt, gps, ticks, use_graph=True):
    b = lt.Batch(gps, use_graph=use_graph)
    b.step(ticks)
    out = [gp.status() for gp in gps]
    b.close()
    return out


@pytest.mark.parametrize("precondition", [True, False])
def test_batch_mix_matches_oracle(lt, precondition):
    iters = 60
    ps = _problems(iters)
    gps = [_gpu_problem(lt, p, precondition=precondition) for p in ps]
    st = _run(lt, gps, iters)
    for p, gp, (rep, done) in zip(ps, gps, st):
        s = p.schedule
        Xo, _ = o.complete_pga(p.M, p.mask, o.mats_for(p.shape, list(p.kinds)), mu0=s["mu0"], nu=s["nu"],
                               mu_bar=s["mu_bar"], max_iter=iters)
        err = rel(lt.to_host(gp.X), Xo)
        say(p.name, p.shape, "err", err, rep)
        assert done == 2 and rep["iters"] == iters
        assert np.linalg.norm(Xo) > 0
        assert err < 1e-4


def test_batch_alone_equals_mix_bitwise(lt):
    iters = 30
    ps = _problems(iters, seed0=400)
    mix = [_gpu_problem(lt, p) for p in ps]
    _run(lt, mix, iters)
    for i in (0, 3, 5):
        alone = _gpu_problem(lt, ps[i])
        _run(lt, [alone], iters)
        assert np.array_equal(lt.to_host(alone.X), lt.to_host(mix[i].X)), ps[i].name


def test_batch_graph_equals_eager(lt):
    iters = 25
    ps = _problems(iters, seed0=500)
    g = [_gpu_problem(lt, p) for p in ps]
    e = [_gpu_problem(lt, p) for p in ps]
    _run(lt, g, iters, use_graph=True)
    _run(lt, e, iters, use_graph=False)
    for a, b in zip(g, e):
        assert np.array_equal(lt.to_host(a.X), lt.to_host(b.X))


def test_problem_joins_running_batch(lt):
    """Continuous batching: B and C run 12 ticks, then A joins; every result
    equals the one obtained alone."""
    iters = 30
    ps = _problems(iters, seed0=600)
    A, B, C = ps[0], ps[2], ps[4]
    gA, gB, gC = (_gpu_problem(lt, p) for p in (A, B, C))
    b1 = lt.Batch([gB, gC])
    b1.step(12)
    b1.close()
    b2 = lt.Batch([gA, gB, gC])
    b2.step(iters)        # B and C finish after 18 more ticks and then sit idle
    b2.close()
    (rA, dA), (rB, dB), (rC, dC) = gA.status(), gB.status(), gC.status()
    assert (dA, dB, dC) == (2, 2, 2) and rA["iters"] == rB["iters"] == rC["iters"] == iters
    for p, gp in ((A, gA), (B, gB), (C, gC)):
        ref = _gpu_problem(lt, p)
        _run(lt, [ref], iters)
        assert np.array_equal(lt.to_host(ref.X), lt.to_host(gp.X)), p.name


def test_batch_stopping_rule_per_problem(lt):
    iters = 400
    ps = _problems(iters, tol=1e-4, seed0=700)[:4]
    gps = [_gpu_problem(lt, p) for p in ps]
    st = _run(lt, gps, iters)
    for p, gp, (rep, done) in zip(ps, gps, st):
        s = p.schedule
        Xo, info = o.complete_pga(p.M, p.mask, o.mats_for(p.shape, list(p.kinds)), mu0=s["mu0"], nu=s["nu"],
                                  mu_bar=s["mu_bar"], tol=1e-4, max_iter=iters)
        say(p.name, rep, info)
        assert done == 1 and info["converged"]
        assert abs(rep["iters"] - info["iters"]) <= 1
        assert rel(lt.to_host(gp.X), Xo) < 1e-3


def test_batch_matches_single_problem_path(lt):
    p = wl.config1(trailing=(3, 4))
    p.schedule["max_iter"] = 80
    gp = _gpu_problem(lt, p)
    _run(lt, [gp], 80)
    import torch
    s = p.schedule
    # the same algorithm (both preconditioned and warm-started with the default
    # cold-start period): equal to FP32 rounding
    assert lt.pga_warm(p.shape, p.kinds)
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], max_iter=80)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)
    assert rel(lt.to_host(gp.X), lt.to_host(X).astype(np.float64)) < 1e-6
    # every Jacobi from a cold start: the same result to the Jacobi tolerance
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], max_iter=80, warm_restart=-1)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)
    assert rel(lt.to_host(gp.X), lt.to_host(X).astype(np.float64)) < 5e-5
    # the Jacobi on the slices themselves: the same result to the Jacobi tolerance
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], max_iter=80, precondition=False)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)
    assert rel(lt.to_host(gp.X), lt.to_host(X).astype(np.float64)) < 5e-5
