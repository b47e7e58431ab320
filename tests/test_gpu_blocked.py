"""GPU parity of the blocked Jacobi kernels (slices with more than 256 columns,
or columns too long for the register-resident kernel) and of the
global-memory Cholesky of the preconditioned path (n > 200): SVT, completion
and the batch engine against the FP64 oracle, on the slices themselves and on
their Cholesky factors, alone equal to in a mix.  The single-problem calls
run both blocked kernels: the wide one (their default: one workgroup per block
pair) and, with LT_WIDE=0, the one-workgroup kernel the batch engine uses."""
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


@pytest.fixture(params=["wide", "one-workgroup"])
def kernel(request, monkeypatch):
    """Which blocked kernel the single-problem calls take (read per call)."""
    if request.param == "one-workgroup":
        monkeypatch.setenv("LT_WIDE", "0")
    else:
        monkeypatch.delenv("LT_WIDE", raising=False)
    return request.param


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


# working matrices 512 x 512 (32 lanes per pair, 16 blocks of 32 columns),
# 300 x 280 (ragged: 10 blocks of 28), 600 x 260 from a 260 x 600 slice
# (transposed, 64 lanes per pair, 18 blocks of 16 with 28 padding columns),
# 2048 x 300 (64 lanes per pair and 32 rows per lane), 600 x 256 (preconditioned:
# the global-memory Cholesky and the register kernel on the 256 x 256 factor)
BLK_SHAPES = [((512, 512, 2), ("dct",)), ((300, 280, 3), ("dct",)), ((260, 600, 2), ("dct",)),
              ((2048, 300, 1), ("identity",)), ((600, 256, 2), ("dct",))]


@pytest.mark.parametrize("precondition", [False, True])
@pytest.mark.parametrize("shape,kinds", BLK_SHAPES)
def test_svt_blocked_matches_oracle(lt, kernel, shape, kinds, precondition):
    say("svt blocked", kernel, shape, kinds, lt.svt_path(shape, kinds, precondition=precondition))
    rng = np.random.default_rng(110)
    r = 12
    mats = o.mats_for(shape, list(kinds))
    A = o.lproduct(rng.standard_normal((shape[0], r) + shape[2:]),
                   rng.standard_normal((r, shape[1]) + shape[2:]), mats)
    A = A + 0.05 * rng.standard_normal(shape)
    s = o.singular_values(A, mats)
    for tau in (0.0, float(np.quantile(s, 0.7)), float(s.max()) * 1.01):
        D, rank, sweeps = lt.svt_prox(lt.to_device(A), tau, kinds, precondition=precondition)
        ref = o.svt(A, tau, mats)
        err = rel(lt.to_host(D), ref) if np.linalg.norm(ref) > 0 else float(np.abs(lt.to_host(D)).max())
        say("  tau", tau, "err", err, "sweeps", lt.to_host(sweeps).max(), "rank", lt.to_host(rank))
        assert err < 2e-5
        rk = lt.to_host(rank)
        ref_rk = o.svt_ranks(A, tau, mats)
        near = (np.abs(s - tau) < 1e-4 * max(s.max(), 1e-30)).sum(axis=1)
        assert np.all(np.abs(rk - ref_rk) <= near)


@pytest.mark.parametrize("precondition", [False, True])
def test_svt_blocked_rank_deficient(lt, kernel, precondition):
    """Zero slice, rank one, repeated columns: zero pairs never rotate (and the
    Cholesky zeroes the dependent columns) and the exact ranks come out."""
    rng = np.random.default_rng(111)
    m, n = 320, 300
    A = np.zeros((m, n, 3))
    A[:, :, 1] = np.outer(rng.standard_normal(m), rng.standard_normal(n))
    B = rng.standard_normal((m, n // 2))
    A[:, :, 2] = np.concatenate([B, B], axis=1)
    mats = o.mats_for(A.shape, ["identity"])
    tau = 1e-3 * float(o.singular_values(A, mats).max())
    D, rank, _ = lt.svt_prox(lt.to_device(A), tau, ("identity",), precondition=precondition)
    assert rel(lt.to_host(D), o.svt(A, tau, mats)) < 2e-5
    assert list(lt.to_host(rank)) == [0, 1, n // 2]


@pytest.mark.parametrize("precondition", [False, True])
def test_pga_blocked_fixed_threshold(lt, kernel, precondition):
    """512 x 512 x 3 completion with a fixed threshold (the iterate carries rank
    from the first iteration), 12 iterations against the oracle."""
    import torch
    p = wl.make_problem((512, 512, 3), 10, 0.3, seed=112)
    mats = o.mats_for(p.shape, list(p.kinds))
    mu = 0.05 * float(np.linalg.norm(p.M * p.mask))
    params = lt.pga_params(mu0=mu, max_iter=12, fixed_mu=True, precondition=precondition)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)
    Xo, _ = o.complete_pga(p.M, p.mask, mats, mu0=mu, max_iter=12, fixed_mu=mu)
    err = rel(lt.to_host(X), Xo)
    say("pga 512x512x3 fixed mu: err", err, rep)
    assert np.linalg.norm(Xo) > 0
    assert err < 1e-4


@pytest.mark.parametrize("precondition", [False, True])
def test_pga_blocked_continuation(lt, kernel, precondition):
    """300 x 280 x 2 x 2 completion with the continuation schedule, 40 iterations."""
    import torch
    p = wl.make_problem((300, 280, 2, 2), 5, 0.4, seed=113)
    s = wl.pga_schedule_params(p.M, p.mask)
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], max_iter=40,
                           precondition=precondition)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)
    Xo, _ = o.complete_pga(p.M, p.mask, o.mats_for(p.shape, list(p.kinds)), mu0=s["mu0"], nu=s["nu"],
                           mu_bar=s["mu_bar"], max_iter=40)
    err = rel(lt.to_host(X), Xo)
    say("pga 300x280x2x2: err", err, rep)
    assert np.linalg.norm(Xo) > 0
    assert err < 1e-4


def _gpu_problem(lt, p, precondition=True):
    import torch
    s = p.schedule
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], tol=0.0, max_iter=s["max_iter"],
                           precondition=precondition)
    return lt.Problem(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)


def _mix(iters, seed0):
    # two blocked problems (16 and 32 lanes per pair) among register-resident ones
    specs = [((300, 280, 2), 4, 0.4), ((40, 32, 3), 3, 0.5), ((260, 600, 2), 4, 0.35),
             ((96, 64, 4), 4, 0.4)]
    out = []
    for i, (shape, r, f) in enumerate(specs):
        p = wl.make_problem(shape, r, f, seed=seed0 + i, name="bmix%d" % i)
        p.schedule = dict(wl.pga_schedule_params(p.M, p.mask), max_iter=iters, tol=0.0)
        out.append(p)
    return out


@pytest.mark.parametrize("precondition", [False, True])
def test_batch_with_blocked_problems(lt, precondition):
    iters = 30
    ps = _mix(iters, 900)
    gps = [_gpu_problem(lt, p, precondition) for p in ps]
    b = lt.Batch(gps)
    b.step(iters)
    b.close()
    for p, gp in zip(ps, gps):
        rep, done = gp.status()
        s = p.schedule
        Xo, _ = o.complete_pga(p.M, p.mask, o.mats_for(p.shape, list(p.kinds)), mu0=s["mu0"], nu=s["nu"],
                               mu_bar=s["mu_bar"], max_iter=iters)
        err = rel(lt.to_host(gp.X), Xo)
        say(p.name, p.shape, "err", err)
        assert done == 2 and rep["iters"] == iters
        assert np.linalg.norm(Xo) > 0
        assert err < 1e-4
    # alone equals in the mix, bitwise
    for i in (0, 2):
        alone = _gpu_problem(lt, ps[i], precondition)
        b = lt.Batch([alone])
        b.step(iters)
        b.close()
        assert np.array_equal(lt.to_host(alone.X), lt.to_host(gps[i].X)), ps[i].name
