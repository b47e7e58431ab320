"""GPU tests of the C-ABI entry points beyond the single-tensor operations:
full *_L-SVD factors (Alg. 3 shapes), the multirank, the batched SVT
(lt_svt_prox_batched), the nuclear norm of the completion report (Theorem 21),
the pair dot-product precision option, and slices whose singular values
cluster at the threshold -- each against the FP64 oracle."""
import numpy as np
import pytest

import oracle as o
import parity
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


# ------------------------------------------------------------ full factors --

@pytest.mark.parametrize("shape,kinds", [((12, 9, 5), ("dct",)), ((9, 14, 3, 2), ("dct", "dct")),
                                         ((8, 8, 4), ("dct",)), ((70, 20, 3), ("identity",)),
                                         ((10, 8, 3), ("dct",))])
@pytest.mark.parametrize("transform_domain", [False, True])
def test_lsvd_full_factors(lt, shape, kinds, transform_domain):
    """economy = 0: U is I1 x I1, S is I1 x I2, V is I2 x I2 per slice (Alg. 3);
    U *_L S *_L V^T = A, L(U)^p and L(V)^p orthogonal, L(S)^p diagonal with the
    oracle's singular values in descending order.  (10, 8, 3): rank 2, so most
    columns of both factors are basis completions."""
    say("lsvd full", shape, kinds, "transform domain", transform_domain)
    rng = np.random.default_rng(sum(shape) + 7)
    mats = o.mats_for(shape, list(kinds))
    if shape == (10, 8, 3):
        A = o.lproduct(rng.standard_normal((10, 2, 3)), rng.standard_normal((2, 8, 3)), mats)
    else:
        A = rng.standard_normal(shape)
    U, S, V, sig = lt.lsvd(lt.to_device(A), kinds, transform_domain=transform_domain, economy=False)
    I1, I2 = shape[:2]
    assert tuple(U.shape) == (I1, I1) + shape[2:] and tuple(S.shape) == (I1, I2) + shape[2:]
    assert tuple(V.shape) == (I2, I2) + shape[2:]
    U, S, V = (lt.to_host(x).astype(np.float64) for x in (U, S, V))
    if transform_domain:
        Uh, Sh, Vh = o.slices(U), o.slices(S), o.slices(V)
        U, S, V = (o.inverse_transform(x, mats) for x in (U, S, V))
    else:
        Uh, Sh, Vh = (o.slices(o.transform(x, mats)) for x in (U, S, V))
    R = o.lproduct(o.lproduct(U, S, mats), o.ttranspose(V, mats), mats)
    assert rel(R, A) < 2e-5
    sref = o.singular_values(A, mats)
    smax = sref.max()
    n = min(I1, I2)
    for p in range(Sh.shape[0]):
        d = np.diag(Sh[p])
        assert np.abs(Sh[p] - _diag_embed(d, I1, I2)).max() < 1e-6 * smax
        assert np.abs(d[:n] - sref[p]).max() < 2e-5 * smax
        assert np.all(np.diff(d[:n]) <= 1e-6 * smax)
    for Qh, k in ((Uh, I1), (Vh, I2)):
        for q in Qh:
            assert q.shape == (k, k)
            assert np.abs(q.T @ q - np.eye(k)).max() < 1e-4


def _diag_embed(d, I1, I2):
    D = np.zeros((I1, I2))
    k = min(I1, I2)
    D[np.arange(k), np.arange(k)] = d[:k]
    return D


# ------------------------------------------------------------- batched SVT --

BATCH = [((32, 48, 3), ("dct",), 0.5), ((64, 40, 3, 2), ("dct", "dct"), 0.3),
         ((144, 176, 3), ("dct",), 0.4),              # preconditioned, LDS Cholesky
         ((256, 256, 2), ("identity",), 0.6),         # register kernel, n = 256
         ((300, 220, 2), ("dct",), 0.5),              # preconditioned, global Cholesky + blocked Jacobi
         ((20, 20, 16), ("dct",), 0.0),               # tau = 0: the identity
         ((1, 7, 3), ("dct",), 0.2)]                  # n = 1


def test_svt_prox_batched_matches_oracle(lt):
    rng = np.random.default_rng(400)
    As, taus, kinds, refs, rranks = [], [], [], [], []
    for shape, k, q in BATCH:
        A = rng.standard_normal(shape)
        mats = o.mats_for(shape, list(k))
        s = o.singular_values(A, mats)
        tau = float(np.quantile(s, q)) if q > 0 else 0.0
        As.append(A)
        taus.append(tau)
        kinds.append(k)
        refs.append(o.svt(A, tau, mats))
        rranks.append(o.svt_ranks(A, tau, mats))
    Ds, ranks = lt.svt_prox_batched([lt.to_device(A) for A in As], taus, kinds)
    for (shape, k, q), D, ref, r, rr in zip(BATCH, Ds, refs, ranks, rranks):
        say("batched svt", shape, k, "path", lt.svt_path(shape, k))
        parity.check(lt.to_host(D), ref, 2e-5, label=str(shape))
        assert np.array_equal(lt.to_host(r), np.asarray(rr))
    # each tensor's result equals its own lt_svt_prox call up to rounding
    for A, tau, k, D in zip(As, taus, kinds, Ds):
        D1, _, _ = lt.svt_prox(lt.to_device(A), tau, k)
        assert rel(lt.to_host(D), lt.to_host(D1).astype(np.float64)) < 2e-5


def test_svt_prox_batched_in_place_and_errors(lt):
    rng = np.random.default_rng(401)
    A = rng.standard_normal((24, 18, 5))
    mats = o.mats_for(A.shape, ["dct"])
    tau = float(np.median(o.singular_values(A, mats)))
    Ad = lt.to_device(A)
    Ds, _ = lt.svt_prox_batched([Ad], [tau], outs=[Ad])     # D aliases A
    assert Ds[0].data_ptr() == Ad.data_ptr()
    assert rel(lt.to_host(Ad), o.svt(A, tau, mats)) < 2e-5
    with pytest.raises(lt.LtError) as e:
        lt.svt_prox_batched([lt.to_device(A)], [-1.0])
    assert e.value.status == lt.ERR_ARG
    with pytest.raises((lt.LtError, ValueError)):           # Fourier modes: not in the batch engine
        lt.svt_prox_batched([lt.to_device(A)], [tau], [("dft",)])


# ---------------------------------------------------- nuclear norm, report --

@pytest.mark.parametrize("shape,kinds", [((24, 20, 3, 2), ("dct", "dct")), ((16, 12, 4), ("dft",)),
                                         ((16, 12, 5), ("dft",)), ((30, 26, 3), ("identity",))])
def test_pga_report_nuclear_norm(lt, shape, kinds):
    """rep.nuclear_norm = ||X||_* of the returned iterate (Theorem 21: the
    transform-domain singular values over alpha; alpha = P under the DFT)."""
    import torch
    p = wl.make_problem(shape, 2, 0.6, seed=11, kinds=kinds)
    sch = wl.pga_schedule_params(p.M, p.mask)
    params = lt.pga_params(mu0=sch["mu0"], nu=sch["nu"], mu_bar=sch["mu_bar"], max_iter=40)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, kinds)
    Xg = lt.to_host(X).astype(np.float64)
    nn = o.nuclear_norm(Xg, o.mats_for(shape, list(kinds)))
    say("nuclear norm", shape, kinds, rep["nuclear_norm"], nn)
    assert nn > 0
    assert abs(rep["nuclear_norm"] - nn) <= 2e-5 * nn


def test_pga_report_slowest_sweeps(lt):
    """rep.slowest_sweeps sums, over the iterations, the largest sweep count
    among the slices: at least the mean, at most the sweep limit, and exactly
    iterations x limit when every slice runs to the limit."""
    import torch
    p = wl.make_problem((48, 40, 3, 2), 3, 0.5, seed=13)
    sch = wl.pga_schedule_params(p.M, p.mask)
    M, mask = lt.to_device(p.M), lt.to_device(p.mask, torch.uint8)
    _, rep, _ = lt.complete_pga(M, mask, lt.pga_params(mu0=sch["mu0"], nu=sch["nu"], mu_bar=sch["mu_bar"],
                                                         max_iter=12))
    P = 6
    say("slowest sweeps", rep["slowest_sweeps"], "total", rep["total_sweeps"])
    assert rep["total_sweeps"] / P <= rep["slowest_sweeps"] <= 12 * 40
    assert rep["slowest_sweeps"] >= 12
    _, rep, _ = lt.complete_pga(M, mask, lt.pga_params(mu0=sch["mu0"], nu=sch["nu"], mu_bar=sch["mu_bar"],
                                                         max_iter=5, jacobi_tol=1e-300, max_sweeps=3))
    assert rep["slowest_sweeps"] == 5 * 3 and rep["total_sweeps"] == 5 * 3 * P


def test_batch_status_nuclear_norm(lt):
    import torch
    p = wl.make_problem((40, 36, 3, 2), 3, 0.5, seed=12)
    sch = wl.pga_schedule_params(p.M, p.mask)
    params = lt.pga_params(mu0=sch["mu0"], nu=sch["nu"], mu_bar=sch["mu_bar"], max_iter=30)
    gp = lt.Problem(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params)
    rep0, _ = gp.status()
    assert np.isnan(rep0["nuclear_norm"])         # before any iteration
    b = lt.Batch([gp], use_graph=False)
    b.step(30)
    rep, done = gp.status()
    b.close()
    nn = o.nuclear_norm(lt.to_host(gp.X).astype(np.float64), o.mats_for(p.shape, ["dct", "dct"]))
    assert done == 2 and abs(rep["nuclear_norm"] - nn) <= 2e-5 * nn


# ------------------------------------------------- pair dot-product precision --

@pytest.mark.parametrize("fp32_dots", [False, True])
@pytest.mark.parametrize("shape,precondition", [((144, 176, 6), True), ((144, 176, 6), False),
                                                ((256, 256, 3), True), ((520, 300, 2), False)])
def test_svt_dot_precision(lt, fp32_dots, shape, precondition):
    """Both pair dot-product precisions on the register, preconditioned and
    blocked kernels match the oracle SVT slice by slice."""
    rng = np.random.default_rng(402)
    A = rng.standard_normal(shape)
    mats = o.mats_for(shape, ["dct"])
    tau = float(np.median(o.singular_values(A, mats)))
    D, rank, sweeps = lt.svt_prox(lt.to_device(A), tau, precondition=precondition, fp32_dots=fp32_dots)
    say("svt dots", "fp32" if fp32_dots else "fp64", shape, lt.svt_path(shape, precondition=precondition),
        "mean sweeps", float(lt.to_host(sweeps).mean()))
    parity.check(lt.to_host(D), o.svt(A, tau, mats), 2e-5, label="dots")


# ---------------------------------------------- spectra clustered at tau --

@pytest.mark.parametrize("precondition", [True, False])
@pytest.mark.parametrize("spread", [1e-2, 1e-4])
def test_svt_clustered_at_threshold(lt, precondition, spread):
    """Slices whose singular values crowd around tau (half just above, half
    just below, relative gaps ~spread/n): the Jacobi's early stop must still
    separate kept from dropped values.  Identity transform, so each slice is
    given its singular values exactly; compared slice by slice."""
    rng = np.random.default_rng(403)
    I1, I2, P = 96, 80, 6
    n = min(I1, I2)
    tau = 1.0
    A = np.empty((I1, I2, P))
    for p in range(P):
        Uq, _ = np.linalg.qr(rng.standard_normal((I1, n)))
        Vq, _ = np.linalg.qr(rng.standard_normal((I2, n)))
        s = tau * (1.0 + spread * rng.uniform(-1.0, 1.0, n))
        s[: n // 8] = tau * rng.uniform(2.0, 5.0, n // 8)      # a few clear ones above
        A[:, :, p] = (Uq * s) @ Vq.T
    mats = o.mats_for(A.shape, ["identity"])
    D, rank, sweeps = lt.svt_prox(lt.to_device(A), tau, ("identity",), precondition=precondition)
    ref = o.svt(A, tau, mats)
    say("clustered", spread, "precondition", precondition, "sweeps", lt.to_host(sweeps))
    parity.check(lt.to_host(D), ref, 1e-4, slice_factor=3.0, label="clustered %g" % spread)
    # kept counts: exact away from the cluster's rounding band
    sv = o.singular_values(A, mats)
    band = np.abs(sv - tau) <= 1e-5 * tau
    lo = (sv > tau * (1 + 1e-5)).sum(axis=1)
    hi = lo + band.sum(axis=1)
    r = lt.to_host(rank)
    assert np.all((r >= lo) & (r <= hi))
