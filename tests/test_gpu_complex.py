"""GPU tests of the complex Hermitian Jacobi that thresholds Fourier slices
(one per conjugate pair, Section 2's t-SVD under the DFT), on the complex
slices and on their complex Cholesky-QR factors: against the FP64 oracle's
complex SVT slice by slice, against the real-embedding path it replaces, and
inside the completion.  The cases reach every instantiated (lanes per pair,
rows per lane) and both orientations of the slice."""
import os

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


def _low_rank_plus_noise(shape, kinds, seed):
    rng = np.random.default_rng(seed)
    mats = o.mats_for(shape, list(kinds))
    r = max(1, min(shape[0], shape[1]) // 4)
    A = o.lproduct(rng.standard_normal((shape[0], r) + shape[2:]),
                   rng.standard_normal((r, shape[1]) + shape[2:]), mats).real
    return A + 0.05 * rng.standard_normal(shape), mats


# (shape, kinds): G and rows per lane of the complex working matrix without
# preconditioning (2 max(I1, I2) interleaved rows by min(I1, I2) columns); on
# the factor (2 min(I1, I2) rows) they reach G 8 with 8, 16, 32, 48 rows and
# G 16 with 16
CX_CASES = [
    ((8, 6, 5), ("dft",)),              # G 8, R 8; P = 5: one self-conjugate slice
    ((5, 9, 6), ("dft",)),              # transposed; P = 6: two self-conjugate slices
    ((60, 51, 4), ("dft",)),            # G 8, R 16, odd n
    ((100, 80, 4), ("dft",)),           # G 16, R 16
    ((96, 190, 2), ("dft",)),           # G 16, R 24, transposed
    ((256, 64, 3), ("dft",)),           # G 16, R 32
    ((60, 300, 2), ("dft",)),           # G 16, R 40, transposed
    ((380, 12, 3), ("dft",)),           # G 16, R 48
    ((128, 100, 2), ("dft",)),          # G 8, R 32
    ((130, 101, 3), ("dft",)),          # G 8, R 36
    ((120, 150, 2), ("dft",)),          # G 8, R 40, transposed
    ((10, 7, 4, 3), ("dft", "dct")),    # mixed transforms
    ((190, 192, 2), ("dft",)),          # G 8, R 48, one exchange buffer, transposed
]


@pytest.mark.parametrize("precondition", [False, True])
@pytest.mark.parametrize("shape,kinds", CX_CASES)
def test_svt_complex_matches_oracle(lt, shape, kinds, precondition):
    assert lt.svt_path(shape, kinds, precondition=precondition) == ("precond+complex" if precondition else "complex")
    A, mats = _low_rank_plus_noise(shape, kinds, sum(shape))
    s = o.singular_values(A, mats)
    for tau in (0.0, float(np.quantile(s, 0.5)), float(s.max()) * 1.01):
        D, rank, sweeps = lt.svt_prox(lt.to_device(A), tau, kinds, precondition=precondition)
        ref = o.svt(A, tau, mats)
        rk, ref_rk = lt.to_host(rank), np.asarray(o.svt_ranks(A, tau, mats))
        say("complex svt", shape, kinds, "tau", tau, "ranks", rk[:6], "sweeps", lt.to_host(sweeps)[:6])
        if np.linalg.norm(ref) > 0:
            parity.check(lt.to_host(D), ref, 2e-5, label="%s tau %.3g" % (shape, tau))
        else:
            assert float(np.abs(lt.to_host(D)).max()) == 0.0
        near = (np.abs(s - tau) < 1e-4 * max(s.max(), 1e-30)).sum(axis=1)
        assert np.all(np.abs(rk - ref_rk) <= near)


@pytest.mark.parametrize("shape,kinds", [((7, 1, 4), ("dft",)), ((1, 9, 3), ("dft",)), ((10, 8, 1), ("dft",)),
                                         ((6, 5, 2, 1), ("dft", "dft"))])
def test_svt_complex_degenerate_shapes(lt, shape, kinds):
    """One-column slices (n = 1: nothing to precondition), a single row, and
    trailing modes of size 1 (every slice its own conjugate) against the
    oracle."""
    rng = np.random.default_rng(sum(shape) + 3)
    mats = o.mats_for(shape, list(kinds))
    A = rng.standard_normal(shape)
    s = o.singular_values(A, mats)
    assert "complex" in lt.svt_path(shape, kinds)
    for tau in (0.0, float(np.median(s))):
        D, rank, _ = lt.svt_prox(lt.to_device(A), tau, kinds)
        ref = o.svt(A, tau, mats)
        say("degenerate complex", shape, "tau", tau, "ranks", lt.to_host(rank))
        if np.linalg.norm(ref) > 0:
            parity.check(lt.to_host(D), ref, 2e-5, label="%s tau %.3g" % (shape, tau))
        near = (np.abs(s - tau) < 1e-4 * max(s.max(), 1e-30)).sum(axis=1)
        assert np.all(np.abs(lt.to_host(rank) - np.asarray(o.svt_ranks(A, tau, mats))) <= near)


def test_noalloc_fourier_equals_workspace_entry_point(lt):
    """The entry point that allocates nothing runs the same complex kernels on
    its static scratch: the same bits as lt_svt_prox, twice in a row (the
    second call smaller)."""
    import torch
    rng = np.random.default_rng(510)
    for shape, kinds in (((144, 176, 3, 6), ("dft", "dft")), ((40, 30, 5), ("dft",))):
        assert lt.workspace_bytes(shape, kinds, "svt") <= lt.NOALLOC_SCRATCH_BYTES
        A = rng.standard_normal(shape)
        tau = float(np.median(o.singular_values(A, o.mats_for(shape, list(kinds)))))
        Ad = lt.to_device(A)
        D1, r1, _ = lt.svt_prox(Ad, tau, kinds)
        D2 = lt.fortran_empty(shape)
        P = int(np.prod(shape[2:]))
        r2 = torch.empty(P, dtype=torch.int32, device="cuda")
        assert lt.svt_prox_noalloc(Ad, tau, D2, r2, None, kinds) == 0
        torch.cuda.synchronize()
        assert np.array_equal(lt.to_host(D1), lt.to_host(D2))
        assert np.array_equal(lt.to_host(r1), lt.to_host(r2))


@pytest.mark.parametrize("shape,r", [((40, 30, 5), 7), ((20, 64, 4), 5), ((144, 176, 3, 2), 10)])
def test_svt_complex_precond_rank_deficient(lt, shape, r):
    """Slices of exact rank r < n: singular Gram matrices in the complex
    preconditioner (its zeroed pivots), at tau = 0 (D = A) and at a threshold in
    the spectrum, against the oracle, with the exact ranks."""
    kinds = ("dft",) * (len(shape) - 2)
    rng = np.random.default_rng(sum(shape) + r)
    mats = o.mats_for(shape, list(kinds))
    A = o.lproduct(rng.standard_normal((shape[0], r) + shape[2:]),
                   rng.standard_normal((r, shape[1]) + shape[2:]), mats).real
    assert lt.svt_path(shape, kinds) == "precond+complex"
    s = o.singular_values(A, mats)
    for tau in (0.0, float(np.quantile(s[:, :r], 0.5))):
        D, rank, _ = lt.svt_prox(lt.to_device(A), tau, kinds)
        ref = o.svt(A, tau, mats)
        say("rank-deficient complex", shape, r, "tau", tau, "ranks", lt.to_host(rank)[:6])
        parity.check(lt.to_host(D), ref, 2e-5, label="rank %d tau %.3g" % (r, tau))
        ref_rk = np.asarray(o.svt_ranks(A, tau, mats))
        near = (np.abs(s - tau) < 1e-4 * s.max()).sum(axis=1)
        assert np.all(np.abs(lt.to_host(rank) - ref_rk) <= near)
        if tau == 0.0:
            assert np.all(lt.to_host(rank) == r)


def test_svt_complex_video_against_embedding(lt):
    """The 144 x 176 x 3 x 50 video with the DFT along both trailing modes (76
    representatives, 2 self-conjugate): the complex path and the real
    embedding against the oracle, the same ranks, and a gap threshold's ranks
    exactly."""
    shape, kinds = (144, 176, 3, 50), ("dft", "dft")
    A, mats = _low_rank_plus_noise(shape, kinds, 144)
    s = o.singular_values(A, mats)
    tau = float(np.quantile(s, 0.9))
    ref = o.svt(A, tau, mats)
    Dc, rc, sc = lt.svt_prox(lt.to_device(A), tau, kinds)
    Du, ru, su = lt.svt_prox(lt.to_device(A), tau, kinds, precondition=False)
    os.environ["LT_DFT_EMBED"] = "1"
    try:
        assert lt.svt_path(shape, kinds) != "complex"
        De, re_, se = lt.svt_prox(lt.to_device(A), tau, kinds)
    finally:
        del os.environ["LT_DFT_EMBED"]
    say("video dft: complex sweeps", lt.to_host(sc).mean(), "(on the slices", lt.to_host(su).mean(), ")",
        "embedding sweeps", lt.to_host(se).mean())
    parity.check(lt.to_host(Dc), ref, 2e-5, label="complex, preconditioned")
    parity.check(lt.to_host(Du), ref, 2e-5, label="complex")
    parity.check(lt.to_host(De), ref, 2e-5, label="embedding")
    near = (np.abs(s - tau) < 1e-4 * s.max()).sum(axis=1)
    assert np.all(np.abs(lt.to_host(rc) - np.asarray(o.svt_ranks(A, tau, mats))) <= near)
    assert np.all(np.abs(lt.to_host(rc) - lt.to_host(re_)) <= near)
    assert np.all(np.abs(lt.to_host(ru) - lt.to_host(re_)) <= near)
    # a threshold in the gap between the rank-36 signal and the noise
    tau = float(0.5 * (s[:, 35].min() + s[:, 36].max()))
    assert s[:, 35].min() > 1.2 * s[:, 36].max()
    D, rank, _ = lt.svt_prox(lt.to_device(A), tau, kinds)
    assert np.all(lt.to_host(rank) == 36)
    parity.check(lt.to_host(D), o.svt(A, tau, mats), 2e-5, label="gap")


@pytest.mark.parametrize("shape,kinds", [((8, 6, 5), ("dft",)), ((5, 9, 6), ("dft",)),
                                         ((20, 14, 4, 3), ("dft", "dct")), ((33, 40, 4), ("dft",)),
                                         ((100, 80, 3), ("dft",))])
def test_lsvd_fourier_invariants(lt, shape, kinds):
    """The t-SVD (economy *_L-SVD under the DFT): A = U *_L S *_L V^H with the
    oracle's products and conjugate transpose, the transform-domain slices of U
    and V orthonormal (complex), S's the diagonal of the sorted singular values,
    which match the oracle's; both orientations, self-conjugate slices."""
    rng = np.random.default_rng(sum(shape) + 7)
    A = rng.standard_normal(shape)
    mats = o.mats_for(shape, list(kinds))
    U, S, V, sig = lt.lsvd(lt.to_device(A), kinds)
    U, S, V, sig = (lt.to_host(x).astype(np.float64) for x in (U, S, V, sig))
    R = o.lproduct(o.lproduct(U, S, mats), o.ttranspose(V, mats), mats)
    assert np.abs(np.imag(R)).max() < 1e-9 * np.abs(A).max()
    parity.check(np.real(R), A, 2e-5, label="t-SVD %s" % (shape,))
    sv = o.singular_values(A, mats)
    say("lsvd dft", shape, kinds, "sigma err", np.abs(sig - sv).max() / sv.max())
    assert np.abs(sig - sv).max() < 2e-5 * sv.max()
    for Q in (U, V):
        for q in o.slices(o.transform(Q, mats)):
            assert np.abs(q.conj().T @ q - np.eye(q.shape[1])).max() < 2e-5
    for sh, sg in zip(o.slices(o.transform(S, mats)), sv):
        assert np.abs(sh - np.diag(sg)).max() < 2e-5 * sv.max()


@pytest.mark.parametrize("shape,kinds", [((12, 9, 5), ("dft",)), ((9, 14, 4), ("dft",)),
                                         ((20, 14, 4, 3), ("dft", "dct")), ((64, 48, 3), ("dft",))])
def test_ltruncate_fourier_matches_oracle(lt, shape, kinds):
    """Eckart-Young under the DFT: A_k against the oracle on a rank-3 signal
    plus small noise, for k = 0, 3 and min(I1, I2); the error norm equals the
    tail of the transform-domain singular values over sqrt(alpha), alpha = P
    for the unnormalised Fourier matrix (Section 3.2)."""
    rng = np.random.default_rng(sum(shape) + 11)
    mats = o.mats_for(shape, list(kinds))
    A = o.lproduct(rng.standard_normal((shape[0], 3) + shape[2:]),
                   rng.standard_normal((3, shape[1]) + shape[2:]), mats).real
    A = A + 0.01 * rng.standard_normal(shape)
    s = o.singular_values(A, mats)
    alpha = o.transform_alpha(mats)
    n = min(shape[0], shape[1])
    for k in (0, 3, n):
        Ak = lt.to_host(lt.ltruncate(lt.to_device(A), k, kinds)).astype(np.float64)
        if k == 0:
            assert np.abs(Ak).max() == 0.0
            continue
        parity.check(Ak, o.truncate(A, k, mats), 2e-5, label="%s k %d" % (shape, k))
        tail = float(np.sqrt((s[:, k:] ** 2).sum() / alpha))
        resid = float(np.linalg.norm(A - Ak))
        say("  truncate dft", shape, "k", k, "residual", resid, "tail", tail)
        assert abs(resid - tail) <= 1e-4 * np.linalg.norm(A) + 1e-3 * tail


@pytest.mark.parametrize("shape,kinds", [((20, 16, 5), ("dft",)), ((12, 30, 4, 3), ("dft", "dct"))])
def test_multirank_fourier_low_rank_product(lt, shape, kinds):
    """The multirank of a rank-4 product under the DFT: 4 on every slice (the
    partners of each conjugate pair included), as the oracle counts it."""
    rng = np.random.default_rng(sum(shape) + 13)
    mats = o.mats_for(shape, list(kinds))
    A = o.lproduct(rng.standard_normal((shape[0], 4) + shape[2:]),
                   rng.standard_normal((4, shape[1]) + shape[2:]), mats).real
    rho, avg, tubal = lt.multirank(lt.to_device(A), kinds)
    rho = lt.to_host(rho)
    assert np.all(rho == 4) and avg == 4.0 and tubal == 4
    assert np.array_equal(rho, o.multirank(A, mats, rtol=1e-5)[0])


def test_pga_video_dft(lt):
    """Completion of the 144 x 176 x 3 x 50 video tensor under the DFT (the
    t-product's TNN-PGA-F) through the preconditioned complex path, 30
    iterations of the default schedule (the iterate's rank builds up from 0),
    against the oracle."""
    import torch
    p = wl.make_problem((144, 176, 3, 50), 10, 0.3, seed=5, kinds=("dft", "dft"))
    assert lt.svt_path(p.shape, p.kinds) == "precond+complex"
    s = wl.pga_schedule_params(p.M, p.mask)
    iters = 30
    params = lt.pga_params(mu0=s["mu0"], nu=s["nu"], mu_bar=s["mu_bar"], max_iter=iters)
    X, rep, st = lt.complete_pga(lt.to_device(p.M), lt.to_device(p.mask, torch.uint8), params, p.kinds)
    Xo, _ = o.complete_pga(p.M, p.mask, o.mats_for(p.shape, list(p.kinds)), mu0=s["mu0"], nu=s["nu"],
                           mu_bar=s["mu_bar"], max_iter=iters)
    say("pga video dft:", rep)
    assert np.linalg.norm(Xo) > 0
    parity.check(lt.to_host(X), Xo, 1e-4, label="video dft pga")
