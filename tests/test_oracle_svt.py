"""Pins of the oracle's *_L-SVD and singular value thresholding: the SVD
theorem and its corollaries, Eckart-Young, and Theorem 23's optimality
conditions checked through SciPy's DCT (not the oracle's transform)."""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle as o


def _dctn(X):
    axes = list(range(2, X.ndim))
    return sfft.dctn(X, type=2, norm="ortho", axes=axes)


def _idctn(X):
    axes = list(range(2, X.ndim))
    return sfft.idctn(X, type=2, norm="ortho", axes=axes)


@pytest.mark.parametrize("shape,kinds", [((4, 3, 5), ["dct"]), ((3, 5, 2, 3), ["dct", "dct"]),
                                         ((4, 3, 5), ["dft"]), ((3, 4, 3, 2), ["dft", "dct"])])
def test_lsvd_reconstructs_and_is_orthogonal(shape, kinds):
    A = np.random.default_rng(20).standard_normal(shape)
    mats = o.mats_for(shape, kinds)
    U, S, V = o.lsvd(A, mats)
    R = o.lproduct(o.lproduct(U, S, mats), o.ttranspose(V, mats), mats)
    assert np.abs(R - A).max() < 1e-11
    for Q in (U, V):
        Qh = o.slices(o.transform(Q, mats))
        for p in range(Qh.shape[0]):
            assert np.abs(Qh[p].conj().T @ Qh[p] - np.eye(Qh.shape[1])).max() < 1e-11
    Sh = o.slices(o.transform(S, mats))
    for p in range(Sh.shape[0]):
        off = Sh[p] - np.diag(np.diag(Sh[p])) if Sh.shape[1] == Sh.shape[2] else Sh[p].copy()
        if Sh.shape[1] != Sh.shape[2]:
            k = min(Sh.shape[1:])
            off[np.arange(k), np.arange(k)] = 0
        assert np.abs(off).max() < 1e-11          # f-diagonal


def test_lsvd_norm_identity_and_ordering():
    # Corollary: ||A||^2 = ||S||^2 = sum_i ||S_i||^2 and ||S_1|| >= ||S_2|| >= ...
    A = np.random.default_rng(21).standard_normal((5, 4, 3, 2))
    mats = o.mats_for(A.shape, ["dct", "dct"])
    U, S, V = o.lsvd(A, mats)
    assert abs(o.fro(S) - o.fro(A)) < 1e-12 * o.fro(A)
    tubes = [o.fro(S[i, i]) for i in range(4)]
    assert abs(sum(t * t for t in tubes) - o.fro(A) ** 2) < 1e-10
    assert all(tubes[i] >= tubes[i + 1] - 1e-12 for i in range(3))


def test_eckart_young_error():
    # ||A - A_k||^2 = sum_{i > k} ||S_i||^2 (Eckart-Young theorem, Section 3.2).
    A = np.random.default_rng(22).standard_normal((6, 5, 4))
    mats = o.mats_for(A.shape, ["dct"])
    U, S, V = o.lsvd(A, mats)
    k = 2
    Ak = o.lproduct(o.lproduct(U[:, :k], S[:k, :k], mats), o.ttranspose(V[:, :k], mats), mats)
    tubes = [o.fro(S[i, i]) ** 2 for i in range(5)]
    assert abs(o.fro(A - Ak) ** 2 - sum(tubes[k:])) < 1e-10


@pytest.mark.parametrize("kinds", [["dct"], ["dft"], ["dct", "identity"]])
def test_truncate_is_the_eckart_young_tensor(kinds):
    """truncate(A, k) equals the theorem's U(:,1:k) *_L S(1:k,1:k) *_L V(:,1:k)^T
    built from lsvd and lproduct, its error is the tail of the singular tubes,
    and no product X *_L Y with k lateral slices does better."""
    rng = np.random.default_rng(24)
    shape = (7, 5) + ((4,) if len(kinds) == 1 else (3, 2))
    A = rng.standard_normal(shape)
    mats = o.mats_for(shape, kinds)
    U, S, V = o.lsvd(A, mats)
    for k in (1, 2, 4):
        Ak = o.truncate(A, k, mats)
        ref = o.lproduct(o.lproduct(U[:, :k], S[:k, :k], mats), o.ttranspose(V[:, :k], mats), mats)
        assert np.abs(Ak - ref).max() < 1e-10
        tails = sum(o.fro(S[i, i]) ** 2 for i in range(k, 5))
        err = o.fro(A - Ak)
        assert abs(err ** 2 - tails) < 1e-9 * o.fro(A) ** 2
        for _ in range(20):
            X = rng.standard_normal((7, k) + shape[2:])
            Y = rng.standard_normal((k, 5) + shape[2:])
            B = o.lproduct(X, Y, mats)
            if np.iscomplexobj(B):
                B = B.real
            assert o.fro(A - B) >= err - 1e-12
        rho, _ = o.multirank(Ak, mats, rtol=1e-9)
        assert np.all(rho <= k)


def test_truncate_limits():
    A = np.random.default_rng(25).standard_normal((6, 4, 3))
    mats = o.mats_for(A.shape, ["dct"])
    assert np.abs(o.truncate(A, 4, mats) - A).max() < 1e-12
    assert np.abs(o.truncate(A, 9, mats) - A).max() < 1e-12
    assert np.abs(o.truncate(A, 0, mats)).max() == 0.0


def test_multirank_of_product():
    rng = np.random.default_rng(23)
    mats = o.mats_for((8, 7, 3, 2), ["dct", "dct"])
    A = rng.standard_normal((8, 3, 3, 2))
    B = rng.standard_normal((3, 7, 3, 2))
    rho, avg = o.multirank(o.lproduct(A, B, mats), mats)
    assert np.all(rho == 3) and avg == 3


def _nuclear_dct(Y):
    Yh = _dctn(Y)
    flat = Yh.reshape(Yh.shape[0], Yh.shape[1], -1, order="F")
    return sum(np.linalg.svd(flat[:, :, p], compute_uv=False).sum() for p in range(flat.shape[2]))


@pytest.mark.parametrize("shape", [(6, 4, 3), (4, 7, 2, 3)])
def test_svt_optimality_conditions(shape):
    # Theorem 23: D_tau(A) is the unique minimiser of tau ||Y||_* + 1/2 ||Y - A||^2.
    # Per transform-domain slice: A^p - D^p = tau U_r V_r^T + W, ||W||_2 <= tau,
    # U_r^T W = 0, W V_r = 0 (subgradient of the nuclear norm).
    rng = np.random.default_rng(24)
    A = rng.standard_normal(shape)
    mats = o.mats_for(shape, ["dct"] * (len(shape) - 2))
    s_all = o.singular_values(A, mats)
    tau = float(np.median(s_all))
    D = o.svt(A, tau, mats)
    Ah = _dctn(A).reshape(shape[0], shape[1], -1, order="F")
    Dh = _dctn(D).reshape(shape[0], shape[1], -1, order="F")
    for p in range(Ah.shape[2]):
        U, s, Vt = np.linalg.svd(Dh[:, :, p], full_matrices=False)
        r = int((s > 1e-9).sum())
        Ur, Vr = U[:, :r], Vt[:r].T
        W = Ah[:, :, p] - Dh[:, :, p] - tau * Ur @ Vr.T
        assert np.linalg.norm(W, 2) <= tau * (1 + 1e-9)
        assert np.abs(Ur.T @ W).max() < 1e-10
        assert np.abs(W @ Vr).max() < 1e-10
    # objective is not improved by random perturbations
    f0 = tau * _nuclear_dct(D) + 0.5 * o.fro(D - A) ** 2
    for _ in range(5):
        E = rng.standard_normal(shape) * 1e-3
        f1 = tau * _nuclear_dct(D + E) + 0.5 * o.fro(D + E - A) ** 2
        assert f1 >= f0 - 1e-12


def test_svt_special_cases():
    rng = np.random.default_rng(25)
    A = rng.standard_normal((5, 4, 3, 2))
    mats = o.mats_for(A.shape, ["dct", "dct"])
    assert np.abs(o.svt(A, 0.0, mats) - A).max() < 1e-12
    smax = o.singular_values(A, mats).max()
    assert np.abs(o.svt(A, smax * 1.0001, mats)).max() == 0.0
    # I1 = I2 = 1: soft thresholding of the transform coefficients (textbook)
    a = rng.standard_normal((1, 1, 5, 3))
    ma = o.mats_for(a.shape, ["dct", "dct"])
    ah = _dctn(a)
    expect = _idctn(np.sign(ah) * np.maximum(np.abs(ah) - 0.3, 0.0))
    assert np.abs(o.svt(a, 0.3, ma) - expect).max() < 1e-12


def test_svt_nonexpansive_and_dft_real():
    rng = np.random.default_rng(26)
    A = rng.standard_normal((4, 5, 6))
    B = A + 0.1 * rng.standard_normal(A.shape)
    mats = o.mats_for(A.shape, ["dct"])
    assert o.fro(o.svt(A, 0.5, mats) - o.svt(B, 0.5, mats)) <= o.fro(A - B) * (1 + 1e-12)
    mf = o.mats_for(A.shape, ["dft"])
    D = o.svt(A, 0.5, mf)
    assert not np.iscomplexobj(D)
    # the full complex result is real up to rounding
    Ah = o.slices(o.transform(A, mf))
    Dh = []
    for p in range(Ah.shape[0]):
        U, s, Vt = np.linalg.svd(Ah[p], full_matrices=False)
        Dh.append((U * np.maximum(s - 0.5, 0)) @ Vt)
    Dc = o.inverse_transform(o.unslices(np.stack(Dh), A.shape), mf)
    assert np.abs(Dc.imag).max() < 1e-12
    assert np.abs(Dc.real - D).max() < 1e-12


def test_svt_ranks():
    rng = np.random.default_rng(27)
    A = rng.standard_normal((6, 5, 4))
    mats = o.mats_for(A.shape, ["dct"])
    tau = 1.0
    D = o.svt(A, tau, mats)
    rho, _ = o.multirank(D, mats, rtol=1e-9)
    assert np.array_equal(rho, o.svt_ranks(A, tau, mats))


def test_warm_start_invariance():
    """The warm-started SVT's premise (reading R22): for the n x n factor L and
    any orthogonal Z, L Z has the singular values of L and the same left
    singular subspaces, so the projector sum (1 - tau/sigma_i) u_i u_i^T that
    the preconditioned rebuild uses is unchanged."""
    rng = np.random.default_rng(22)
    n, tau = 12, 0.8
    L = np.tril(rng.standard_normal((n, n)))
    Z, _ = np.linalg.qr(rng.standard_normal((n, n)))

    def proj(A):
        U, s, _ = np.linalg.svd(A)
        keep = s > tau
        return s, (U[:, keep] * (1.0 - tau / s[keep])) @ U[:, keep].T

    s1, P1 = proj(L)
    s2, P2 = proj(L @ Z)
    assert np.allclose(s1, s2, rtol=1e-12, atol=1e-12)
    assert np.allclose(P1, P2, atol=1e-11)
    # and the non-orthogonal case is not invariant (a wrong Z would show)
    s3, _ = proj(L @ (Z + 0.1 * rng.standard_normal((n, n))))
    assert not np.allclose(s1, s3, rtol=1e-3)
