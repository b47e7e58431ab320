"""Pins of the oracle's stopping rule, of its Fourier-transform SVT threshold
and of its nuclear norm, each against something the oracle does not compute
itself: a completion worked by hand, Theorem 23's optimality conditions and
Theorem 21's identity evaluated through NumPy's FFT and SciPy's DCT, and the
dual-norm definition of the nuclear norm (eq. (23))."""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle as o


# ------------------------------------------------------------ stopping rule --

def test_stop_criterion_value():
    """||Y - X||_F / ||X||_F on a pair worked by hand: X = (1, 2, 2, 0) has norm
    3, Y - X = (0, 0, 0, 5), so the ratio is 5/3 (||Y|| = sqrt(34) in the
    denominator would give 0.857, the squared form 25/9)."""
    X = np.array([1.0, 2.0, 2.0, 0.0]).reshape(2, 2, 1)
    Y = np.array([1.0, 2.0, 2.0, 5.0]).reshape(2, 2, 1)
    assert abs(o.stop_criterion(Y, X) - 5.0 / 3.0) < 1e-15
    assert o.stop_criterion(Y, np.zeros_like(X)) == np.inf
    assert o.stop_criterion(X, X) == 0.0


def test_completion_worked_by_hand():
    """A 1 x 1 x 1 tensor m = 3, observed, thresholds mu = 2, 1, 0.5, 0.5
    (mu0 = 2, nu = 0.5, mu_bar = 0.5).  The slice is 1 x 1, so the prox is the
    scalar soft threshold and G = m at every step (Alg. 5 with eq. (51)):
      k = 1: Y = 0,                 X^2 = 3 - 2 = 1,   crit = |0 - 1| / 1 = 1
      k = 2: beta_2 = (t_1 - 1)/t_2 = 0, Y = X^2 = 1,  X^3 = 2,  crit = 1/2
      k = 3: t_2 = (1 + sqrt 5)/2, t_3 = (1 + sqrt(4 t_2^2 + 1))/2 = 2.1935270853,
             beta_3 = (t_2 - 1)/t_3 = 0.2817535251, Y = X^3 + beta_3 (X^3 - X^2)
             = 2.2817535251, X^4 = 2.5, crit = |Y - X^4| / X^4 = 0.0872985899
      k = 4: beta_4 = (t_3 - 1)/t_4 = 0.4340427828, Y = 2.5 + 0.5 beta_4,
             X^5 = 2.5, crit = 0.0868085566
    (mpmath, 30 digits).  A criterion on ||X^{k+1} - X^k|| would give 0.2 at
    k = 3; a momentum weight (t_k - 1)/t_k or (t_{k-1} - 1)/t_{k-1} changes
    the k = 3 and k = 4 values."""
    M = np.full((1, 1, 1), 3.0)
    mask = np.ones(M.shape, bool)
    mats = o.mats_for(M.shape, ["dct"])
    trace = []
    X, info = o.complete_pga(M, mask, mats, mu0=2.0, nu=0.5, mu_bar=0.5, max_iter=4, trace=trace)
    expect = [1.0, 0.5, 0.0872985899498716727249983948015, 0.0868085565560604001222631332899]
    assert np.allclose(trace, expect, rtol=1e-13, atol=0)
    assert abs(X[0, 0, 0] - 2.5) < 1e-15
    # the same run stops at k = 4 once the test may fire (mu_4 = mu_bar) ...
    X, info = o.complete_pga(M, mask, mats, mu0=2.0, nu=0.5, mu_bar=0.5, tol=0.087, max_iter=10)
    assert info["converged"] and info["iters"] == 4
    # ... but not at k = 3 (crit 0.0873 > 0.087), and not before the floor when gated
    X, info = o.complete_pga(M, mask, mats, mu0=2.0, nu=0.5, mu_bar=0.5, tol=0.6, max_iter=10)
    assert info["converged"] and info["iters"] == 3      # mu_3 = 0.5 is the floor
    X, info = o.complete_pga(M, mask, mats, mu0=2.0, nu=0.5, mu_bar=0.5, tol=0.6, max_iter=10,
                             gate_until_floor=False)
    assert info["converged"] and info["iters"] == 2


# --------------------------------------------- transform helpers (library) --

def _lib_forward(X, kinds):
    """L(X) through SciPy's orthonormal DCT-II and NumPy's unnormalised FFT
    (F_n of Section 2), mode by mode; identity modes untouched."""
    Y = X.astype(np.complex128) if "dft" in kinds else X
    for i, k in enumerate(kinds):
        ax = i + 2
        if k == "dct":
            Y = sfft.dct(Y.real, type=2, norm="ortho", axis=ax) + (
                1j * sfft.dct(Y.imag, type=2, norm="ortho", axis=ax) if np.iscomplexobj(Y) else 0)
        elif k == "dft":
            Y = np.fft.fft(Y, axis=ax)
    return Y


def _lib_inverse(Xh, kinds):
    Y = Xh
    for i, k in reversed(list(enumerate(kinds))):
        ax = i + 2
        if k == "dct":
            Y = sfft.idct(Y.real, type=2, norm="ortho", axis=ax) + (
                1j * sfft.idct(Y.imag, type=2, norm="ortho", axis=ax) if np.iscomplexobj(Y) else 0)
        elif k == "dft":
            Y = np.fft.ifft(Y, axis=ax)
    return Y


def _lib_slices(Xh):
    I1, I2 = Xh.shape[:2]
    return np.moveaxis(Xh.reshape(I1, I2, -1, order="F"), 2, 0)


def _alpha(shape, kinds):
    """||L(A)||_F^2 / ||A||_F^2 for these transforms: the product of the DFT
    sizes (NumPy's FFT is unnormalised, the DCT orthonormal)."""
    a = 1.0
    for i, k in enumerate(kinds):
        if k == "dft":
            a *= shape[i + 2]
    return a


def _lib_nuclear(Y, kinds):
    """Theorem 21 / eq. (24): (1/alpha) ||bdiag(L(Y))||_*, bdiag built
    explicitly and its singular values taken in one LAPACK call."""
    S = _lib_slices(_lib_forward(Y, kinds))
    P, I1, I2 = S.shape
    B = np.zeros((P * I1, P * I2), dtype=S.dtype)
    for p in range(P):
        B[p * I1:(p + 1) * I1, p * I2:(p + 1) * I2] = S[p]
    return np.linalg.svd(B, compute_uv=False).sum() / _alpha(Y.shape, kinds)


CASES = [((4, 3, 5), ("dft",)), ((3, 5, 6), ("dft",)), ((3, 4, 3, 2), ("dft", "dct")),
         ((4, 4, 2, 3), ("dft", "dft")), ((5, 3, 4), ("dct",)), ((4, 3, 2, 3), ("identity", "dft"))]


def test_alpha_norm_relation():
    """transform_alpha is the factor of ||L(A)||^2 = alpha ||A||^2 (Section 3.2)."""
    rng = np.random.default_rng(40)
    for shape, kinds in CASES:
        A = rng.standard_normal(shape)
        mats = o.mats_for(shape, list(kinds))
        a = o.transform_alpha(mats)
        assert abs(a - _alpha(shape, kinds)) < 1e-12 * a
        assert abs(np.linalg.norm(_lib_forward(A, kinds)) ** 2 - a * np.linalg.norm(A) ** 2) < 1e-10 * a
    with pytest.raises(ValueError):           # the c-product matrix is not a scaled unitary
        o.transform_alpha(o.mats_for((3, 3, 4), ["cprod"]))


# ------------------------------------------------------------ nuclear norm --

@pytest.mark.parametrize("shape,kinds", CASES)
def test_nuclear_norm_is_theorem_21(shape, kinds):
    """nuclear_norm(A) = (1/alpha) ||bdiag(L(A))||_* (Theorem 21), with L(A)
    from the FFT / DCT libraries and the nuclear norm of the explicit
    block-diagonal matrix."""
    A = np.random.default_rng(41).standard_normal(shape)
    mats = o.mats_for(shape, list(kinds))
    ref = _lib_nuclear(A, kinds)
    assert abs(o.nuclear_norm(A, mats) - ref) < 1e-11 * ref


@pytest.mark.parametrize("shape,kinds", CASES)
def test_nuclear_norm_is_the_dual_norm(shape, kinds):
    """Definition (eq. (23)): ||A||_* = sup over ||B|| <= 1 of |<A, B>|, the
    spectral norm being ||bdiag(L(B))||_2 (the proposition before the
    definition).  The supremum is reached at B = L^{-1}(U_p V_p^H per slice),
    and no B of spectral norm 1 exceeds it."""
    rng = np.random.default_rng(42)
    A = rng.standard_normal(shape)
    mats = o.mats_for(shape, list(kinds))
    nn = o.nuclear_norm(A, mats)
    S = _lib_slices(_lib_forward(A, kinds))
    best = []
    for Sp in S:
        U, s, Vh = np.linalg.svd(Sp, full_matrices=False)
        best.append(U @ Vh)
    I1, I2 = shape[:2]
    Bh = np.moveaxis(np.stack(best), 0, 2).reshape(shape, order="F")
    B = _lib_inverse(Bh, kinds)
    assert np.abs(np.imag(B)).max() < 1e-12        # real A: conjugate-symmetric slices
    B = np.real(B)

    def spectral(T):
        return max(np.linalg.norm(Tp, 2) for Tp in _lib_slices(_lib_forward(T, kinds)))

    assert abs(spectral(B) - 1.0) < 1e-12
    assert abs(np.vdot(A, B) - nn) < 1e-11 * nn
    for _ in range(20):
        R = rng.standard_normal(shape)
        R /= spectral(R)
        assert abs(np.vdot(A, R)) <= nn * (1 + 1e-12)


# ------------------------------------------------------- SVT under the DFT --

@pytest.mark.parametrize("shape,kinds", [c for c in CASES if "dft" in c[1]])
def test_svt_optimality_fourier(shape, kinds):
    """Theorem 23 for transforms with Fourier modes: D = D_tau(A) minimises
    tau ||Y||_* + 1/2 ||Y - A||_F^2 with the nuclear norm of Theorem 21
    (factor 1/alpha, alpha the product of the DFT sizes).  Through the
    libraries' FFT: per slice of L(A) - L(D) = tau U_r V_r^H + W with
    ||W||_2 <= tau, U_r^H W = 0, W V_r = 0 (the subgradient of the slice
    nuclear norm; a threshold scaled by alpha or by its square root fails
    the first condition).  The objective evaluated with that nuclear norm does
    not decrease along the perturbations tried."""
    rng = np.random.default_rng(43)
    A = rng.standard_normal(shape)
    mats = o.mats_for(shape, list(kinds))
    s_all = np.concatenate([np.linalg.svd(Sp, compute_uv=False) for Sp in _lib_slices(_lib_forward(A, kinds))])
    tau = float(np.median(s_all))
    D = o.svt(A, tau, mats)
    assert not np.iscomplexobj(D)
    Ah = _lib_slices(_lib_forward(A, kinds))
    Dh = _lib_slices(_lib_forward(D, kinds))
    kept = 0
    for Ap, Dp in zip(Ah, Dh):
        U, s, Vh = np.linalg.svd(Dp, full_matrices=False)
        r = int((s > 1e-9 * max(s.max(), 1.0)).sum())
        kept += r
        Ur, Vr = U[:, :r], Vh[:r].conj().T
        W = Ap - Dp - tau * Ur @ Vr.conj().T
        assert np.linalg.norm(W, 2) <= tau * (1 + 1e-9)
        if r:
            assert np.abs(Ur.conj().T @ W).max() < 1e-10
            assert np.abs(W @ Vr).max() < 1e-10
    assert kept > 0

    def f(Y):
        return tau * _lib_nuclear(Y, kinds) + 0.5 * np.linalg.norm(Y - A) ** 2

    f0 = f(D)
    for _ in range(8):
        E = rng.standard_normal(shape) * 1e-3
        assert f(D + E) >= f0 - 1e-12
        assert f(D - E) >= f0 - 1e-12
    for c in (0.9, 1.1):          # the threshold rescaled: a worse objective
        assert f(o.svt(A, c * tau, mats)) > f0
