"""Pins of the oracle's transform machinery against closed forms, library
routines the oracle does not call, and the paper's diagonalisation theorems."""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle as o


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9])
def test_dct_orthogonal_and_equals_scipy(n):
    # Section 2: C_n is orthogonal; with the delta_{i,1} reading it is SciPy's
    # orthonormal DCT-II (a library routine the oracle does not call).
    C = o.dct_matrix(n)
    assert np.abs(C @ C.T - np.eye(n)).max() < 1e-14
    x = np.random.default_rng(n).standard_normal(n)
    assert np.abs(C @ x - sfft.dct(x, type=2, norm="ortho")).max() < 1e-13


def test_dct_literal_delta_ij_is_not_orthogonal():
    # Documents the reading: the printed delta_{i,j} scaling breaks orthogonality.
    n = 6
    C = np.array([[np.sqrt((2 - (i == j)) / n) * np.cos(i * (2 * j + 1) * np.pi / (2 * n))
                   for j in range(n)] for i in range(n)])
    assert np.abs(C @ C.T - np.eye(n)).max() > 0.1


@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_dft_closed_form(n):
    # F_n F_n^* = n I (Section 2) and F_n x = numpy.fft.fft(x).
    F = o.dft_matrix(n)
    assert np.abs(F @ F.conj().T - n * np.eye(n)).max() < 1e-12
    x = np.random.default_rng(n).standard_normal(n)
    assert np.abs(F @ x - np.fft.fft(x)).max() < 1e-12


@pytest.mark.parametrize("n", [2, 3, 6])
def test_cprod_matrix_first_column_and_tph_diagonalisation(n):
    # M e_1 = 1 (W = diag(C(:,1))), and eq. (d): C tph(a) C^* = diag(M a).
    M = o.cprod_matrix(n)
    assert np.abs(M[:, 0] - 1.0).max() < 1e-12
    a = np.random.default_rng(n).standard_normal(n)
    C = o.dct_matrix(n)
    lhs = C @ o.tph(a) @ C.T
    assert np.abs(lhs - np.diag(M @ a)).max() < 1e-12


def test_tph_hand_example():
    # Toeplitz-plus-Hankel of (a1, a2, a3) written out by hand from eq. (3.22).
    a1, a2, a3 = 2.0, 3.0, 5.0
    T = np.array([[a1, a2, a3], [a2, a1, a2], [a3, a2, a1]])
    H = np.array([[a2, a3, 0], [a3, 0, a3], [0, a3, a2]])
    assert np.array_equal(o.tph([a1, a2, a3]), T + H)


def test_scalar_tensor_btph_diagonalised_by_kron_dct():
    # Theorem 8, eq. (19), order 4: (C4 x C3) btph(x) (C4 x C3)^* = diag(x x3 M3 x4 M4).
    I3, I4 = 3, 4
    x = np.random.default_rng(1).standard_normal((1, 1, I3, I4))
    K = np.kron(o.dct_matrix(I4), o.dct_matrix(I3))
    lhs = K @ o.btph(x) @ K.T
    xh = o.transform(x, [o.cprod_matrix(I3), o.cprod_matrix(I4)])
    d = o.slices(xh).reshape(-1)
    assert np.abs(lhs - np.diag(d)).max() < 1e-11


@pytest.mark.parametrize("shape", [(2, 3, 4), (2, 2, 3, 2)])
def test_btph_block_diagonalisation_eq20(shape):
    # eq. (20): btph(X) = (C_N^* x .. x C_3^* x I_I1) bdiag(L(X)) (C_N x .. x C_3 x I_I2)
    X = np.random.default_rng(2).standard_normal(shape)
    trailing = shape[2:]
    Ck = np.ones((1, 1))
    for n in trailing:
        Ck = np.kron(o.dct_matrix(n), Ck)
    left = np.kron(Ck.T, np.eye(shape[0]))
    right = np.kron(Ck, np.eye(shape[1]))
    Lx = o.transform(X, [o.cprod_matrix(n) for n in trailing])
    assert np.abs(o.btph(X) - left @ o.bdiag(Lx) @ right).max() < 1e-11


def test_mode_product_brute_force_and_matricisation():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2, 3, 4, 5))
    U = rng.standard_normal((6, 4))
    Y = o.mode_product(X, U, 3)
    Yb = np.zeros((2, 3, 6, 5))
    for a in range(2):
        for b in range(3):
            for j in range(6):
                for d in range(5):
                    Yb[a, b, j, d] = sum(X[a, b, i, d] * U[j, i] for i in range(4))
    assert np.abs(Y - Yb).max() < 1e-12
    # the n-mode products along different modes commute (Section 2)
    V = rng.standard_normal((2, 5))
    assert np.abs(o.mode_product(o.mode_product(X, U, 3), V, 4)
                  - o.mode_product(o.mode_product(X, V, 4), U, 3)).max() < 1e-12


def test_slice_numbering_is_vec_order():
    # eq. (3.5): p = k3 + (k4 - 1) I3 (1-based); 0-based p = k3 + I3 k4.
    X = np.random.default_rng(4).standard_normal((2, 3, 4, 5))
    S = o.slices(X)
    for k3 in range(4):
        for k4 in range(5):
            assert np.array_equal(S[k3 + 4 * k4], X[:, :, k3, k4])
    assert np.array_equal(o.unslices(S, X.shape), X)


def test_norm_scaling_alpha():
    # Section 3.2: ||A|| = alpha^{-1/2} ||L(A)||; orthonormal DCT alpha = 1, DFT
    # along modes 3 and 4: alpha = I3 I4 (reading alpha = prod alpha_i^2).
    A = np.random.default_rng(5).standard_normal((3, 4, 5, 6))
    Ld = o.transform(A, o.mats_for(A.shape, ["dct", "dct"]))
    Lf = o.transform(A, o.mats_for(A.shape, ["dft", "dft"]))
    assert abs(o.fro(Ld) - o.fro(A)) < 1e-12 * o.fro(A)
    assert abs(o.fro(Lf) / o.fro(A) - np.sqrt(30)) < 1e-12


def test_transform_roundtrip_and_scipy_dctn():
    A = np.random.default_rng(6).standard_normal((3, 4, 5, 6))
    mats = o.mats_for(A.shape, ["dct", "dct"])
    Ah = o.transform(A, mats)
    assert np.abs(Ah - sfft.dctn(A, type=2, norm="ortho", axes=[2, 3])).max() < 1e-12
    assert np.abs(o.inverse_transform(Ah, mats) - A).max() < 1e-12
