"""Pins of the oracle's *_L-product: circular convolution (DFT), the
block-Toeplitz-plus-Hankel product (c-product), identity, transpose and ring
properties."""
import itertools

import numpy as np
import pytest

import oracle as o


def _circ_conv(A, B):
    """Brute-force multidimensional circular convolution over the trailing modes
    with matrix products of the frontal slices: the t-product of Kilmer and
    Martin generalised to order N, written from its definition."""
    trailing = A.shape[2:]
    C = np.zeros((A.shape[0], B.shape[1]) + trailing)
    for k in itertools.product(*[range(n) for n in trailing]):
        acc = np.zeros((A.shape[0], B.shape[1]))
        for j in itertools.product(*[range(n) for n in trailing]):
            kj = tuple((a - b) % n for a, b, n in zip(k, j, trailing))
            acc += A[(slice(None), slice(None)) + j] @ B[(slice(None), slice(None)) + kj]
        C[(slice(None), slice(None)) + k] = acc
    return C


@pytest.mark.parametrize("trailing", [(5,), (3, 4)])
def test_dft_product_is_circular_convolution(trailing):
    rng = np.random.default_rng(10)
    A = rng.standard_normal((3, 2) + trailing)
    B = rng.standard_normal((2, 4) + trailing)
    mats = o.mats_for(A.shape, ["dft"] * len(trailing))
    C = o.lproduct(A, B, mats)
    assert np.abs(C.imag).max() < 1e-12
    assert np.abs(C.real - _circ_conv(A, B)).max() < 1e-12


@pytest.mark.parametrize("trailing", [(4,), (3, 2), (2, 3)])
def test_cproduct_equals_btph_product(trailing):
    # Definition 9 / Lemma: btph(A) btph(B) = btph(A *_c B) with L built from M_c.
    rng = np.random.default_rng(11)
    A = rng.standard_normal((2, 3) + trailing)
    B = rng.standard_normal((3, 2) + trailing)
    mats = o.mats_for(A.shape, ["cprod"] * len(trailing))
    C = o.lproduct(A, B, mats)
    assert np.abs(o.btph(A) @ o.btph(B) - o.btph(C)).max() < 1e-11


def test_facewise_brute_force():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((2, 3, 2, 3))
    B = rng.standard_normal((3, 4, 2, 3))
    C = o.facewise(A, B)
    for k3 in range(2):
        for k4 in range(3):
            assert np.abs(C[:, :, k3, k4] - A[:, :, k3, k4] @ B[:, :, k3, k4]).max() < 1e-12


@pytest.mark.parametrize("kinds", [["dct"], ["dft"], ["cprod"], ["dct", "dct"], ["dft", "dct"]])
def test_identity_tensor(kinds):
    trailing = (4, 3)[:len(kinds)]
    A = np.random.default_rng(13).standard_normal((3, 3) + trailing)
    mats = o.mats_for(A.shape, kinds)
    I = o.identity_tensor(3, trailing, mats)
    assert np.abs(o.lproduct(A, I, mats) - A).max() < 1e-11
    assert np.abs(o.lproduct(I, A, mats) - A).max() < 1e-11


@pytest.mark.parametrize("kind", ["dft", "cprod"])
def test_identity_closed_form_first_slice(kind):
    # For F and for M_c (both with M e_1 = 1) the identity is I in the first
    # frontal slice and zero elsewhere.
    mats = o.mats_for((3, 3, 5), [kind])
    I = o.identity_tensor(3, (5,), mats)
    expect = np.zeros((3, 3, 5))
    expect[:, :, 0] = np.eye(3)
    assert np.abs(I - expect).max() < 1e-12


def test_dct_identity_is_not_first_slice():
    mats = o.mats_for((3, 3, 5), ["dct"])
    I = o.identity_tensor(3, (5,), mats)
    assert np.abs(I[:, :, 1:]).max() > 1e-3


@pytest.mark.parametrize("kinds", [["dct", "dct"], ["dft"], ["cprod", "dct"]])
def test_transpose_reverses_product(kinds):
    trailing = (3, 4)[:len(kinds)]
    rng = np.random.default_rng(14)
    A = rng.standard_normal((2, 3) + trailing)
    B = rng.standard_normal((3, 4) + trailing)
    mats = o.mats_for(A.shape, kinds)
    lhs = o.ttranspose(o.lproduct(A, B, mats), mats)
    rhs = o.lproduct(o.ttranspose(B, mats), o.ttranspose(A, mats), mats)
    assert np.abs(lhs - rhs).max() < 1e-11


def test_dft_transpose_is_tproduct_transpose():
    # t-product transpose: transpose each slice, reverse slices 2..n.
    A = np.random.default_rng(15).standard_normal((2, 3, 5))
    mats = o.mats_for(A.shape, ["dft"])
    T = o.ttranspose(A, mats)
    expect = np.stack([A[:, :, (-k) % 5].T for k in range(5)], axis=2)
    assert np.abs(T - expect).max() < 1e-12


def test_entrywise_decomposition_and_ring():
    # Section 3.2 propositions: (X *_L Y)_{ij} = sum_k X_{ik} *_L Y_{kj}; and
    # scalar-tensors form a commutative ring.
    rng = np.random.default_rng(16)
    mats = o.mats_for((1, 1, 3, 4), ["dct", "dct"])
    X = rng.standard_normal((2, 3, 3, 4))
    Y = rng.standard_normal((3, 2, 3, 4))
    Z = o.lproduct(X, Y, mats)
    for i in range(2):
        for j in range(2):
            acc = sum(o.lproduct(X[i:i + 1, k:k + 1], Y[k:k + 1, j:j + 1], mats) for k in range(3))
            assert np.abs(acc - Z[i:i + 1, j:j + 1]).max() < 1e-12
    a, b, c = (rng.standard_normal((1, 1, 3, 4)) for _ in range(3))
    assert np.abs(o.lproduct(a, b, mats) - o.lproduct(b, a, mats)).max() < 1e-12
    assert np.abs(o.lproduct(a, o.lproduct(b, c, mats), mats)
                  - o.lproduct(o.lproduct(a, b, mats), c, mats)).max() < 1e-12
    assert np.abs(o.lproduct(a, b + c, mats)
                  - o.lproduct(a, b, mats) - o.lproduct(a, c, mats)).max() < 1e-12


def test_column_decomposition():
    rng = np.random.default_rng(17)
    mats = o.mats_for((1, 1, 4), ["dct"])
    A = rng.standard_normal((3, 2, 4))
    B = rng.standard_normal((2, 5, 4))
    C = o.lproduct(A, B, mats)
    for j in range(5):
        assert np.abs(o.lproduct(A, B[:, j:j + 1], mats) - C[:, j:j + 1]).max() < 1e-12
