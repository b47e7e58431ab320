"""CPU checks (NumPy, FP64) of the algebra the complex Jacobi path rests on,
independent of the kernels: a complex m x n matrix W is held as 2m interleaved
real rows (row 2i: Re, row 2i + 1: Im); its twinned real form T interleaves
each column w with i w.  Pinned here:
  * T^T T is the real form of W^H W, block (a, b) = [[Re g, -Im g], [Im g, Re g]]
    with g = w_a^H w_b;
  * the real Cholesky factor of T^T T is the real form of the complex one, so
    its even columns are the complex factor's columns;
  * with B' = [b_1, i b_1, ...] (columns twinned), B' B'^T applied to the
    interleaved W gives the interleaved B B^H W, and (T B') B'^T has the
    interleaved (W B) B^H as its even columns;
  * over the interleaved rows, Re(w_a^H w_b) is the real dot of the columns
    and Im(w_a^H w_b) the real dot of w_a with J w_b, J mapping each (Re, Im)
    pair (x, y) to (y, -x): the row's pair partner, negated on odd rows;
  * the Hermitian rotation (phase of a^H b, then the real rotation with
    zeta = (|b|^2 - |a|^2) / (2 |a^H b|)) leaves the pair orthogonal.
"""
import numpy as np


def interleave(W):
    """Complex m x n -> real 2m x n, rows (Re, Im) interleaved."""
    m, n = W.shape
    R = np.empty((2 * m, n))
    R[0::2] = W.real
    R[1::2] = W.imag
    return R


def deinterleave(R):
    return R[0::2] + 1j * R[1::2]


def times_i(R):
    """i w for interleaved columns: (Re, Im) -> (-Im, Re)."""
    S = np.empty_like(R)
    S[0::2] = -R[1::2]
    S[1::2] = R[0::2]
    return S


def twin(R):
    """Columns w_1, i w_1, w_2, i w_2, ... of interleaved columns."""
    m2, n = R.shape
    T = np.empty((m2, 2 * n))
    T[:, 0::2] = R
    T[:, 1::2] = times_i(R)
    return T


def real_form(C):
    """Complex n x n -> 2n x 2n with 2 x 2 blocks [[Re, -Im], [Im, Re]]."""
    n = C.shape[0]
    R = np.empty((2 * n, 2 * n))
    R[0::2, 0::2] = C.real
    R[1::2, 1::2] = C.real
    R[1::2, 0::2] = C.imag
    R[0::2, 1::2] = -C.imag
    return R


def _rand(rng, m, n):
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def test_twinned_gram_is_the_real_form_of_the_complex_gram():
    rng = np.random.default_rng(1)
    W = _rand(rng, 13, 7)
    T = twin(interleave(W))
    G = W.conj().T @ W
    assert np.allclose(T.T @ T, real_form(G), rtol=0, atol=1e-12 * np.abs(G).max())
    # one block, with the signs the Gram kernel writes: rows 2a, 2a + 1,
    # columns 2b, 2b + 1 of [[Re g, -Im g], [Im g, Re g]], g = w_a^H w_b
    a, b = 4, 2
    g = W[:, a].conj() @ W[:, b]
    blk = (T.T @ T)[2 * a:2 * a + 2, 2 * b:2 * b + 2]
    assert np.allclose(blk, [[g.real, -g.imag], [g.imag, g.real]])


def test_complex_gram_from_two_real_dots():
    rng = np.random.default_rng(5)
    W = _rand(rng, 23, 9)
    Wi = interleave(W)
    JW = np.empty_like(Wi)
    k = np.arange(Wi.shape[0])
    sign = np.where(k % 2 == 1, -1.0, 1.0)
    JW[:] = sign[:, None] * Wi[k ^ 1]                 # partner row, odd rows negated
    G = W.conj().T @ W                                # G[a, b] = w_a^H w_b
    assert np.allclose(Wi.T @ Wi, G.real)
    assert np.allclose(Wi.T @ JW, G.imag)
    # with G[a, b] in rows 2a, 2a + 1 and columns 2b, 2b + 1 of the real form
    assert np.allclose(real_form(G), twin(Wi).T @ twin(Wi))


def test_real_cholesky_of_the_twinned_gram_is_the_real_form_of_the_complex_factor():
    rng = np.random.default_rng(2)
    W = _rand(rng, 20, 9)
    G = W.conj().T @ W
    L = np.linalg.cholesky(G)                         # complex, lower, positive diagonal
    Lr = np.linalg.cholesky(twin(interleave(W)).T @ twin(interleave(W)))
    assert np.allclose(Lr, real_form(L), atol=1e-10)
    # the even columns, interleaved, are the complex factor's columns
    assert np.allclose(deinterleave(Lr[:, 0::2]), L, atol=1e-10)


def test_twinned_rebuilds_form_the_complex_products():
    rng = np.random.default_rng(3)
    W = _rand(rng, 11, 6)
    B = _rand(rng, 11, 3)                             # kept columns of the slice (U side)
    Wi, Bt = interleave(W), twin(interleave(B))
    assert np.allclose(deinterleave(Bt @ (Bt.T @ Wi)), B @ (B.conj().T @ W))
    # preconditioned form: B over the n columns (V side), D = (W B) B^H
    V = _rand(rng, 6, 2)
    T, Vt = twin(interleave(W)), twin(interleave(V))
    D = (T @ Vt) @ Vt.T
    assert np.allclose(deinterleave(D[:, 0::2]), (W @ V) @ V.conj().T)


def test_hermitian_rotation_orthogonalises_the_pair():
    rng = np.random.default_rng(4)
    for _ in range(20):
        a, b = _rand(rng, 17, 1)[:, 0], _rand(rng, 17, 1)[:, 0]
        g = a.conj() @ b
        pa, pb = np.vdot(a, a).real, np.vdot(b, b).real
        d = abs(g)
        e = g / d                                     # phase of a^H b
        zeta = (pb - pa) / (2 * d)
        t = np.sign(zeta) / (abs(zeta) + np.sqrt(1 + zeta * zeta)) if zeta != 0 else 1.0
        c = 1 / np.sqrt(1 + t * t)
        s = c * t
        y = b * np.conj(e)                            # a^H y = |g|, real
        a2, b2 = c * a - s * y, c * y + s * a
        assert abs(a2.conj() @ b2) < 1e-12 * np.sqrt(pa * pb)
        # the norm updates the kernel uses
        assert np.isclose(np.vdot(a2, a2).real, pa - t * d)
        assert np.isclose(np.vdot(b2, b2).real, pb + t * d)
        # interleaved: the real dot of the rows is Re a^H b, and the cross sum
        # Re a Im b - Im a Re b is its imaginary part
        ai, bi = interleave(a[:, None])[:, 0], interleave(b[:, None])[:, 0]
        assert np.isclose(ai @ bi, g.real)
        assert np.isclose((ai[0::2] * bi[1::2] - ai[1::2] * bi[0::2]).sum(), g.imag)
