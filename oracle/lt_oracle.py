"""FP64 CPU oracle for *_L-product tensor completion (Bentbib, Elalj, El Hachimi,
Jbilou, Ratnani: "Generalized L-product for high order tensors with applications
using GPU computations", arXiv 2202.02870).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with the
HIP library: it is a plain, slow, obviously-correct NumPy implementation of the
paper's definitions, in float64 (complex128 for the Fourier transform).

Conventions
-----------
* A tensor of order N is an ndarray of shape (I1, I2, I3, ..., IN).
* Frontal slice p (0-based) is X[:, :, k3, ..., kN] with p the column-major
  (first-index-fastest) linear index of (k3, ..., kN): the paper's Vec numbering,
  eq. (3.5).  `slices` returns them stacked as an array of shape (P, I1, I2).
* A transform is described by a list `mats` with one entry per trailing mode
  3..N: an (Ii x Ii) matrix M_i, or None for the identity.

Where the paper's text is garbled or silent, the reading taken is stated in the
docstring of the function that takes it.

Parity status: every public function here is pinned by `-m "not gpu"` tests in
tests/test_oracle_*.py against closed forms, library routines the oracle does
not call, brute force or the paper's theorems.
"""
import numpy as np

# ---------------------------------------------------------------------------
# Transform matrices (Section 2, definitions of F_n, C_n and M)
# ---------------------------------------------------------------------------


def dct_matrix(n):
    """Orthonormal DCT-II matrix C_n (Section 2, definition of C_{I3}).

    Entry (i, j), 1-based: sqrt((2 - delta_{i,1}) / n) cos((i-1)(2j-1) pi / (2n)).
    Reading: the Kronecker delta is delta_{i,1} (first row scaled by sqrt(1/n));
    the printed delta_{i,j} would not give the orthogonal matrix the text says C_n
    is.
    """
    C = np.empty((n, n), dtype=np.float64)
    for i in range(n):          # 0-based row: (i-1) of the paper
        scale = np.sqrt((1.0 if i == 0 else 2.0) / n)
        for j in range(n):      # 0-based column: (2j-1) of the paper is 2j+1 here
            C[i, j] = scale * np.cos(i * (2 * j + 1) * np.pi / (2.0 * n))
    return C


def dft_matrix(n):
    """Fourier matrix F_n = [w^{(i-1)(j-1)}], w = exp(-2 pi i / n), n x n
    (Section 2, t-product transform).  Reading: i, j run over 1..n (the printed
    range 1..n-1 would not give F_n F_n^* = n I)."""
    F = np.empty((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            F[i, j] = np.exp(-2j * np.pi * i * j / n)
    return F


def cprod_matrix(n):
    """c-product transform M = W^{-1} C (I + Z) (Section 2, eq. (m); Section 3.1
    definition of L): W = diag(C(:,1)), Z the upshift matrix with ones on the
    first superdiagonal."""
    C = dct_matrix(n)
    W = np.diag(C[:, 0])
    Z = np.diag(np.ones(n - 1), 1)
    return np.linalg.inv(W) @ C @ (np.eye(n) + Z)


# ---------------------------------------------------------------------------
# Mode products, slices, transform L (Section 2 eq. (3); Section 3.2)
# ---------------------------------------------------------------------------


def mode_product(X, U, mode):
    """n-mode product X x_n U (Section 2, eq. (3)); `mode` is 1-based.

    (X x_n U)[..., j, ...] = sum_{i_n} X[..., i_n, ...] U[j, i_n].
    """
    ax = mode - 1
    Y = np.tensordot(U, X, axes=([1], [ax]))   # new axis 0 is j
    return np.moveaxis(Y, 0, ax)


def transform(X, mats):
    """L(X) = X x_3 M_3 x_4 M_4 ... x_N M_N (Section 3.2).  mats[i] is the matrix
    for mode i+3, or None for the identity."""
    Y = X
    for i, M in enumerate(mats):
        if M is not None:
            Y = mode_product(Y, M, i + 3)
    return Y


def inverse_transform(Xh, mats):
    """L^{-1}(X^) = X^ x_N M_N^{-1} ... x_3 M_3^{-1} (Section 3.2)."""
    Y = Xh
    for i in reversed(range(len(mats))):
        M = mats[i]
        if M is not None:
            Y = mode_product(Y, np.linalg.inv(M), i + 3)
    return Y


def n_slices(shape):
    P = 1
    for d in shape[2:]:
        P *= d
    return P


def slices(X):
    """Frontal slices X^p in the paper's Vec order (eq. (3.5)): shape (P, I1, I2)."""
    I1, I2 = X.shape[0], X.shape[1]
    P = n_slices(X.shape)
    flat = X.reshape((I1, I2, P), order="F")
    return np.ascontiguousarray(np.moveaxis(flat, 2, 0))


def unslices(S, shape):
    """Inverse of `slices`."""
    I1, I2 = shape[0], shape[1]
    flat = np.moveaxis(S, 0, 2)
    return flat.reshape(tuple(shape), order="F")


def facewise(A, B):
    """Generalised face-wise product C^p = A^p B^p (Section 3.1 definition)."""
    SA, SB = slices(A), slices(B)
    SC = np.stack([SA[p] @ SB[p] for p in range(SA.shape[0])])
    shape = (A.shape[0], B.shape[1]) + tuple(A.shape[2:])
    return unslices(SC, shape)


def lproduct(A, B, mats):
    """A *_L B = L^{-1}(L(A) face-wise L(B)) (Section 3.2 definition; Alg. 2)."""
    return inverse_transform(facewise(transform(A, mats), transform(B, mats)), mats)


def ttranspose(A, mats):
    """Tensor transpose: L(A^T)^p = (L(A)^p)^T (Section 3.2 definition).
    Reading: for a complex transform the slice transpose is the conjugate
    transpose, so that a real tensor has a real transpose (for the DFT this is
    the t-product transpose)."""
    Ah = slices(transform(A, mats))
    T = np.stack([Ah[p].conj().T for p in range(Ah.shape[0])])
    shape = (A.shape[1], A.shape[0]) + tuple(A.shape[2:])
    return inverse_transform(unslices(T, shape), mats)


def identity_tensor(n, trailing, mats):
    """Identity tensor: L(I)^p = I_n for every p (Section 3.2 definition)."""
    P = 1
    for d in trailing:
        P *= d
    Ih = unslices(np.stack([np.eye(n) for _ in range(P)]), (n, n) + tuple(trailing))
    return inverse_transform(Ih, mats)


# ---------------------------------------------------------------------------
# Conjugate pairing of DFT slices (real input -> conjugate-symmetric slices)
# ---------------------------------------------------------------------------


def _conj_partner(p, trailing, kinds):
    """Slice index q such that L(X)^q = conj(L(X)^p) for real X when the modes
    listed as 'dft' in `kinds` use F and the others a real matrix."""
    ks = []
    rem = p
    for d in trailing:
        ks.append(rem % d)
        rem //= d
    q = 0
    stride = 1
    for k, d, kind in zip(ks, trailing, kinds):
        kk = (-k) % d if kind == "dft" else k
        q += kk * stride
        stride *= d
    return q


def _kinds(mats):
    return ["dft" if (M is not None and np.iscomplexobj(M)) else "real" for M in mats]


# ---------------------------------------------------------------------------
# *_L-SVD, SVT, norms, ranks (Section 3.2: Theorem tsvd1, Alg. 3, Alg. 4,
# Definition of D_tau, Theorem 23, nuclear norm eq. (24), multirank)
# ---------------------------------------------------------------------------


def lsvd(A, mats):
    """*_L-SVD (Alg. 3): per slice SVD of L(A)^p, then U = L^{-1}(U^),
    S = L^{-1}(S^), V = L^{-1}(V^).  Full factors: U is I1 x I1, V is I2 x I2.
    Singular values of every slice are sorted in descending order.  For a real
    input under the DFT the factors of conjugate-partner slices are taken as
    conjugates of each other, so U, S, V are real (up to rounding)."""
    I1, I2 = A.shape[0], A.shape[1]
    trailing = tuple(A.shape[2:])
    Ah = slices(transform(A, mats))
    P = Ah.shape[0]
    cplx = np.iscomplexobj(Ah)
    dt = np.complex128 if cplx else np.float64
    Uh = np.zeros((P, I1, I1), dtype=dt)
    Sh = np.zeros((P, I1, I2), dtype=dt)
    Vh = np.zeros((P, I2, I2), dtype=dt)
    kinds = _kinds(mats)
    real_input = not np.iscomplexobj(A)
    for p in range(P):
        q = _conj_partner(p, trailing, kinds) if (cplx and real_input) else p
        if q < p:
            Uh[p], Sh[p], Vh[p] = Uh[q].conj(), Sh[q].conj(), Vh[q].conj()
            continue
        Ap = Ah[p]
        if cplx and real_input and q == p:
            Ap = Ap.real
        U, s, Vt = np.linalg.svd(Ap, full_matrices=True)
        Uh[p] = U
        for i, si in enumerate(s):
            Sh[p, i, i] = si
        Vh[p] = Vt.conj().T
    U = inverse_transform(unslices(Uh, (I1, I1) + trailing), mats)
    S = inverse_transform(unslices(Sh, (I1, I2) + trailing), mats)
    V = inverse_transform(unslices(Vh, (I2, I2) + trailing), mats)
    if cplx and real_input:
        U, S, V = U.real, S.real, V.real
    return U, S, V


def singular_values(A, mats):
    """Singular values of every transform-domain slice, shape (P, min(I1, I2)),
    descending."""
    Ah = slices(transform(A, mats))
    return np.stack([np.linalg.svd(Ah[p], compute_uv=False) for p in range(Ah.shape[0])])


def svt(A, tau, mats):
    """Tensor singular value thresholding D_tau(A) (Section 3.2 definition of
    D_tau; Alg. 4): for every slice of L(A), sigma <- max(sigma - tau, 0) and
    rebuild; then L^{-1}.  The threshold is applied to the transform-domain
    singular values as is (for the orthonormal DCT alpha = 1)."""
    Ah = slices(transform(A, mats))
    P = Ah.shape[0]
    Dh = np.empty_like(Ah)
    for p in range(P):
        U, s, Vt = np.linalg.svd(Ah[p], full_matrices=False)
        s = np.maximum(s - tau, 0.0)
        Dh[p] = (U * s) @ Vt
    D = inverse_transform(unslices(Dh, A.shape), mats)
    if np.iscomplexobj(D) and not np.iscomplexobj(A):
        D = D.real
    return D


def truncate(A, k, mats):
    """Rank-k approximation A_k = U(:, 1:k) *_L S(1:k, 1:k) *_L V(:, 1:k)^T of
    the Eckart-Young theorem (Section 3.2): the best approximation of A by
    X *_L Y with X of k lateral slices; per slice of L(A), the k largest
    singular triplets, then L^{-1}."""
    Ah = slices(transform(A, mats))
    P = Ah.shape[0]
    Th = np.empty_like(Ah)
    for p in range(P):
        U, s, Vt = np.linalg.svd(Ah[p], full_matrices=False)
        kk = max(0, min(int(k), s.size))
        Th[p] = (U[:, :kk] * s[:kk]) @ Vt[:kk]
    T = inverse_transform(unslices(Th, A.shape), mats)
    if np.iscomplexobj(T) and not np.iscomplexobj(A):
        T = T.real
    return T


def svt_ranks(A, tau, mats):
    """Number of transform-domain singular values above tau, per slice: the rank
    of every slice of L(D_tau(A)) (multirank of the SVT result)."""
    s = singular_values(A, mats)
    return (s > tau).sum(axis=1)


def multirank(A, mats, rtol=1e-10):
    """Multirank rho_p = rank L(A)^p and average rank (Section 3.2 definition)."""
    s = singular_values(A, mats)
    smax = s.max() if s.size else 0.0
    rho = (s > rtol * max(smax, 1e-300)).sum(axis=1)
    return rho, rho.mean()


def transform_alpha(mats):
    """alpha of Section 3.2 for L = x_3 M_3 ... x_N M_N with M_i = alpha_i R_i,
    R_i unitary.  Reading: alpha = prod alpha_i^2, the factor with
    ||L(A)||_F^2 = alpha ||A||_F^2 (the printed alpha = prod alpha_i would not
    give the norm relation the section states); alpha_i^2 is read off
    M_i M_i^H = alpha_i^2 I.  Orthonormal DCT: 1; DFT of size n: n.  Raises
    ValueError for a matrix that is not a scaled unitary (the c-product's
    W^{-1} C (I + Z)), for which the section's norm relations do not hold."""
    alpha = 1.0
    for M in mats:
        if M is None:
            continue
        G = M @ M.conj().T
        a2 = float(np.real(np.trace(G))) / M.shape[0]
        if np.abs(G - a2 * np.eye(M.shape[0])).max() > 1e-10 * a2:
            raise ValueError("mode matrix is not a scaled unitary")
        alpha *= a2
    return alpha


def nuclear_norm(A, mats):
    """Tensor nuclear norm (Theorem 21, eq. (24)): (1/alpha) times the sum of
    the singular values of every transform-domain slice L(A)^p, alpha as in
    `transform_alpha`."""
    return singular_values(A, mats).sum() / transform_alpha(mats)


def fro(X):
    return float(np.sqrt(np.sum(np.abs(X) ** 2)))


# ---------------------------------------------------------------------------
# Block Toeplitz-plus-Hankel structure of the c-product (Section 3, eq. (3.22),
# the order-N construction, bdiag eq. (bd), eq. (20))
# ---------------------------------------------------------------------------


def _tph_pattern(n):
    """Index pattern of a Toeplitz-plus-Hankel matrix of a length-n sequence.
    Returns two integer arrays (T, H) of shape (n, n); entry -1 means zero.
    Toeplitz part: a_{|i-j|+1}.  Hankel part (1-based i, j): a_{i+j} when
    i+j <= n, 0 when i+j = n+1, a_{2n+2-i-j} when i+j > n+1 (reading of the
    anti-diagonal drawing in eq. (3.22))."""
    T = np.empty((n, n), dtype=np.int64)
    H = np.empty((n, n), dtype=np.int64)
    for i in range(n):
        for j in range(n):
            T[i, j] = abs(i - j)
            s = (i + 1) + (j + 1)
            if s <= n:
                H[i, j] = s - 1
            elif s == n + 1:
                H[i, j] = -1
            else:
                H[i, j] = 2 * n + 2 - s - 1
    return T, H


def btph(X):
    """Block Toeplitz-plus-Hankel matrix of an order-N tensor (eq. (3.22) for
    order 3; order N built from order N-1 blocks with the outer block level on
    mode N).  Size (I1 P) x (I2 P)."""
    if X.ndim == 2:
        return X.copy()
    n = X.shape[-1]
    blocks = [btph(X[..., k]) for k in range(n)]
    bh, bw = blocks[0].shape
    T, H = _tph_pattern(n)
    out = np.zeros((n * bh, n * bw), dtype=np.result_type(X.dtype, np.float64))
    for i in range(n):
        for j in range(n):
            blk = blocks[T[i, j]].copy()
            if H[i, j] >= 0:
                blk = blk + blocks[H[i, j]]
            out[i * bh:(i + 1) * bh, j * bw:(j + 1) * bw] = blk
    return out


def tph(a):
    """Toeplitz-plus-Hankel matrix of a tube (eq. (d))."""
    return btph(np.asarray(a, dtype=np.float64).reshape(1, 1, -1))


def bdiag(X):
    """Block-diagonal matrix of the frontal slices (eq. (bd))."""
    S = slices(X)
    P, I1, I2 = S.shape
    out = np.zeros((P * I1, P * I2), dtype=S.dtype)
    for p in range(P):
        out[p * I1:(p + 1) * I1, p * I2:(p + 1) * I2] = S[p]
    return out


# ---------------------------------------------------------------------------
# Tensor completion by the proximal gradient algorithm (Section 4: eqs.
# (48)-(53), Alg. 5; parameters and stopping rule of Section 5)
# ---------------------------------------------------------------------------


def pga_schedule(max_iter, mu0, nu, mu_bar, fixed_mu=None):
    """Scalars of Alg. 5 that depend on no data: for k = 1..max_iter, the
    momentum weight beta_k = (t_{k-1} - 1) / t_k of eq. (52) and the threshold
    mu_k used by the prox at iteration k.

    Readings: t_0 = t_1 = 1 (the printed t_0 = t_1 = 0 divides 0 by 0 at k = 1);
    t_{k+1} = (1 + sqrt(4 t_k^2 + 1)) / 2; iteration k uses mu_k with mu_1 = mu0
    and the update mu_{k+1} = max(nu mu_k, mu_bar) follows the prox.  With
    `fixed_mu` every iteration uses that threshold.
    """
    betas, mus = [], []
    t_prev, t = 1.0, 1.0
    mu = mu0
    for _ in range(max_iter):
        betas.append((t_prev - 1.0) / t)
        mus.append(fixed_mu if fixed_mu is not None else mu)
        t_prev, t = t, (1.0 + np.sqrt(4.0 * t * t + 1.0)) / 2.0
        mu = max(nu * mu, mu_bar)
    return np.array(betas), np.array(mus)


def pga_step(X, X_prev, M, mask, beta, mu, mats):
    """One iteration of Alg. 5.  Returns (X_next, Y).

    eq. (52): Y = X + beta (X - X_prev).
    eq. (51): G = Y - (P_Omega(Y) - P_Omega(M)) = P_{Omega^c}(Y) + P_Omega(M)
              (reading: the sign after the second equality is +, as the first
              equality gives), with step 1/l_f = 1.
    eq. (53): X_next = D_mu(G).
    """
    Y = X + beta * (X - X_prev)
    G = np.where(mask, M, Y)
    return svt(G, mu, mats), Y


def stop_criterion(Y, X_next):
    """||Y - X_next||_F / ||X_next||_F (Section 5).  Reading: infinite when
    X_next = 0, so that an all-zero iterate never counts as converged."""
    den = fro(X_next)
    if den == 0.0:
        return np.inf
    return fro(Y - X_next) / den


def complete_pga(M, mask, mats, mu0, nu=0.9, mu_bar=None, tol=0.0, max_iter=100,
                 fixed_mu=None, gate_until_floor=True, trace=None):
    """Tensor completion by PGA (Alg. 5), X^0 = X^1 = 0.

    Runs until the stopping rule of Section 5 holds (when tol > 0; with
    `gate_until_floor` only once mu_k has reached mu_bar) or max_iter
    iterations.  Returns (X, info) with info = dict(iters, crit, converged).
    Reading: mu_bar is an explicit parameter (the printed mu_bar = nu mu0 with
    mu0 = nu ||M||_F would keep X at zero); default 1e-4 mu0.
    """
    if mu_bar is None:
        mu_bar = 1e-4 * mu0
    betas, mus = pga_schedule(max_iter, mu0, nu, mu_bar, fixed_mu)
    X_prev = np.zeros(M.shape)
    X = np.zeros(M.shape)
    crit = np.inf
    iters = 0
    converged = False
    for k in range(max_iter):
        X_next, Y = pga_step(X, X_prev, M, mask, betas[k], mus[k], mats)
        crit = stop_criterion(Y, X_next)
        X_prev, X = X, X_next
        iters = k + 1
        if trace is not None:
            trace.append(crit)
        at_floor = (fixed_mu is not None) or (mus[k] <= mu_bar)
        if tol > 0 and crit <= tol and (at_floor or not gate_until_floor):
            converged = True
            break
    return X, dict(iters=iters, crit=crit, converged=converged)


# ---------------------------------------------------------------------------
# Quality metrics (Section 5)
# ---------------------------------------------------------------------------


def rse(X_obt, X_ori):
    """Relative error ||X_obt - X_ori||_F / ||X_ori||_F.  Reading: the printed
    squared ratio over ||X_obt|| does not reproduce the paper's PSNR/RSE pairs."""
    return fro(X_obt - X_ori) / fro(X_ori)


def psnr(X_obt, X_ori, peak=1.0):
    """PSNR = 10 log10(N_el peak^2 / ||X_obt - X_ori||_F^2) (Section 5; reading:
    the per-entry mean square error, peak 1 for data in [0, 1])."""
    err2 = fro(X_obt - X_ori) ** 2
    return 10.0 * np.log10(X_ori.size * peak * peak / err2)


# ---------------------------------------------------------------------------
# Convenience: transform lists from mode kinds
# ---------------------------------------------------------------------------


def mats_for(shape, kinds):
    """Build the mode matrices for modes 3..N.  kinds[i] in {'dct', 'dft',
    'identity', 'cprod'} or an explicit matrix."""
    mats = []
    for i, kind in enumerate(kinds):
        n = shape[i + 2]
        if isinstance(kind, np.ndarray):
            mats.append(np.asarray(kind))
        elif kind == "dct":
            mats.append(dct_matrix(n))
        elif kind == "dft":
            mats.append(dft_matrix(n))
        elif kind == "cprod":
            mats.append(cprod_matrix(n))
        elif kind == "identity":
            mats.append(None)
        else:
            raise ValueError(kind)
    return mats
