"""Seeded synthetic completion workloads (inputs only).

Stand-ins for the paper's colour videos (Section 5, Tables 2 and 9), which are
not available: tensors in [0, 1] of prescribed low L-rank, shaped like the
paper's 144x176x3xF videos, with a uniform Bernoulli observation mask.

This module draws random numbers and assembles inputs; it holds none of the
completion arithmetic (no SVD, thresholding, momentum or transform matrices of
the library or of the oracle).  A tensor of prescribed L-rank is assembled as
A *_L B from random factors; that one product is done with SciPy's orthonormal
DCT-II (`scipy.fft.dctn` / `idctn`), its FFT for Fourier modes, and a per-slice
matmul, library routines that neither the oracle nor the HIP library uses.

Draw order for one problem: factor A, factor B, noise, mask (all float64 from
`numpy.random.default_rng(seed)`, PCG64).
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft


@dataclass
class Problem:
    X_true: np.ndarray          # float64, shape (I1, I2, I3, ..., IN)
    M: np.ndarray               # float64 observed tensor (X_true plus noise)
    mask: np.ndarray            # bool, True where observed
    kinds: tuple                # transform kind per trailing mode ('dct' / 'identity')
    name: str = ""
    schedule: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.X_true.shape


def _dct_axes(kinds):
    return [i + 2 for i, k in enumerate(kinds) if k == "dct"]


def _dft_axes(kinds):
    return [i + 2 for i, k in enumerate(kinds) if k == "dft"]


def _low_lrank(A, B, kinds):
    """A *_L B for L = orthonormal DCT-II along the modes marked 'dct' and the
    DFT along those marked 'dft' (identity elsewhere), via SciPy's DCT / FFT and
    per-slice matmul; real part (exact for real factors)."""
    dct, dft = _dct_axes(kinds), _dft_axes(kinds)

    def fwd(X):
        X = sfft.dctn(X, type=2, norm="ortho", axes=dct) if dct else X
        return sfft.fftn(X, axes=dft) if dft else X

    Ch = np.einsum("ik...,kj...->ij...", fwd(A), fwd(B))
    C = sfft.ifftn(Ch, axes=dft) if dft else Ch
    C = sfft.idctn(C.real if dft else C, type=2, norm="ortho", axes=dct) if dct else C
    return np.real(C)


def make_problem(shape, rank, observed, seed, kinds=None, dist="uniform",
                 rescale=True, noise_var=0.0, name=""):
    """One completion problem.

    shape: (I1, I2, I3, ..., IN); rank: inner dimension of A (I1 x r x ...) and
    B (r x I2 x ...); observed: Bernoulli probability of each entry being in
    Omega; dist: 'uniform' (U[0,1]) or 'normal' (N(0,1)) factors; rescale: map
    the product to [0, 1] by min-max; noise_var: variance of i.i.d. Gaussian
    noise added to the observed tensor M.
    """
    shape = tuple(int(s) for s in shape)
    if kinds is None:
        kinds = ("dct",) * (len(shape) - 2)
    rng = np.random.default_rng(seed)
    trailing = shape[2:]
    a_shape = (shape[0], rank) + trailing
    b_shape = (rank, shape[1]) + trailing
    if dist == "uniform":
        A = rng.random(a_shape)
        B = rng.random(b_shape)
    elif dist == "normal":
        A = rng.standard_normal(a_shape)
        B = rng.standard_normal(b_shape)
    else:
        raise ValueError(dist)
    X = _low_lrank(A, B, kinds)
    if rescale:
        lo, hi = X.min(), X.max()
        X = (X - lo) / (hi - lo)
    noise = rng.standard_normal(shape) * np.sqrt(noise_var) if noise_var > 0 else None
    mask = rng.random(shape) < observed
    M = X + noise if noise is not None else X.copy()
    return Problem(X_true=X, M=M, mask=mask, kinds=tuple(kinds), name=name)


# ---------------------------------------------------------------------------
# The benchmark configurations
# ---------------------------------------------------------------------------


def pga_schedule_params(M, mask, nu=0.9, floor_ratio=1e-4):
    """mu0 = nu ||P_Omega(M)||_F, mu_bar = floor_ratio mu0 (continuation
    parameters of the completion runs)."""
    mu0 = nu * float(np.sqrt(np.sum(np.where(mask, M, 0.0) ** 2)))
    return dict(mu0=mu0, nu=nu, mu_bar=floor_ratio * mu0)


def config0():
    """Order-3 plain completion: 32x32x8 = A *_L B, A 32x3x8, B 3x32x8 ~ N(0,1),
    DCT along mode 3, 50% observed; fixed threshold 0.1 ||X||_F / sqrt(8192);
    100 iterations."""
    p = make_problem((32, 32, 8), 3, 0.5, seed=0, dist="normal", rescale=False,
                     name="order3-32x32x8-r3-obs0.5")
    tau = 0.1 * float(np.sqrt(np.sum(p.X_true ** 2))) / np.sqrt(p.X_true.size)
    p.schedule = dict(fixed_mu=tau, mu0=tau, nu=1.0, mu_bar=tau, max_iter=100, tol=0.0)
    return p


def config1(trailing=(3, 50), transform="dct"):
    """Order-4 video-shaped completion: 144x176x3x50 of L-rank 10 (DCT along
    modes 3 and 4; transform="dft": the DFT, the t-product form), factors
    U[0,1], rescaled to [0,1], 30% observed; 200 iterations with continuation
    mu0 = 0.9 ||P_Omega M||, nu = 0.9, mu_bar = 1e-4 mu0."""
    kinds = (transform,) * len(trailing)
    p = make_problem((144, 176) + tuple(trailing), 10, 0.3, seed=1, kinds=kinds,
                     name="video-144x176x%s-r10-obs0.3%s" % ("x".join(map(str, trailing)),
                                                             "" if transform == "dct" else "-" + transform))
    p.schedule = dict(pga_schedule_params(p.M, p.mask), max_iter=200, tol=0.0)
    return p


def config2(trailing=(3, 100)):
    """Order-4 larger completion: 256x256x3x100 of L-rank 20 plus N(0, 1e-3)
    noise (variance), 20% observed; 300 iterations."""
    p = make_problem((256, 256) + tuple(trailing), 20, 0.2, seed=2, noise_var=1e-3,
                     name="large-256x256x%s-r20-obs0.2" % "x".join(map(str, trailing)))
    p.schedule = dict(pga_schedule_params(p.M, p.mask), max_iter=300, tol=0.0)
    return p


def config3_specs(n=64, seed=3):
    """Shapes of the batched uneven mix: per problem, order 3 or 4 by a fair
    coin, I1, I2 from {32,64,96,128,192,256}, I3 from {3,8,16}, I4 from
    {1,10,30} when order 4, L-rank in [2,16] clipped to min(I1,I2), observed
    fraction U[0.15,0.60].  Returns a list of dicts (with a child seed each)."""
    children = np.random.SeedSequence(seed).spawn(n)
    sizes = [32, 64, 96, 128, 192, 256]
    specs = []
    for i, child in enumerate(children):
        rng = np.random.default_rng(child)
        order = 4 if rng.random() < 0.5 else 3
        I1 = int(rng.choice(sizes))
        I2 = int(rng.choice(sizes))
        I3 = int(rng.choice([3, 8, 16]))
        trailing = (I3,) if order == 3 else (I3, int(rng.choice([1, 10, 30])))
        r = int(min(rng.integers(2, 17), min(I1, I2)))
        f = float(rng.uniform(0.15, 0.60))
        specs.append(dict(shape=(I1, I2) + trailing, rank=r, observed=f,
                          seed=int(rng.integers(0, 2**31 - 1)), index=i))
    return specs


def config3(n=64, seed=3, max_iter=100):
    probs = []
    for s in config3_specs(n, seed):
        p = make_problem(s["shape"], s["rank"], s["observed"], s["seed"],
                         name="mix%02d-%s" % (s["index"], "x".join(map(str, s["shape"]))))
        p.schedule = dict(pga_schedule_params(p.M, p.mask), max_iter=max_iter, tol=0.0)
        probs.append(p)
    return probs


FRAME_SHAPES = {1080: (1080, 1920), 2160: (2160, 3840)}


def config_frames(height=1080, frames=2, rank=10, observed=0.1, seed=6):
    """Large-frame completion: height x width x 3 x frames of L-rank `rank`
    (DCT along modes 3 and 4), factors U[0,1] rescaled to [0,1], `observed`
    fraction observed (Table 9's 1080 x 1920 and 2160 x 3840 colour frames;
    sr 0.1 as in the GPU experiments); continuation schedule as the video
    workload.  Frontal slices are 1080 x 1920 or 2160 x 3840."""
    I1, I2 = FRAME_SHAPES[height]
    p = make_problem((I1, I2, 3, frames), rank, observed, seed=seed,
                     name="frames-%dx%dx3x%d-r%d-obs%g" % (I1, I2, frames, rank, observed))
    p.schedule = dict(pga_schedule_params(p.M, p.mask), max_iter=100, tol=0.0)
    return p


LARGE_REQUEST_SHAPE = (512, 512, 3, 64)


def config4_specs(n=200, seed=4, large_frac=0.1):
    """Requests of the served stream: the uneven-mix distribution of
    config3_specs, except that a request is, with probability large_frac, a
    512x512x3x64 tensor (192 frontal slices of 512 x 512; L-rank and observed
    fraction drawn as for the mix).  Same dict layout as config3_specs."""
    specs = config3_specs(n, seed)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 512]))
    for sp in specs:
        big = rng.random() < large_frac
        r = int(rng.integers(2, 17))
        f = float(rng.uniform(0.15, 0.60))
        if big:
            sp.update(shape=LARGE_REQUEST_SHAPE, rank=r, observed=f)
    return specs


def config4_large():
    """One large request of the served stream on its own: 512x512x3x64 of
    L-rank 10, factors U[0,1], rescaled to [0,1], 30% observed, continuation
    schedule as the video workload."""
    p = make_problem(LARGE_REQUEST_SHAPE, 10, 0.3, seed=5, name="large-request-512x512x3x64-r10-obs0.3")
    p.schedule = dict(pga_schedule_params(p.M, p.mask), max_iter=500, tol=0.0)
    return p


def n_slices(shape):
    P = 1
    for d in shape[2:]:
        P *= d
    return P
