"""Thin ctypes binding of liblt.so (include/lt.h).

Argument marshalling only: every step of every operation runs in the HIP
kernels of liblt.so.  PyTorch provides device memory (tensors) and the stream
(torch.cuda.current_stream()).  Importing this module raises ImportError when
the built library is missing; there is no fallback.

Tensor convention: a tensor of logical shape (I1, I2, I3, ..., IN) is a float32
CUDA tensor in column-major (Fortran) order, i.e. strides (1, I1, I1*I2, ...).
`to_device` / `to_host` convert from and to NumPy arrays of that shape.
"""
import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LT_LIBRARY", os.path.join(_HERE, "liblt.so"))
if not os.path.exists(LIB_PATH):
    raise ImportError("liblt.so not built (%s); run python -m paper_2202_02870_amd.build" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

MAX_ORDER = 8
OK = 0
ERR_ARG, ERR_SHAPE, ERR_UNSUPPORTED, ERR_NONFINITE, ERR_HIP, ERR_WORKSPACE = -1, -2, -3, -4, -5, -6
WARN_MAXSWEEPS, WARN_NOT_CONVERGED = 1, 2
KIND = {"dct": 0, "dft": 1, "identity": 2, "custom": 3}
PREC = {"f32": 0, "bf16x3": 1}
OP = {"lproduct": 0, "lsvd": 1, "svt": 2, "pga": 3, "truncate": 4, "lsvd_full": 5}


class Desc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("kind", ctypes.c_int32 * MAX_ORDER),
                ("dims", ctypes.c_int64 * MAX_ORDER), ("custom", ctypes.c_void_p * MAX_ORDER)]


class SvdOpts(ctypes.Structure):
    _fields_ = [("jacobi_tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("no_precondition", ctypes.c_int32),
                ("warm_restart", ctypes.c_int32), ("fp32_dots", ctypes.c_int32)]


class PgaParams(ctypes.Structure):
    _fields_ = [("mu0", ctypes.c_double), ("nu", ctypes.c_double), ("mu_bar", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("gate_until_floor", ctypes.c_int32),
                ("fixed_mu", ctypes.c_int32), ("svd", SvdOpts), ("start_iter", ctypes.c_int32)]


class PgaReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("max_sweeps_hit", ctypes.c_int32), ("slowest_sweeps", ctypes.c_int32),
                ("last_crit", ctypes.c_double), ("total_sweeps", ctypes.c_int64),
                ("total_slices", ctypes.c_int64), ("total_rotations", ctypes.c_int64),
                ("nuclear_norm", ctypes.c_double)]


class ProblemC(ctypes.Structure):
    _fields_ = [("desc", ctypes.POINTER(Desc)), ("M", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("params", PgaParams), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t)]


PROF_CLASSES = ("forward", "jacobi", "rebuild", "inverse", "other", "precond")
SVT_PATHS = ("register", "precond", "blocked", "precond+blocked",   # LT_SVT_PRECOND / LT_SVT_BLOCKED bits
             None, None, "blocked+wide", "precond+blocked+wide",    # ... and LT_SVT_WIDE
             "complex", "precond+complex")                          # LT_SVT_COMPLEX (Fourier slices)


class Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64 * 6), ("ms", ctypes.c_double * 6), ("dropped", ctypes.c_int64)]


_vp = ctypes.c_void_p
_sig = {
    "lt_create": (ctypes.c_int, [ctypes.POINTER(_vp), _vp]),
    "lt_destroy": (ctypes.c_int, [_vp]),
    "lt_set_stream": (ctypes.c_int, [_vp, _vp]),
    "lt_last_error": (ctypes.c_char_p, [_vp]),
    "lt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lt_profile_begin": (ctypes.c_int, [_vp]),
    "lt_profile_end": (ctypes.c_int, [_vp, ctypes.POINTER(Profile)]),
    "lt_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Desc), ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_int]),
    "lt_lproduct": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, ctypes.POINTER(Desc), _vp, _vp,
                                   ctypes.c_int, _vp, ctypes.c_size_t]),
    "lt_lsvd": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(SvdOpts), _vp, ctypes.c_size_t]),
    "lt_multirank": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, ctypes.c_double, _vp,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(SvdOpts), _vp, ctypes.c_size_t]),
    "lt_svt_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(ctypes.POINTER(Desc)),
                                                         ctypes.POINTER(SvdOpts)]),
    "lt_svt_prox_batched": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.POINTER(Desc)),
                                           ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(SvdOpts),
                                           _vp, ctypes.c_size_t]),
    "lt_svt_path": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.POINTER(SvdOpts)]),
    "lt_pga_warm": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.POINTER(SvdOpts)]),
    "lt_ltruncate": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, ctypes.c_int32, _vp,
                                    ctypes.POINTER(SvdOpts), _vp, ctypes.c_size_t]),
    "lt_svt_prox": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, ctypes.c_double, _vp, _vp, _vp,
                                   ctypes.POINTER(SvdOpts), _vp, ctypes.c_size_t]),
    "lt_svt_prox_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, ctypes.c_double, _vp, _vp, _vp,
                                           ctypes.POINTER(SvdOpts)]),
    "lt_complete_pga": (ctypes.c_int, [_vp, ctypes.POINTER(Desc), _vp, _vp, ctypes.POINTER(PgaParams),
                                       _vp, ctypes.POINTER(PgaReport), _vp, ctypes.c_size_t]),
    "lt_problem_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Desc), ctypes.POINTER(PgaParams)]),
    "lt_problem_init": (ctypes.c_int, [_vp, ctypes.POINTER(ProblemC)]),
    "lt_problem_status": (ctypes.c_int, [_vp, ctypes.POINTER(ProblemC), ctypes.POINTER(PgaReport),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "lt_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(ProblemC)]),
    "lt_batch_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ProblemC), _vp, ctypes.c_size_t,
                                       ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    "lt_batch_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lt_batch_destroy": (ctypes.c_int, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class LtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_lib.lt_status_string(status).decode(), status, msg))
        self.status = status


_handles = {}


def _handle():
    dev = torch.cuda.current_device()
    h = _handles.get(dev)
    if h is None:
        h = _vp()
        st = _lib.lt_create(ctypes.byref(h), _vp(torch.cuda.current_stream().cuda_stream))
        if st != OK:
            raise LtError(st, "lt_create failed")
        _handles[dev] = h
    _lib.lt_set_stream(h, _vp(torch.cuda.current_stream().cuda_stream))
    return h


def _check(h, st, allow_warn=True):
    if st < 0 or (st > 0 and not allow_warn):
        raise LtError(st, _lib.lt_last_error(h).decode())
    return st


def make_desc(shape, kinds=None):
    """lt_desc for a tensor of shape (I1, I2, I3, ..., IN); kinds per trailing
    mode: 'dct' | 'identity' | 'dft' | a NumPy (Ii x Ii) matrix (custom).  The
    returned object keeps custom matrices alive."""
    shape = tuple(int(s) for s in shape)
    if kinds is None:
        kinds = ("dct",) * (len(shape) - 2)
    if len(kinds) != len(shape) - 2:
        raise ValueError("one kind per trailing mode")
    d = Desc()
    d.order = len(shape)
    keep = []
    for i, s in enumerate(shape):
        d.dims[i] = s
    for i, k in enumerate(kinds):
        if isinstance(k, np.ndarray):
            m = np.ascontiguousarray(k, dtype=np.float64)
            keep.append(m)
            d.kind[i + 2] = KIND["custom"]
            d.custom[i + 2] = m.ctypes.data
        else:
            d.kind[i + 2] = KIND[k]
    d._keep = keep
    return d


def fortran_empty(shape, dtype=torch.float32, device="cuda"):
    strides = []
    acc = 1
    for s in shape:
        strides.append(acc)
        acc *= int(s)
    return torch.empty_strided(tuple(int(s) for s in shape), tuple(strides), dtype=dtype, device=device)


def is_fortran(t):
    acc = 1
    for s, st in zip(t.shape, t.stride()):
        if s > 1 and st != acc:
            return False
        acc *= s
    return True


def to_device(a, dtype=torch.float32):
    a = np.asarray(a)
    t = fortran_empty(a.shape, dtype=dtype)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)).to(dtype))
    return t


def to_host(t):
    return t.detach().cpu().numpy()


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp()


def _check_tensor(t, shape, dtype=torch.float32, name="tensor"):
    if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not is_fortran(t):
        raise ValueError("%s must be a column-major %s CUDA tensor of shape %s" % (name, dtype, tuple(shape)))


def workspace_bytes(shape, kinds=None, op="svt", precision="f32", shape_b=None, kinds_b=None):
    da = make_desc(shape, kinds)
    db = make_desc(shape_b, kinds_b if kinds_b is not None else kinds) if shape_b is not None else None
    n = _lib.lt_workspace_bytes(ctypes.byref(da), ctypes.byref(db) if db is not None else None,
                                OP[op], PREC[precision])
    if n == 0:
        raise ValueError("invalid descriptor")
    return int(n)


def _workspace(nbytes, ws):
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small")
        return ws
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def svd_opts(jacobi_tol=0.0, max_sweeps=0, precision="f32", precondition=True, warm_restart=0,
             fp32_dots=False):
    """warm_restart (completion only): 0 a cold Jacobi start every 256 iterations,
    k > 0 every k, < 0 every iteration (no warm start).  fp32_dots: FP32 pair dot
    products in the Jacobi (default FP64)."""
    return SvdOpts(jacobi_tol, max_sweeps, PREC[precision], 0 if precondition else 1, int(warm_restart),
                   1 if fp32_dots else 0)


def ltruncate(A, k, kinds=None, jacobi_tol=0.0, max_sweeps=0, precision="f32", out=None, ws=None):
    """Rank-k approximation A_k = U(:, 1:k) *_L S(1:k, 1:k) *_L V(:, 1:k)^T
    (Eckart-Young theorem); out may be A."""
    shape = tuple(A.shape)
    _check_tensor(A, shape, name="A")
    d = make_desc(shape, kinds)
    Ak = out if out is not None else fortran_empty(shape)
    _check_tensor(Ak, shape, name="Ak")
    nb = workspace_bytes(shape, kinds, "truncate", precision)
    w = _workspace(nb, ws)
    h = _handle()
    o = svd_opts(jacobi_tol, max_sweeps, precision)
    _check(h, _lib.lt_ltruncate(h, ctypes.byref(d), _ptr(A), int(k), _ptr(Ak), ctypes.byref(o), _ptr(w), nb))
    return Ak


def multirank(A, kinds=None, rtol=1e-5, jacobi_tol=0.0, max_sweeps=0, precision="f32", ws=None):
    """lt_multirank: the rank of every slice of L(A) (singular values above rtol
    times the largest of the tensor) as an int32 CUDA tensor, the average rank
    and the tubal rank (slices up to 256 columns; Fourier modes through the
    complex Jacobi)."""
    shape = tuple(A.shape)
    _check_tensor(A, shape, name="A")
    d = make_desc(shape, kinds)
    P = int(np.prod(shape[2:])) if len(shape) > 2 else 1
    rank = torch.empty(P, dtype=torch.int32, device="cuda")
    nb = workspace_bytes(shape, kinds, "lsvd", precision)
    w = _workspace(nb, ws)
    h = _handle()
    o = svd_opts(jacobi_tol, max_sweeps, precision)
    avg = ctypes.c_double()
    tubal = ctypes.c_int32()
    _check(h, _lib.lt_multirank(h, ctypes.byref(d), _ptr(A), float(rtol), _ptr(rank), ctypes.byref(avg),
                                ctypes.byref(tubal), ctypes.byref(o), _ptr(w), nb))
    return rank, float(avg.value), int(tubal.value)


def svt_path(shape, kinds=None, precondition=True):
    """How the SVT of these slices runs: "register" (register-resident Jacobi
    on the slice), "precond" (on its Cholesky-QR factor), "blocked" (blocked
    Jacobi on the slice), "precond+blocked" (blocked, on the factor), and
    "blocked+wide" / "precond+blocked+wide" (the wide blocked Jacobi, one
    workgroup per block pair), "complex" / "precond+complex" (Fourier slices:
    the Hermitian Jacobi on the complex slices or on their complex Cholesky-QR
    factors; otherwise the real embeddings take one of the others); host only,
    LtError if no kernel takes the shape."""
    d = make_desc(tuple(shape), kinds)
    o = svd_opts(precondition=precondition)
    st = _lib.lt_svt_path(ctypes.byref(d), ctypes.byref(o))
    if st < 0:
        raise LtError(st, "no Jacobi kernel takes slices of %s" % (tuple(shape),))
    return SVT_PATHS[st]


def pga_warm(shape, kinds=None, precondition=True, warm_restart=0):
    """True if complete_pga warm-starts the Jacobi of these slices (host only)."""
    d = make_desc(tuple(shape), kinds)
    o = svd_opts(precondition=precondition, warm_restart=warm_restart)
    st = _lib.lt_pga_warm(ctypes.byref(d), ctypes.byref(o))
    if st < 0:
        raise LtError(st, "invalid shape %s" % (tuple(shape),))
    return st == 1


def svt_prox(A, tau, kinds=None, jacobi_tol=0.0, max_sweeps=0, precision="f32", out=None, ws=None,
             precondition=True, fp32_dots=False):
    """D_tau(A) (Alg. 4).  Returns (D, rank[P] int32, sweeps[P] int32)."""
    shape = tuple(A.shape)
    _check_tensor(A, shape, name="A")
    d = make_desc(shape, kinds)
    P = int(np.prod(shape[2:])) if len(shape) > 2 else 1
    D = out if out is not None else fortran_empty(shape)
    _check_tensor(D, shape, name="D")
    rank = torch.empty(P, dtype=torch.int32, device="cuda")
    sweeps = torch.empty(P, dtype=torch.int32, device="cuda")
    nb = workspace_bytes(shape, kinds, "svt", precision)
    w = _workspace(nb, ws)
    h = _handle()
    o = svd_opts(jacobi_tol, max_sweeps, precision, precondition, fp32_dots=fp32_dots)
    st = _lib.lt_svt_prox(h, ctypes.byref(d), _ptr(A), float(tau), _ptr(D), _ptr(rank), _ptr(sweeps),
                          ctypes.byref(o), _ptr(w), nb)
    _check(h, st)
    return D, rank, sweeps


def svt_prox_batched(As, taus, kinds=None, jacobi_tol=0.0, max_sweeps=0, precision="f32", outs=None,
                     precondition=True, fp32_dots=False):
    """lt_svt_prox_batched: D_i = D_{tau_i}(A_i) for a list of column-major
    tensors (shapes and orders may differ) in one pass of the batch engine.
    kinds: None (DCT on every trailing mode) or one kinds tuple per tensor.
    Returns (list of D_i, list of rank_i int32 tensors)."""
    n = len(As)
    if len(taus) != n:
        raise ValueError("one tau per tensor")
    kl = kinds if kinds is not None else [None] * n
    descs = [make_desc(tuple(A.shape), k) for A, k in zip(As, kl)]
    Ds = list(outs) if outs is not None else [fortran_empty(tuple(A.shape)) for A in As]
    ranks = []
    for A, D in zip(As, Ds):
        _check_tensor(A, tuple(A.shape), name="A")
        _check_tensor(D, tuple(A.shape), name="D")
        P = int(np.prod(A.shape[2:])) if A.dim() > 2 else 1
        ranks.append(torch.empty(P, dtype=torch.int32, device="cuda"))
    darr = (ctypes.POINTER(Desc) * n)(*[ctypes.pointer(d) for d in descs])
    aarr = (_vp * n)(*[A.data_ptr() for A in As])
    tarr = (ctypes.c_double * n)(*[float(t) for t in taus])
    oarr = (_vp * n)(*[D.data_ptr() for D in Ds])
    rarr = (_vp * n)(*[r.data_ptr() for r in ranks])
    o = svd_opts(jacobi_tol, max_sweeps, precision, precondition, fp32_dots=fp32_dots)
    nb = int(_lib.lt_svt_batched_workspace_bytes(n, darr, ctypes.byref(o)))
    if nb == 0:
        raise ValueError("a tensor of the batch is not supported by the batch engine")
    w = torch.empty(nb, dtype=torch.uint8, device="cuda")
    h = _handle()
    _check(h, _lib.lt_svt_prox_batched(h, n, darr, aarr, tarr, oarr, rarr, ctypes.byref(o), _ptr(w), nb))
    return Ds, ranks


NOALLOC_SCRATCH_BYTES = 64 << 20   # LT_NOALLOC_SCRATCH_BYTES


def svt_prox_noalloc(A, tau, D, rank=None, sweeps=None, kinds=None, jacobi_tol=0.0, max_sweeps=0,
                     precision="f32", precondition=True, fp32_dots=False):
    """lt_svt_prox_noalloc: D_tau(A) into the caller's D (and optional int32
    rank / sweeps tensors of P entries) with the library's static scratch as
    workspace; allocates nothing.  Returns the status."""
    shape = tuple(A.shape)
    _check_tensor(A, shape, name="A")
    _check_tensor(D, shape, name="D")
    d = make_desc(shape, kinds)
    h = _handle()
    o = svd_opts(jacobi_tol, max_sweeps, precision, precondition, fp32_dots=fp32_dots)
    return _check(h, _lib.lt_svt_prox_noalloc(h, ctypes.byref(d), _ptr(A), float(tau), _ptr(D), _ptr(rank),
                                              _ptr(sweeps), ctypes.byref(o)))


def lproduct(A, B, kinds=None, precision="f32", out=None, ws=None):
    """A *_L B (Alg. 2)."""
    sa, sb = tuple(A.shape), tuple(B.shape)
    _check_tensor(A, sa, name="A")
    _check_tensor(B, sb, name="B")
    da, db = make_desc(sa, kinds), make_desc(sb, kinds)
    sc = (sa[0], sb[1]) + sa[2:]
    C = out if out is not None else fortran_empty(sc)
    _check_tensor(C, sc, name="C")
    nb = workspace_bytes(sa, kinds, "lproduct", precision, shape_b=sb)
    w = _workspace(nb, ws)
    h = _handle()
    st = _lib.lt_lproduct(h, ctypes.byref(da), _ptr(A), ctypes.byref(db), _ptr(B), _ptr(C),
                          PREC[precision], _ptr(w), nb)
    _check(h, st)
    return C


def lsvd(A, kinds=None, transform_domain=False, jacobi_tol=0.0, max_sweeps=0, precision="f32", ws=None,
         economy=True):
    """*_L-SVD (Alg. 3): returns (U, S, V, sigma).  Economy: U: I1 x n x ...,
    S: n x n x ..., V: I2 x n x ...; full (economy=False): U: I1 x I1 x ...,
    S: I1 x I2 x ..., V: I2 x I2 x ....  sigma: P x n (transform domain,
    descending)."""
    shape = tuple(A.shape)
    _check_tensor(A, shape, name="A")
    d = make_desc(shape, kinds)
    I1, I2 = shape[0], shape[1]
    n = min(I1, I2)
    tr = shape[2:]
    P = int(np.prod(tr)) if tr else 1
    ku, kv, (sr, sc) = (n, n, (n, n)) if economy else (I1, I2, (I1, I2))
    U = fortran_empty((I1, ku) + tr)
    S = fortran_empty((sr, sc) + tr)
    V = fortran_empty((I2, kv) + tr)
    sig = torch.empty((P, n), dtype=torch.float32, device="cuda")
    nb = workspace_bytes(shape, kinds, "lsvd" if economy else "lsvd_full", precision)
    w = _workspace(nb, ws)
    h = _handle()
    o = svd_opts(jacobi_tol, max_sweeps, precision)
    st = _lib.lt_lsvd(h, ctypes.byref(d), _ptr(A), _ptr(U), _ptr(S), _ptr(V), _ptr(sig),
                      1 if economy else 0, 1 if transform_domain else 0, ctypes.byref(o), _ptr(w), nb)
    _check(h, st)
    return U, S, V, sig


def pga_params(mu0, nu=0.9, mu_bar=None, tol=0.0, max_iter=100, check_every=10,
               gate_until_floor=True, fixed_mu=False, jacobi_tol=0.0, max_sweeps=0, precision="f32",
               precondition=True, warm_restart=0, fp32_dots=False, start_iter=0):
    """start_iter > 0 (complete_pga only): continue the run that the previous
    call with the same workspace and output tensor ended at that iteration."""
    if mu_bar is None:
        mu_bar = 1e-4 * mu0
    return PgaParams(float(mu0), float(nu), float(mu_bar), float(tol), int(max_iter), int(check_every),
                     1 if gate_until_floor else 0, 1 if fixed_mu else 0,
                     svd_opts(jacobi_tol, max_sweeps, precision, precondition, warm_restart, fp32_dots),
                     int(start_iter))


def complete_pga(M, mask, params, kinds=None, out=None, ws=None):
    """Completion by PGA (Alg. 5).  mask: uint8 CUDA tensor (same layout).
    Returns (X, report dict, status)."""
    shape = tuple(M.shape)
    _check_tensor(M, shape, name="M")
    _check_tensor(mask, shape, dtype=torch.uint8, name="mask")
    d = make_desc(shape, kinds)
    prec = {v: k for k, v in PREC.items()}[params.svd.precision]
    X = out if out is not None else fortran_empty(shape)
    _check_tensor(X, shape, name="X")
    nb = workspace_bytes(shape, kinds, "pga", prec)
    w = _workspace(nb, ws)
    h = _handle()
    rep = PgaReport()
    st = _lib.lt_complete_pga(h, ctypes.byref(d), _ptr(M), _ptr(mask), ctypes.byref(params), _ptr(X),
                              ctypes.byref(rep), _ptr(w), nb)
    _check(h, st)
    return X, _report(rep), st


def profile_begin():
    """Start timing every kernel launch of this device's handle (HIP events on
    the current stream)."""
    h = _handle()
    _check(h, _lib.lt_profile_begin(h))


def profile_end():
    """Stop timing; returns {class: (calls, total_ms)} and the dropped count."""
    h = _handle()
    pr = Profile()
    _check(h, _lib.lt_profile_end(h, ctypes.byref(pr)))
    return {c: (int(pr.calls[i]), float(pr.ms[i])) for i, c in enumerate(PROF_CLASSES)}, int(pr.dropped)


# ---------------------------------------------------------------------------
# Batched completion engine
# ---------------------------------------------------------------------------


def _report(rep):
    return dict(iters=rep.iters, converged=bool(rep.converged), max_sweeps_hit=rep.max_sweeps_hit,
                last_crit=rep.last_crit, total_sweeps=rep.total_sweeps, total_slices=rep.total_slices,
                total_rotations=rep.total_rotations, nuclear_norm=rep.nuclear_norm,
                slowest_sweeps=rep.slowest_sweeps)


class Problem:
    """One completion problem of the batch engine: owns its device iterate,
    workspace and descriptor.  M and mask are column-major CUDA tensors (float32,
    uint8) that must stay alive while the problem runs."""

    def __init__(self, M, mask, params, kinds=None, out=None):
        shape = tuple(M.shape)
        _check_tensor(M, shape, name="M")
        _check_tensor(mask, shape, dtype=torch.uint8, name="mask")
        self.shape = shape
        self.desc = make_desc(shape, kinds)
        self.params = params
        self.M, self.mask = M, mask
        self.X = out if out is not None else fortran_empty(shape)
        _check_tensor(self.X, shape, name="X")
        nb = _lib.lt_problem_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(params))
        if nb == 0:
            raise ValueError("invalid problem")
        self.ws_bytes = int(nb)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.c = ProblemC(ctypes.pointer(self.desc), _ptr(M), _ptr(mask), _ptr(self.X), params,
                          _ptr(self.ws), self.ws_bytes)
        self.reset()

    def reset(self):
        """(Re)initialise: X^0 = X^1 = 0, iteration 0."""
        h = _handle()
        _check(h, _lib.lt_problem_init(h, ctypes.byref(self.c)))

    @property
    def nbytes(self):
        """Device bytes this problem holds (M, mask, X and workspace)."""
        n = int(np.prod(self.shape))
        return 4 * n + n + 4 * n + self.ws_bytes

    def status(self):
        """(report, done) -- synchronises; once done the result is in self.X."""
        h = _handle()
        rep = PgaReport()
        done = ctypes.c_int32()
        _check(h, _lib.lt_problem_status(h, ctypes.byref(self.c), ctypes.byref(rep), ctypes.byref(done)))
        return _report(rep), int(done.value)


class Batch:
    """Work tables of a set of initialised problems; step(k) enqueues k ticks
    (one PGA iteration of every unfinished problem per tick)."""

    def __init__(self, problems, use_graph=True, jacobi_lanes=0):
        """jacobi_lanes: lanes per column pair of the Jacobi kernel (0 = built-in
        choice, "auto" = timed choice of paper_2202_02870_amd.autotune)."""
        self.problems = list(problems)
        n = len(self.problems)
        if jacobi_lanes == "auto":
            from . import autotune
            jacobi_lanes, _ = autotune.tune([p.shape for p in self.problems])
        self.jacobi_lanes = int(jacobi_lanes)
        arr = (ProblemC * n)(*[p.c for p in self.problems])
        self._arr = arr
        nb = _lib.lt_batch_workspace_bytes(n, arr)
        if nb == 0:
            raise ValueError("invalid batch")
        self.ws = torch.empty(int(nb), dtype=torch.uint8, device="cuda")
        h = _handle()
        self.b = _vp()
        _check(h, _lib.lt_batch_create(h, n, arr, _ptr(self.ws), int(nb), 1 if use_graph else 0,
                                       int(jacobi_lanes), ctypes.byref(self.b)))

    def step(self, ticks=1):
        h = _handle()
        _check(h, _lib.lt_batch_step(self.b, int(ticks)))

    def close(self):
        if self.b:
            _lib.lt_batch_destroy(self.b)
            self.b = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
