/*
 * lt.h -- C-ABI of the MI355X (gfx950) *_L-product tensor-completion library.
 *
 * Operations follow Bentbib, Elalj, El Hachimi, Jbilou, Ratnani, "Generalized
 * L-product for high order tensors with applications using GPU computations"
 * (arXiv 2202.02870):
 *   lt_lproduct      A *_L B                       (Section 3.2, Alg. 2)
 *   lt_lsvd          *_L-SVD  A = U *_L S *_L V^T  (Section 3.2 theorem, Alg. 3)
 *   lt_svt_prox      D_tau(A), the prox of tau ||.||_* (Theorem 23, Alg. 4)
 *   lt_complete_pga  completion by PGA             (Section 4, eqs. (48)-(53), Alg. 5)
 *
 * Tensors.  A tensor of order N (2 <= N <= LT_MAX_ORDER) with dims I1..IN is a
 * float32 array in column-major (first-index-fastest) order over
 * (i1, i2, i3, ..., iN).  Frontal slice p -- the paper's representative matrix
 * X^p of eq. (3.5), p the column-major index of (i3, ..., iN) -- therefore
 * starts at element p*I1*I2 and is an I1 x I2 column-major matrix with leading
 * dimension I1.  (A C-contiguous array of shape (IN, ..., I3, I2, I1) has this
 * layout.)  The transform L multiplies mode i (i = 3..N) by the matrix M_i
 * selected by lt_desc.kind[i-1] (Section 3.2: L(A) = A x_3 M_3 ... x_N M_N).
 *
 * Memory and streams.  Every tensor pointer argument is a DEVICE pointer owned
 * by the caller; the library never frees or retains it.  `ws` is a device
 * workspace of at least lt_workspace_bytes(...) bytes, owned by the caller.
 * No call allocates device memory.  All calls are asynchronous on the handle's
 * stream unless stated otherwise; results are ready once that stream is
 * synchronised.  A handle must not be used from two threads at once.
 *
 * Errors.  Every function returns an int status: 0 on success, a negative
 * LT_ERR_* code on failure (nothing has been launched, outputs untouched unless
 * stated), a positive LT_WARN_* code when results were produced with a caveat.
 * lt_last_error(h) returns a message for the last failure on that handle.  No
 * C++ exception crosses this interface.
 */
#ifndef LT_H
#define LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LT_MAX_ORDER 8

/* ---- status codes ------------------------------------------------------ */
#define LT_OK 0
#define LT_ERR_ARG (-1)          /* null pointer, bad enum or parameter value */
#define LT_ERR_SHAPE (-2)        /* dims inconsistent or beyond a kernel's limits */
#define LT_ERR_UNSUPPORTED (-3)  /* valid request this GPU library does not run */
#define LT_ERR_NONFINITE (-4)    /* NaN or Inf found in an input that is checked */
#define LT_ERR_HIP (-5)          /* a HIP runtime call failed */
#define LT_ERR_WORKSPACE (-6)    /* ws is NULL or smaller than lt_workspace_bytes */
#define LT_WARN_MAXSWEEPS 1      /* some slice SVD stopped at max_sweeps */
#define LT_WARN_NOT_CONVERGED 2  /* PGA reached max_iter with tol > 0 unmet */

/* ---- transform kinds (one per trailing mode) ----------------------------- */
typedef enum {
  LT_DCT = 0,       /* orthonormal DCT-II C_n (Section 2; the transform of TNN-PGA-C) */
  LT_DFT = 1,       /* Fourier matrix F_n (Section 2); complex transform-domain slices, taken by
                       lt_lproduct, lt_svt_prox and lt_complete_pga (FP32 transforms) */
  LT_IDENTITY = 2,  /* M_i = I (mode i not transformed) */
  LT_CUSTOM = 3     /* caller-given invertible M_i (e.g. the c-product W^{-1} C (I+Z)) */
} lt_mode_kind;

/* Transform precision of the L / L^{-1} GEMMs. */
typedef enum {
  LT_PREC_F32 = 0,     /* FP32 MFMA, FP32 accumulate */
  LT_PREC_BF16X3 = 1   /* BF16 MFMA on hi/lo splits of both operands
                          (hi*hi + hi*lo + lo*hi), FP32 accumulate */
} lt_precision;

/* Operations, for lt_workspace_bytes. */
typedef enum { LT_OP_LPRODUCT = 0, LT_OP_LSVD = 1, LT_OP_SVT = 2, LT_OP_PGA = 3,
               LT_OP_TRUNCATE = 4, LT_OP_LSVD_FULL = 5 } lt_op;
/* LT_OP_LSVD: lt_lsvd with economy != 0 and lt_multirank; LT_OP_LSVD_FULL:
 * lt_lsvd with economy == 0. */

/* Tensor shape and transform.  Host struct, read during the call only. */
typedef struct {
  int32_t order;                        /* N, 2..LT_MAX_ORDER (N = 2: one slice, no transform) */
  int32_t kind[LT_MAX_ORDER];           /* kind[i-1] is the lt_mode_kind of mode i, i = 3..N */
  int64_t dims[LT_MAX_ORDER];           /* dims[i-1] = I_i >= 1 */
  const double* custom[LT_MAX_ORDER];   /* HOST pointer, row-major I_i x I_i matrix, read when
                                           kind[i-1] == LT_CUSTOM; must be invertible */
} lt_desc;

/* One-sided Jacobi SVD options (Alg. 3 / Alg. 4 per-slice SVD). */
typedef struct {
  double jacobi_tol;    /* a column pair is rotated while |a_i.a_j| > tol ||a_i|| ||a_j||;
                           <= 0 selects 1e-7 */
  int32_t max_sweeps;   /* sweep limit per slice; <= 0 selects 40 */
  int32_t precision;    /* lt_precision of the transform GEMMs */
  int32_t no_precondition; /* SVT paths: 0 runs the Jacobi on the Cholesky-QR factor R^T of
                              each slice with 2 <= n <= 200 (n = min(I1, I2)), and with
                              any larger n where the slice itself would need the blocked
                              or the wide kernel (fewer sweeps, same result to the Jacobi
                              tolerance); nonzero runs it on the slice itself.  lt_lsvd
                              always uses the slice itself. */
  int32_t warm_restart; /* lt_complete_pga on preconditioned slices of real transforms held by
                           the register-resident kernel: the Jacobi of iteration k runs on
                           L Z, Z the rotations accumulated since the last cold start
                           (Z = I), which its columns leave nearly orthogonal (fewer
                           sweeps, same result to the Jacobi tolerance).  0: a cold start
                           every 256 iterations; k > 0: every k; < 0: every iteration (no
                           warm start).  Ignored by the other entry points. */
  int32_t fp32_dots;    /* 0 (default): the column-pair dot products that decide each rotation
                           are formed in FP64 (exact products of the FP32 columns, FP64 sums),
                           as are the column norms and the rotation angle; the columns are
                           rotated in FP32.  Nonzero: the pair dot products use FP32 products
                           and per-lane FP32 sums (FP64 across lanes) -- faster, with a
                           rounding error of about 1e-6 of |a_i| |a_j|, above the
                           default tolerance: the rotate-or-skip decision near it is
                           then decided by rounding. */
} lt_svd_opts;

/* Largest min(I1, I2) the one-workgroup preconditioned paths take (the
 * per-slice FP64 Cholesky runs in LDS up to n = 200, in global memory up to
 * 512); beyond it the wide path factors each slice's Gram matrix by a
 * multi-launch blocked Cholesky, up to 2304 columns. */
#define LT_PRECOND_MAX_N 512

/* Jacobi kernels of the per-slice SVD (Alg. 3 / Alg. 4), chosen by slice shape
 * (m = max(I1, I2), n = min(I1, I2)).  The Jacobi's working matrix is the
 * slice (m x n) or, with LT_SVT_PRECOND set, the slice's n x n Cholesky-QR
 * factor (see no_precondition).  It runs
 *   register-resident (LT_SVT_BLOCKED clear): its columns held in one
 *                    workgroup's registers (n <= 256 and ceil(n/2) column pairs
 *                    of G lanes holding all rows at 32 rows per lane, G <= 64,
 *                    ceil(n/2) G <= 1024);
 *   blocked (LT_SVT_BLOCKED set): the other working matrices with n <= 512 and
 *                    at most 2048 rows: columns in a per-slice working buffer of
 *                    the workspace, swept block pair by block pair by one
 *                    workgroup per slice (a much longer kernel);
 *   wide (LT_SVT_BLOCKED and LT_SVT_WIDE set): the blocked layout with one
 *                    workgroup per block pair and one launch per block round,
 *                    and one host synchronisation per sweep, up to 2304 columns
 *                    (preconditioned: the factor is n x n; otherwise also at most
 *                    2304 rows; the 1080 x 1920 and 2160 x 3840 video frames).
 *                    lt_svt_prox and lt_complete_pga run every working matrix
 *                    the register-resident kernel cannot hold through it; the
 *                    batch engine (graph-captured ticks) uses the one-workgroup
 *                    blocked kernel up to 512 columns and refuses wider slices.
 * Larger slices are LT_ERR_SHAPE.  lt_lsvd runs the register kernel only.
 * Fourier slices (complex, one per conjugate pair, Section 2's t-SVD of the
 * DFT) take
 *   complex (LT_SVT_COMPLEX): a one-sided Jacobi with Hermitian rotations (the
 *                    pair's a^H b and the angle in FP64), register-resident, on
 *                    complex columns held as interleaved (Re, Im) real rows:
 *                    with LT_SVT_PRECOND also set (preconditioning requested,
 *                    2 <= n, 2n <= LT_PRECOND_MAX_N) on the n x n complex
 *                    Cholesky-QR factor (2n rows), taken from the real Cholesky
 *                    factor of the real form [w_1, i w_1, ...] of the slice;
 *                    otherwise on the m x n slice (2m rows).  It needs
 *                    ceil(n/2) G <= 768 with G = 16 or 8 lanes per pair, at
 *                    most 48 rows per lane and its exchange buffer within the
 *                    LDS (e.g. the 144 x 176 video slices: G = 8, 36 rows per
 *                    lane on the factor, 44 on the slice);
 *   otherwise the kernels above on the real embedding [[X, -Y], [Y, X]]
 *                    (2 I1 x 2 I2; also with LT_DFT_EMBED=1 in the
 *                    environment).
 * lt_svt_path reports the single-problem calls' choice. */
#define LT_SVT_REGISTER 0
#define LT_SVT_PRECOND 1   /* bit */
#define LT_SVT_BLOCKED 2   /* bit */
#define LT_SVT_WIDE 4      /* bit (with LT_SVT_BLOCKED): the wide blocked Jacobi, see above */
#define LT_SVT_COMPLEX 8   /* the complex Hermitian Jacobi of Fourier slices (with LT_SVT_PRECOND: on the
                              complex Cholesky-QR factor), see above */

/* Parameters of Alg. 5 (values used in the paper's Section 5: nu = 0.9,
 * mu0 = nu ||M||_F, tol = 1e-4, itermax 100). */
typedef struct {
  double mu0;             /* threshold of the first iteration, > 0 */
  double nu;              /* continuation factor, 0 < nu <= 1: mu_{k+1} = max(nu mu_k, mu_bar) */
  double mu_bar;          /* threshold floor, 0 < mu_bar <= mu0 */
  double tol;             /* stop when ||Y^k - X^{k+1}||_F / ||X^{k+1}||_F <= tol; <= 0: never */
  int32_t max_iter;       /* iteration limit, >= 1 */
  int32_t check_every;    /* the stopping test syncs the host every this many iterations (>= 1) */
  int32_t gate_until_floor; /* nonzero: the test may stop the run only once mu_k == mu_bar */
  int32_t fixed_mu;       /* nonzero: every iteration thresholds at mu0 */
  lt_svd_opts svd;
  int32_t start_iter;     /* lt_complete_pga: 0 starts from X^0 = X^1 = 0; k0 > 0 continues a run
                             that the previous call on the same workspace (same descriptor and
                             parameters apart from max_iter and start_iter) ended at iteration
                             k0: X holds X^k0 and the workspace X^(k0-1) and the accumulated
                             rotations; the call then runs iterations k0 + 1 .. k0 + max_iter
                             with the schedule's t_k and mu_k.  The batch engine ignores it. */
} lt_pga_params;

typedef struct {
  int32_t iters;          /* iterations performed */
  int32_t converged;      /* 1 if the stopping rule fired */
  int32_t max_sweeps_hit; /* number of slice SVDs that stopped at max_sweeps */
  int32_t slowest_sweeps; /* lt_complete_pga: the largest sweep count among the slices of each
                             iteration, summed over the iterations (the slices run side by
                             side, so a Jacobi launch lasts as long as its slowest slice);
                             0 from lt_problem_status */
  double last_crit;       /* last evaluated stopping ratio (inf if X = 0; NaN if never evaluated) */
  int64_t total_sweeps;   /* Jacobi sweeps summed over all slices and iterations */
  int64_t total_slices;   /* slice SVDs performed (iters x P) */
  int64_t total_rotations; /* column-pair rotations applied, summed likewise */
  double nuclear_norm;    /* tensor nuclear norm of the returned iterate (Theorem 21, eq. (24)):
                             (1/alpha) x the sum of the singular values of its transform-domain
                             slices, here the last prox's sigma_i - mu_k over the kept ones
                             (alpha = 1 for DCT and identity modes, x I_i per Fourier mode);
                             NaN with custom mode matrices or before any iteration */
} lt_pga_report;

/* Kernel timing, recorded with HIP events on the handle's stream around every
 * kernel launch of the classes below while profiling is on. */
#define LT_PROF_FORWARD 0   /* L: transform GEMM (with the fused momentum/mask step in PGA) */
#define LT_PROF_JACOBI 1    /* per-slice one-sided Jacobi SVD + threshold */
#define LT_PROF_REBUILD 2   /* rank-r rebuild of the thresholded slices */
#define LT_PROF_INVERSE 3   /* L^{-1}: transform GEMM (with the fused stopping norms in PGA) */
#define LT_PROF_OTHER 4     /* small reductions, transform-matrix builds, face-wise products */
#define LT_PROF_PRECOND 5   /* Gram matrices and Cholesky factors of the preconditioned SVT */
#define LT_PROF_NCLASS 6
typedef struct {
  int64_t calls[LT_PROF_NCLASS];
  double ms[LT_PROF_NCLASS];   /* summed event-to-event durations */
  int64_t dropped;             /* launches not timed because the event pool was full */
} lt_profile;

typedef struct lt_handle lt_handle;

/* Create a handle bound to the current HIP device and `stream` (a hipStream_t;
 * NULL = the legacy default stream).  Allocates only host memory. */
int lt_create(lt_handle** h, void* stream);
int lt_destroy(lt_handle* h);
int lt_set_stream(lt_handle* h, void* stream);
const char* lt_last_error(const lt_handle* h);
const char* lt_status_string(int status);

/* Start recording kernel durations on this handle (allocates HIP events the
 * first time; call outside graph capture).  lt_profile_end synchronises the
 * stream, returns the totals since lt_profile_begin and stops recording. */
int lt_profile_begin(lt_handle* h);
int lt_profile_end(lt_handle* h, lt_profile* out);

/* Bytes of device workspace an operation needs.  `b` is read only for
 * LT_OP_LPRODUCT.  Returns 0 if the descriptor is invalid. */
size_t lt_workspace_bytes(const lt_desc* a, const lt_desc* b, int op, int precision);

/* C = A *_L B (Alg. 2).  a: I1 x l x I3..IN, b: l x I2 x I3..IN (same trailing
 * dims and kinds), C: I1 x I2 x I3..IN.  Transform precision: `precision`. */
int lt_lproduct(lt_handle* h, const lt_desc* a, const float* A, const lt_desc* b,
                const float* B, float* C, int precision, void* ws, size_t ws_bytes);

/* *_L-SVD (Alg. 3): A = U *_L S *_L V^T with L(U)^p, L(V)^p orthogonal and
 * L(S)^p diagonal for every slice p (Section 3.2).
 *   economy == 0: Alg. 3's shapes, U: I1 x I1 x I3..IN, S: I1 x I2 x I3..IN,
 *     V: I2 x I2 x I3..IN; the factor of the longer side is the economy one
 *     completed by an orthonormal basis of the complement of its columns (any
 *     basis is valid: the extra columns meet zero rows of S).  Workspace:
 *     lt_workspace_bytes(a, NULL, LT_OP_LSVD_FULL, prec).
 *   economy != 0: with n = min(I1, I2), U: I1 x n x ..., S: n x n x ...,
 *     V: I2 x n x ....  Workspace: LT_OP_LSVD.
 * Transform-domain singular values of every slice are sorted in descending
 * order; singular vectors of zero singular values are some orthonormal
 * completion.  transform_domain != 0 returns L(U), L(S), L(V) (the per-slice
 * factors) instead.  sigma (may be NULL): P x n float array of
 * transform-domain singular values, slice-major.  Slices up to
 * min(I1, I2) <= 256 and max(I1, I2) <= 2048 (LT_ERR_SHAPE beyond).
 * Fourier modes (Section 2's t-SVD; FP32 transforms): economy factors in the
 * spatial domain only (LT_ERR_UNSUPPORTED for economy == 0 or
 * transform_domain != 0), with A = U *_L S *_L V^H (the transpose of the
 * Fourier L-product conjugates each slice), from the complex Jacobi, so for the
 * slices it holds (LT_ERR_SHAPE otherwise, see LT_SVT_COMPLEX). */
int lt_lsvd(lt_handle* h, const lt_desc* a, const float* A, float* U, float* S,
            float* V, float* sigma, int economy, int transform_domain, const lt_svd_opts* opts,
            void* ws, size_t ws_bytes);

/* Multirank of A (Section 3.2: rank of every transform-domain slice L(A)^p),
 * counting singular values above rtol times the largest singular value of all
 * slices: rank (device, P int32) per slice; avg (host, may be NULL) their mean
 * (the average rank), tubal (host, may be NULL) their maximum (the tubal
 * rank).  Synchronises the stream when avg or tubal is requested.  Same slice
 * limits as lt_lsvd (Fourier modes: the complex Jacobi's, the two slices of a
 * conjugate pair sharing their singular values); workspace
 * lt_workspace_bytes(a, NULL, LT_OP_LSVD, prec). */
int lt_multirank(lt_handle* h, const lt_desc* a, const float* A, double rtol, int32_t* rank,
                 double* avg, int32_t* tubal, const lt_svd_opts* opts, void* ws, size_t ws_bytes);

/* A_k = U(:, 1:k) *_L S(1:k, 1:k) *_L V(:, 1:k)^T, the best approximation of A
 * by products X *_L Y with X of k lateral slices (Eckart-Young theorem,
 * Section 3.2): every slice of L(A) keeps its k largest singular triplets
 * (all of them when k >= min(I1, I2); A_k = 0 when k <= 0), then L^{-1}.
 * Same slice limits as lt_lsvd (min(I1, I2) <= 256, max(I1, I2) <= 2048; under
 * Fourier modes those of the complex Jacobi, FP32 transforms, with V^H for
 * V^T).  Ak may alias A.  Workspace: lt_workspace_bytes(a, NULL, LT_OP_TRUNCATE,
 * prec). */
int lt_ltruncate(lt_handle* h, const lt_desc* a, const float* A, int32_t k, float* Ak,
                 const lt_svd_opts* opts, void* ws, size_t ws_bytes);

/* How the SVT of descriptor a's slices runs with options opts (may be NULL):
 * LT_SVT_PRECOND and LT_SVT_BLOCKED bits (0: the register kernel on the slice),
 * or a negative status if no kernel takes the shape.  Host only: lets a
 * scheduler keep requests of the long-running blocked kernel apart. */
int lt_svt_path(const lt_desc* a, const lt_svd_opts* opts);

/* 1 if lt_complete_pga with options opts warm-starts the Jacobi of descriptor
 * a's slices (see lt_svd_opts.warm_restart: preconditioned slices of real
 * transforms with n = min(I1, I2) small enough for the register-resident
 * kernel to hold the factor's rows and those of the accumulated rotations), 0
 * if not, a negative status for an invalid descriptor.  Host only. */
int lt_pga_warm(const lt_desc* a, const lt_svd_opts* opts);

/* D = D_tau(A) (Alg. 4): every slice of L(A) has its singular values
 * soft-thresholded by tau >= 0, then L^{-1}.  rank_out (device, P int32, may
 * be NULL): per slice, the number of singular values above tau.  sweeps_out
 * (device, P int32, may be NULL): Jacobi sweeps used per slice.  D may alias A. */
int lt_svt_prox(lt_handle* h, const lt_desc* a, const float* A, double tau, float* D,
                int32_t* rank_out, int32_t* sweeps_out, const lt_svd_opts* opts,
                void* ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lt_svt_prox with the
 * workspace taken from a static device array of LT_NOALLOC_SCRATCH_BYTES bytes
 * that the library holds on each GPU until the process ends (its address is
 * resolved for the handle's device by lt_create).  Arguments and results as
 * lt_svt_prox; the call allocates nothing.  LT_ERR_WORKSPACE when the shape
 * needs more workspace than the array holds (lt_workspace_bytes(a, NULL,
 * LT_OP_SVT, prec) > LT_NOALLOC_SCRATCH_BYTES); LT_ERR_ARG when the current
 * device is not the handle's.  Every call on one GPU shares that GPU's array
 * (nothing in it needs clearing between calls: each call writes what it
 * reads): calls that overlap on one GPU -- on two streams, two handles or two
 * threads -- race and must be serialised by the caller. */
#define LT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lt_svt_prox_noalloc(lt_handle* h, const lt_desc* a, const float* A, double tau, float* D,
                        int32_t* rank_out, int32_t* sweeps_out, const lt_svd_opts* opts);

/* Batched SVT: D[i] = D_{tau[i]}(A[i]) (Alg. 4, Theorem 23) for n tensors of
 * possibly different shapes and orders (real transforms), as one pass of the
 * batch engine below: one grouped forward-transform launch over all tensors,
 * the Jacobi SVDs of all their frontal slices in one launch per kernel family
 * (register-resident items packed longest first, preconditioned ones, blocked
 * ones), one rebuild launch and one grouped inverse-transform launch.  a, A,
 * D: arrays of n descriptors (host) and device pointers; tau: host array,
 * tau[i] >= 0; D[i] may alias A[i].  rank_out (host array of n device
 * pointers, or NULL; entries may be NULL): per slice of tensor i, the number of
 * singular values above tau[i].  Workspace: lt_svt_batched_workspace_bytes
 * (same n, a, opts).  Set-up synchronises the stream (tables are uploaded); the
 * SVT itself is then asynchronous.  Fourier modes: LT_ERR_UNSUPPORTED. */
size_t lt_svt_batched_workspace_bytes(int n, const lt_desc* const* a, const lt_svd_opts* opts);
int lt_svt_prox_batched(lt_handle* h, int n, const lt_desc* const* a, const float* const* A,
                        const double* tau, float* const* D, int32_t* const* rank_out,
                        const lt_svd_opts* opts, void* ws, size_t ws_bytes);

/* Completion by PGA (Alg. 5) from X^0 = X^1 = 0 (or continued, see
 * lt_pga_params.start_iter); on return X holds the last iterate and the
 * workspace the one before it.  M: observed tensor; mask:
 * uint8 per entry, nonzero = observed (the set Omega of eq. (48)); X: output,
 * the last iterate.  Checks M on Omega for NaN/Inf (LT_ERR_NONFINITE).
 * Synchronises the host with the stream when tol > 0 (every check_every
 * iterations) and at the end (to fill rep).  rep may be NULL. */
int lt_complete_pga(lt_handle* h, const lt_desc* a, const float* M, const uint8_t* mask,
                    const lt_pga_params* p, float* X, lt_pga_report* rep,
                    void* ws, size_t ws_bytes);

/* ---- batched completion engine ------------------------------------------
 * Many independent completion problems (Alg. 5 each, possibly of different
 * shapes and orders) advance together: one tick runs one PGA iteration of every
 * unfinished problem with a fixed sequence of six launches -- tick start,
 * forward L of all problems (one grouped GEMM launch), the one-sided Jacobi SVT
 * of every frontal slice of every problem (one launch over a longest-first work
 * list; small slices of one problem are packed several per workgroup), the
 * rank-r rebuild (one launch), inverse L with the stopping norms (one grouped
 * launch), tick end (stopping rule evaluated on the device).  The slices of
 * problems that lt_complete_pga would warm-start (lt_svd_opts.warm_restart,
 * lt_pga_warm) take the warm-started Jacobi instead, one slice per workgroup
 * (plus one launch forming L Z per slice before it, and one Jacobi launch per
 * kernel configuration), cold every warm_restart iterations of the problem.
 * A problem's whole state (iterates, scalars, counters, accumulated rotations)
 * lives in its own workspace, so problems can join or leave between ticks by
 * building a new batch. */
typedef struct {
  const lt_desc* desc;   /* shape and transform (host, read during lt_problem_init) */
  const float* M;        /* device, observed tensor */
  const uint8_t* mask;   /* device, 1 byte per entry, nonzero = observed */
  float* X;              /* device, the iterate; holds the result once finished */
  lt_pga_params params;  /* Alg. 5 parameters; svd.precision selects the transform */
  void* ws;              /* device workspace of lt_problem_workspace_bytes(desc, &params) */
  size_t ws_bytes;
} lt_problem;

size_t lt_problem_workspace_bytes(const lt_desc* a, const lt_pga_params* p);

/* Validate, check M on the mask for NaN/Inf (synchronises), build the
 * transforms and the schedule, zero the iterates (X^0 = X^1 = 0). */
int lt_problem_init(lt_handle* h, const lt_problem* p);

/* Synchronise the handle's stream and read a problem's progress.  done is 0
 * while running, 1 when the stopping rule fired, 2 at max_iter.  Once done, the
 * last iterate is in p->X (copied there by this call if needed). */
int lt_problem_status(lt_handle* h, const lt_problem* p, lt_pga_report* rep, int32_t* done);

typedef struct lt_batch lt_batch;

/* Device bytes for the batch's work tables. */
size_t lt_batch_workspace_bytes(int n, const lt_problem* probs);

/* Build the work tables of n initialised problems (all with the same
 * svd.precision, jacobi_tol and max_sweeps).  use_graph != 0 captures one tick
 * as a HIP graph on first use and replays it.  jacobi_lanes selects the lanes
 * per column pair of the Jacobi kernel (4, 8, 16, 32 or 64; 0 = built-in
 * choice), e.g. from an autotuning run; LT_ERR_SHAPE if it cannot hold every
 * slice of the batch.  bws: device workspace of lt_batch_workspace_bytes bytes
 * (caller-owned, must outlive the batch). */
int lt_batch_create(lt_handle* h, int n, const lt_problem* probs, void* bws, size_t bws_bytes,
                    int use_graph, int jacobi_lanes, lt_batch** out);
/* Enqueue `ticks` ticks on the handle's stream (asynchronous). */
int lt_batch_step(lt_batch* b, int ticks);
int lt_batch_destroy(lt_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LT_H */
