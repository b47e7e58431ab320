// Internal declarations shared by the HIP sources of liblt.so (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---- bf16 helpers (round to nearest even; inputs here are finite) ---------
__host__ __device__ inline uint16_t f32_to_bf16_bits(float v) {
  union { float f; uint32_t u; } x;
  x.f = v;
  uint32_t u = x.u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t h) {
  union { float f; uint32_t u; } x;
  x.u = ((uint32_t)h) << 16;
  return x.f;
}

// ---- transform GEMM: out[q, e] = sum_p K[q, p] in[p, e] ----------------------
// Rows are transform-domain slice indices (q, p < P); columns are the I1*I2
// entries of a slice (e < N).  in/out are row-major P x N (ld = N), which is
// exactly the tensor layout (slice p starts at p*N).
enum ProMode { PRO_PLAIN = 0, PRO_PGA = 1 };
enum EpiMode { EPI_PLAIN = 0, EPI_PGA = 1 };

struct GemmArgs {
  const float* K;          // P x P row-major (FP32 path)
  const uint16_t* Khi;     // bf16 split of the same matrix (BF16X3 path)
  const uint16_t* Klo;
  int P;
  long long N;
  // prologue: PRO_PLAIN reads B; PRO_PGA builds G = mask ? M : X + beta (X - Xp)
  const float* B;
  const float* X;
  const float* Xp;
  const float* M;
  const uint8_t* mask;
  float beta;
  // epilogue: EPI_PLAIN stores out; EPI_PGA also forms Y = X + beta (X - Xp) at
  // the output position and accumulates ||Y - out||^2, ||out||^2 per workgroup
  float* out;
  double* partials;        // [gridDim.x * gridDim.y][2]
  // Fourier transforms (stacked real form): output rows Mo and contraction
  // length Kd when nonzero (K is Mo x Kd row-major), else P and P
  int Mo, Kd;
};

hipError_t launch_transform_gemm(const GemmArgs& a, int precision, int pro, int epi,
                                 hipStream_t s, int* n_partials);

// Build the Kronecker transform K = M_N (x) ... (x) M_3 (P x P, row-major) and
// optionally its bf16 hi/lo split.  Per mode: kind (0 DCT, 2 identity, 3 custom),
// size, and for custom a device pointer to the row-major matrix (double).
// inverse != 0 builds (x) M_i^{-1} (for DCT: transposes; custom matrices must
// then already be the inverses).
struct KronDesc {
  int nmodes;
  int n[8];
  int kind[8];
  const double* custom[8];
};
hipError_t launch_build_kron(const KronDesc& d, int P, int inverse, float* K,
                             uint16_t* Khi, uint16_t* Klo, hipStream_t s);

hipError_t launch_reduce_partials(const double* partials, int n, double* out2, hipStream_t s,
                                  const int32_t* sweeps = nullptr, int nsl = 0,
                                  unsigned long long* slowest = nullptr);
// Transforms with Fourier modes (kind 1 in KronDesc), stacked real form:
// forward [Re K; Im K] (2P x P), inverse [Re K^{-1}, -Im K^{-1}] (P x 2P).
hipError_t launch_build_kron_dft(const KronDesc& d, int P, int inverse, float* K, hipStream_t s);
// Complex slices (planes Re, Im: P x I1 x I2) <-> real embeddings of the
// representatives rep[0..npairs) of their conjugate pairs (2 I1 x 2 I2 each).
hipError_t launch_dft_embed(const float* Re, const float* Im, const int* rep, int npairs, int I1, int I2,
                            float* E, hipStream_t s);
hipError_t launch_dft_extract(const float* E, const int* rep, const int* partner, int npairs, int I1, int I2,
                              float* Re, float* Im, const int32_t* rankE, int32_t* rank,
                              const int32_t* sweepsE, int32_t* sweeps, const double* nucE, double* nuc,
                              hipStream_t s);
// The same slices <-> complex working matrices of the Hermitian Jacobi (2 max(I1,
// I2) interleaved rows by min(I1, I2) columns, 2 I1 I2 floats each; twin: each
// column followed by its product by i, 4 I1 I2 floats), and the results back
// with the partners' conjugates (twin: read from the even columns).
hipError_t launch_dft_stack(const float* Re, const float* Im, const int* rep, int npairs, int I1, int I2,
                            float* W, hipStream_t s, bool twin = false);
hipError_t launch_dft_unstack(const float* W, const int* rep, const int* partner, int npairs, int I1, int I2,
                              float* Re, float* Im, const int32_t* rankE, int32_t* rank,
                              const int32_t* sweepsE, int32_t* sweeps, const double* nucE, double* nuc,
                              hipStream_t s, bool twin = false);
// Columns 0, 2, ..., 2 (ncols - 1) of rows-row column-major matrices (src_stride
// floats apart) into contiguous rows x ncols ones (dst_stride apart).
hipError_t launch_even_columns(const float* src, long long src_stride, float* dst, long long dst_stride, int rows,
                               int ncols, int nslices, hipStream_t s);
// Columns j < k of complex matrices (2 m interleaved rows) and their products
// by i as columns 2j, 2j + 1 of Bk; per-representative values to both slices
// of each conjugate pair (P x n).
hipError_t launch_twin_columns(const float* U, long long u_stride, int rows2, int k, float* Bk, long long bk_stride,
                               int nslices, hipStream_t s);
hipError_t launch_expand_pairs(const double* v, const int* rep, const int* partner, int npairs, int n, double* out,
                               hipStream_t s);
// out[0] = scale * (v[0] + ... + v[n-1]) in a fixed summation order (one workgroup).
hipError_t launch_sum_scaled(const double* v, int n, double scale, double* out, hipStream_t s);

// C^p = A^p B^p for p < P; A^p: I1 x L (ld I1), B^p: L x I2 (ld L), C^p: I1 x I2.
// complex_planes: complex slices, each operand a plane of real parts followed
// by one of imaginary parts (the Fourier transform's output layout).
hipError_t launch_facewise(const float* A, const float* B, float* C, int I1, int L,
                           int I2, int P, hipStream_t s, bool complex_planes = false);

// count of non-finite values among entries with mask != 0 (mask may be null)
hipError_t launch_count_nonfinite(const float* X, const uint8_t* mask, long long n,
                                  unsigned int* count, hipStream_t s);

// ---- one-sided Jacobi SVT ----------------------------------------------------
// Per slice (one workgroup each), working matrix W = slice (I1 >= I2) or
// slice^T (I1 < I2), m = max(I1, I2) rows, n = min(I1, I2) columns.
struct JacobiArgs {
  const float* src;        // slices, slice s at src + s * slice_stride
  long long slice_stride;
  int I1, I2;
  int nslices;
  double tau;              // SVT threshold (svt mode)
  double tol;              // rotate while |a.b| > tol |a||b|
  int max_sweeps;
  int qeff;                // 4-row chunks per lane that carry rows (set by launch_jacobi)
  int mode;                // 0: SVT (write kept, scaled columns); 1: all columns + norms
  float* bk;               // out, slice s at bk + s * bk_stride: m x r columns (ld m)
  long long bk_stride;     // 0: slice_stride
  int32_t* rank;           // out [nslices] (svt mode: r; lsvd mode: n)
  int32_t* sweeps;         // out [nslices]
  double* sigma;           // lsvd mode: out [nslices][n] column norms (unsorted)
  unsigned long long* sweep_total;  // optional: atomic sum of sweeps
  unsigned long long* rot_total;    // optional: atomic sum of rotations
  unsigned int* maxsweep_hits;      // optional: atomic count of slices at max_sweeps
  double* nuc;             // optional, SVT mode: [nslices] sum of (sigma_i - tau) over kept columns
  // blocked kernel only: per-slice working buffers (work_stride floats each) and
  // the block layout (set by launch_jacobi_blk)
  float* work;
  long long work_stride;
  int blk_b, blk_n, blk_nbuf;
};

struct JacobiConfig {
  int G;        // lanes per column pair
  int R;        // rows per lane (register-resident)
  int threads;  // workgroup size
  int nbuf;     // LDS exchange buffers (2: one barrier pair per round; 1: two)
  size_t lds;   // dynamic LDS bytes
};

// Pick a kernel configuration for an m x n working matrix (0 on success).
int jacobi_pick_config(int m, int n, int max_lds, JacobiConfig* cfg, int force_G);
hipError_t launch_jacobi(const JacobiArgs& a, const JacobiConfig& cfg, hipStream_t s);

// Warm-started Jacobi on the preconditioned factors (one slice per workgroup):
// the Jacobi runs on M = L Z, L = R^T the slice's n x n Cholesky factor and Z
// the orthogonal matrix of the rotations accumulated since the last cold start
// (Z = I, M = L), and rewrites Z with this call's rotations appended.
struct WarmArgs {
  const float* M;          // slice s at M + s * m_stride (n x n, column-major): L Z, or L when cold
  long long m_stride;
  float* Z;                // slice s at Z + s * n * n (column-major): read unless cold, rewritten
  float* bk;               // kept columns, scaled (as JacobiArgs::bk in SVT mode)
  long long bk_stride;
  int32_t* rank;
  int32_t* sweeps;
  unsigned long long* sweep_total;
  unsigned long long* rot_total;
  unsigned int* hits;
  double* nuc;             // optional: [nslices] sum of (sigma_i - tau) over kept columns
  double tau;
  double tol;
  int n;
  int nslices;
  int max_sweeps;
  int cold;
};
// Configuration for n x n factors (0 on success, -1 if the kernel cannot hold
// them), launch, and the product M = L Z (FP32 MFMA, no LDS).
int jacobi_warm_config(int n, int max_lds, JacobiConfig* cfg, int force_G = 0);
// Complex (Hermitian) Jacobi for Fourier slices on their stacked working
// matrices (ms = 2 m interleaved rows, n columns, SVT mode): configuration (0 on
// success, -1 if the kernel cannot hold them) and launch.  Bk takes 2 r
// columns of ms rows per slice (each kept column and its product by i).
int jacobi_cx_config(int ms, int n, int max_lds, JacobiConfig* cfg);
hipError_t launch_jacobi_cx(const JacobiArgs& a, const JacobiConfig& cfg, hipStream_t s);
hipError_t launch_jacobi_warm(const WarmArgs& a, const JacobiConfig& cfg, hipStream_t s);
hipError_t launch_warm_product(const float* L, long long l_stride, const float* Z, float* M,
                               long long m_stride, int n, int nslices, hipStream_t s);

// The register-resident kernel can hold an m x n working matrix (shape limits
// only; the device's LDS is checked by jacobi_pick_config).
bool jacobi_reg_shape(int m, int n);
// Blocked Jacobi for working matrices the register-resident kernel cannot hold
// (n <= 512, m <= 2048): columns live in a per-slice working buffer and one
// workgroup per slice sweeps them block pair by block pair.
// Kernel variants (lanes per pair G, rows per lane R): {16,16}, {32,16},
// {64,16}, {64,32}.
constexpr int kBlkNumVariants = 4;
extern const int kBlkVariants[kBlkNumVariants][2];
struct JacobiBlkConfig {
  int G, R;              // lanes per column pair, register rows per lane
  int variant;           // index into kBlkVariants
  int b, nblk;           // block width (even) and block count (even)
  int qeff;              // 4-row chunks per lane (rows held: 4 G qeff)
  int threads;
  int nbuf;              // LDS exchange buffers (2 when they fit: one barrier per ring round)
  size_t lds;
  long long work_floats; // working buffer per slice
};
int jacobi_blk_pick_config(int m, int n, int max_lds, JacobiBlkConfig* cfg);
hipError_t launch_jacobi_blk(const JacobiArgs& a, const JacobiBlkConfig& cfg, hipStream_t s);

// Wide blocked Jacobi (many columns, few slices): the blocked layout with one
// workgroup per block pair, one launch per block round, and per-slice state on
// the device between launches.  Host loop: launch_wide_copy_in (also clears the
// state), launch_wide_sweep until *active (device) reads 0 after a sweep or the
// sweep limit, then launch_wide_out (kept columns, rank, sweeps, nuc, totals as
// the SVT mode of the other kernels).
constexpr size_t kWideStateBytes = 32;
struct WideArgs {
  const float* src;        // slices (working orientation as JacobiArgs), slice s at src + s * slice_stride
  long long slice_stride;
  int I1, I2, nslices;
  float* work;             // per-slice working buffers, work_stride floats each
  long long work_stride;
  void* state;             // nslices x kWideStateBytes
  double tau, tol;
  int max_sweeps;
  float* bk;               // kept columns, slice s at bk + s * bk_stride (m x r, ld m)
  long long bk_stride;
  int32_t* rank;
  int32_t* sweeps;
  double* nuc;
  unsigned long long* sweep_total;
  unsigned long long* rot_total;
  unsigned int* hits;
};
struct JacobiWideConfig {
  int G, R, variant, b, nblk, qeff, threads, nbuf;
  size_t lds;
  long long work_floats;
};
int jacobi_wide_pick_config(int m, int n, int max_lds, JacobiWideConfig* cfg);
hipError_t launch_wide_copy_in(const WideArgs& a, const JacobiWideConfig& c, hipStream_t s);
hipError_t launch_wide_sweep(const WideArgs& a, const JacobiWideConfig& c, int* active, hipStream_t s);
hipError_t launch_wide_out(const WideArgs& a, const JacobiWideConfig& c, hipStream_t s);

// D (slice orientation) = rebuild from kept columns: D_W = Bk Bk^T W
struct RebuildArgs {
  const float* W;          // transform-domain slices (the Jacobi input)
  float* D;                // output slices (may equal W)
  const float* bk;
  const int32_t* rank;
  long long slice_stride;
  int I1, I2, nslices;
  int flip;                // 0: D_W = Bk (Bk^T W), Bk m x r; 1: D_W = (W B) B^T, B n x r
  int rcap;                // set by launch_rebuild: kept-column capacity of its LDS
  long long bk_stride;     // between the slices' kept columns (0: slice_stride)
  int kmax;                // bound on the kept counts (0: min(I1, I2))
};

// Cholesky-QR preconditioning of the Jacobi SVD (lt_precond.hip).
struct GramArgs {
  const float* W;          // slices (working orientation as for the Jacobi kernel)
  long long slice_stride;
  double* C;               // out: n x n FP64 per slice at C + s * c_stride (lower triangle)
  long long c_stride;      // >= n * n
  int I1, I2, nslices;
};
hipError_t launch_gram(const GramArgs& a, hipStream_t s);
// The Gram matrix (2n x 2n lower triangle, FP64, c_stride doubles per slice) of
// the real form [w_1, i w_1, w_2, i w_2, ...] of complex m x n slices whose
// columns w_a are interleaved (Re, Im) rows col_stride floats apart (slices
// w_stride floats apart): the real form of W^H W.
hipError_t launch_gram_cx(const float* W, long long w_stride, long long col_stride, int m, int n, double* C,
                          long long c_stride, int nslices, hipStream_t s);

struct CholArgs {
  double* C;               // in: Gram lower triangles; out: L (FP32 n x n) over each slice's region
  long long c_stride;      // doubles between slices (L slice s at (float*)(C + s * c_stride))
  int n, nslices;
};
size_t chol_lds_bytes(int n);
hipError_t launch_chol(const CholArgs& a, hipStream_t s);
// Gram matrix and Cholesky in one launch (one workgroup per slice, the Gram on
// FP64 MFMA into LDS): the same L as launch_gram + launch_chol, for
// min(I1, I2) <= kGramCholMaxN; C receives only L (FP32, first half).
constexpr int kGramCholMaxN = 176;
hipError_t launch_gram_chol(const GramArgs& g, hipStream_t s);
// Cholesky for any n (multi-launch, many workgroups per slice): C (n x n FP64,
// lower triangle, c_stride doubles per slice) factored in place, then the FP32
// factor written to L (n x n per slice, l_stride floats, zero above the
// diagonal; col_step 2: only the even columns, n x ceil(n/2)); thr: scratch,
// one double per slice.
hipError_t launch_chol_big(double* C, long long c_stride, int n, int nslices, float* L, long long l_stride,
                           double* thr, hipStream_t s, int col_step = 1);
hipError_t launch_rebuild(const RebuildArgs& a, hipStream_t s);

// lsvd finalisation: sort, normalise, V = W^T U diag(1/sigma), write factors
struct LsvdArgs {
  const float* W;          // transform-domain slices
  const float* cols;       // Jacobi final columns (m x n per slice, ld m)
  const double* sigma;     // [nslices][n]
  long long slice_stride;
  int I1, I2, nslices;
  float* U;                // I1 x n per slice (slice stride I1*n)
  float* S;                // n x n per slice
  float* V;                // I2 x n per slice
  float* sig_out;          // optional [nslices][n]
};
hipError_t launch_lsvd_finalize(const LsvdArgs& a, hipStream_t s);
// Economy factors of complex (Fourier) slices from the complex Jacobi's
// all-columns output, one conjugate-pair representative per workgroup: W and
// cols are its working matrix and final columns (2 m interleaved rows x n,
// w_stride floats apart), sigma their norms; U, S, V receive real-part planes
// then imaginary-part planes (P slices each, I1 x n, n x n, I2 x n) for the
// representative and, conjugated, its partner; sig_out (optional) P x n.
// scratch: 2 m n + 2 n^2 floats per representative (scratch_stride apart).
struct LsvdCxArgs {
  const float* W;
  const float* cols;
  const double* sigma;
  long long w_stride;
  const int* rep;
  const int* partner;
  int npairs, P, I1, I2;
  float* U;
  float* S;
  float* V;
  float* sig_out;
  float* scratch;
  long long scratch_stride;
};
hipError_t launch_lsvd_finalize_cx(const LsvdCxArgs& a, hipStream_t s);

// Full factors and multirank (lt_factors.hip).  dst (rd x cd per slice) = src
// (rs x cs per slice) padded with zeros; complete_basis fills columns n..m-1 of
// each slice's m x m factor Q (first n columns orthonormal, m <= 2048) with an
// orthonormal basis of their complement, H (P x m x n FP64) and beta (P x n)
// being scratch; multirank counts sigma (P x n) above rtol * max sigma per
// slice into rank and writes their mean and maximum to out[0], out[1].
hipError_t launch_pad_copy(const float* src, float* dst, int rs, int cs, int rd, int cd, int P, hipStream_t s);
// The SVT rebuild (as launch_rebuild) for any kept count, through two batched
// GEMMs; T: scratch of nslices x I1 x I2 floats.
hipError_t launch_rebuild_gemm(const RebuildArgs& r, float* T, hipStream_t s);
hipError_t launch_complete_basis(float* Q, double* H, double* beta, int m, int n, int P, hipStream_t s);
hipError_t launch_multirank(const double* sigma, int P, int n, double rtol, int32_t* rank, double* out,
                            hipStream_t s);

// ---- batched completion engine (many problems, one tick = one PGA iteration) --
// Device-resident state of one problem.  Static fields are written once at
// initialisation; the dynamic fields advance on the device every tick.
struct ProbDev {
  int I1, I2, P, pad0;
  long long N, nel;
  const float* M;
  const uint8_t* mask;
  float* Xa;                 // iterate buffers: X^k is in Xa when parity == 0
  float* Xb;
  float* Gh;                 // transform-domain slices (thresholded in place)
  float* Bk;                 // kept columns of the Jacobi SVT
  int32_t* rank;
  int32_t* sweeps;
  double* nuc;               // [P] per slice: sum of (sigma_i - mu_k) over the kept singular values
  const float* K;            // forward / inverse Kronecker transforms (FP32)
  const float* Kinv;
  const uint16_t *Khi, *Klo, *Kihi, *Kilo;   // bf16 splits
  const double* betas;       // [max_iter] momentum weights beta_k (eq. (52))
  const double* mus;         // [max_iter] thresholds mu_k
  double* partials;          // [n_partials][2] norms of the inverse GEMM tiles
  int n_partials;
  int max_iter;
  double tol, mu_bar;
  int gate_until_floor, enabled;
  double* C;                 // preconditioning: per-slice Gram matrix / Cholesky factor (or null)
  int precond, pad2;         // nonzero: the SVT runs the Jacobi on R^T (n x n) and rebuilds (W B) B^T
  float* work;               // blocked Jacobi: per-slice working buffers (or null)
  long long work_stride;
  int blk_b, blk_n, blk_q, blk_variant, blk_nbuf, pad3;
  float* Z;                  // warm-started Jacobi: per-slice accumulated rotations (n x n), or null
  int warm_period, pad4;     // cold start (Z = I) when iter % warm_period == 0; 0: always cold
  // dynamic
  int iter, parity, done, active;   // done: 1 converged, 2 iteration limit
  double beta, tau, num, den, crit;
  unsigned long long sweep_total, rot_total;
  unsigned int maxsweep_hits, pad1;
};

struct GemmTile { int prob, tx, ty, part; };          // one 64x64 output tile
struct SvtItem { int prob, slice0, nsub, qeff; };    // nsub same-shape slices, qeff row chunks
struct RebuildTile { int prob, slice, j0, pad; };    // 16 working columns of one slice
struct GramTile { int prob, slice, tile, pad; };     // one lower-triangle 32x32 tile of C = W^T W
struct CholItem { int prob, slice; };                // one slice's Cholesky factorization

hipError_t launch_gemm_grouped(ProbDev* const* probs, const GemmTile* tiles, int ntiles, int precision,
                               int inverse, hipStream_t s);
hipError_t launch_batch_begin(ProbDev* const* probs, int nprob, hipStream_t s);
hipError_t launch_batch_end(ProbDev* const* probs, int nprob, hipStream_t s);
// wide: tiles of slices with more than 256 columns (up to 512 kept columns);
// kmax: the largest min(I1, I2) of the tiles' problems (bounds the kept count)
hipError_t launch_rebuild_tiles(ProbDev* const* probs, const RebuildTile* tiles, int ntiles, int wide,
                                int kmax, hipStream_t s);
hipError_t launch_gram_tiles(ProbDev* const* probs, const GramTile* tiles, int ntiles, hipStream_t s);
hipError_t launch_chol_items(ProbDev* const* probs, const CholItem* items, int nitems, int nmax,
                             hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

struct JacobiBatchConfig {
  int G, RMAX, threads, nbuf;
  size_t lds;   // per workgroup (max over items)
};
// Choose a kernel for a batch of slices shapes (m_i x n_i) and each item's pack
// size; returns 0 on success.
int jacobi_batch_config(const int* m, const int* n, int count, int max_lds, int force_G,
                        JacobiBatchConfig* cfg, int* nsub_out, int* qeff_out);
hipError_t launch_jacobi_items(ProbDev* const* probs, const SvtItem* items, int nitems,
                               const JacobiBatchConfig& cfg, double tol, int max_sweeps,
                               hipStream_t s);
// Blocked kernel over items (problem, slice) of problems with blk_variant == variant.
hipError_t launch_jacobi_blk_items(ProbDev* const* probs, const CholItem* items, int nitems, int variant,
                                   int threads, size_t lds, double tol, int max_sweeps, hipStream_t s);
// Warm-started Jacobi over items (problem, slice) of warm-started problems
// sharing one configuration (G, R, nbuf; threads and LDS the items' maxima),
// and the products M = L Z they need (nmax: the items' largest n).
hipError_t launch_jacobi_warm_items(ProbDev* const* probs, const CholItem* items, int nitems,
                                    const JacobiConfig& cfg, double tol, int max_sweeps, hipStream_t s);
hipError_t launch_warm_product_items(ProbDev* const* probs, const CholItem* items, int nitems, int nmax,
                                     hipStream_t s);

}  // namespace lt
