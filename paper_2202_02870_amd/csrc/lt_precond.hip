// Preconditioning of the per-slice one-sided Jacobi SVD by a QR factor
// computed as Cholesky-QR (the SVD step of Alg. 3 / Alg. 4; how the SVD is
// computed is not part of the method).
//
// For a working slice W (m x n, m >= n), C = W^T W = R^T R with R upper
// triangular; W and R have the same singular values and right singular
// vectors.  One-sided Jacobi applied to L = R^T (n x n) turns L J into
// V Sigma, i.e. its converged columns are sigma_i v_i with v_i the right
// singular vectors of W, and the SVT result is D_W = sum (1 - tau/sigma_i)
// sigma_i u_i v_i^T = W (sum g_i v_i v_i^T) = W B B^T with B = [sqrt(g_i) v_i].
// The Jacobi kernel writes B exactly as it writes its left-vector output on
// the unpreconditioned path (kept columns scaled by sqrt(1 - tau/sigma)/sigma),
// and the rebuild kernel forms (W B) B^T by treating W^T as its working matrix.
//
// Why: on the slices of the completion iterates the Jacobi sweeps needed on
// R^T are about half of those on W once the iterate has become low-rank plus
// noise, and R^T has n rows instead of m.
//
// Accuracy: C is accumulated in FP64 from FP32 products (exact), so the
// eigenvalues sigma_i^2 carry an absolute error of about n eps64 sigma_max^2;
// a pivot below n * 64 eps64 * max diag(C) (a column numerically in the span of
// the earlier ones) is set to zero with its column of L, which perturbs the
// singular values by at most about 1e-6 sigma_max.  L is handed to the Jacobi
// kernel in FP32, the precision the slice itself has.
#include "lt_internal.h"

#include <float.h>
#include <math.h>

namespace lt {

namespace {

__device__ inline float w_elem(const float* W, bool trans, int I1, int row, int col) {
  return trans ? W[(long long)row * I1 + col] : W[(long long)col * I1 + row];
}

constexpr int GT = 32;   // Gram output tile (GT x GT)

typedef double ct_v4d __attribute__((ext_vector_type(4)));

// C (lower triangle, n x n column-major FP64) = W^T W for one slice: one
// lower-triangle GT x GT tile (ti >= tj, index t) per workgroup of four waves,
// each wave a 16 x 16 quarter on FP64 MFMA (the FP32 entries of W are exact in
// FP64, the products and sums are FP64), W staged through LDS GK rows at a
// time, coalesced along whichever dimension W keeps contiguous.
constexpr int GK = 64;   // rows of W per LDS chunk
__device__ __attribute__((always_inline)) void gram_tile(const float* W, int I1, int I2, double* C, int t) {
  __shared__ float Ai[GK][GT + 1];
  __shared__ float Aj[GK][GT + 1];
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int tj = t - ti * (ti + 1) / 2;
  const bool trans = I1 < I2;
  const int m = trans ? I2 : I1;
  const int n = trans ? I1 : I2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const int wa = wave & 1, wb = wave >> 1;
  const bool live = !(ti == tj && wa < wb);   // a quarter wholly above the diagonal skips the products
  // MFMA 16x16x4: lane l gives A[l % 16][l / 16] (from the tj columns) and
  // B[l / 16][l % 16] (from the ti columns) and holds D[l / 16 + 4 q][l % 16]:
  // C(i, j) with i = GT ti + 16 wa + l % 16, j = GT tj + 16 wb + l / 16 + 4 q
  ct_v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += GK) {
    for (int idx = tid; idx < GK * GT; idx += 256) {
      int kk, c;
      if (trans) {   // W(row, col) = A[row * I1 + col]: columns contiguous
        c = idx % GT;
        kk = idx / GT;
      } else {       // W(row, col) = A[col * I1 + row]: rows contiguous
        kk = idx % GK;
        c = idx / GK;
      }
      const int row = k0 + kk, ci = ti * GT + c, cj = tj * GT + c;
      Ai[kk][c] = (row < m && ci < n) ? w_elem(W, trans, I1, row, ci) : 0.f;
      Aj[kk][c] = (row < m && cj < n) ? w_elem(W, trans, I1, row, cj) : 0.f;
    }
    __syncthreads();
    if (live) {
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)Aj[kk + lq][16 * wb + lr], (double)Ai[kk + lq][16 * wa + lr],
                                                   acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if (!live) return;
  const int i = ti * GT + 16 * wa + lr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = tj * GT + 16 * wb + lq + 4 * q;
    if (i < n && j < n && i >= j) C[i + (long long)j * n] = acc[q];
  }
}

// The Gram matrix of a complex slice's real form T = [w_1, i w_1, w_2, ...]
// (complex columns w_a of m entries held as 2m interleaved (Re, Im) rows,
// col_stride floats apart): its 2 x 2 blocks are [[Re g, -Im g], [Im g, Re g]]
// with g = w_a^H w_b, so one complex product per block (half the multiply-adds
// of the real Gram of T).  Over the interleaved rows Re g is the real dot of
// the two columns and Im g the real dot of w_a with J w_b, where J maps each
// (Re, Im) pair (x, y) to (y, -x).  One 32 x 32 tile of complex products
// (lower, ta >= tb, index blockIdx.x) per workgroup of four waves, each wave a
// 16 x 16 quarter on FP64 MFMA with two accumulators (Re g, Im g), the columns
// staged through LDS 64 interleaved rows at a time; the FP32 entries are exact
// in FP64, the products and sums are FP64.  C is the 2n x 2n lower triangle.
constexpr int GCX = 32;     // complex columns per tile side
constexpr int GCX_K = 64;   // interleaved rows per LDS chunk (even: pairs stay whole)

__global__ __launch_bounds__(256) void k_gram_cx(const float* W, long long w_stride, long long col_stride, int m,
                                                 int n, double* C, long long c_stride) {
  __shared__ float As[GCX_K][GCX + 1], Bs[GCX_K][GCX + 1];
  const float* Ws = W + (long long)blockIdx.y * w_stride;
  double* Cs = C + (long long)blockIdx.y * c_stride;
  const int t = blockIdx.x;
  int ta = 0;
  while ((ta + 1) * (ta + 2) / 2 <= t) ++ta;
  const int tb = t - ta * (ta + 1) / 2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lq = lane >> 4;
  const int wa = wave & 1, wb = wave >> 1;
  const int a0 = GCX * ta, b0 = GCX * tb;
  const bool live = !(ta == tb && wa < wb);   // a quarter wholly above the diagonal skips the products
  const int rows = 2 * m;
  // MFMA 16x16x4: lane l gives A[l % 16][l / 16] and B[l / 16][l % 16] and holds
  // D[l / 16 + 4 q][l % 16]; A from the b columns (w_b, or J w_b: the row's
  // pair partner, negated on odd rows), B from the a columns, so lane l holds
  // the products of column a = a0 + 16 wa + l % 16 with b = b0 + 16 wb + l / 16 + 4 q
  const double sgn = (lq & 1) ? -1.0 : 1.0;
  ct_v4d re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < rows; k0 += GCX_K) {
    for (int e = tid; e < GCX_K * GCX; e += 256) {   // consecutive lanes: consecutive rows of a column
      const int r = e % GCX_K, c = e / GCX_K;
      const int row = k0 + r, ca = a0 + c, cb = b0 + c;
      As[r][c] = (row < rows && ca < n) ? Ws[ca * col_stride + row] : 0.f;
      Bs[r][c] = (row < rows && cb < n) ? Ws[cb * col_stride + row] : 0.f;
    }
    __syncthreads();
    if (live) {
#pragma unroll
      for (int kk = 0; kk < GCX_K; kk += 4) {
        const double x = Bs[kk + lq][16 * wb + lr];
        const double xj = sgn * (double)Bs[kk + (lq ^ 1)][16 * wb + lr];
        const double y = As[kk + lq][16 * wa + lr];
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(xj, y, im, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (!live) return;
  const long long n2 = 2LL * n;
  const int a = a0 + 16 * wa + lr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = b0 + 16 * wb + lq + 4 * q;
    if (a < n && b < n && a >= b) {   // real form rows 2a, 2a + 1, columns 2b, 2b + 1 (lower part)
      Cs[(2 * a) + (2 * b) * n2] = re[q];
      Cs[(2 * a + 1) + (2 * b) * n2] = im[q];
      Cs[(2 * a + 1) + (2 * b + 1) * n2] = re[q];
      if (a > b) Cs[(2 * a) + (2 * b + 1) * n2] = -im[q];
    }
  }
}

__global__ __launch_bounds__(256) void k_gram(GramArgs a) {
  const int s = blockIdx.y;
  gram_tile(a.W + (long long)s * a.slice_stride, a.I1, a.I2, a.C + (long long)s * a.c_stride, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_gram_tiles(ProbDev* const* probs, const GramTile* tiles) {
  const GramTile t = tiles[blockIdx.x];
  const ProbDev* pd = probs[t.prob];
  if (!pd->active) return;
  const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
  gram_tile(pd->Gh + (long long)t.slice * pd->N, pd->I1, pd->I2, pd->C + (long long)t.slice * n * n, t.tile);
}

__device__ inline int tri_off(int j, int n) { return j * n - (j * (j - 1)) / 2; }   // column j of a packed lower triangle

constexpr int CH_NMAX = 200;   // largest n of the Cholesky in LDS
constexpr int CB = 16;         // block width

// 1 / sqrt(x) for x > 0: hardware estimate and two Newton steps (FP64 accuracy)
__device__ inline double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double h = 0.5 * x * y;
    y = fma(y, fma(-h, y, 0.5), y);
  }
  return y;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky C = L L^T of one slice's Gram matrix, blocked right-looking, on a
// packed lower triangle in LDS (FP64).  Per block of CB columns: wave 0 factors
// the CB x CB diagonal block (no workgroup barrier inside), every lane solves
// one row of the panel below it against that block, and the workgroup applies
// the block's rank-CB update to the trailing triangle: three barriers per
// block.  A pivot at or below n * 64 eps64 * max diag(C) zeroes its column.
// Writes L in FP32 (n x n column-major, zero above the diagonal) over the first
// half of the slice's own C region.
// PANEL_IN_LDS: solve the panel rows in place in LDS (the batch kernel, where
// a register copy of the row spilled) rather than in registers.
template <bool PANEL_IN_LDS>
__device__ __attribute__((always_inline)) void chol_slice(double* Cs, int n) {
  extern __shared__ __attribute__((aligned(16))) double T[];
  __shared__ double dmax_s;
  __shared__ double dinv_s[CB];   // reciprocals of the current block's diagonal (0: zeroed column)
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* C = Cs;
  float* L = reinterpret_cast<float*>(Cs);
  // one flat pass (independent loads in flight), lower triangle only
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    if (i >= j) T[tri_off(j, n) + i - j] = C[e];
  }
  __syncthreads();
  if (tid < 64) {   // max of the diagonal, one wave
    double d = 0.0;
    for (int j = tid; j < n; j += 64) d = fmax(d, T[tri_off(j, n)]);
    for (int o = 32; o >= 1; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
    if (tid == 0) dmax_s = d;
  }
  __syncthreads();
  const double thr = dmax_s * (64.0 * n * DBL_EPSILON);
  const int lane = tid & 63, wave = tid >> 6;
  const int l32 = tid & 31, grp = tid >> 5, ngrp = nt >> 5;
  for (int K = 0; K < n; K += CB) {
    const int kb = min(CB, n - K);
    // (a) diagonal block, column by column, by wave 0; each step loads all
    // its operands before storing (no load waits on a store)
    if (wave == 0) {
      for (int k = K; k < K + kb; ++k) {
        const int ok = tri_off(k, n);
        const double piv = T[ok];
        const bool live = piv > thr;
        const double inv = live ? rsq64(piv) : 0.0;   // 1 / L(k, k)
        if (lane > 0 && k + lane < K + kb) T[ok + lane] *= inv;
        wave_sync();
        // T(i, j) -= L(i, k) L(j, k), k < j <= i < K + kb (offsets in a CB x CB square, 4 per lane)
        const int r = K + kb - 1 - k;   // rows below k in the block
        int ii[4], jj[4];
        bool ok2[4];
        double ti[4], tj[4], tt[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = lane + 64 * u;   // index into the r x r square, lower part used
          ii[u] = k + 1 + e / CB;
          jj[u] = k + 1 + e % CB;
          ok2[u] = e < CB * CB && e / CB < r && e % CB <= e / CB;
          ti[u] = ok2[u] ? T[ok + ii[u] - k] : 0.0;
          tj[u] = ok2[u] ? T[ok + jj[u] - k] : 0.0;
          tt[u] = ok2[u] ? T[tri_off(jj[u], n) + ii[u] - jj[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (ok2[u]) T[tri_off(jj[u], n) + ii[u] - jj[u]] = fma(-ti[u], tj[u], tt[u]);
        if (lane == 0) {
          T[ok] = piv * inv;   // L(k, k) = sqrt(piv); 0 for a zeroed column
          dinv_s[k - K] = inv;
        }
        wave_sync();
      }
    }
    __syncthreads();
    // (b) panel: row i >= K + kb solves x L11^T = T(i, K .. K + kb - 1) (each
    // lane owns its row)
    for (int i = K + kb + tid; i < n; i += nt) {
      if (PANEL_IN_LDS) {
        for (int q = 0; q < kb; ++q) {
          double acc = T[tri_off(K + q, n) + i - K - q];
          for (int p = 0; p < q; ++p)
            acc = fma(-T[tri_off(K + p, n) + i - K - p], T[tri_off(K + p, n) + q - p], acc);
          T[tri_off(K + q, n) + i - K - q] = acc * dinv_s[q];
        }
      } else {
        double x[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) {
          if (q < kb) {
            double acc = T[tri_off(K + q, n) + i - K - q];
#pragma unroll
            for (int p = 0; p < q; ++p) acc = fma(-x[p], T[tri_off(K + p, n) + q - p], acc);
            x[q] = acc * dinv_s[q];
            T[tri_off(K + q, n) + i - K - q] = x[q];
          }
        }
      }
    }
    __syncthreads();
    // (c) trailing triangle: T(i, j) -= sum_q L(i, K+q) L(j, K+q), K + kb <= j <= i
    for (int i = K + kb + grp; i < n; i += ngrp) {
      double li[CB];
#pragma unroll
      for (int q = 0; q < CB; ++q) li[q] = q < kb ? T[tri_off(K + q, n) + i - K - q] : 0.0;
      for (int j = K + kb + l32; j <= i; j += 32) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < CB; ++q)
          if (q < kb) acc = fma(li[q], T[tri_off(K + q, n) + j - K - q], acc);
        T[tri_off(j, n) + i - j] -= acc;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    L[e] = i >= j ? (float)T[tri_off(j, n) + i - j] : 0.f;
  }
}

// ---- Tiled LDS Cholesky (n <= CT_NMAX) -----------------------------------------
// The same factorization (right-looking, blocks of CT = 16 columns, pivots at
// or below 64 n eps64 max diag(C) zero their column), with the matrix held in
// LDS as 16 x 16 tiles (tile (ti, tj), ti >= tj, column-major inside, the
// diagonal tiles full and symmetric, padding beyond n set to the identity):
//   (a) one wave factors the diagonal tile in registers: lane j + 16 g holds
//       rows 4 g .. 4 g + 3 of column j of the symmetric tile; step k
//       broadcasts column k within each 16-lane row (DPP) and row k of column
//       j (= column k of row j, by symmetry) across the row groups, so every
//       step is a rank-1 update in registers with no LDS round trip;
//   (b) every lane solves one row of the panel tiles below against it;
//   (c) the trailing tiles get C -= X_i X_j^T on FP64 MFMA (16x16x4, exact
//       FP64 products and sums), one tile per wave at a time.
constexpr int CT = 16;
constexpr int CT_NMAX = 192;    // 78 tiles + the current factor: the LDS of one CU

__host__ __device__ inline int ct_ntiles(int nb) { return nb * (nb + 1) / 2; }
__device__ inline int ct_index(int ti, int tj) { return ti * (ti + 1) / 2 + tj; }
__host__ __device__ inline size_t ct_lds_bytes(int n) {
  const int nb = (n + CT - 1) / CT;
  return ((size_t)ct_ntiles(nb) * CT * CT + CT * CT + CT) * sizeof(double);
}

// row index of entry t of a packed lower triangle of tiles (t = ti (ti + 1) / 2 + tj)
__device__ inline int ct_row(int t) {
  int ti = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
  while (ti * (ti + 1) / 2 > t) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  return ti;
}

__device__ inline double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}


// Lane k of each 16-lane row to the whole row (DPP row_newbcast), FP64.
template <int K>
__device__ inline double row_bcast_k(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + K, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + K, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ inline double row_bcast(double v, int k) {
  switch (k) {
    case 0: return row_bcast_k<0>(v);
    case 1: return row_bcast_k<1>(v);
    case 2: return row_bcast_k<2>(v);
    case 3: return row_bcast_k<3>(v);
    case 4: return row_bcast_k<4>(v);
    case 5: return row_bcast_k<5>(v);
    case 6: return row_bcast_k<6>(v);
    case 7: return row_bcast_k<7>(v);
    case 8: return row_bcast_k<8>(v);
    case 9: return row_bcast_k<9>(v);
    case 10: return row_bcast_k<10>(v);
    case 11: return row_bcast_k<11>(v);
    case 12: return row_bcast_k<12>(v);
    case 13: return row_bcast_k<13>(v);
    case 14: return row_bcast_k<14>(v);
    default: return row_bcast_k<15>(v);
  }
}

// Factor the tiles already in LDS (padding set) and write L in FP32 (n x n
// column-major, zero above the diagonal) to L.
__device__ __attribute__((always_inline)) void chol_tiles_factor(double* T, int n, float* L) {
  __shared__ double dmax_s;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = (n + CT - 1) / CT;
  const int ntl = ct_ntiles(nb);
  double* L11 = T + (size_t)ntl * CT * CT;   // the current diagonal factor, column-major
  double* dinv = L11 + CT * CT;              // its pivot reciprocals (0: zeroed column)
  if (tid < 64) {   // max of the diagonal, one wave
    double d = 0.0;
    for (int j = tid; j < n; j += 64) d = fmax(d, T[(size_t)ct_index(j / CT, j / CT) * CT * CT + (CT + 1) * (j % CT)]);
    for (int o = 32; o >= 1; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
    if (tid == 0) dmax_s = d;
  }
  __syncthreads();
  const double thr = dmax_s * (64.0 * n * DBL_EPSILON);
  const int wave = tid >> 6, lane = tid & 63, nwv = nt >> 6;
  for (int tk = 0; tk < nb; ++tk) {
    // (a) the diagonal tile, by wave 0: lane (j, g) = j + 16 g holds rows
    // 4 g .. 4 g + 3 of column j of the symmetric tile
    if (wave == 0) {
      double* D = T + (size_t)ct_index(tk, tk) * CT * CT;
      const int j = lane & 15, g = lane >> 4;
      double c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) c[u] = D[(4 * g + u) + CT * j];
#pragma unroll
      for (int k = 0; k < CT; ++k) {
        const int kg = k >> 2, ku = k & 3;
        const double piv = readlane_d(c[ku], k + 16 * kg);
        const double inv = piv > thr ? rsq64(piv) : 0.0;   // 1 / L(k, k); 0 zeroes the column
        double tik[4];   // T(4 g + u, k): column k's rows of this row group, from lane (k, g)
#pragma unroll
        for (int u = 0; u < 4; ++u) tik[u] = row_bcast(c[u], k);
        const double tkj = __shfl(c[ku], j + 16 * kg, 64);   // T(k, j) = T(j, k)
        if (j > k) {
          // T(i, j) -= L(i, k) L(j, k) = T(i, k) T(k, j) / T(k, k), rows i > k
          const double w = tkj * (inv * inv);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (4 * g + u > k) c[u] = fma(-tik[u], w, c[u]);
        } else if (j == k) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = 4 * g + u;
            c[u] = i < k ? 0.0 : (i == k ? piv * inv : tik[u] * inv);
          }
        }
        if (lane == 0) dinv[k] = inv;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        D[(4 * g + u) + CT * j] = c[u];
        L11[(4 * g + u) + CT * j] = c[u];
      }
    }
    __syncthreads();
    // (b) panel rows: x L11^T = c for each row of the tiles (ti, tk), ti > tk
    const int prows = (nb - tk - 1) * CT;
    for (int e = tid; e < prows; e += nt) {
      const int ti = tk + 1 + (e >> 4), r = e & 15;
      double* X = T + (size_t)ct_index(ti, tk) * CT * CT;
      double x[CT];
#pragma unroll
      for (int q = 0; q < CT; ++q) {
        double acc = X[r + CT * q];
#pragma unroll
        for (int p = 0; p < q; ++p) acc = fma(-x[p], L11[q + CT * p], acc);
        x[q] = acc * dinv[q];
      }
#pragma unroll
      for (int q = 0; q < CT; ++q) X[r + CT * q] = x[q];
    }
    __syncthreads();
    // (c) trailing tiles (ti, tj), tk < tj <= ti: C -= X_ti X_tj^T.  MFMA
    // 16x16x4 operands: lane l gives A[l % 16][l / 16] and B[l / 16][l % 16]
    // and holds D[l / 16 + 4 q][l % 16], q = 0..3.  The product is formed
    // transposed, D = -X_tj X_ti^T, so that lane l's D entries are the tile's
    // (row l % 16, column l / 16 + 4 q): consecutive lanes touch consecutive
    // doubles of the column-major tile (no LDS bank conflicts)
    const int mt = nb - tk - 1;
    const int ntr = mt * (mt + 1) / 2;
    const int lr = lane & 15, lq = lane >> 4;
    for (int t = wave; t < ntr; t += nwv) {
      const int a = ct_row(t), b = t - a * (a + 1) / 2;
      const int ti = tk + 1 + a, tj = tk + 1 + b;
      const double* Xi = T + (size_t)ct_index(ti, tk) * CT * CT;
      const double* Xj = T + (size_t)ct_index(tj, tk) * CT * CT;
      double* Cij = T + (size_t)ct_index(ti, tj) * CT * CT;
      ct_v4d acc;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = Cij[lr + CT * (lq + 4 * q)];
#pragma unroll
      for (int ks = 0; ks < CT / 4; ++ks) {
        const double av = -Xj[lr + CT * (4 * ks + lq)];
        const double bv = Xi[lr + CT * (4 * ks + lq)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Cij[lr + CT * (lq + 4 * q)] = acc[q];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    L[e] = i >= j ? (float)T[(size_t)ct_index(i / CT, j / CT) * CT * CT + (i % CT) + CT * (j % CT)] : 0.f;
  }
}

// Cholesky of one slice's Gram matrix C (n x n FP64, lower triangle): the tiles
// loaded from C; L in FP32 over the first half of the slice's region.
__device__ __attribute__((always_inline)) void chol_tiles(double* Cs, int n) {
  extern __shared__ __attribute__((aligned(16))) double T[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = (n + CT - 1) / CT;
  const int ntl = ct_ntiles(nb);
  const double* C = Cs;
  // the lower triangle into tiles; the diagonal tiles get the symmetric upper
  // part too, the padding the identity
  for (int e = tid; e < ntl * CT * CT; e += nt) {
    const int t = e >> 8, r = e & 15, c = (e >> 4) & 15;
    const int ti = ct_row(t), tj = t - ti * (ti + 1) / 2;
    const int i = CT * ti + r, j = CT * tj + c;
    double v;
    if (i < n && j < n) v = i >= j ? C[i + (long long)j * n] : C[j + (long long)i * n];
    else v = i == j ? 1.0 : 0.0;
    T[e] = v;
  }
  __syncthreads();
  chol_tiles_factor(T, n, reinterpret_cast<float*>(Cs));
}

// The Gram matrix C = W^T W of one slice formed straight into the tiles on
// FP64 MFMA (the FP32 entries of W are exact in FP64, the products and sums are
// FP64, as in k_gram), then factored as chol_tiles: no FP64 copy of C goes
// through memory.  W: the slice in working orientation (m x n, n <= CTG_NMAX),
// staged through LDS sixteen rows at a time (coalesced loads, each entry read
// once); each wave accumulates up to CTG_TPW tiles across the chunks.
constexpr int CTG_NMAX = 176;   // tiles (132 KiB at 176) + a 16-row chunk of W
constexpr int CTG_TPW = 5;      // tiles per wave: 66 tiles at n = 176 over 16 waves
constexpr int CTG_ROWS = 16;

__host__ __device__ inline size_t ctg_lds_bytes(int n) {
  const int nb = (n + CT - 1) / CT;
  return ct_lds_bytes(n) + (size_t)CTG_ROWS * CT * nb * sizeof(float);
}

__device__ __attribute__((always_inline)) void gram_chol_tiles(const float* W, int I1, int I2, double* Cs) {
  extern __shared__ __attribute__((aligned(16))) double T[];
  const bool trans = I1 < I2;
  const int m = trans ? I2 : I1;
  const int n = trans ? I1 : I2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63, nwv = nt >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int nb = (n + CT - 1) / CT;
  const int npad = CT * nb;
  const int ntl = ct_ntiles(nb);
  // the chunk of W after the tiles, the current factor and its reciprocals
  float* Wst = reinterpret_cast<float*>(T + (size_t)ntl * CT * CT + CT * CT + CT);
  // tile (ti, tj): lane l gives A[l % 16][l / 16] = W(k + l / 16, 16 tj + l % 16) and
  // B[l / 16][l % 16] = W(k + l / 16, 16 ti + l % 16), so D = A B holds
  // C(16 tj + l / 16 + 4 q, 16 ti + l % 16) = C(16 ti + l % 16, 16 tj + l / 16 + 4 q):
  // the tile's (row l % 16, column l / 16 + 4 q), consecutive in LDS across lanes
  ct_v4d acc[CTG_TPW];
  int toff_i[CTG_TPW], toff_j[CTG_TPW];
#pragma unroll
  for (int u = 0; u < CTG_TPW; ++u) {
    acc[u] = ct_v4d{0.0, 0.0, 0.0, 0.0};
    const int t = wave + u * nwv;
    const int ti = t < ntl ? ct_row(t) : 0, tj = t < ntl ? t - ti * (ti + 1) / 2 : 0;
    toff_i[u] = CT * ti + lr;
    toff_j[u] = CT * tj + lr;
  }
  for (int k0 = 0; k0 < m; k0 += CTG_ROWS) {
    // stage rows k0 .. k0 + 15 of W (zero beyond m and n); entry e of the
    // staging order is (r, c) = (e / npad, e % npad) when columns are
    // contiguous (trans), (e % 16, e / 16) otherwise; each lane starts at
    // e0 = tid and steps by nt
    {
      const int lim = trans ? npad : CTG_ROWS;
      int b = tid / lim, a = tid - b * lim;
      const int qb = nt / lim, qa = nt - qb * lim;
      for (int e = tid; e < CTG_ROWS * npad; e += nt) {
        const int r = trans ? b : a, c = trans ? a : b;
        const int row = k0 + r;
        Wst[r * npad + c] = (row < m && c < n) ? w_elem(W, trans, I1, row, c) : 0.f;
        a += qa;
        b += qb;
        if (a >= lim) {
          a -= lim;
          ++b;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CTG_TPW; ++u) {
      if (wave + u * nwv < ntl) {
#pragma unroll
        for (int st = 0; st < CTG_ROWS / 4; ++st) {
          const float* row = Wst + (4 * st + lq) * npad;
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)row[toff_j[u]], (double)row[toff_i[u]], acc[u],
                                                        0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < CTG_TPW; ++u) {
    const int t = wave + u * nwv;
    if (t < ntl) {
      double* Tt = T + (size_t)t * CT * CT;
#pragma unroll
      for (int q = 0; q < 4; ++q) Tt[lr + CT * (lq + 4 * q)] = acc[u][q];
    }
  }
  __syncthreads();
  for (int i = n + tid; i < npad; i += nt)   // padding: identity on the diagonal
    T[(size_t)ct_index(i / CT, i / CT) * CT * CT + (CT + 1) * (i % CT)] = 1.0;
  __syncthreads();
  chol_tiles_factor(T, n, reinterpret_cast<float*>(Cs));
}

constexpr int CG = 32;          // block width of the global-memory Cholesky
constexpr int CG_NMAX = 512;    // largest n it takes

// LDS of the global-memory Cholesky: the diagonal block and the panel rows.
__host__ __device__ inline size_t cholg_lds_doubles(int n) {
  return (size_t)CG * (CG + 1) + (size_t)(n > CG ? n - CG : 0) * CG;
}

// Cholesky C = L L^T of one slice's Gram matrix for n beyond the LDS kernel,
// in place in global memory (FP64 lower triangle), blocked right-looking with
// CG columns per block.  Per block: the diagonal block goes to LDS and wave 0
// factors it; every lane solves one panel row against it, into LDS; then the
// block's columns of L are written in FP32 (the layout of the LDS kernel's
// output: n x n column-major over the first half of the slice's region, zero
// above the diagonal) while the workgroup applies the block's rank-CG update to
// the trailing lower triangle in global memory, 4 x 4 entries per lane.  The
// FP32 columns of a block overwrite FP64 columns that are no longer read (those
// of this and earlier blocks).  Pivots: as the LDS kernel.
__device__ __attribute__((always_inline)) void chol_slice_global(double* Cs, int n) {
  extern __shared__ __attribute__((aligned(16))) double S[];
  double* Dg = S;                      // CG x (CG + 1), row-major: Dg[i][j] = block (i, j)
  double* Pn = S + CG * (CG + 1);      // panel rows, row-major CG wide
  __shared__ double red_s[16];
  __shared__ double dinv_s[CG];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  double* C = Cs;
  float* L = reinterpret_cast<float*>(Cs);
  {   // max of the diagonal
    double d = 0.0;
    for (int j = tid; j < n; j += nt) d = fmax(d, C[j + (long long)j * n]);
    for (int o = 32; o >= 1; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
    if (lane == 0) red_s[wave] = d;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int w = 0; w < nt / 64; ++w) m = fmax(m, red_s[w]);
      red_s[0] = m;
    }
    __syncthreads();
  }
  const double thr = red_s[0] * (64.0 * n * DBL_EPSILON);
  for (int K = 0; K < n; K += CG) {
    const int kb = min(CG, n - K);
    const int t = n - K - kb;   // trailing rows (and columns)
    // (a) diagonal block
    for (int e = tid; e < kb * kb; e += nt) {
      const int i = e % kb, j = e / kb;
      Dg[i * (CG + 1) + j] = i >= j ? C[(K + i) + (long long)(K + j) * n] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      for (int k = 0; k < kb; ++k) {
        const double piv = Dg[k * (CG + 1) + k];
        const double inv = piv > thr ? rsq64(piv) : 0.0;   // 1 / L(k, k); 0 zeroes the column
        if (lane > k && lane < kb) Dg[lane * (CG + 1) + k] *= inv;
        wave_sync();
        const int r = kb - 1 - k;   // rows below k in the block
        for (int e = lane; e < r * r; e += 64) {
          const int ii = k + 1 + e / r, jj = k + 1 + e % r;
          if (jj <= ii) Dg[ii * (CG + 1) + jj] = fma(-Dg[ii * (CG + 1) + k], Dg[jj * (CG + 1) + k],
                                                     Dg[ii * (CG + 1) + jj]);
        }
        if (lane == 0) {
          Dg[k * (CG + 1) + k] = piv * inv;   // sqrt(piv), or 0
          dinv_s[k] = inv;
        }
        wave_sync();
      }
    }
    __syncthreads();
    // (b) panel: row K + kb + r solves x L11^T = C(row, K .. K + kb - 1), in
    // place in its LDS row (each lane owns its row)
    for (int r = tid; r < t; r += nt) {
      const int i = K + kb + r;
      double* x = Pn + (size_t)r * CG;
      for (int q = 0; q < kb; ++q) x[q] = C[i + (long long)(K + q) * n];
      for (int q = 0; q < kb; ++q) {
        double acc = x[q];
        for (int p = 0; p < q; ++p) acc = fma(-x[p], Dg[q * (CG + 1) + p], acc);
        x[q] = acc * dinv_s[q];
      }
    }
    __syncthreads();
    // (c) FP32 columns K .. K + kb - 1 of L
    for (long long e = tid; e < (long long)kb * n; e += nt) {
      const int j = K + (int)(e / n), i = (int)(e % n);
      double v = 0.0;
      if (i >= j) v = i < K + kb ? Dg[(i - K) * (CG + 1) + (j - K)] : Pn[(size_t)(i - K - kb) * CG + (j - K)];
      L[(long long)j * n + i] = (float)v;
    }
    // (d) trailing update C(i, j) -= sum_q P(i, q) P(j, q), K + kb <= j <= i < n,
    // in 4 x 4 tiles (bi >= bj) of the trailing triangle
    const int T4 = (t + 3) / 4;
    const int ntiles = T4 * (T4 + 1) / 2;
    for (int tt = tid; tt < ntiles; tt += nt) {
      int bi = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
      while ((bi + 1) * (bi + 2) / 2 <= tt) ++bi;
      while (bi * (bi + 1) / 2 > tt) --bi;
      const int bj = tt - bi * (bi + 1) / 2;
      const int i0 = 4 * bi, j0 = 4 * bj;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int q = 0; q < kb; ++q) {
        double pa[4], pb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          pa[a] = i0 + a < t ? Pn[(size_t)(i0 + a) * CG + q] : 0.0;
          pb[a] = j0 + a < t ? Pn[(size_t)(j0 + a) * CG + q] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(pa[a], pb[b], acc[a][b]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = K + kb + j0 + b;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = K + kb + i0 + a;
          if (i0 + a < t && j0 + b < t && i >= j) C[i + (long long)j * n] -= acc[a][b];
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_chol_global(CholArgs a) {
  chol_slice_global(a.C + (long long)blockIdx.x * a.c_stride, a.n);
}

__global__ __launch_bounds__(1024) void k_chol_global_items(ProbDev* const* probs, const CholItem* items) {
  const CholItem it = items[blockIdx.x];
  const ProbDev* pd = probs[it.prob];
  if (!pd->active) return;
  const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
  chol_slice_global(pd->C + (long long)it.slice * n * n, n);
}

__global__ __launch_bounds__(1024) void k_chol(CholArgs a) {
  chol_slice<false>(a.C + (long long)blockIdx.x * a.c_stride, a.n);
}

__global__ __launch_bounds__(1024) void k_chol_tiles(CholArgs a) {
  chol_tiles(a.C + (long long)blockIdx.x * a.c_stride, a.n);
}

__global__ __launch_bounds__(1024) void k_gram_chol_tiles(GramArgs g) {
  const int s = blockIdx.x;
  gram_chol_tiles(g.W + (long long)s * g.slice_stride, g.I1, g.I2, g.C + (long long)s * g.c_stride);
}

__global__ __launch_bounds__(1024) void k_chol_items(ProbDev* const* probs, const CholItem* items) {
  const CholItem it = items[blockIdx.x];
  const ProbDev* pd = probs[it.prob];
  if (!pd->active) return;
  const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
  chol_slice<true>(pd->C + (long long)it.slice * n * n, n);
}

__global__ __launch_bounds__(1024) void k_chol_tiles_items(ProbDev* const* probs, const CholItem* items) {
  const CholItem it = items[blockIdx.x];
  const ProbDev* pd = probs[it.prob];
  if (!pd->active) return;
  const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
  chol_tiles(pd->C + (long long)it.slice * n * n, n);
}

// ---- Cholesky for large n (the 1080- and 2160-column frames) -----------------
// The same right-looking blocked factorization (blocks of CG columns, pivots as
// above), with every stage a launch over all slices and, for the panel and the
// trailing update, many workgroups per slice: the FP64 lower triangle is
// factored in place in global memory, then written as an FP32 factor (zero
// above the diagonal) to its own buffer.

// thr[s] = 64 n eps64 max diag(C_s): pivots at or below it zero their column.
__global__ __launch_bounds__(256) void k_cholb_thr(const double* C, long long c_stride, int n, double* thr) {
  __shared__ double red[4];
  const double* Cs = C + (long long)blockIdx.x * c_stride;
  double d = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) d = fmax(d, Cs[j + (long long)j * n]);
  for (int o = 32; o >= 1; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0)
    thr[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * (64.0 * n * DBL_EPSILON);
}

// Diagonal block K..K+kb-1 of one slice factored in place by one wave, the
// block in registers: lane i holds row i (columns 0..i), so in step k the pivot
// and the entries L(j, k) of the scaled column reach every lane by readlane at
// indices fixed by the unrolled loops, and each lane updates its own row
// (pivots as above).  A short last block is padded to CG columns with a
// diagonal above the threshold and zero coupling, and each step masks column k
// to the rows below the pivot once, so the steps run without branches: every
// lane applies every update, which changes only entries above the diagonal
// (never read, never stored); the entries of the factor see the same operations
// in the same order as with per-entry guards.  With Dg, the factored block
// (zero above the diagonal) is also left in LDS for a panel solve.
__device__ __attribute__((always_inline)) void cholb_diag_wave(double* Cs, int n, int K, double t,
                                                               double (*Dg)[CG + 1]) {
  const int kb = min(CG, n - K);
  const int lane = threadIdx.x & 63;
  const double pad = 1.0 + 2.0 * t;   // > t (t >= 0): padded pivots keep their column
  const int lr = min(lane, kb - 1);   // clamped: every lane loads in bounds
  double v[CG];
#pragma unroll
  for (int j = 0; j < CG; ++j) {
    const double x = Cs[(K + lr) + (long long)(K + min(j, kb - 1)) * n];
    v[j] = (lane < kb && j <= lane) ? x : (lane == j ? pad : 0.0);
  }
#pragma unroll
  for (int k = 0; k < CG; ++k) {
    const double piv = readlane_d(v[k], k);
    const double inv = piv > t ? rsq64(piv) : 0.0;
    v[k] = lane == k ? piv * inv : v[k] * inv;
    const double vk = lane > k ? v[k] : 0.0;   // L(lane, k) below the pivot
#pragma unroll
    for (int j = k + 1; j < CG; ++j) {
      v[j] = fma(-vk, readlane_d(v[k], j), v[j]);
      // keeps the broadcast L(j, k) values from being hoisted en masse (they
      // would spill out of the scalar registers)
      if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
  }
  // fresh copies of n and K: the stores' column offsets are recomputed here
  // rather than kept in scalar registers from the loads through the steps
  int ns = n, Ks = K;
  asm volatile("" : "+s"(ns), "+s"(Ks));
#pragma unroll
  for (int j = 0; j < CG; ++j)
    if (lane < kb && j <= lane) Cs[(Ks + lane) + (long long)(Ks + j) * ns] = v[j];
  if (Dg && lane < kb) {
#pragma unroll
    for (int j = 0; j < CG; ++j)
      if (j < kb) Dg[lane][j] = j <= lane ? v[j] : 0.0;
  }
}

// Row i of the panel below the diagonal block: x L11^T = C(i, K..K+kb-1),
// solved in place against the factored block Dg and its reciprocal pivots
// (loaded first, solved and stored second).
__device__ __attribute__((always_inline)) void cholb_panel_load(const double* Cs, int n, int K, int kb, int i,
                                                                double (&x)[CG]) {
#pragma unroll
  for (int q = 0; q < CG; ++q) x[q] = q < kb ? Cs[i + (long long)(K + q) * n] : 0.0;
}

__device__ __attribute__((always_inline)) void cholb_panel_solve(double* Cs, int n, int K, int kb, int i,
                                                                 const double (*Dg)[CG + 1], const double* dinv,
                                                                 double (&x)[CG]) {
#pragma unroll
  for (int q = 0; q < CG; ++q) {
    if (q < kb) {
      double acc = x[q];
#pragma unroll
      for (int p2 = 0; p2 < CG; ++p2)
        if (p2 < q) acc = fma(-x[p2], Dg[q][p2], acc);
      x[q] = acc * dinv[q];
    }
  }
#pragma unroll
  for (int q = 0; q < CG; ++q)
    if (q < kb) Cs[i + (long long)(K + q) * n] = x[q];
}

__global__ __launch_bounds__(64) void k_cholb_diag(double* C, long long c_stride, int n, int K,
                                                  const double* thr) {
  cholb_diag_wave(C + (long long)blockIdx.x * c_stride, n, K, thr[blockIdx.x], nullptr);
}

// Panel rows K+kb .. n-1, one lane per row, against the block factored by
// k_cholb_diag (read back from C).
__global__ __launch_bounds__(256) void k_cholb_panel(double* C, long long c_stride, int n, int K) {
  __shared__ double Dg[CG][CG + 1];
  __shared__ double dinv[CG];
  double* Cs = C + (long long)blockIdx.y * c_stride;
  const int kb = min(CG, n - K);
  for (int e = threadIdx.x; e < kb * kb; e += 256) {
    const int i = e % kb, j = e / kb;
    Dg[i][j] = i >= j ? Cs[(K + i) + (long long)(K + j) * n] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < kb) {
    const double d = Dg[threadIdx.x][threadIdx.x];
    dinv[threadIdx.x] = d > 0.0 ? 1.0 / d : 0.0;
  }
  __syncthreads();
  const int i = K + kb + blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    double x[CG];
    cholb_panel_load(Cs, n, K, kb, i, x);
    cholb_panel_solve(Cs, n, K, kb, i, Dg, dinv, x);
  }
}

// Both in one launch when the panel is short: wave 0 factors the block into C
// and LDS while the other waves, one panel row per lane, load their rows; then
// they solve them.  This saves a launch and a read of the block per step and
// overlaps the row loads with the factorization; the same arithmetic as the
// two kernels above.
constexpr int CHOLB_FUSED_ROWS = 256;   // panel rows up to which the step is fused

__global__ __launch_bounds__(64 + CHOLB_FUSED_ROWS) void k_cholb_diag_panel(double* C, long long c_stride, int n,
                                                                            int K, const double* thr) {
  __shared__ double Dg[CG][CG + 1];
  __shared__ double dinv[CG];
  double* Cs = C + (long long)blockIdx.x * c_stride;
  const int kb = min(CG, n - K);
  const int tid = threadIdx.x;
  const int i = K + kb + tid - 64;
  const bool prow = tid >= 64 && i < n;
  double x[CG];
  if (tid < 64) cholb_diag_wave(Cs, n, K, thr[blockIdx.x], Dg);
  else if (prow) cholb_panel_load(Cs, n, K, kb, i, x);
  __syncthreads();
  if (tid < kb) {
    const double d = Dg[tid][tid];
    dinv[tid] = d > 0.0 ? 1.0 / d : 0.0;
  }
  __syncthreads();
  if (prow) cholb_panel_solve(Cs, n, K, kb, i, Dg, dinv, x);
}

// Trailing update C(i, j) -= sum_q P(i, q) P(j, q) over the trailing lower
// triangle (rows and columns K+kb ..), one 64 x 64 tile (bi >= bj) per
// workgroup, the two panel row blocks staged in LDS, 4 x 4 outputs per lane.
__global__ __launch_bounds__(256) void k_cholb_update(double* C, long long c_stride, int n, int K) {
  __shared__ double Pi[64][CG + 1];
  __shared__ double Pj[64][CG + 1];
  double* Cs = C + (long long)blockIdx.y * c_stride;
  const int kb = min(CG, n - K);
  const int T0 = K + kb;
  int bi = (int)((sqrt(8.0 * blockIdx.x + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= (int)blockIdx.x) ++bi;
  while (bi * (bi + 1) / 2 > (int)blockIdx.x) --bi;
  const int bj = blockIdx.x - bi * (bi + 1) / 2;
  const int i0 = T0 + 64 * bi, j0 = T0 + 64 * bj;
  for (int e = threadIdx.x; e < 64 * CG; e += 256) {
    const int r = e % 64, q = e / 64;
    Pi[r][q] = (q < kb && i0 + r < n) ? Cs[(i0 + r) + (long long)(K + q) * n] : 0.0;
    Pj[r][q] = (q < kb && j0 + r < n) ? Cs[(j0 + r) + (long long)(K + q) * n] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int q = 0; q < kb; ++q) {
    double pa[4], pb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      pa[a] = Pi[tx + 16 * a][q];
      pb[a] = Pj[ty + 16 * a][q];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(pa[a], pb[b], acc[a][b]);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int j = j0 + ty + 16 * b;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + tx + 16 * a;
      if (i < n && j < n && i >= j) Cs[i + (long long)j * n] -= acc[a][b];
    }
  }
}

// FP32 factor: L[i + j n] = C(i, c) with c = j col_step, for i >= c, 0 above
// the diagonal; j < ncols (col_step 2: the even columns only).
__global__ __launch_bounds__(256) void k_cholb_fp32(const double* C, long long c_stride, float* L,
                                                   long long l_stride, int n, int ncols, int col_step) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)n * ncols) return;
  const int j = (int)(e / n), i = (int)(e - (long long)j * n);
  const int c = j * col_step;
  const double* Cs = C + (long long)blockIdx.y * c_stride;
  L[(long long)blockIdx.y * l_stride + e] = i >= c ? (float)Cs[(long long)c * n + i] : 0.f;
}

}  // namespace

hipError_t launch_chol_big(double* C, long long c_stride, int n, int nslices, float* L, long long l_stride,
                           double* thr, hipStream_t s, int col_step) {
  if (nslices <= 0) return hipSuccess;
  if (n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cholb_thr, dim3(nslices), dim3(256), 0, s, C, c_stride, n, thr);
  hipError_t e = hipGetLastError();
  for (int K = 0; K < n && e == hipSuccess; K += CG) {
    const int kb = n - K < CG ? n - K : CG;
    const int t = n - K - kb;
    if (t <= CHOLB_FUSED_ROWS) {
      hipLaunchKernelGGL(k_cholb_diag_panel, dim3(nslices), dim3(64 + CHOLB_FUSED_ROWS), 0, s, C, c_stride, n, K,
                         thr);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if (t <= 0) break;
    } else {
      hipLaunchKernelGGL(k_cholb_diag, dim3(nslices), dim3(64), 0, s, C, c_stride, n, K, thr);
      if ((e = hipGetLastError()) != hipSuccess) break;
      hipLaunchKernelGGL(k_cholb_panel, dim3((t + 255) / 256, nslices), dim3(256), 0, s, C, c_stride, n, K);
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    const int T64 = (t + 63) / 64;
    hipLaunchKernelGGL(k_cholb_update, dim3(T64 * (T64 + 1) / 2, nslices), dim3(256), 0, s, C, c_stride, n, K);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  const int ncols = (n + col_step - 1) / col_step;
  const long long nn = (long long)n * ncols;
  hipLaunchKernelGGL(k_cholb_fp32, dim3((unsigned)((nn + 255) / 256), nslices), dim3(256), 0, s, C, c_stride,
                     L, l_stride, n, ncols, col_step);
  return hipGetLastError();
}

// LDS of the LDS Cholesky kernel for slices up to n columns: the tiled
// kernel's up to CT_NMAX, the packed triangle's beyond.
size_t chol_lds_bytes(int n) {
  return n <= CT_NMAX ? ct_lds_bytes(n) : (size_t)n * (n + 1) / 2 * sizeof(double);
}

hipError_t launch_gram_cx(const float* W, long long w_stride, long long col_stride, int m, int n, double* C,
                          long long c_stride, int nslices, hipStream_t s) {
  if (nslices <= 0) return hipSuccess;
  if (m < 1 || n < 1 || c_stride < 4LL * n * n) return hipErrorInvalidValue;
  const int nt = (n + GCX - 1) / GCX;
  hipLaunchKernelGGL(k_gram_cx, dim3(nt * (nt + 1) / 2, nslices), dim3(256), 0, s, W, w_stride, col_stride, m, n, C,
                     c_stride);
  return hipGetLastError();
}

hipError_t launch_gram(const GramArgs& a, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  const int n = a.I1 < a.I2 ? a.I1 : a.I2;
  const int nt = (n + GT - 1) / GT;
  hipLaunchKernelGGL(k_gram, dim3(nt * (nt + 1) / 2, a.nslices), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gram_tiles(ProbDev* const* probs, const GramTile* tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_tiles, dim3(ntiles), dim3(256), 0, s, probs, tiles);
  return hipGetLastError();
}

hipError_t launch_chol_items(ProbDev* const* probs, const CholItem* items, int nitems, int nmax,
                             hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (nmax > CH_NMAX) {
    // items of slices beyond the LDS kernel (every item of this list)
    if (nmax > CG_NMAX) return hipErrorInvalidValue;
    const size_t lds = cholg_lds_doubles(nmax) * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)k_chol_global_items,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chol_global_items, dim3(nitems), dim3(1024), lds, s, probs, items);
    return hipGetLastError();
  }
  if (nmax < 1) return hipErrorInvalidValue;
  // every item by the tiled kernel when all fit it, else by the packed one
  const void* fn = nmax <= CT_NMAX ? (const void*)k_chol_tiles_items : (const void*)k_chol_items;
  const size_t lds = chol_lds_bytes(nmax);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nmax <= CT_NMAX)
    hipLaunchKernelGGL(k_chol_tiles_items, dim3(nitems), dim3(nmax <= 64 ? 256 : 1024), lds, s, probs, items);
  else
    hipLaunchKernelGGL(k_chol_items, dim3(nitems), dim3(1024), lds, s, probs, items);
  return hipGetLastError();
}

hipError_t launch_gram_chol(const GramArgs& g, hipStream_t s) {
  if (g.nslices <= 0) return hipSuccess;
  const int n = g.I1 < g.I2 ? g.I1 : g.I2;
  if (n < 1 || n > CTG_NMAX) return hipErrorInvalidValue;
  const size_t lds = ctg_lds_bytes(n);
  hipError_t e = hipFuncSetAttribute((const void*)k_gram_chol_tiles, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_chol_tiles, dim3(g.nslices), dim3(n <= 64 ? 256 : 1024), lds, s, g);
  return hipGetLastError();
}

hipError_t launch_chol(const CholArgs& a, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  if (a.n > CH_NMAX) {
    if (a.n > CG_NMAX) return hipErrorInvalidValue;
    const size_t lds = cholg_lds_doubles(a.n) * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)k_chol_global, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chol_global, dim3(a.nslices), dim3(1024), lds, s, a);
    return hipGetLastError();
  }
  if (a.n < 1) return hipErrorInvalidValue;
  const void* fn = a.n <= CT_NMAX ? (const void*)k_chol_tiles : (const void*)k_chol;
  const size_t lds = chol_lds_bytes(a.n);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (a.n <= CT_NMAX)
    hipLaunchKernelGGL(k_chol_tiles, dim3(a.nslices), dim3(a.n <= 64 ? 256 : 1024), lds, s, a);
  else
    hipLaunchKernelGGL(k_chol, dim3(a.nslices), dim3(1024), lds, s, a);
  return hipGetLastError();
}

}  // namespace lt
