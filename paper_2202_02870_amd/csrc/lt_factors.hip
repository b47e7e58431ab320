// Factor post-processing of the *_L-SVD (Alg. 3) and the multirank of
// Section 3.2, on the transform-domain slices:
//   * full factors: Alg. 3 returns U (I1 x I1), S (I1 x I2), V (I2 x I2) per
//     slice.  The Jacobi gives the economy factors (n = min(I1, I2) columns);
//     the longer side's factor is completed with an orthonormal basis of the
//     orthogonal complement of its n columns, taken from a Householder QR of
//     those columns (Q = H_0 ... H_{n-1} [R; 0], and the last m - n columns of
//     H_0 ... H_{n-1} span the complement), and S is padded with zeros;
//   * multirank: the number of singular values of each slice of L(A) above a
//     tolerance relative to the largest of the tensor, their mean and maximum
//     (the average rank and tubal rank).
#include "lt_internal.h"

#include <math.h>

namespace lt {

namespace {

__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic sum over a 256-thread workgroup (result in every thread).
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum64(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// dst (rd x cd per slice, column-major) = src (rs x cs per slice) padded with zeros.
__global__ void k_pad_copy(const float* src, float* dst, int rs, int cs, int rd, int cd) {
  const long long p = blockIdx.y;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rd * cd) return;
  const int j = (int)(e / rd), i = (int)(e - (long long)j * rd);
  dst[p * rd * cd + e] = (i < rs && j < cs) ? src[p * rs * cs + (long long)j * rs + i] : 0.f;
}

// Householder QR of the first n columns of each slice's m x m factor Q (FP32),
// in FP64: H (m x n per slice) receives the reflector vectors v_k (rows k..m-1
// of column k; v_k[k] = x_k - alpha_k), beta[k] = 2 / (v_k^T v_k) (0 for an
// already reduced column).  One workgroup (4 waves) per slice; the trailing
// columns are updated one wave per column.
__global__ __launch_bounds__(256) void k_householder(const float* Q, double* H, double* beta, int m, int n) {
  __shared__ double red[4];
  const long long p = blockIdx.x;
  const float* Qs = Q + p * m * m;
  double* Hs = H + p * m * n;
  double* bs = beta + p * n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (long long e = tid; e < (long long)m * n; e += 256) Hs[e] = (double)Qs[e];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double* x = Hs + (long long)k * m;
    double part = 0.0;
    for (int i = k + 1 + tid; i < m; i += 256) part += x[i] * x[i];
    const double tail = block_sum(part, red);
    const double x0 = x[k];
    const double nrm = sqrt(x0 * x0 + tail);
    // v = x - alpha e_k with alpha = -sign(x0) ||x||: no cancellation in v_k
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vtv = v0 * v0 + tail;
    const double b = vtv > 0.0 ? 2.0 / vtv : 0.0;
    __syncthreads();   // every thread has read x[k]
    if (tid == 0) {
      x[k] = v0;
      bs[k] = b;
    }
    __syncthreads();
    // A(k:m, j) -= b v (v^T A(k:m, j)) for the columns j > k
    for (int j = k + 1 + w; j < n; j += 4) {
      double* a = Hs + (long long)j * m;
      double d = 0.0;
      for (int i = k + l; i < m; i += 64) d += x[i] * a[i];
      d = wave_sum64(d) * b;
      for (int i = k + l; i < m; i += 64) a[i] -= d * x[i];
    }
    __syncthreads();
  }
}

// Columns n..m-1 of each slice's factor: Q[:, n + c] = H_0 H_1 ... H_{n-1} e_{n+c}
// (the reflectors applied last to first), one wave per column, the column in
// registers (m <= 64 * kRows).
constexpr int kRows = 32;
__global__ __launch_bounds__(256) void k_complement(const double* H, const double* beta, float* Q, int m, int n) {
  const long long p = blockIdx.y;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (n + c >= m) return;   // wave-uniform
  const double* Hs = H + p * m * n;
  const double* bs = beta + p * n;
  const int col = n + c;
  double v[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) v[r] = (l + 64 * r == col) ? 1.0 : 0.0;
  for (int k = n - 1; k >= 0; --k) {
    const double* x = Hs + (long long)k * m;
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int i = l + 64 * r;
      if (i >= k && i < m) d += x[i] * v[r];
    }
    d = wave_sum64(d) * bs[k];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int i = l + 64 * r;
      if (i >= k && i < m) v[r] -= d * x[i];
    }
  }
  float* out = Q + p * m * m + (long long)col * m;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = l + 64 * r;
    if (i < m) out[i] = (float)v[r];
  }
}

// Multirank: sigma is P x n (FP64, slice-major).  rank[p] = #{i : sigma[p][i] >
// rtol * max(sigma)}; out[0] = the mean of rank, out[1] = its maximum.  One
// workgroup, fixed summation order.
__global__ __launch_bounds__(256) void k_multirank(const double* sigma, int P, int n, double rtol, int32_t* rank,
                                                   double* out) {
  __shared__ double red[4];
  __shared__ double mx[256];
  const int tid = threadIdx.x;
  double m = 0.0;
  for (long long e = tid; e < (long long)P * n; e += 256) m = fmax(m, sigma[e]);
  mx[tid] = m;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) mx[tid] = fmax(mx[tid], mx[tid + o]);
    __syncthreads();
  }
  const double cut = rtol * fmax(mx[0], 1e-300);
  __syncthreads();
  double sum = 0.0, top = 0.0;
  for (int p = tid; p < P; p += 256) {
    int r = 0;
    for (int i = 0; i < n; ++i) r += sigma[(long long)p * n + i] > cut;
    rank[p] = r;
    sum += (double)r;
    top = fmax(top, (double)r);
  }
  sum = block_sum(sum, red);
  mx[tid] = top;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) mx[tid] = fmax(mx[tid], mx[tid + o]);
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = P > 0 ? sum / (double)P : 0.0;
    out[1] = mx[0];
  }
}

// Batched FP32 GEMM for the rebuild of slices with many kept columns:
// C_s = op(A_s) op(B_s), column-major, op(A) M x K, op(B) K x N, with the
// slice's kept count limiting N (rank_dim 1) or K (rank_dim 2).  64 x 64 output
// tile per workgroup, K in chunks of 16 through LDS, 4 x 4 outputs per lane,
// FP32 accumulation.
struct BGemm {
  const float* A;
  long long lda, sA;
  int tA;
  const float* B;
  long long ldb, sB;
  int tB;
  float* C;
  long long ldc, sC;
  int M, N, K;
  const int32_t* rank;
  int rank_dim;
};

__global__ __launch_bounds__(256) void k_bgemm(BGemm g) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int s = blockIdx.z;
  const int r = g.rank ? g.rank[s] : 0;
  const int N = g.rank_dim == 1 ? min(g.N, r) : g.N;
  const int K = g.rank_dim == 2 ? min(g.K, r) : g.K;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (j0 >= N) return;
  const float* A = g.A + (long long)s * g.sA;
  const float* B = g.B + (long long)s * g.sB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      // A tile: rows i0..i0+63 of op(A), columns k0..k0+15; B tile likewise
      int kk, ii;
      if (g.tA) { kk = e % 16; ii = e / 16; } else { ii = e % 64; kk = e / 64; }
      const int i = i0 + ii, k = k0 + kk;
      As[kk][ii] = (i < g.M && k < K) ? (g.tA ? A[k + (long long)i * g.lda] : A[i + (long long)k * g.lda]) : 0.f;
      int kb, jj;
      if (g.tB) { jj = e % 64; kb = e / 64; } else { kb = e % 16; jj = e / 16; }
      const int j = j0 + jj, k2 = k0 + kb;
      Bs[kb][jj] = (j < N && k2 < K) ? (g.tB ? B[j + (long long)k2 * g.ldb] : B[k2 + (long long)j * g.ldb]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        av[a] = As[kk][tx + 16 * a];
        bv[a] = Bs[kk][ty + 16 * a];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  float* C = g.C + (long long)s * g.sC;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int j = j0 + ty + 16 * b;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + tx + 16 * a;
      if (i < g.M && j < N) C[i + (long long)j * g.ldc] = acc[a][b];
    }
  }
}

hipError_t bgemm(const BGemm& g, int nslices, hipStream_t s) {
  dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64), (unsigned)nslices);
  hipLaunchKernelGGL(k_bgemm, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace

// The SVT rebuild from the kept columns for any kept count, as two batched
// GEMMs through T (P x I1 x I2 floats).  Slice S (I1 x I2); working matrix W = S
// (I1 >= I2) or S^T.  flip 0 (Bk: m x r): D_W = Bk (Bk^T W), i.e. D = Bk (Bk^T S)
// or D = (S Bk) Bk^T; flip 1 (B: n x r, the preconditioned path): D_W = (W B) B^T,
// i.e. D = (S B) B^T or D = B (B^T S).
hipError_t launch_rebuild_gemm(const RebuildArgs& r, float* T, hipStream_t s) {
  if (r.nslices <= 0) return hipSuccess;
  const bool trans = r.I1 < r.I2;
  const int I1 = r.I1, I2 = r.I2;
  const int m = trans ? I2 : I1, n = trans ? I1 : I2;
  const long long N = (long long)I1 * I2;
  const int rows_b = r.flip ? n : m;   // rows of the kept-column matrix
  // left = 1: D = X (X^T S) with X the kept columns (rows I1); left = 0: D = (S X) X^T (rows I2)
  const bool left = r.flip ? trans : !trans;
  (void)rows_b;
  BGemm g1{}, g2{};
  if (left) {
    // T = X^T S (r x I2), D = X T
    g1.A = r.bk; g1.lda = I1; g1.sA = r.slice_stride; g1.tA = 1;
    g1.B = r.W; g1.ldb = I1; g1.sB = r.slice_stride; g1.tB = 0;
    g1.C = T; g1.ldc = n; g1.sC = N;
    g1.M = n; g1.N = I2; g1.K = I1; g1.rank = r.rank; g1.rank_dim = 0;
    // rows of T beyond the kept count are never read (K of the second product)
    g2.A = r.bk; g2.lda = I1; g2.sA = r.slice_stride; g2.tA = 0;
    g2.B = T; g2.ldb = n; g2.sB = N; g2.tB = 0;
    g2.C = r.D; g2.ldc = I1; g2.sC = r.slice_stride;
    g2.M = I1; g2.N = I2; g2.K = n; g2.rank = r.rank; g2.rank_dim = 2;
  } else {
    // T = S X (I1 x r), D = T X^T
    g1.A = r.W; g1.lda = I1; g1.sA = r.slice_stride; g1.tA = 0;
    g1.B = r.bk; g1.ldb = I2; g1.sB = r.slice_stride; g1.tB = 0;
    g1.C = T; g1.ldc = I1; g1.sC = N;
    g1.M = I1; g1.N = n; g1.K = I2; g1.rank = r.rank; g1.rank_dim = 1;
    g2.A = T; g2.lda = I1; g2.sA = N; g2.tA = 0;
    g2.B = r.bk; g2.ldb = I2; g2.sB = r.slice_stride; g2.tB = 1;
    g2.C = r.D; g2.ldc = I1; g2.sC = r.slice_stride;
    g2.M = I1; g2.N = I2; g2.K = n; g2.rank = r.rank; g2.rank_dim = 2;
  }
  hipError_t e = bgemm(g1, r.nslices, s);
  if (e != hipSuccess) return e;
  return bgemm(g2, r.nslices, s);
}

hipError_t launch_pad_copy(const float* src, float* dst, int rs, int cs, int rd, int cd, int P, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  const long long e = (long long)rd * cd;
  dim3 grid((unsigned)((e + 255) / 256), (unsigned)P);
  hipLaunchKernelGGL(k_pad_copy, grid, dim3(256), 0, s, src, dst, rs, cs, rd, cd);
  return hipGetLastError();
}

hipError_t launch_complete_basis(float* Q, double* H, double* beta, int m, int n, int P, hipStream_t s) {
  if (P <= 0 || n >= m) return hipSuccess;
  if (m > 64 * kRows || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_householder, dim3((unsigned)P), dim3(256), 0, s, Q, H, beta, m, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((m - n + 3) / 4), (unsigned)P);
  hipLaunchKernelGGL(k_complement, grid, dim3(256), 0, s, H, beta, Q, m, n);
  return hipGetLastError();
}

hipError_t launch_multirank(const double* sigma, int P, int n, double rtol, int32_t* rank, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_multirank, dim3(1), dim3(256), 0, s, sigma, P, n, rtol, rank, out);
  return hipGetLastError();
}

}  // namespace lt
