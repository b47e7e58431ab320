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

}  // namespace

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
