// Transform-domain kernels: the invertible transform L as one GEMM with the
// Kronecker matrix K = M_N (x) ... (x) M_3 (Section 3.2: L(A) = A x_3 M_3 ...
// x_N M_N; with the Vec slice order of eq. (3.5), L(A)^q = sum_p K[q,p] A^p),
// the masked momentum step of eqs. (51)-(52) fused into the forward GEMM's
// operand load, and the stopping-rule norms of Section 5 fused into the
// inverse GEMM's store.
#include "lt_internal.h"

#include <math.h>

namespace lt {

namespace {

constexpr int TQ = 64;   // output rows (transform-domain slices) per workgroup
constexpr int TE = 64;   // output columns (slice entries) per workgroup
constexpr int TPK = 32;  // contraction chunk staged in LDS

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic workgroup sum of two doubles (256 threads), result in thread 0.
// Workgroups of 4, 8 or 12 waves (a multiple of four, at most 16): the waves'
// sums in groups of four, each group pairwise, the groups in order.
__device__ inline void block_sum2(double& s1, double& s2) {
  __shared__ double red[2][16];
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = (int)(blockDim.x >> 6);
  if (l == 0) { red[0][w] = s1; red[1][w] = s2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nw; i += 4) {
      a += (red[0][i] + red[0][i + 1]) + (red[0][i + 2] + red[0][i + 3]);
      b += (red[1][i] + red[1][i + 1]) + (red[1][i + 2] + red[1][i + 3]);
    }
    s1 = a;
    s2 = b;
  }
}

template <int PRO>
__device__ inline float load_operand(const GemmArgs& a, long long g) {
  if (PRO == PRO_PLAIN) return a.B[g];
  if (!a.mask) return a.M[g];                           // every entry observed: G = M
  const float x = a.X[g];
  const float y = x + a.beta * (x - a.Xp[g]);          // eq. (52)
  return a.mask[g] ? a.M[g] : y;                        // eq. (51), step 1/l_f = 1
}

template <int EPI>
__device__ inline void store_result(const GemmArgs& a, long long g, float o, double& s1,
                                    double& s2) {
  if (EPI == EPI_PGA) {
    const float x = a.X[g];
    const float y = x + a.beta * (x - a.Xp[g]);
    const double d = (double)y - (double)o;
    s1 += d * d;
    s2 += (double)o * (double)o;
  }
  a.out[g] = o;
}

// FP32 MFMA (v_mfma_f32_16x16x4_f32).  Workgroup = NW waves; tile (16 NW) x 64;
// wave w owns output rows 16w..16w+15 and four 16-column sub-tiles.  NW = 4
// in general; with up to 192 output rows one workgroup of NW = 4, 8 or 12
// waves takes them all, so the staged input (with the momentum prologue's four
// reads per entry) is read from memory once instead of once per 64 rows.
// Operand lane layout of the 16x16x4 instruction: A[i][k] at lane i + 16k,
// B[k][j] at lane j + 16k, D[i][j] in element i%4 of lane j + 16(i/4).
template <int PRO, int EPI, int NW = 4>
__device__ void gemm_f32_tile(const GemmArgs& a, int tx, int ty, double* part) {
  constexpr int TQW = 16 * NW;
  constexpr int NT = 64 * NW;
  __shared__ float Ks[TQW][TPK + 1];
  __shared__ float Bs[TPK][TE + 4];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const long long e0 = (long long)tx * TE;
  const int q0 = ty * TQW;
  const int Mo = a.Mo ? a.Mo : a.P;   // output rows
  const int Kd = a.Kd ? a.Kd : a.P;   // contraction length (input rows)
  const long long N = a.N;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int p0 = 0; p0 < Kd; p0 += TPK) {
    for (int idx = tid; idx < TQW * TPK; idx += NT) {
      const int i = idx / TPK, k = idx - i * TPK;
      const int q = q0 + i, p = p0 + k;
      Ks[i][k] = (q < Mo && p < Kd) ? a.K[(long long)q * Kd + p] : 0.f;
    }
    for (int idx = tid; idx < TPK * TE; idx += NT) {
      const int k = idx / TE, j = idx - k * TE;
      const int p = p0 + k;
      const long long e = e0 + j;
      Bs[k][j] = (p < Kd && e < N) ? load_operand<PRO>(a, (long long)p * N + e) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TPK; kk += 4) {
      const float av = Ks[16 * w + (l & 15)][kk + (l >> 4)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float bv = Bs[kk + (l >> 4)][16 * t + (l & 15)];
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = q0 + 16 * w + 4 * (l >> 4) + v;
      const long long e = e0 + 16 * t + (l & 15);
      if (q < Mo && e < N) store_result<EPI>(a, (long long)q * N + e, acc[t][v], s1, s2);
    }
  }
  if (EPI == EPI_PGA) {
    block_sum2(s1, s2);
    if (threadIdx.x == 0) {
      part[0] = s1;
      part[1] = s2;
    }
  }
}

template <int PRO, int EPI, int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_f32(GemmArgs a) {
  gemm_f32_tile<PRO, EPI, NW>(a, blockIdx.x, blockIdx.y,
                              a.partials + 2 * ((long long)blockIdx.y * gridDim.x + blockIdx.x));
}

// BF16 MFMA (v_mfma_f32_16x16x32_bf16) on hi/lo splits: K ~ Kh + Kl and
// in ~ Bh + Bl, product Kh Bh + Kh Bl + Kl Bh with FP32 accumulation.
// Lane layout of the 16x16x32 instruction: A[i][8c..8c+7] at lane i + 16c,
// B[8c..8c+7][j] at lane j + 16c, D as for the FP32 instruction.
template <int PRO, int EPI>
__device__ void gemm_bf16x3_tile(const GemmArgs& a, int tx, int ty, double* part) {
  constexpr int KP = TPK + 8;  // row pitch in halves (80 B: keeps 16-B alignment)
  __shared__ __attribute__((aligned(16))) uint16_t Kh[TQ][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Kl[TQ][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[TE][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[TE][KP];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const long long e0 = (long long)tx * TE;
  const int q0 = ty * TQ;
  const int Mo = a.Mo ? a.Mo : a.P;
  const int Kd = a.Kd ? a.Kd : a.P;
  const long long N = a.N;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int p0 = 0; p0 < Kd; p0 += TPK) {
    for (int idx = tid; idx < TQ * TPK; idx += 256) {
      const int i = idx / TPK, k = idx - i * TPK;
      const int q = q0 + i, p = p0 + k;
      const bool in = (q < Mo && p < Kd);
      Kh[i][k] = in ? a.Khi[(long long)q * Kd + p] : (uint16_t)0;
      Kl[i][k] = in ? a.Klo[(long long)q * Kd + p] : (uint16_t)0;
    }
    for (int idx = tid; idx < TPK * TE; idx += 256) {
      const int k = idx / TE, j = idx - k * TE;
      const int p = p0 + k;
      const long long e = e0 + j;
      const float v = (p < Kd && e < N) ? load_operand<PRO>(a, (long long)p * N + e) : 0.f;
      const uint16_t h = f32_to_bf16_bits(v);
      Bh[j][k] = h;
      Bl[j][k] = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
    }
    __syncthreads();
    const int c = l >> 4;
    const uint4 ah = *reinterpret_cast<const uint4*>(&Kh[16 * w + (l & 15)][8 * c]);
    const uint4 al = *reinterpret_cast<const uint4*>(&Kl[16 * w + (l & 15)][8 * c]);
    const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah);
    const bf16x8 Al = __builtin_bit_cast(bf16x8, al);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint4 bh = *reinterpret_cast<const uint4*>(&Bh[16 * t + (l & 15)][8 * c]);
      const uint4 bl = *reinterpret_cast<const uint4*>(&Bl[16 * t + (l & 15)][8 * c]);
      const bf16x8 Bhv = __builtin_bit_cast(bf16x8, bh);
      const bf16x8 Blv = __builtin_bit_cast(bf16x8, bl);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Blv, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bhv, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bhv, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }

  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = q0 + 16 * w + 4 * (l >> 4) + v;
      const long long e = e0 + 16 * t + (l & 15);
      if (q < Mo && e < N) store_result<EPI>(a, (long long)q * N + e, acc[t][v], s1, s2);
    }
  }
  if (EPI == EPI_PGA) {
    block_sum2(s1, s2);
    if (threadIdx.x == 0) {
      part[0] = s1;
      part[1] = s2;
    }
  }
}

template <int PRO, int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(GemmArgs a) {
  gemm_bf16x3_tile<PRO, EPI>(a, blockIdx.x, blockIdx.y,
                             a.partials + 2 * ((long long)blockIdx.y * gridDim.x + blockIdx.x));
}

// Grouped transform GEMMs of a batch: one workgroup per (problem, tile).  The
// forward pass builds G from the problem's current iterates (parity) and writes
// the transform-domain slices; the inverse pass writes X^{k+1} over X^{k-1} and
// the per-tile stopping norms.
template <int PREC, int INV>
__global__ __launch_bounds__(256) void k_gemm_grouped(ProbDev* const* probs, const GemmTile* tiles) {
  const GemmTile t = tiles[blockIdx.x];
  const ProbDev* pd = probs[t.prob];
  if (!pd->active) return;
  GemmArgs a{};
  a.P = pd->P;
  a.N = pd->N;
  a.K = INV ? pd->Kinv : pd->K;
  a.Khi = INV ? pd->Kihi : pd->Khi;
  a.Klo = INV ? pd->Kilo : pd->Klo;
  float* cur = pd->parity ? pd->Xb : pd->Xa;
  float* prev = pd->parity ? pd->Xa : pd->Xb;
  a.X = cur;
  a.Xp = prev;
  a.beta = (float)pd->beta;
  if constexpr (!INV) {
    a.M = pd->M;
    a.mask = pd->mask;
    a.out = pd->Gh;
    if constexpr (PREC != 0) gemm_bf16x3_tile<PRO_PGA, EPI_PLAIN>(a, t.tx, t.ty, nullptr);
    else gemm_f32_tile<PRO_PGA, EPI_PLAIN>(a, t.tx, t.ty, nullptr);
  } else {
    a.B = pd->Gh;
    a.out = prev;
    double* part = pd->partials + 2 * (long long)t.part;
    if constexpr (PREC != 0) gemm_bf16x3_tile<PRO_PLAIN, EPI_PGA>(a, t.tx, t.ty, part);
    else gemm_f32_tile<PRO_PLAIN, EPI_PGA>(a, t.tx, t.ty, part);
  }
}

// Start of a tick: problems that are enabled and not finished take part and
// load this iteration's scalars (Alg. 5: beta_k of eq. (52), threshold mu_k).
__global__ void k_batch_begin(ProbDev* const* probs, int nprob) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nprob) return;
  ProbDev* p = probs[i];
  const int act = p->enabled && !p->done && p->iter < p->max_iter;
  p->active = act;
  if (act) {
    p->beta = p->betas[p->iter];
    p->tau = p->mus[p->iter];
  }
}

// End of a tick: stopping ratio ||Y - X^{k+1}|| / ||X^{k+1}|| from the tile
// partials (fixed summation order), iteration count, iterate parity, and the
// stopping rule (gated until mu_k reaches mu_bar when requested).
__global__ __launch_bounds__(256) void k_batch_end(ProbDev* const* probs, int nprob) {
  ProbDev* p = probs[blockIdx.x];
  if (!p->active) return;
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < p->n_partials; i += 256) {
    s1 += p->partials[2 * i];
    s2 += p->partials[2 * i + 1];
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) {
    const double crit = s2 > 0.0 ? sqrt(s1) / sqrt(s2) : INFINITY;
    const bool at_floor = p->mus[p->iter] <= p->mu_bar;
    p->num = s1;
    p->den = s2;
    p->crit = crit;
    p->iter += 1;
    p->parity ^= 1;
    if (p->tol > 0.0 && crit <= p->tol && (at_floor || !p->gate_until_floor)) p->done = 1;
    else if (p->iter >= p->max_iter) p->done = 2;
  }
}

__global__ void k_fill_zero(uint32_t* p, long long nwords) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Entry (r, c) of the mode matrix: orthonormal DCT-II
// sqrt((2 - delta_{r,0}) / n) cos(r (2c + 1) pi / (2n)) (0-based indices).
__device__ inline double dct_entry(int r, int c, int n) {
  const double s = sqrt((r == 0 ? 1.0 : 2.0) / (double)n);
  return s * cos((double)r * (double)(2 * c + 1) * M_PI / (2.0 * (double)n));
}

__global__ void k_build_kron(KronDesc d, int P, int inverse, float* K, uint16_t* Khi,
                             uint16_t* Klo) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)P * P) return;
  int rq = (int)(idx / P), rp = (int)(idx % P);
  double v = 1.0;
  for (int m = 0; m < d.nmodes; ++m) {
    const int n = d.n[m];
    const int j = rq % n, k = rp % n;
    rq /= n;
    rp /= n;
    double e;
    if (d.kind[m] == 0) {
      e = inverse ? dct_entry(k, j, n) : dct_entry(j, k, n);   // C^{-1} = C^T
    } else if (d.kind[m] == 2) {
      e = (j == k) ? 1.0 : 0.0;
    } else {
      e = d.custom[m][(long long)j * n + k];
    }
    v *= e;
  }
  const float f = (float)v;
  K[idx] = f;
  if (Khi) {
    const uint16_t h = f32_to_bf16_bits(f);
    Khi[idx] = h;
    Klo[idx] = f32_to_bf16_bits(f - bf16_bits_to_f32(h));
  }
}

// Stacked real form of a transform with Fourier modes (Section 2: F_n =
// [w^{jk}], w = exp(-2 pi i / n), F_n^{-1} = F_n^* / n).  Forward: [Re K; Im K]
// (2P x P, row-major), so that for a real input the GEMM writes the real plane
// (rows 0..P-1) and the imaginary plane (rows P..2P-1) of the transform-domain
// slices.  Inverse: [Re K^{-1}, -Im K^{-1}] (P x 2P), so that the GEMM over both
// planes writes Re(K^{-1} (Dr + i Di)), the (real) result for
// conjugate-symmetric slices.
__global__ void k_build_kron_dft(KronDesc d, int P, int inverse, float* K) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)P * P) return;
  const int q = (int)(idx / P), p = (int)(idx % P);
  int rq = q, rp = p;
  double vr = 1.0, vi = 0.0;
  for (int m = 0; m < d.nmodes; ++m) {
    const int n = d.n[m];
    const int j = rq % n, k = rp % n;
    rq /= n;
    rp /= n;
    double er, ei = 0.0;
    if (d.kind[m] == 1) {
      const double ang = 2.0 * M_PI * (double)(((long long)j * k) % n) / (double)n;
      er = cos(ang);
      ei = inverse ? sin(ang) : -sin(ang);
      if (inverse) {
        er /= n;
        ei /= n;
      }
    } else if (d.kind[m] == 0) {
      er = inverse ? dct_entry(k, j, n) : dct_entry(j, k, n);
    } else if (d.kind[m] == 2) {
      er = (j == k) ? 1.0 : 0.0;
    } else {
      er = d.custom[m][(long long)j * n + k];
    }
    const double tr = vr * er - vi * ei;
    vi = vr * ei + vi * er;
    vr = tr;
  }
  if (!inverse) {
    K[(long long)q * P + p] = (float)vr;
    K[(long long)(P + q) * P + p] = (float)vi;
  } else {
    K[(long long)q * 2 * P + p] = (float)vr;
    K[(long long)q * 2 * P + P + p] = (float)(-vi);
  }
}

// Real embedding [[X, -Y], [Y, X]] (2 I1 x 2 I2, column-major) of the complex
// slice X + iY of every representative slice rep[t] of a conjugate pair: its
// singular values are those of X + iY, each twice, and its SVT is the
// embedding of the complex SVT.
__global__ void k_dft_embed(const float* __restrict__ Re, const float* __restrict__ Im, const int* rep,
                            int I1, int I2, long long N, float* __restrict__ E) {
  const int t = blockIdx.y;
  const long long n4 = 4 * N;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n4) return;
  const int r = (int)(e % (2 * I1)), c = (int)(e / (2 * I1));
  const bool top = r < I1, left = c < I2;
  const int i = top ? r : r - I1, j = left ? c : c - I2;
  const long long src = (long long)rep[t] * N + (long long)j * I1 + i;
  const float x = Re[src], y = Im[src];
  E[(long long)t * n4 + e] = top ? (left ? x : -y) : (left ? y : x);
}

// Complex SVT result of slice rep[t] from the thresholded embedding (its left
// block column holds [Re D; Im D]); the partner slice gets the conjugate, a
// self-conjugate slice a zero imaginary part.  Ranks and sweeps per slice (the
// embedding counts every singular value twice).
__global__ void k_dft_extract(const float* __restrict__ E, const int* rep, const int* partner, int I1,
                              int I2, long long N, float* __restrict__ Re, float* __restrict__ Im,
                              const int32_t* rankE, int32_t* rank, const int32_t* sweepsE,
                              int32_t* sweeps, const double* nucE, double* nuc) {
  const int t = blockIdx.y;
  const int p = rep[t], q = partner[t];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) {
    // the embedding holds every singular value of the complex slice twice; the
    // partner slice (its conjugate) has the same ones
    if (rank) rank[p] = rank[q] = rankE[t] / 2;
    if (sweeps) sweeps[p] = sweeps[q] = sweepsE[t];
    if (nuc) nuc[p] = nuc[q] = 0.5 * nucE[t];
  }
  if (e >= N) return;
  const int i = (int)(e % I1), j = (int)(e / I1);
  const float* Et = E + (long long)t * 4 * N + (long long)j * 2 * I1;
  const float re = Et[i], im = Et[I1 + i];
  Re[(long long)p * N + e] = re;
  if (q == p) {
    Im[(long long)p * N + e] = 0.f;
  } else {
    Im[(long long)p * N + e] = im;
    Re[(long long)q * N + e] = re;
    Im[(long long)q * N + e] = -im;
  }
}

// Complex working matrices of the representatives rep[t] for the Hermitian
// Jacobi: ms = 2 m interleaved rows (row 2r: Re, 2r + 1: Im) by n columns,
// column-major, 2N floats per representative.  I1 >= I2: the slice's columns
// (entry (i, j) at row pair i of column j); I1 < I2: its rows (entry (i, j) at
// row pair j of column i, the plain transpose, whose SVT is the transpose of
// the slice's).  twin: 2n columns, 4N floats per representative, column 2j
// the working column j and column 2j + 1 its product by i ((Re, Im) ->
// (-Im, Re)): the real form of the complex matrix, whose real Gram matrix and
// Cholesky factor are the real forms of the complex ones.  A 32 x 32 tile per
// workgroup goes through LDS so that reads and writes are both coalesced.
__global__ __launch_bounds__(256) void k_dft_stack(const float* __restrict__ Re, const float* __restrict__ Im,
                                                   const int* rep, int I1, int I2, long long N,
                                                   float* __restrict__ W, int twin) {
  __shared__ float2 T[32][33];   // T[j - j0][i - i0]
  const int t = blockIdx.y;
  const int ti = (I1 + 31) / 32;
  const int i0 = 32 * (int)(blockIdx.x % ti), j0 = 32 * (int)(blockIdx.x / ti);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const long long src = (long long)rep[t] * N;
  for (int jj = ty; jj < 32; jj += 8) {
    const int i = i0 + tx, j = j0 + jj;
    if (i < I1 && j < I2) {
      const long long e = src + (long long)j * I1 + i;
      T[jj][tx] = make_float2(Re[e], Im[e]);
    }
  }
  __syncthreads();
  float2* Wt = reinterpret_cast<float2*>(W + (long long)t * (twin ? 4 : 2) * N);
  const int m = I1 >= I2 ? I1 : I2;
  const long long cp = twin ? 2LL * m : m;   // float2 entries between working columns
  if (I1 >= I2) {
    for (int jj = ty; jj < 32; jj += 8) {
      const int i = i0 + tx, j = j0 + jj;
      if (i < I1 && j < I2) {
        const float2 v = T[jj][tx];
        Wt[(long long)j * cp + i] = v;
        if (twin) Wt[(long long)j * cp + m + i] = make_float2(-v.y, v.x);
      }
    }
  } else {
    for (int ii = ty; ii < 32; ii += 8) {
      const int i = i0 + ii, j = j0 + tx;
      if (i < I1 && j < I2) {
        const float2 v = T[tx][ii];
        Wt[(long long)i * cp + j] = v;
        if (twin) Wt[(long long)i * cp + m + j] = make_float2(-v.y, v.x);
      }
    }
  }
}

// Columns j < k of per-slice complex matrices (rows2 = 2 m interleaved rows,
// u_stride floats apart) written with their products by i ((Re, Im) ->
// (-Im, Re)) as columns 2j and 2j + 1 of Bk (bk_stride apart): the real
// rebuild over the interleaved rows then forms U_k U_k^H W.
__global__ __launch_bounds__(256) void k_twin_columns(const float* __restrict__ U, long long u_stride, int rows2,
                                                      int k, float* __restrict__ Bk, long long bk_stride) {
  const int t = blockIdx.y;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)rows2 * k) return;
  const int j = (int)(e / rows2), r = (int)(e - (long long)j * rows2);
  const float* u = U + t * u_stride + (long long)j * rows2;
  float* b = Bk + t * bk_stride + (long long)(2 * j) * rows2;
  b[r] = u[r];
  b[rows2 + r] = (r & 1) ? u[r - 1] : -u[r + 1];
}

// Per-representative values (n each) copied to the representative's slice and
// its partner's (P x n).
__global__ __launch_bounds__(256) void k_expand_pairs(const double* __restrict__ v, const int* rep,
                                                      const int* partner, int n, double* __restrict__ out) {
  const int t = blockIdx.x;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double x = v[(long long)t * n + k];
    out[(long long)rep[t] * n + k] = x;
    out[(long long)partner[t] * n + k] = x;
  }
}

// Columns 0, 2, 4, ... of per-slice column-major rows x (2 ncols) matrices
// (leading dimension rows, src_stride floats apart) into rows x ncols ones
// (dst_stride floats apart): the complex Cholesky factor out of the real
// factor of the twinned matrix.
__global__ __launch_bounds__(256) void k_even_columns(const float* __restrict__ src, long long src_stride,
                                                      float* __restrict__ dst, long long dst_stride, int rows,
                                                      int ncols) {
  const int t = blockIdx.y;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)rows * ncols) return;
  const int j = (int)(e / rows), r = (int)(e - (long long)j * rows);
  dst[t * dst_stride + e] = src[t * src_stride + (long long)(2 * j) * rows + r];
}

// The complex SVT results back to the planes: slice rep[t] from its working
// matrix (layout of k_dft_stack), its partner the conjugate, a self-conjugate
// slice a zero imaginary part.  Ranks, sweeps and nuclear-norm shares as
// k_dft_extract (the Jacobi counts each kept complex column twice).
__global__ __launch_bounds__(256) void k_dft_unstack(const float* __restrict__ W, const int* rep,
                                                     const int* partner, int I1, int I2, long long N,
                                                     float* __restrict__ Re, float* __restrict__ Im,
                                                     const int32_t* rankE, int32_t* rank, const int32_t* sweepsE,
                                                     int32_t* sweeps, const double* nucE, double* nuc, int twin) {
  __shared__ float2 T[32][33];
  const int t = blockIdx.y;
  const int p = rep[t], q = partner[t];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (rank) rank[p] = rank[q] = rankE[t] / 2;
    if (sweeps) sweeps[p] = sweeps[q] = sweepsE[t];
    if (nuc) nuc[p] = nuc[q] = 0.5 * nucE[t];
  }
  const int ti = (I1 + 31) / 32;
  const int i0 = 32 * (int)(blockIdx.x % ti), j0 = 32 * (int)(blockIdx.x / ti);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const float2* Wt = reinterpret_cast<const float2*>(W + (long long)t * (twin ? 4 : 2) * N);
  const long long cp = twin ? 2LL * (I1 >= I2 ? I1 : I2) : (I1 >= I2 ? I1 : I2);
  if (I1 >= I2) {
    for (int jj = ty; jj < 32; jj += 8) {
      const int i = i0 + tx, j = j0 + jj;
      if (i < I1 && j < I2) T[jj][tx] = Wt[(long long)j * cp + i];
    }
  } else {
    for (int ii = ty; ii < 32; ii += 8) {
      const int i = i0 + ii, j = j0 + tx;
      if (i < I1 && j < I2) T[tx][ii] = Wt[(long long)i * cp + j];
    }
  }
  __syncthreads();
  for (int jj = ty; jj < 32; jj += 8) {
    const int i = i0 + tx, j = j0 + jj;
    if (i < I1 && j < I2) {
      const float2 v = T[jj][tx];
      const long long e = (long long)j * I1 + i;
      Re[(long long)p * N + e] = v.x;
      if (q == p) {
        Im[(long long)p * N + e] = 0.f;
      } else {
        Im[(long long)p * N + e] = v.y;
        Re[(long long)q * N + e] = v.x;
        Im[(long long)q * N + e] = -v.y;
      }
    }
  }
}

// out = scale * sum of v[0..n): per-thread sums over a fixed stride, then the
// fixed-order workgroup sum (the same bits on every call).
__global__ __launch_bounds__(256) void k_sum_scaled(const double* v, int n, double scale, double* out) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += v[i];
  block_sum2(a, b);
  if (threadIdx.x == 0) *out = scale * a;
}

// Also, when sweeps is given, adds the largest of the nsl per-slice sweep counts
// of this iteration to *slowest (the Jacobi launch lasts as long as its slowest
// slice).
__global__ __launch_bounds__(256) void k_reduce_partials(const double* p, int n, double* out,
                                                         const int32_t* sweeps, int nsl,
                                                         unsigned long long* slowest) {
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    s1 += p[2 * i];
    s2 += p[2 * i + 1];
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) {
    out[0] = s1;
    out[1] = s2;
  }
  if (sweeps) {
    __shared__ int smax[4];
    int m = 0;
    for (int i = threadIdx.x; i < nsl; i += 256) m = max(m, sweeps[i]);
    for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      *slowest += (unsigned long long)max(max(smax[0], smax[1]), max(smax[2], smax[3]));
  }
}

// Face-wise product (Section 3.1 definition): one 16x16 output tile of one slice
// per workgroup, contraction staged through LDS in chunks of 16.
__global__ __launch_bounds__(256) void k_facewise(const float* A, const float* B, float* C,
                                                  int I1, int L, int I2) {
  __shared__ float As[16][17];
  __shared__ float Bs[16][17];
  const int p = blockIdx.z;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  const int i = blockIdx.x * 16 + ti, j = blockIdx.y * 16 + tj;
  const float* Ap = A + (long long)p * I1 * L;
  const float* Bp = B + (long long)p * L * I2;
  float acc = 0.f;
  for (int k0 = 0; k0 < L; k0 += 16) {
    // A tile: rows i (ti), cols k0 + tj ; B tile: rows k0 + ti, cols j (tj)
    const int ka = k0 + tj, kb = k0 + ti;
    As[ti][tj] = (i < I1 && ka < L) ? Ap[(long long)ka * I1 + i] : 0.f;
    Bs[ti][tj] = (kb < L && j < I2) ? Bp[(long long)j * L + kb] : 0.f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = fmaf(As[ti][k], Bs[k][tj], acc);
    __syncthreads();
  }
  if (i < I1 && j < I2) C[(long long)p * I1 * I2 + (long long)j * I1 + i] = acc;
}

// The face-wise product of complex slices (Fourier modes), each operand in two
// planes (real parts of all P slices, then imaginary parts; plane strides
// P I1 L, P L I2 and P I1 I2): C = (Ar Br - Ai Bi) + i (Ar Bi + Ai Br).
__global__ __launch_bounds__(256) void k_facewise_cx(const float* A, const float* B, float* C, int I1, int L,
                                                     int I2, int P) {
  __shared__ float Ar[16][17], Ai[16][17];
  __shared__ float Br[16][17], Bi[16][17];
  const int p = blockIdx.z;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  const int i = blockIdx.x * 16 + ti, j = blockIdx.y * 16 + tj;
  const long long pa = (long long)P * I1 * L, pb = (long long)P * L * I2;
  const float* Ap = A + (long long)p * I1 * L;
  const float* Bp = B + (long long)p * L * I2;
  float cr = 0.f, ci = 0.f;
  for (int k0 = 0; k0 < L; k0 += 16) {
    const int ka = k0 + tj, kb = k0 + ti;
    const bool ina = i < I1 && ka < L, inb = kb < L && j < I2;
    Ar[ti][tj] = ina ? Ap[(long long)ka * I1 + i] : 0.f;
    Ai[ti][tj] = ina ? Ap[pa + (long long)ka * I1 + i] : 0.f;
    Br[ti][tj] = inb ? Bp[(long long)j * L + kb] : 0.f;
    Bi[ti][tj] = inb ? Bp[pb + (long long)j * L + kb] : 0.f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      cr = fmaf(Ar[ti][k], Br[k][tj], cr);
      cr = fmaf(-Ai[ti][k], Bi[k][tj], cr);
      ci = fmaf(Ar[ti][k], Bi[k][tj], ci);
      ci = fmaf(Ai[ti][k], Br[k][tj], ci);
    }
    __syncthreads();
  }
  if (i < I1 && j < I2) {
    const long long e = (long long)p * I1 * I2 + (long long)j * I1 + i;
    C[e] = cr;
    C[(long long)P * I1 * I2 + e] = ci;
  }
}

__global__ void k_count_nonfinite(const float* X, const uint8_t* mask, long long n,
                                  unsigned int* count) {
  unsigned int c = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    if (mask && !mask[i]) continue;
    if (!isfinite(X[i])) ++c;
  }
  if (c) atomicAdd(count, c);
}

}  // namespace

hipError_t launch_gemm_grouped(ProbDev* const* probs, const GemmTile* tiles, int ntiles, int precision,
                               int inverse, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int key = (precision ? 2 : 0) | (inverse ? 1 : 0);
  switch (key) {
    case 0: hipLaunchKernelGGL((k_gemm_grouped<0, 0>), dim3(ntiles), dim3(256), 0, s, probs, tiles); break;
    case 1: hipLaunchKernelGGL((k_gemm_grouped<0, 1>), dim3(ntiles), dim3(256), 0, s, probs, tiles); break;
    case 2: hipLaunchKernelGGL((k_gemm_grouped<1, 0>), dim3(ntiles), dim3(256), 0, s, probs, tiles); break;
    default: hipLaunchKernelGGL((k_gemm_grouped<1, 1>), dim3(ntiles), dim3(256), 0, s, probs, tiles); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_begin(ProbDev* const* probs, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_begin, dim3((nprob + 63) / 64), dim3(64), 0, s, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_batch_end(ProbDev* const* probs, int nprob, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_end, dim3(nprob), dim3(256), 0, s, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const long long nw = (long long)(bytes / 4);
  if (nw <= 0) return hipSuccess;
  long long blocks = (nw + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, nw);
  return hipGetLastError();
}

hipError_t launch_transform_gemm(const GemmArgs& a, int precision, int pro, int epi,
                                 hipStream_t s, int* n_partials) {
  if (a.P <= 0 || a.N <= 0) return hipErrorInvalidValue;
  const int Mo = a.Mo ? a.Mo : a.P;
  // FP32: all output rows in one workgroup when they fit 12 waves
  const int nw = precision ? 4 : (Mo <= 64 ? 4 : (Mo <= 128 ? 8 : (Mo <= 192 ? 12 : 4)));
  const int rows = 16 * nw;
  dim3 grid((unsigned)((a.N + TE - 1) / TE), (unsigned)((Mo + rows - 1) / rows));
  if (n_partials) *n_partials = (int)(grid.x * grid.y);
  const int key = (precision ? 4 : 0) | (pro << 1) | epi;
  const dim3 blk(64 * nw);
  switch (key) {
    case 0:
      if (nw == 12) hipLaunchKernelGGL((k_gemm_f32<0, 0, 12>), grid, blk, 0, s, a);
      else if (nw == 8) hipLaunchKernelGGL((k_gemm_f32<0, 0, 8>), grid, blk, 0, s, a);
      else hipLaunchKernelGGL((k_gemm_f32<0, 0, 4>), grid, blk, 0, s, a);
      break;
    case 1:
      if (nw == 12) hipLaunchKernelGGL((k_gemm_f32<0, 1, 12>), grid, blk, 0, s, a);
      else if (nw == 8) hipLaunchKernelGGL((k_gemm_f32<0, 1, 8>), grid, blk, 0, s, a);
      else hipLaunchKernelGGL((k_gemm_f32<0, 1, 4>), grid, blk, 0, s, a);
      break;
    case 2:
      if (nw == 12) hipLaunchKernelGGL((k_gemm_f32<1, 0, 12>), grid, blk, 0, s, a);
      else if (nw == 8) hipLaunchKernelGGL((k_gemm_f32<1, 0, 8>), grid, blk, 0, s, a);
      else hipLaunchKernelGGL((k_gemm_f32<1, 0, 4>), grid, blk, 0, s, a);
      break;
    case 3:
      if (nw == 12) hipLaunchKernelGGL((k_gemm_f32<1, 1, 12>), grid, blk, 0, s, a);
      else if (nw == 8) hipLaunchKernelGGL((k_gemm_f32<1, 1, 8>), grid, blk, 0, s, a);
      else hipLaunchKernelGGL((k_gemm_f32<1, 1, 4>), grid, blk, 0, s, a);
      break;
    case 4: hipLaunchKernelGGL((k_gemm_bf16x3<0, 0>), grid, dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_gemm_bf16x3<0, 1>), grid, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_gemm_bf16x3<1, 0>), grid, dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_gemm_bf16x3<1, 1>), grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_build_kron(const KronDesc& d, int P, int inverse, float* K, uint16_t* Khi,
                             uint16_t* Klo, hipStream_t s) {
  const long long n = (long long)P * P;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_build_kron, dim3(blocks), dim3(256), 0, s, d, P, inverse, K, Khi, Klo);
  return hipGetLastError();
}

hipError_t launch_build_kron_dft(const KronDesc& d, int P, int inverse, float* K, hipStream_t s) {
  const long long n = (long long)P * P;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_build_kron_dft, dim3(blocks), dim3(256), 0, s, d, P, inverse, K);
  return hipGetLastError();
}

hipError_t launch_dft_embed(const float* Re, const float* Im, const int* rep, int npairs, int I1, int I2,
                            float* E, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const long long N = (long long)I1 * I2;
  dim3 grid((unsigned)((4 * N + 255) / 256), (unsigned)npairs);
  hipLaunchKernelGGL(k_dft_embed, grid, dim3(256), 0, s, Re, Im, rep, I1, I2, N, E);
  return hipGetLastError();
}

hipError_t launch_dft_extract(const float* E, const int* rep, const int* partner, int npairs, int I1, int I2,
                              float* Re, float* Im, const int32_t* rankE, int32_t* rank,
                              const int32_t* sweepsE, int32_t* sweeps, const double* nucE, double* nuc,
                              hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const long long N = (long long)I1 * I2;
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)npairs);
  hipLaunchKernelGGL(k_dft_extract, grid, dim3(256), 0, s, E, rep, partner, I1, I2, N, Re, Im, rankE, rank,
                     sweepsE, sweeps, nuc ? nucE : nullptr, nuc);
  return hipGetLastError();
}

hipError_t launch_dft_stack(const float* Re, const float* Im, const int* rep, int npairs, int I1, int I2,
                            float* W, hipStream_t s, bool twin) {
  if (npairs <= 0) return hipSuccess;
  const long long tiles = (long long)((I1 + 31) / 32) * ((I2 + 31) / 32);
  hipLaunchKernelGGL(k_dft_stack, dim3((unsigned)tiles, (unsigned)npairs), dim3(256), 0, s, Re, Im, rep, I1, I2,
                     (long long)I1 * I2, W, twin ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_dft_unstack(const float* W, const int* rep, const int* partner, int npairs, int I1, int I2,
                              float* Re, float* Im, const int32_t* rankE, int32_t* rank,
                              const int32_t* sweepsE, int32_t* sweeps, const double* nucE, double* nuc,
                              hipStream_t s, bool twin) {
  if (npairs <= 0) return hipSuccess;
  const long long tiles = (long long)((I1 + 31) / 32) * ((I2 + 31) / 32);
  hipLaunchKernelGGL(k_dft_unstack, dim3((unsigned)tiles, (unsigned)npairs), dim3(256), 0, s, W, rep, partner, I1,
                     I2, (long long)I1 * I2, Re, Im, rankE, rank, sweepsE, sweeps, nuc ? nucE : nullptr, nuc,
                     twin ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_twin_columns(const float* U, long long u_stride, int rows2, int k, float* Bk, long long bk_stride,
                               int nslices, hipStream_t s) {
  if (nslices <= 0 || k <= 0) return hipSuccess;
  const long long e = (long long)rows2 * k;
  hipLaunchKernelGGL(k_twin_columns, dim3((unsigned)((e + 255) / 256), (unsigned)nslices), dim3(256), 0, s, U,
                     u_stride, rows2, k, Bk, bk_stride);
  return hipGetLastError();
}

hipError_t launch_expand_pairs(const double* v, const int* rep, const int* partner, int npairs, int n, double* out,
                               hipStream_t s) {
  if (npairs <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_pairs, dim3((unsigned)npairs), dim3(256), 0, s, v, rep, partner, n, out);
  return hipGetLastError();
}

hipError_t launch_even_columns(const float* src, long long src_stride, float* dst, long long dst_stride, int rows,
                               int ncols, int nslices, hipStream_t s) {
  if (nslices <= 0 || rows <= 0 || ncols <= 0) return hipSuccess;
  const long long e = (long long)rows * ncols;
  hipLaunchKernelGGL(k_even_columns, dim3((unsigned)((e + 255) / 256), (unsigned)nslices), dim3(256), 0, s, src,
                     src_stride, dst, dst_stride, rows, ncols);
  return hipGetLastError();
}

hipError_t launch_sum_scaled(const double* v, int n, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_scaled, dim3(1), dim3(256), 0, s, v, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partials, int n, double* out2, hipStream_t s,
                                  const int32_t* sweeps, int nsl, unsigned long long* slowest) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, n, out2, sweeps, nsl, slowest);
  return hipGetLastError();
}

hipError_t launch_facewise(const float* A, const float* B, float* C, int I1, int L, int I2,
                           int P, hipStream_t s, bool complex_planes) {
  dim3 grid((I1 + 15) / 16, (I2 + 15) / 16, P);
  if (complex_planes) hipLaunchKernelGGL(k_facewise_cx, grid, dim3(256), 0, s, A, B, C, I1, L, I2, P);
  else hipLaunchKernelGGL(k_facewise, grid, dim3(256), 0, s, A, B, C, I1, L, I2);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* X, const uint8_t* mask, long long n,
                                  unsigned int* count, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, X, mask, n,
                     count);
  return hipGetLastError();
}

}  // namespace lt
