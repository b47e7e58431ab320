// Per-slice SVD by one-sided (Hestenes) Jacobi and the singular value
// soft-threshold of Alg. 4 / the prox of Theorem 23, batched over frontal
// slices: one workgroup per slice.
//
// Working matrix: W = slice (I1 >= I2) or slice^T (I1 < I2), m x n with
// m = max(I1, I2) rows and n = min(I1, I2) columns.  Columns of W are rotated
// in pairs until every pair is orthogonal to within `tol`; the final columns
// are u_i sigma_i with sigma_i their norms (W J = U Sigma, J orthogonal).
//
// Layout in the workgroup: pair slot g (0 <= g < ceil(n/2)) is held by a group
// of G lanes; each lane keeps R rows of the slot's two columns in registers
// (FP32), as R/4 chunks of 4 consecutive rows interleaved across the group
// (chunk c of a column belongs to lane c mod G), so a group moves a column
// through LDS as contiguous 16-byte pieces.  Column norms, pair dot products
// (exact FP32 x FP32 products summed in FP64) and rotation angles are FP64;
// the columns are rotated in FP32.  FP32 pair dot products are an opt-in.
//
// Pair schedule (one sweep meets every column pair exactly once, in
// 2*ceil(n/2) - 1 rounds).  The ceil(n/2) slots form one range of c slots; while
// c is even the range runs a ring phase: tops stay, bottoms shift one slot along
// the range after each of its c rounds, so every top meets every bottom; then one
// swap (the first half's bottoms trade places with the second half's tops) turns
// the range into two ranges of c/2 slots, one holding the former tops and one the
// former bottoms, and each continues the same way.  A range of odd size c finishes
// with the round-robin (circle) tournament over its 2c columns (2c - 1 rounds).
// A ring round moves one column per slot through LDS where the circle moves two;
// the ordering is a reordering of the cyclic Jacobi sweep, not of the arithmetic
// of a rotation.
//
// SVT output: with g_i = 1 - tau / sigma_i for sigma_i > tau, the result of
// Alg. 4 in working orientation is D_W = sum_i g_i u_i u_i^T W (because
// u_i^T W = sigma_i v_i^T), so the kernel writes only the kept columns
// sqrt(g_i) u_i (compacted, deterministic order) and their count; the rebuild
// kernel forms D_W = Bk (Bk^T W) from the untouched input.
#include "lt_internal.h"

#include <math.h>

namespace lt {

namespace {

// Sum over the G lanes of a group; every lane gets the bitwise-same result.
// Steps within 8 lanes use DPP (quad permutations, half-row mirror), wider
// steps use cross-lane shuffles.
__device__ inline double dpp_add(double v, int ctrl_sel) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int plo, phi;
  switch (ctrl_sel) {
    case 0:   // lane ^ 1
      plo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      phi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:   // lane ^ 2
      plo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      phi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    default:  // mirror within each half row of 8 lanes (pairs quad 0 with quad 1)
      plo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
      phi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
      break;
  }
  return v + __hiloint2double(phi, plo);
}

template <int G>
__device__ inline double group_sum(double v) {
  v = dpp_add(v, 0);
  if (G >= 4) v = dpp_add(v, 1);
  if (G >= 8) v = dpp_add(v, 2);
  if (G >= 16) v += __shfl_xor(v, 8, 64);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// The same group sum for FP32 values (DPP modifiers on the adds).
__device__ inline float dpp_addf(float v, int ctrl_sel) {
  const int x = __float_as_int(v);
  int y;
  switch (ctrl_sel) {
    case 0: y = __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); break;
    case 1: y = __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false); break;
    default: y = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false); break;
  }
  return v + __int_as_float(y);
}

template <int G>
__device__ inline float group_sumf(float v) {
  v = dpp_addf(v, 0);
  if (G >= 4) v = dpp_addf(v, 1);
  if (G >= 8) v = dpp_addf(v, 2);
  if (G >= 16) v += __shfl_xor(v, 8, 64);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// FP64 dot product of two FP32 register columns (FP32 x FP32 products are exact
// in FP64) over all R rows of the lane: the chunks beyond the slice's qeff hold
// zeros (see get_rows), so no per-chunk predicate is needed.  The scheduling
// barriers keep the compiler from converting a whole column to FP64 ahead of use.
template <int R>
__device__ inline double dot64(const float (&x)[R], const float (&y)[R]) {
  double d0 = 0.0, d1 = 0.0;
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    const int r = 4 * q;
    d0 = fma((double)x[r], (double)y[r], d0);
    d1 = fma((double)x[r + 1], (double)y[r + 1], d1);
    d0 = fma((double)x[r + 2], (double)y[r + 2], d0);
    d1 = fma((double)x[r + 3], (double)y[r + 3], d1);
    __builtin_amdgcn_sched_barrier(0);
  }
  return d0 + d1;
}

// The same dot product with FP32 products and two FP32 accumulators per lane
// (interleaved rows), the opt-in FP32 form: with the FP32 group sum the error
// bound is about (R/2 + 2 + log2 G) * 2^-24 of sum |x_i y_i| (about 2e-6 at 32
// rows per lane and G = 8), the same order as a 1e-6 orthogonality test, so
// near the tolerance the rotate-or-skip decision is decided by rounding.
template <int R>
__device__ inline float dot32x(const float (&x)[R], const float (&y)[R]) {
  float d0 = 0.f, d1 = 0.f;
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    const int r = 4 * q;
    d0 = fmaf(x[r], y[r], d0);
    d1 = fmaf(x[r + 1], y[r + 1], d1);
    d0 = fmaf(x[r + 2], y[r + 2], d0);
    d1 = fmaf(x[r + 3], y[r + 3], d1);
  }
  return d0 + d1;
}

// Complex columns (Fourier slices) are held with their real and imaginary
// parts in consecutive rows (row 2i: Re, row 2i + 1: Im), so that a lane's
// 4-row chunks hold whole entries.  a^H b = sum conj(a_i) b_i: its real part is
// the plain dot product of the interleaved rows, its imaginary part sums
// Re a_i Im b_i - Im a_i Re b_i.  Both in FP64 from the exact FP32 products.
template <int R>
__device__ inline void dot64c(const float (&x)[R], const float (&y)[R], double& re, double& im) {
  double r0 = 0.0, r1 = 0.0, i0 = 0.0, i1 = 0.0;
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    const int r = 4 * q;
    const double xr0 = x[r], xi0 = x[r + 1], xr1 = x[r + 2], xi1 = x[r + 3];
    const double yr0 = y[r], yi0 = y[r + 1], yr1 = y[r + 2], yi1 = y[r + 3];
    r0 = fma(xr0, yr0, r0);
    r1 = fma(xr1, yr1, r1);
    i0 = fma(xr0, yi0, i0);
    i1 = fma(xr1, yi1, i1);
    r0 = fma(xi0, yi0, r0);
    r1 = fma(xi1, yi1, r1);
    i0 = fma(-xi0, yr0, i0);
    i1 = fma(-xi1, yr1, i1);
    __builtin_amdgcn_sched_barrier(0);
  }
  re = r0 + r1;
  im = i0 + i1;
}

// Hardware FP64 reciprocal refined by one Newton step (about 1e-15 relative):
// it only forms the rotation's zeta, which is then rounded to FP32, so the
// IEEE-exact division sequence is not needed.
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Hardware FP64 reciprocal square root refined by one Newton step,
// y <- y + y (1 - x y^2) / 2 (about 1e-15 relative for the arguments >= 1 it
// gets here: 1 + zeta^2 and 1 + t^2).
__device__ inline double rsq64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// The rotation that zeroes the off-diagonal entry of the 2 x 2 Gram matrix
// [[pa, d], [d, pb]] of a column pair (d != 0), all in FP64:
// zeta = (pb - pa) / (2 d), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) (the
// smaller root of t^2 + 2 zeta t - 1 = 0, so |angle| <= pi/4),
// c = 1 / sqrt(1 + t^2), s = c t.  c and s are then rounded to FP32, the
// precision the columns are rotated in; t stays FP64 for the norm updates
// pa - t d and pb + t d.  zeta is clamped so zeta^2 cannot overflow (t is then
// below 1e-100 either way).
__device__ inline void jacobi_angle(double d, double pa, double pb, double& t, float& cf, float& sf) {
  const double zeta = fmin(fmax((pb - pa) * (0.5 * rcp64(d)), -1e100), 1e100);
  const double az = fabs(zeta);
  const double z2 = fma(az, az, 1.0);
  const double tt = rcp64(fma(z2, rsq64(z2), az));   // 1 / (|zeta| + sqrt(1 + zeta^2))
  t = zeta < 0.0 ? -tt : tt;
  const double c = rsq64(fma(tt, tt, 1.0));
  cf = (float)c;
  sf = (float)(c * t);
}

// A wave-uniform FP64 value moved to scalar registers.
__device__ inline double uniform_d(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// Pair dot-product precision travels with the Jacobi tolerance: a negative
// tolerance asks for FP32 products and per-lane FP32 sums (an opt-in of the
// library's svd options); decode_tol restores the magnitude and returns that
// request.  The default is FP64 dot products of the FP32 columns.
__device__ inline bool decode_tol(double& tol) {
  const bool fp32 = tol < 0.0;
  tol = fabs(tol);
  return fp32;
}

// (x, y) <- (c x - s y, c y + s x) on every row: s y and s x rounded, then one
// fma each (the rounding every Jacobi kernel here applies).  Written
// as VALU-only inline assembly whose outputs are tied to its inputs, so that a
// wave-uniform branch around it updates the column registers in place (the
// compiler would otherwise rotate into fresh registers and copy back at the
// join).  The leading s_nop covers the wait a transcendental result (c comes
// from v_rsq) needs before a VALU reads it.
template <int R>
__device__ inline void rotate_in_place(float (&av)[R], float (&bv)[R], float cf, float sf) {
  asm volatile("s_nop 1" ::);
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    float t0, t1;
    asm volatile(
        "v_mul_f32 %8, %10, %4\n\t"
        "v_mul_f32 %9, %10, %0\n\t"
        "v_fma_f32 %0, %11, %0, -%8\n\t"
        "v_fma_f32 %4, %11, %4, %9\n\t"
        "v_mul_f32 %8, %10, %5\n\t"
        "v_mul_f32 %9, %10, %1\n\t"
        "v_fma_f32 %1, %11, %1, -%8\n\t"
        "v_fma_f32 %5, %11, %5, %9\n\t"
        "v_mul_f32 %8, %10, %6\n\t"
        "v_mul_f32 %9, %10, %2\n\t"
        "v_fma_f32 %2, %11, %2, -%8\n\t"
        "v_fma_f32 %6, %11, %6, %9\n\t"
        "v_mul_f32 %8, %10, %7\n\t"
        "v_mul_f32 %9, %10, %3\n\t"
        "v_fma_f32 %3, %11, %3, -%8\n\t"
        "v_fma_f32 %7, %11, %7, %9"
        : "+v"(av[4 * q]), "+v"(av[4 * q + 1]), "+v"(av[4 * q + 2]), "+v"(av[4 * q + 3]),
          "+v"(bv[4 * q]), "+v"(bv[4 * q + 1]), "+v"(bv[4 * q + 2]), "+v"(bv[4 * q + 3]),
          "=&v"(t0), "=&v"(t1)
        : "v"(sf), "v"(cf));
  }
}

// Columns are stored as R/4 chunks of 4 rows; chunk q of lane l holds rows
// 4 (l + G q) .. 4 (l + G q) + 3.  Only the first qeff chunks carry rows; the
// others are zero in every lane from the first load on (get_rows,
// load_work_col), stay zero under rotations, and are neither stored nor
// reloaded, so dots and rotations run over all R rows without predicates.  An
// LDS column slot is ldw = G R + 4 floats: the rows, then 16 bytes of metadata
// (an FP64 value and an int: the column's norm and id while sweeping, the
// output scale and destination when writing out), moved with the column.
template <int G, int R>
__device__ inline void put_col(float* buf, int ldw, int idx, int l, const float (&v)[R], int qeff,
                               double meta_d, int meta_i) {
  float* col = buf + (size_t)idx * ldw;
  float4* p = reinterpret_cast<float4*>(col);
#pragma unroll
  for (int q = 0; q < R / 4; ++q)
    if (q < qeff) p[l + G * q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  if (l == 0)
    *reinterpret_cast<float4*>(col + ldw - 4) =
        make_float4(__int_as_float(__double2loint(meta_d)), __int_as_float(__double2hiint(meta_d)),
                    __int_as_float(meta_i), 0.f);
}

template <int G, int R>
__device__ inline void get_col(const float* buf, int ldw, int idx, int l, float (&v)[R], int qeff,
                               double& meta_d, int& meta_i) {
  const float* col = buf + (size_t)idx * ldw;
  const float4* p = reinterpret_cast<const float4*>(col);
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    if (q < qeff) {
      const float4 t = p[l + G * q];
      v[4 * q] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    }
  }
  const float4 m = *reinterpret_cast<const float4*>(col + ldw - 4);
  meta_d = __hiloint2double(__float_as_int(m.y), __float_as_int(m.x));
  meta_i = __float_as_int(m.z);
}

template <int G, int R>
__device__ inline void get_rows(const float* buf, int ldw, int idx, int l, float (&v)[R], int qeff) {
  const float4* p = reinterpret_cast<const float4*>(buf + (size_t)idx * ldw);
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    const float4 t = (q < qeff) ? p[l + G * q] : make_float4(0.f, 0.f, 0.f, 0.f);
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}

// Stage one half of the working columns (half 0: column p, half 1: column
// 2*npairs - 1 - p, for p < npairs) into LDS column p, rows 0 .. mpad - 1, with
// zeros beyond the slice.  The lanes of the slice cooperate; reads are
// coalesced along the slice's contiguous dimension.
__device__ inline void stage_in(const float* __restrict__ A, float* buf, int ldw, bool trans, int I1,
                                int m, int n, int npairs, int mpad, int half, int t2, int tps) {
  const int total = npairs * mpad;
  if (!trans) {
    for (int e = t2; e < total; e += tps) {   // W(row, col) = A[col * I1 + row]
      const int p = e / mpad, row = e - p * mpad;
      const int col = half ? 2 * npairs - 1 - p : p;
      buf[(size_t)p * ldw + row] = (row < m && col < n) ? A[(long long)col * I1 + row] : 0.f;
    }
  } else {
    for (int e = t2; e < total; e += tps) {   // W(row, col) = A[row * I1 + col]
      const int row = e / npairs, p = e - row * npairs;
      const int col = half ? 2 * npairs - 1 - p : p;
      buf[(size_t)p * ldw + row] = (row < m && col < n) ? A[(long long)row * I1 + col] : 0.f;
    }
  }
}

// Write LDS column p (rows 0 .. m-1), scaled by its metadata value, to the
// output column its metadata int names (none when negative).  Coalesced along
// the rows.
__device__ inline void stage_out(float* __restrict__ out, const float* buf, int ldw, int m, int npairs,
                                 int t2, int tps) {
  const int total = npairs * m;
  for (int e = t2; e < total; e += tps) {
    const int p = e / m, row = e - p * m;
    const float* col = buf + (size_t)p * ldw;
    const int d = __float_as_int(col[ldw - 2]);
    if (d >= 0) {
      const double sc = __hiloint2double(__float_as_int(col[ldw - 3]), __float_as_int(col[ldw - 4]));
      out[(long long)d * m + row] = col[row] * (float)sc;
    }
  }
}

// stage_out for complex columns: output column d takes the scaled column and
// column d + 1 its product with i ((Re, Im) -> (-Im, Re) per entry), so that
// the real rebuild over the interleaved rows, D = B B^T W with B = [b, i b],
// forms b b^H W.  m is even.
__device__ inline void stage_out_cx(float* __restrict__ out, const float* buf, int ldw, int m, int npairs,
                                    int t2, int tps) {
  const int total = npairs * m;
  for (int e = t2; e < total; e += tps) {
    const int p = e / m, row = e - p * m;
    const float* col = buf + (size_t)p * ldw;
    const int d = __float_as_int(col[ldw - 2]);
    if (d >= 0) {
      const float sc = (float)__hiloint2double(__float_as_int(col[ldw - 3]), __float_as_int(col[ldw - 4]));
      out[(long long)d * m + row] = col[row] * sc;
      out[(long long)(d + 1) * m + row] = ((row & 1) ? col[row - 1] : -col[row + 1]) * sc;
    }
  }
}

// Exchange positions of one buffer: the ring phases use one per slot; the
// circle phase of the odd-sized ranges uses c + 1 per range of c slots (one
// extra for the bottom of the range's first slot).
__host__ __device__ inline int exch_positions(int npairs) {
  int c = npairs;
  while (c > 1 && (c & 1) == 0) c >>= 1;
  return c > 1 ? npairs + npairs / c : npairs;
}

// Per-slice LDS region: two (or one) exchange buffers of exch_positions
// columns (rows + metadata) and the slice's control words.
__host__ __device__ inline size_t slice_lds_bytes(int npairs, int ldw, int nbuf) {
  const size_t np = (size_t)exch_positions(npairs);
  size_t b = (size_t)nbuf * np * ldw * sizeof(float) + ((size_t)npairs + 4) * sizeof(int);
  return (b + 15) & ~size_t(15);
}
constexpr size_t kWgCtlBytes = 16;   // workgroup-wide rotation counters

// A lane's rotation count holds two counts: rotations in the low 16 bits and
// large rotations (the pair's |a_i . a_j| / (|a_i| |a_j|) above sqrt(tol)) in
// the high 16.  Cyclic Jacobi converges quadratically, so after a sweep whose
// rotations all had cosines below sqrt(tol) the next sweep's would fall near
// tol: a slice stops after such a sweep instead of running a last sweep that
// only checks.
constexpr unsigned kBigOne = 1u << 16;
__device__ inline double big_rotation2(double tol) { return tol; }

// One workgroup's work: nsub slices of identical shape (I1 x I2), slice q at
// src + q * stride; outputs likewise.
struct Job {
  const float* src;
  float* out;
  int32_t* rank;
  int32_t* sweeps;
  double* sigma;
  long long stride;       // between the packed slices' inputs
  long long out_stride;   // between their outputs
  int I1, I2, nsub, qeff, mode;
  double tau;
  unsigned long long* sweep_total;
  unsigned long long* rot_total;
  unsigned int* hits;
  double* nuc;   // SVT: sum of (sigma_i - tau) over the kept columns (may be null)
};

// CX: complex columns (interleaved rows, see dot64c) under Hermitian
// rotations.  SVT mode: each kept column is written with its product by i
// (stage_out_cx) and counted twice in the rank and the nuclear-norm share, so
// the output has the layout of the real SVT of the embedding [[X, -Y], [Y, X]];
// all-columns mode: as for real columns (interleaved rows, norms).
// Out of line: inlined into the kernels it needs more registers.
template <int G, int R, bool CX = false>
__device__ __attribute__((noinline)) void jacobi_body(const Job& jb, double tol, int max_sweeps, int nbuf, int ldw,
                                                     unsigned char* smem) {
  const int I1 = jb.I1, I2 = jb.I2, qeff = jb.qeff;
  const bool trans = I1 < I2;
  const int m = trans ? I2 : I1;
  const int n = trans ? I1 : I2;
  const int npairs = (n + 1) >> 1;
  const int npos = exch_positions(npairs);   // columns per exchange buffer
  const int tps = npairs * G;   // lanes per slice
  const int tid = threadIdx.x;
  const int sub = tid / tps;
  const int t2 = tid - sub * tps;
  const int g = t2 / G, l = t2 - (t2 / G) * G;
  const bool active = sub < jb.nsub;
  const int subr = active ? sub : 0;   // idle lanes point at slice 0's region, never write
  const size_t sbytes = slice_lds_bytes(npairs, ldw, nbuf);
  int* wg_ctl = reinterpret_cast<int*>(smem);
  unsigned char* base = smem + kWgCtlBytes + (size_t)subr * sbytes;
  float* bufA = reinterpret_cast<float*>(base);
  float* bufB = (nbuf == 2) ? bufA + (size_t)npos * ldw : bufA;
  // ctl[0], ctl[1]: the slice's rotation counters of even / odd sweeps;
  // ctl[2]: kept total; ctl[3 + g]: per-slot output offsets
  int* ctl = reinterpret_cast<int*>(bufA + (size_t)nbuf * npos * ldw);
  const float* __restrict__ A = jb.src + (long long)subr * jb.stride;

  // ---- load: slot g holds columns g (top) and 2*npairs - 1 - g (bottom) ----
  float av[R], bv[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {   // idle lanes too: every lane's rotation is finite
    av[e] = 0.f;
    bv[e] = 0.f;
  }
  int ida = g, idb = 2 * npairs - 1 - g;
  const int mpad = 4 * G * qeff;   // rows a lane group holds per column (>= m)
  if (active) stage_in(A, bufA, ldw, trans, I1, m, n, npairs, mpad, 0, t2, tps);
  __syncthreads();
  if (active) get_rows<G, R>(bufA, ldw, g, l, av, qeff);
  __syncthreads();
  if (active) stage_in(A, bufA, ldw, trans, I1, m, n, npairs, mpad, 1, t2, tps);
  __syncthreads();
  if (active) get_rows<G, R>(bufA, ldw, g, l, bv, qeff);
  if (active && t2 == 0) {
    ctl[0] = 0;
    ctl[1] = 0;
  }
  if (tid == 0) {
    wg_ctl[0] = 0;
    wg_ctl[1] = 0;
  }
  __syncthreads();

  double na = 0.0, nb = 0.0;
  int sweep = 0;
  int my_sweeps = 0;            // sweeps this slice needed (first sweep without rotations)
  bool converged = false;
  long long rotations = 0;
  // pair dot products in FP64 (exact FP32 products, FP64 sums) unless the
  // caller asked for FP32 ones (tolerance passed negated, see decode_tol)
  const bool dot32 = decode_tol(tol);
  const double big2 = big_rotation2(tol);
  // single-exit loop (max_sweeps >= 1): the columns stay in one register set
  for (;;) {
    na = group_sum<G>(dot64<R>(av, av));
    nb = group_sum<G>(dot64<R>(bv, bv));
    unsigned my_rot = 0;   // this lane's rotations | large rotations << 16
    // a converged slice stays frozen in place (no rotations, no moves) while
    // the rest of its pack finishes, so its result and column order do not
    // depend on what it is packed with
    const bool moving = active && !converged;
    // phase state: ranges of c slots; ring phase while c is even, circle
    // tournament once c is odd; r counts the rounds of the current phase
    int c = npairs;
    bool ring = (c & 1) == 0;
    int s0 = 0, i = g, r = 0;
    const int nrounds = 2 * npairs - 1;
    for (int k = 0; k < nrounds; ++k) {
      // one rotation of the slot's pair (av, bv).  The angle is found per lane;
      // the rows are rotated on every lane, lanes without a rotation taking
      // c = 1, s = 0 (the identity on finite values, up to the sign of a zero),
      // so the column registers are updated in place rather than merged lane by
      // lane after a divergent branch.
      float cf = 1.f, sf = 0.f;
      float er = 1.f, ei = 0.f;   // CX: the phase of a^H b
      double t = 0.0;
      double d = 0.0, pa = 0.0, pb = 0.0;
      bool rot = false;
      if (moving) {
        pa = fmax(na, 0.0);
        pb = fmax(nb, 0.0);
        if (CX) {
          // Hermitian rotation: with a^H b = |g| e^{i phi}, b e^{-i phi} meets a
          // with the real product |g|, and the real rotation of that pair
          // orthogonalises it
          double gr, gi;
          dot64c<R>(av, bv, gr, gi);
          gr = group_sum<G>(gr);
          gi = group_sum<G>(gi);
          const double g2 = fma(gr, gr, gi * gi);
          rot = g2 != 0.0 && g2 > tol * tol * (pa * pb);   // |g| > tol sqrt(pa pb)
          if (rot) {
            d = sqrt(g2);
            jacobi_angle(d, pa, pb, t, cf, sf);
            const double id = 1.0 / d;
            er = (float)(gr * id);
            ei = (float)(gi * id);
          }
        } else {
          d = dot32 ? (double)group_sumf<G>(dot32x<R>(av, bv)) : group_sum<G>(dot64<R>(av, bv));
          rot = d != 0.0 && d * d > tol * tol * (pa * pb);   // |d| > tol sqrt(pa pb)
          if (rot) jacobi_angle(d, pa, pb, t, cf, sf);
        }
      }
      // (the in-place update with a wave-uniform skip, rotate_in_place, leaves
      // this out-of-line body's columns in registers the LDS exchange cannot
      // store as float4 tuples: the update stays unconditional here)
      if (CX) {
#pragma unroll
        for (int e = 0; e < R; e += 2) {
          const float xr = av[e], xi = av[e + 1], br = bv[e], bi = bv[e + 1];
          const float yr = fmaf(er, br, ei * bi);      // b e^{-i phi}
          const float yi = fmaf(er, bi, -(ei * br));
          av[e] = fmaf(cf, xr, -(sf * yr));
          av[e + 1] = fmaf(cf, xi, -(sf * yi));
          bv[e] = fmaf(cf, yr, sf * xr);
          bv[e + 1] = fmaf(cf, yi, sf * xi);
        }
      } else {
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const float x = av[e], y = bv[e];
          const float sy = sf * y, sx = sf * x;
          av[e] = fmaf(cf, x, -sy);
          bv[e] = fmaf(cf, y, sx);
        }
      }
      if (rot) {
        na = fma(-t, d, pa);
        nb = fma(t, d, pb);
        my_rot += (l == 0) ? 1u + (d * d > big2 * (pa * pb) ? kBigOne : 0u) : 0u;
      }
      if (k + 1 == nrounds) break;   // no exchange after the sweep's last round
      if (ring && r + 1 < c) {
        // ring: bottoms move one slot down the range, one barrier.  Two buffers
        // alternate; with one, slot i writes position (i + r) mod c of its range
        // and reads (i + 1 + r) mod c, slot i+1's, and the position it writes in
        // the next round is the one only it read in this one.
        const int wpos = (nbuf == 2) ? i : (i + r < c ? i + r : i + r - c);
        const int rpos = wpos + 1 == c ? 0 : wpos + 1;
        float* buf = (nbuf == 2 && (r & 1)) ? bufB : bufA;
        if (moving) put_col<G, R>(buf, ldw, s0 + wpos, l, bv, qeff, nb, idb);
        __syncthreads();
        if (moving) get_col<G, R>(buf, ldw, s0 + rpos, l, bv, qeff, nb, idb);
        ++r;
      } else if (ring) {
        // end of a ring phase: the first half's bottoms and the second half's
        // tops trade places, leaving two ranges of c/2 slots
        const int h = c >> 1;
        const bool first = i < h;
        if (nbuf == 1 && r > 0) __syncthreads();   // the last ring round's reads (one buffer)
        if (moving) {
          if (first) put_col<G, R>(bufB, ldw, g, l, bv, qeff, nb, idb);
          else put_col<G, R>(bufB, ldw, g, l, av, qeff, na, ida);
        }
        __syncthreads();
        if (moving) {
          if (first) get_col<G, R>(bufB, ldw, g + h, l, bv, qeff, nb, idb);
          else get_col<G, R>(bufB, ldw, g - h, l, av, qeff, na, ida);
        }
        if (nbuf == 1) __syncthreads();
        c = h;
        ring = (c & 1) == 0;
        s0 = (g / c) * c;
        i = g - s0;
        r = 0;
      } else {
        // circle tournament over the range's 2c columns: slot 0 keeps its top,
        // the other tops move one slot up (slot 1 takes slot 0's bottom), the
        // bottoms move one slot down and the last slot's top becomes its
        // bottom.  The range owns exchange positions pos0 .. pos0 + c of bufA;
        // phase 1 stores tops at pos0 + i (slot 0's bottom at pos0 + c), phase 2
        // stores the bottoms of slots 1.. one position lower, so that position
        // pos0 + i then holds slot i's new bottom, the last slot's included.
        const int pos0 = s0 + s0 / c;
        if (moving) {
          put_col<G, R>(bufA, ldw, pos0 + i, l, av, qeff, na, ida);
          if (i == 0) put_col<G, R>(bufA, ldw, pos0 + c, l, bv, qeff, nb, idb);
        }
        __syncthreads();
        if (moving && i != 0) {
          get_col<G, R>(bufA, ldw, pos0 + (i == 1 ? c : i - 1), l, av, qeff, na, ida);
          put_col<G, R>(bufA, ldw, pos0 + i - 1, l, bv, qeff, nb, idb);
        }
        __syncthreads();
        if (moving) get_col<G, R>(bufA, ldw, pos0 + i, l, bv, qeff, nb, idb);
        ++r;
      }
    }
    // counters of the next sweep are cleared before the barrier that precedes
    // any of their increments
    // both halves of the sums stay below 2^16: at most 1024 / G slots of a
    // workgroup, each meeting 2 ceil(n/2) - 1 <= 255 pairs per sweep
    if (my_rot) {
      atomicAdd(reinterpret_cast<unsigned*>(&ctl[sweep & 1]), my_rot);
      atomicAdd(reinterpret_cast<unsigned*>(&wg_ctl[sweep & 1]), my_rot);
    }
    __syncthreads();
    const unsigned mine = static_cast<unsigned>(ctl[sweep & 1]);
    const unsigned any = static_cast<unsigned>(wg_ctl[sweep & 1]);
    if (active && t2 == 0) ctl[(sweep + 1) & 1] = 0;
    if (tid == 0) wg_ctl[(sweep + 1) & 1] = 0;
    __syncthreads();
    ++sweep;
    if (!converged) {
      rotations += mine & 0xFFFFu;
      my_sweeps = sweep;
      converged = (mine >> 16) == 0;
    }
    if ((any >> 16) == 0 || sweep >= max_sweeps) break;
  }

  // ---- output -------------------------------------------------------------
  na = group_sum<G>(dot64<R>(av, av));
  nb = group_sum<G>(dot64<R>(bv, bv));
  const double sa = sqrt(na), sb = sqrt(nb);
  bool ka, kb;
  if (jb.mode == 0) {
    ka = active && ida < n && sa > jb.tau;
    kb = active && idb < n && sb > jb.tau;
  } else {
    ka = active && ida < n;
    kb = active && idb < n;
  }
  __syncthreads();
  // per slot: kept count, and the slot's share of the slice's nuclear norm
  // (the exchange buffer is free here), summed below in slot order
  double* nucs = reinterpret_cast<double*>(bufA);
  if (active && l == 0) {
    ctl[3 + g] = (int)ka + (int)kb;
    nucs[g] = (ka ? sa - jb.tau : 0.0) + (kb ? sb - jb.tau : 0.0);
  }
  __syncthreads();
  if (active && t2 == 0) {
    int acc = 0;
    double nsum = 0.0;
    for (int i = 0; i < npairs; ++i) {
      const int c = ctl[3 + i];
      ctl[3 + i] = acc;
      acc += c;
      nsum += nucs[i];
    }
    ctl[2] = acc;
    if (jb.mode == 0 && jb.nuc) jb.nuc[sub] = CX ? 2.0 * nsum : nsum;
  }
  __syncthreads();
  // kept columns, scaled, through LDS: tops, then bottoms
  float* out = jb.out + (long long)subr * jb.out_stride;
  const int j0 = active ? ctl[3 + g] : 0;
  double sca, scb;
  int da, db;
  if (jb.mode == 0) {
    sca = ka ? sqrt(1.0 - jb.tau / sa) / sa : 0.0;
    scb = kb ? sqrt(1.0 - jb.tau / sb) / sb : 0.0;
    da = ka ? (CX ? 2 * j0 : j0) : -1;
    db = kb ? (CX ? 2 * (j0 + (int)ka) : j0 + (int)ka) : -1;
  } else {
    // all columns, at their original column index, plus their norms
    sca = 1.0;
    scb = 1.0;
    da = ka ? ida : -1;
    db = kb ? idb : -1;
    if (l == 0 && ka) jb.sigma[(long long)subr * n + ida] = sa;
    if (l == 0 && kb) jb.sigma[(long long)subr * n + idb] = sb;
  }
  if (active) put_col<G, R>(bufA, ldw, g, l, av, qeff, sca, da);
  __syncthreads();
  if (active) {
    if (CX && jb.mode == 0) stage_out_cx(out, bufA, ldw, m, npairs, t2, tps);
    else stage_out(out, bufA, ldw, m, npairs, t2, tps);
  }
  __syncthreads();
  if (active) put_col<G, R>(bufA, ldw, g, l, bv, qeff, scb, db);
  __syncthreads();
  if (active) {
    if (CX && jb.mode == 0) stage_out_cx(out, bufA, ldw, m, npairs, t2, tps);
    else stage_out(out, bufA, ldw, m, npairs, t2, tps);
  }
  if (active && t2 == 0) {
    if (jb.rank) jb.rank[sub] = (CX && jb.mode == 0) ? 2 * ctl[2] : ctl[2];
    if (jb.sweeps) jb.sweeps[sub] = my_sweeps;
    if (jb.sweep_total) atomicAdd(jb.sweep_total, (unsigned long long)my_sweeps);
    if (jb.rot_total) atomicAdd(jb.rot_total, (unsigned long long)rotations);
    if (!converged && jb.hits) atomicAdd(jb.hits, 1u);
  }
}

// The rounds of one sweep for the slot's pair (av, bv), for the blocked kernel
// below: one rotation per round, then the move the pair schedule prescribes.
// With ring_only, only the first ring phase runs (npairs rounds, npairs even),
// in which every top meets every bottom once.  Returns this lane's count of
// applied rotations (lane 0 of each group counts; large ones also in the high
// half, see kBigOne).  The register-resident body
// keeps its own copy of these rounds: calling this function from it (inlined)
// changed its register allocation and grew its stack frame.
template <int G, int R>
__device__ __attribute__((always_inline)) inline unsigned sweep_rounds(
    float (&av)[R], float (&bv)[R], double& na, double& nb, int& ida, int& idb, bool moving,
    bool dot32, double tol, int npairs, int g, int l, int qeff, float* bufA, float* bufB, int nbuf,
    int ldw, bool ring_only) {
  unsigned my_rot = 0;
  const double big2 = big_rotation2(tol);
  // phase state: ranges of c slots; ring phase while c is even, circle
  // tournament once c is odd; r counts the rounds of the current phase
  int c = npairs;
  bool ring = (c & 1) == 0;
  int s0 = 0, i = g, r = 0;
  const int nrounds = ring_only ? npairs : 2 * npairs - 1;
  for (int k = 0; k < nrounds; ++k) {
    // one rotation of the slot's pair (av, bv).  The angle is found per lane;
    // the rows are rotated under a wave-uniform branch in which lanes without a
    // rotation take c = 1, s = 0 (the identity on finite values, up to the sign
    // of a zero), so the column registers are updated in place rather than
    // merged lane by lane after a divergent branch.
    float cf = 1.f, sf = 0.f;
      double t = 0.0;
    double d = 0.0, pa = 0.0, pb = 0.0;
    bool rot = false;
    if (moving) {
      d = dot32 ? (double)group_sumf<G>(dot32x<R>(av, bv)) : group_sum<G>(dot64<R>(av, bv));
      pa = fmax(na, 0.0);
      pb = fmax(nb, 0.0);
      rot = d != 0.0 && d * d > tol * tol * (pa * pb);   // |d| > tol sqrt(pa pb)
      if (rot) {
        // rotation that zeroes the off-diagonal of [[pa, d], [d, pb]]:
        // zeta = (pb - pa) / (2 d), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
        // c = 1 / sqrt(1 + t^2), s = c t.  zeta is formed in FP64 (a
        // difference of FP64 norms) and clamped where t falls below FP32
        // resolution; t, c and s are FP32, the precision the rotation is
        // applied in.  Every multiply-add is an explicit fma, so the rounding
        // does not depend on how the compiler contracts an instantiation.
        jacobi_angle(d, pa, pb, t, cf, sf);
      }
    }
    // waves without a rotation skip the column update
    if (__builtin_amdgcn_ballot_w64(rot) != 0) rotate_in_place<R>(av, bv, cf, sf);
    if (rot) {
      na = fma(-t, d, pa);
      nb = fma(t, d, pb);
      my_rot += (l == 0) ? 1u + (d * d > big2 * (pa * pb) ? kBigOne : 0u) : 0u;
    }
    if (k + 1 == nrounds) break;   // no exchange after the sweep's last round
    if (ring && r + 1 < c) {
      // ring: bottoms move one slot down the range, one barrier.  Two buffers
      // alternate; with one, slot i writes position (i + r) mod c of its range
      // and reads (i + 1 + r) mod c, slot i+1's, and the position it writes in
      // the next round is the one only it read in this one.
      const int wpos = (nbuf == 2) ? i : (i + r < c ? i + r : i + r - c);
      const int rpos = wpos + 1 == c ? 0 : wpos + 1;
      float* buf = (nbuf == 2 && (r & 1)) ? bufB : bufA;
      if (moving) put_col<G, R>(buf, ldw, s0 + wpos, l, bv, qeff, nb, idb);
      __syncthreads();
      if (moving) get_col<G, R>(buf, ldw, s0 + rpos, l, bv, qeff, nb, idb);
      ++r;
    } else if (ring) {
      // end of a ring phase: the first half's bottoms and the second half's
      // tops trade places, leaving two ranges of c/2 slots
      const int h = c >> 1;
      const bool first = i < h;
      if (nbuf == 1 && r > 0) __syncthreads();   // the last ring round's reads (one buffer)
      if (moving) {
        if (first) put_col<G, R>(bufB, ldw, g, l, bv, qeff, nb, idb);
        else put_col<G, R>(bufB, ldw, g, l, av, qeff, na, ida);
      }
      __syncthreads();
      if (moving) {
        if (first) get_col<G, R>(bufB, ldw, g + h, l, bv, qeff, nb, idb);
        else get_col<G, R>(bufB, ldw, g - h, l, av, qeff, na, ida);
      }
      if (nbuf == 1) __syncthreads();
      c = h;
      ring = (c & 1) == 0;
      s0 = (g / c) * c;
      i = g - s0;
      r = 0;
    } else {
      // circle tournament over the range's 2c columns: slot 0 keeps its top,
      // the other tops move one slot up (slot 1 takes slot 0's bottom), the
      // bottoms move one slot down and the last slot's top becomes its
      // bottom.  The range owns exchange positions pos0 .. pos0 + c of bufA;
      // phase 1 stores tops at pos0 + i (slot 0's bottom at pos0 + c), phase 2
      // stores the bottoms of slots 1.. one position lower, so that position
      // pos0 + i then holds slot i's new bottom, the last slot's included.
      const int pos0 = s0 + s0 / c;
      if (moving) {
        put_col<G, R>(bufA, ldw, pos0 + i, l, av, qeff, na, ida);
        if (i == 0) put_col<G, R>(bufA, ldw, pos0 + c, l, bv, qeff, nb, idb);
      }
      __syncthreads();
      if (moving && i != 0) {
        get_col<G, R>(bufA, ldw, pos0 + (i == 1 ? c : i - 1), l, av, qeff, na, ida);
        put_col<G, R>(bufA, ldw, pos0 + i - 1, l, bv, qeff, nb, idb);
      }
      __syncthreads();
      if (moving) get_col<G, R>(bufA, ldw, pos0 + i, l, bv, qeff, nb, idb);
      ++r;
    }
  }
  return my_rot;
}

// ---- blocked Jacobi: slices whose columns do not fit one workgroup ----------
//
// The working matrix W (m x n) is copied to a per-slice buffer in the register
// layout (column-major, mpad rows, nblk * b columns, zero padded).  The columns
// form nblk (even) blocks of b (even) columns, and one workgroup runs every
// sweep of its slice as nblk - 1 block rounds of the round-robin tournament over
// the blocks: each block pair (A, B) of a round is loaded into the registers, A's
// columns as the slots' tops and B's as their bottoms, and rotated.  In the
// first block round of a sweep the rotations cover every pair among the 2b
// columns (one sweep of the pair schedule on b slots); later block rounds run
// one ring phase, which meets every column of A with every column of B.  So a
// sweep again meets every column pair once.  Columns carry their index and go
// back to their own place in the buffer; the norms are recomputed exactly at
// every load.  Output: the kept columns in column order, as for the
// register-resident kernel.
struct BlkJob {
  const float* src;
  float* work;
  float* out;
  int32_t* rank;
  int32_t* sweeps;
  int I1, I2, b, nblk, qeff, nbuf;
  double tau;
  unsigned long long* sweep_total;
  unsigned long long* rot_total;
  unsigned int* hits;
  double* nuc;   // SVT: sum of (sigma_i - tau) over the kept columns (may be null)
};

// Columns c0 .. c0 + ncols - 1 of W into LDS columns 0 .. ncols - 1 (rows
// 0 .. mpad - 1, zeros beyond the slice), reads coalesced along the slice's
// contiguous dimension.
__device__ inline void stage_cols(const float* __restrict__ A, float* buf, int ldw, bool trans, int I1,
                                  int m, int n, int c0, int ncols, int mpad, int t, int nt) {
  const int total = ncols * mpad;
  if (!trans) {
    for (int e = t; e < total; e += nt) {
      const int p = e / mpad, row = e - p * mpad;
      const int col = c0 + p;
      buf[(size_t)p * ldw + row] = (row < m && col < n) ? A[(long long)col * I1 + row] : 0.f;
    }
  } else {
    for (int e = t; e < total; e += nt) {
      const int row = e / ncols, p = e - row * ncols;
      const int col = c0 + p;
      buf[(size_t)p * ldw + row] = (row < m && col < n) ? A[(long long)row * I1 + col] : 0.f;
    }
  }
}

// A working-buffer column <-> a lane's register rows (the chunk layout of
// put_col / get_col, ld = mpad = 4 G qeff).
template <int G, int R>
__device__ inline void load_work_col(const float* Wk, int mpad, int col, int l, float (&v)[R], int qeff) {
  const float4* p = reinterpret_cast<const float4*>(Wk + (size_t)col * mpad);
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    const float4 x = (q < qeff) ? p[l + G * q] : make_float4(0.f, 0.f, 0.f, 0.f);
    v[4 * q] = x.x;
    v[4 * q + 1] = x.y;
    v[4 * q + 2] = x.z;
    v[4 * q + 3] = x.w;
  }
}

template <int G, int R>
__device__ inline void store_work_col(float* Wk, int mpad, int col, int l, const float (&v)[R], int qeff) {
  float4* p = reinterpret_cast<float4*>(Wk + (size_t)col * mpad);
#pragma unroll
  for (int q = 0; q < R / 4; ++q)
    if (q < qeff) p[l + G * q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// Block at position pos of block round br in the round-robin tournament over
// nblk blocks: position 0 keeps block 0, the others rotate.
__device__ inline int blk_at(int pos, int br, int nblk) {
  return pos == 0 ? 0 : 1 + (pos - 1 + br) % (nblk - 1);
}

__host__ __device__ inline size_t blk_lds_bytes(int b, int ldw, int nbuf) {
  const size_t bytes = kWgCtlBytes + (size_t)nbuf * exch_positions(b) * ldw * sizeof(float) +
                       ((size_t)b + 4) * sizeof(int);
  return (bytes + 15) & ~size_t(15);
}

template <int G, int R>
__device__ __attribute__((always_inline)) inline void jacobi_blk_body(const BlkJob& jb, double tol, int max_sweeps,
                                                          unsigned char* smem) {
  const int I1 = jb.I1, I2 = jb.I2, qeff = jb.qeff, b = jb.b, nblk = jb.nblk, nbuf = jb.nbuf;
  const bool trans = I1 < I2;
  const int m = trans ? I2 : I1;
  const int n = trans ? I1 : I2;
  const int mpad = 4 * G * qeff;
  const int ldw = mpad + 4;
  const int ncols = nblk * b;
  const int tps = b * G;   // lanes holding slots; the rest of the workgroup only joins barriers
  const int tid = threadIdx.x;
  const bool active = tid < tps;
  const int g = active ? tid / G : 0, l = tid % G;
  int* wg_ctl = reinterpret_cast<int*>(smem);
  // exchange buffers (two: one barrier per ring round) and control words
  float* buf = reinterpret_cast<float*>(smem + kWgCtlBytes);
  float* bufB = nbuf == 2 ? buf + (size_t)exch_positions(b) * ldw : buf;
  // ctl[2]: kept total; ctl[3 + g]: per-slot output offsets
  int* ctl = reinterpret_cast<int*>(buf + (size_t)nbuf * exch_positions(b) * ldw);
  float* __restrict__ Wk = jb.work;

  // ---- copy in: b columns at a time through LDS, written out coalesced ----
  for (int c0 = 0; c0 < ncols; c0 += b) {
    stage_cols(jb.src, buf, ldw, trans, I1, m, n, c0, b, mpad, tid, blockDim.x);
    __syncthreads();
    for (int e = tid; e < b * mpad; e += blockDim.x) {
      const int p = e / mpad, row = e - p * mpad;
      Wk[(size_t)(c0 + p) * mpad + row] = buf[(size_t)p * ldw + row];
    }
    __syncthreads();
  }
  // wg_ctl[0], [1]: rotations of even / odd sweeps; [2], [3]: large rotations
  if (tid == 0) {
    wg_ctl[0] = 0;
    wg_ctl[1] = 0;
    wg_ctl[2] = 0;
    wg_ctl[3] = 0;
  }
  __syncthreads();

  float av[R], bv[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    av[e] = 0.f;
    bv[e] = 0.f;
  }
  const bool dot32 = decode_tol(tol);
  int sweep = 0, my_sweeps = 0;
  bool converged = false;
  long long rotations = 0;
  for (;;) {
    unsigned my_rot = 0;   // per lane at most one rotation per round: < 2^16 per sweep
    for (int br = 0; br < nblk - 1; ++br) {
      for (int pi = 0; pi < nblk / 2; ++pi) {
        const int A = blk_at(pi, br, nblk), B = blk_at(nblk - 1 - pi, br, nblk);
        int ida = A * b + g, idb = B * b + g;
        if (active) {
          load_work_col<G, R>(Wk, mpad, ida, l, av, qeff);
          load_work_col<G, R>(Wk, mpad, idb, l, bv, qeff);
        }
        double na = group_sum<G>(dot64<R>(av, av));
        double nb = group_sum<G>(dot64<R>(bv, bv));
        my_rot += sweep_rounds<G, R>(av, bv, na, nb, ida, idb, active, dot32, tol, b, g, l, qeff, buf,
                                     bufB, nbuf, ldw, br > 0);
        if (active) {
          store_work_col<G, R>(Wk, mpad, ida, l, av, qeff);
          store_work_col<G, R>(Wk, mpad, idb, l, bv, qeff);
        }
        // the next block pair may hold columns other lanes just stored
        __syncthreads();
      }
    }
    if (my_rot & 0xFFFFu) atomicAdd(&wg_ctl[sweep & 1], (int)(my_rot & 0xFFFFu));
    if (my_rot >> 16) atomicAdd(&wg_ctl[2 + (sweep & 1)], (int)(my_rot >> 16));
    __syncthreads();
    const int any = wg_ctl[sweep & 1];
    const int anybig = wg_ctl[2 + (sweep & 1)];
    if (tid == 0) {
      wg_ctl[(sweep + 1) & 1] = 0;
      wg_ctl[2 + ((sweep + 1) & 1)] = 0;
    }
    __syncthreads();
    ++sweep;
    rotations += any;
    my_sweeps = sweep;
    converged = (anybig == 0);
    if (converged || sweep >= max_sweeps) break;
  }

  // ---- output: b columns at a time, kept ones compacted in column order ----
  if (tid == 0) ctl[2] = 0;
  __syncthreads();
  double nsum = 0.0;   // thread 0: nuclear-norm share, in column order
  double* nucs = reinterpret_cast<double*>(buf);
  for (int c0 = 0; c0 < ncols; c0 += b) {
    const int id = c0 + g;
    if (active) load_work_col<G, R>(Wk, mpad, id, l, av, qeff);
    const double sa = sqrt(group_sum<G>(dot64<R>(av, av)));
    const bool ka = active && id < n && sa > jb.tau;
    if (active && l == 0) {
      ctl[3 + g] = ka ? 1 : 0;
      nucs[g] = ka ? sa - jb.tau : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      int acc = ctl[2];
      for (int i = 0; i < b; ++i) {
        const int c = ctl[3 + i];
        ctl[3 + i] = acc;
        acc += c;
        nsum += nucs[i];
      }
      ctl[2] = acc;
    }
    __syncthreads();
    const int d = ka ? ctl[3 + g] : -1;
    const double sc = ka ? sqrt(1.0 - jb.tau / sa) / sa : 0.0;
    if (active) put_col<G, R>(buf, ldw, g, l, av, qeff, sc, d);
    __syncthreads();
    if (active) stage_out(jb.out, buf, ldw, m, b, tid, tps);
    __syncthreads();
  }
  if (tid == 0) {
    if (jb.rank) *jb.rank = ctl[2];
    if (jb.nuc) *jb.nuc = nsum;
    if (jb.sweeps) *jb.sweeps = my_sweeps;
    if (jb.sweep_total) atomicAdd(jb.sweep_total, (unsigned long long)my_sweeps);
    if (jb.rot_total) atomicAdd(jb.rot_total, (unsigned long long)rotations);
    if (!converged && jb.hits) atomicAdd(jb.hits, 1u);
  }
}

// One slice per workgroup (single problem), blocked.  The body is inlined: its
// block loop around the rounds leaves too few registers for 32 rows per lane
// and a call frame (16 rows per lane, inlined, do not spill).
template <int G, int R>
__global__ __launch_bounds__(1024) void k_jacobi_blk(JacobiArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.x;
  BlkJob jb;
  jb.src = a.src + (long long)s * a.slice_stride;
  jb.work = a.work + (long long)s * a.work_stride;
  jb.out = a.bk + (long long)s * (a.bk_stride ? a.bk_stride : a.slice_stride);
  jb.rank = a.rank ? a.rank + s : nullptr;
  jb.sweeps = a.sweeps ? a.sweeps + s : nullptr;
  jb.I1 = a.I1;
  jb.I2 = a.I2;
  jb.b = a.blk_b;
  jb.nblk = a.blk_n;
  jb.nbuf = a.blk_nbuf;
  jb.qeff = a.qeff;
  jb.tau = a.tau;
  jb.sweep_total = a.sweep_total;
  jb.rot_total = a.rot_total;
  jb.hits = a.maxsweep_hits;
  jb.nuc = a.nuc ? a.nuc + s : nullptr;
  jacobi_blk_body<G, R>(jb, a.tol, a.max_sweeps, smem);
}

// Batch: one workgroup per slice of the problems whose slices take the blocked
// kernel with this lane count and row capacity.
template <int G, int R>
__global__ __launch_bounds__(1024) void k_jacobi_blk_items(ProbDev* const* probs, const CholItem* items,
                                                          double tol, int max_sweeps) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const CholItem it = items[blockIdx.x];
  ProbDev* pd = probs[it.prob];
  if (!pd->active) return;
  BlkJob jb;
  if (pd->precond) {
    // the slice's Cholesky factor L = R^T (n x n, FP32 over its FP64 Gram block)
    const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
    jb.src = reinterpret_cast<const float*>(pd->C) + (long long)it.slice * 2 * n * n;
    jb.I1 = n;
    jb.I2 = n;
  } else {
    jb.src = pd->Gh + (long long)it.slice * pd->N;
    jb.I1 = pd->I1;
    jb.I2 = pd->I2;
  }
  jb.work = pd->work + (long long)it.slice * pd->work_stride;
  jb.out = pd->Bk + (long long)it.slice * pd->N;
  jb.rank = pd->rank + it.slice;
  jb.sweeps = pd->sweeps + it.slice;
  jb.b = pd->blk_b;
  jb.nblk = pd->blk_n;
  jb.nbuf = pd->blk_nbuf;
  jb.qeff = pd->blk_q;
  jb.tau = pd->tau;
  jb.sweep_total = &pd->sweep_total;
  jb.rot_total = &pd->rot_total;
  jb.hits = &pd->maxsweep_hits;
  jb.nuc = pd->nuc + it.slice;
  jacobi_blk_body<G, R>(jb, tol, max_sweeps, smem);
}

// One slice per workgroup (single problem); CX: complex slices (SVT mode).
template <int G, int R, int LB, bool CX = false>
__global__ __launch_bounds__(LB) void k_jacobi(JacobiArgs a, int nbuf, int ldw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.x;
  Job jb;
  jb.src = a.src + (long long)s * a.slice_stride;
  jb.out = a.bk + (long long)s * (a.bk_stride ? a.bk_stride : a.slice_stride);
  jb.rank = a.rank ? a.rank + s : nullptr;
  jb.sweeps = a.sweeps ? a.sweeps + s : nullptr;
  const int n = a.I1 < a.I2 ? a.I1 : a.I2;
  jb.sigma = a.sigma ? a.sigma + (long long)s * n : nullptr;
  jb.stride = a.slice_stride;
  jb.out_stride = a.bk_stride ? a.bk_stride : a.slice_stride;
  jb.I1 = a.I1;
  jb.I2 = a.I2;
  jb.nsub = 1;
  jb.qeff = a.qeff;   // a run-time bound keeps the register allocation tighter
  jb.mode = a.mode;
  jb.tau = a.tau;
  jb.sweep_total = a.sweep_total;
  jb.rot_total = a.rot_total;
  jb.hits = a.maxsweep_hits;
  jb.nuc = a.nuc ? a.nuc + s : nullptr;
  jacobi_body<G, R, CX>(jb, a.tol, a.max_sweeps, nbuf, ldw, smem);
}

// Batch: one workgroup per item (nsub same-shape slices of one problem),
// items ordered longest-first by the host; the threshold is the problem's
// current mu_k from its device state.
template <int G, int R, int LB>
__global__ __launch_bounds__(LB) void k_jacobi_items(ProbDev* const* probs, const SvtItem* items,
                                                    double tol, int max_sweeps, int nbuf, int ldw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const SvtItem it = items[blockIdx.x];
  ProbDev* pd = probs[it.prob];
  if (!pd->active) return;
  Job jb;
  jb.out = pd->Bk + (long long)it.slice0 * pd->N;
  jb.out_stride = pd->N;
  if (pd->precond) {
    // Jacobi on the slices' Cholesky factors L = R^T (n x n, FP32 over each
    // slice's FP64 Gram block)
    const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
    jb.src = reinterpret_cast<const float*>(pd->C) + (long long)it.slice0 * 2 * n * n;
    jb.stride = 2LL * n * n;
    jb.I1 = n;
    jb.I2 = n;
  } else {
    jb.src = pd->Gh + (long long)it.slice0 * pd->N;
    jb.stride = pd->N;
    jb.I1 = pd->I1;
    jb.I2 = pd->I2;
  }
  jb.rank = pd->rank + it.slice0;
  jb.sweeps = pd->sweeps + it.slice0;
  jb.sigma = nullptr;
  jb.nsub = it.nsub;
  jb.qeff = it.qeff;
  jb.mode = 0;
  jb.tau = pd->tau;
  jb.sweep_total = &pd->sweep_total;
  jb.rot_total = &pd->rot_total;
  jb.hits = &pd->maxsweep_hits;
  jb.nuc = pd->nuc + it.slice0;
  jacobi_body<G, R>(jb, tol, max_sweeps, nbuf, ldw, smem);
}

// ---- warm-started Jacobi on the preconditioned factor ----------------------------
// Completion thresholds slices that change little from one iteration to the
// next.  The one-sided Jacobi of a preconditioned slice can then run on
// M = L Z instead of L (= R^T, the slice's n x n Cholesky factor), Z orthogonal:
// M has the singular values and left singular vectors of L, all the SVT uses,
// and when Z holds the rotations of the previous iterations M's columns start
// close to orthogonal, so far fewer sweeps are needed.  Each working column
// carries its column of Z below it: rows 0 .. npad-1 hold M (zero beyond n),
// rows npad .. npad+n-1 hold Z, npad = 4 ceil(n / 4).  Every rotation applies
// to the whole column, so Z accumulates them, while the dot products and norms
// take the M rows only.  A cold call starts from Z = I (M = L).  One slice per
// workgroup; pair schedule, angle and stopping rule are those of jacobi_body.

// M = L Z per slice (L lower triangular, both n x n column-major) on FP32 MFMA
// (16x16x4): one 16 x 16 tile of M per wave.  The tile is formed as its
// transpose, M^T = Z^T L^T, so that lane l's results are consecutive rows of
// the column-major M (A[i][k] = Z(k, c0 + i), B[k][j] = L(r0 + j, k); lane l
// holds D[4 (l / 16) + q][l % 16] = M(r0 + l % 16, c0 + 4 (l / 16) + q)).
// Within a chunk of 16 contraction indices, lane group g = l / 16 supplies
// k = 4 g + s at step s, so each lane reads four consecutive entries of its Z
// column.  L is lower triangular: a tile of rows r0 .. r0 + 15 stops at
// k = r0 + 15.  The single-problem and batch kernels share this tile, so both
// paths round M alike.
typedef float wp_v4f __attribute__((ext_vector_type(4)));

__device__ __attribute__((always_inline)) inline void warm_tile_mfma(const float* Ls, const float* Zs, float* Ms,
                                                                    int n, int r0, int c0, int lane) {
  const int lr = lane & 15, g = lane >> 4;
  const int zc = c0 + lr;   // the Z column this lane reads
  const int lrow = r0 + lr; // the L row this lane reads
  const int kend = n < r0 + 16 ? n : r0 + 16;
  wp_v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < kend; k0 += 16) {
    float za[4], lb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * g + u;
      za[u] = (zc < n && k < kend) ? Zs[(long long)zc * n + k] : 0.f;
      lb[u] = (lrow < n && k < kend) ? Ls[(long long)k * n + lrow] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(za[u], lb[u], acc, 0, 0, 0);
  }
  if (lrow < n) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int mc = c0 + 4 * g + q;
      if (mc < n) Ms[(long long)mc * n + lrow] = acc[q];
    }
  }
}

// Single problem: job = 4 blockIdx.x + wave runs over (slice, tile), nb x nb
// tiles per slice (nb = ceil(n / 16)), tile t at rows 16 (t % nb), columns
// 16 (t / nb).
__global__ __launch_bounds__(256) void k_warm_product_mfma(const float* L, long long l_stride, const float* Z,
                                                            float* M, long long m_stride, int n, int nb,
                                                            int nslices) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long job = (long long)blockIdx.x * 4 + wave;
  const long long tiles = (long long)nb * nb;
  const int s = (int)(job / tiles);
  if (s >= nslices) return;
  const int t = (int)(job - (long long)s * tiles);
  warm_tile_mfma(L + (long long)s * l_stride, Z + (long long)s * n * n, M + (long long)s * m_stride, n,
                 16 * (t % nb), 16 * (t / nb), lane);
}

// Whether a batch problem's Jacobi starts cold this iteration (Z = I, M = L).
__device__ inline bool warm_cold(const ProbDev* pd) {
  return pd->warm_period <= 0 || pd->iter % pd->warm_period == 0;
}

// Batch: blockIdx.x is the item (one slice of a warm-started problem: L over
// the first half of its FP64 Gram block, M written over the second half), the
// wave's tile 4 blockIdx.y + wave of that slice's nb x nb; the grid covers the
// largest item, waves past a smaller item's tiles return.  Cold problems skip.
__global__ __launch_bounds__(256) void k_warm_product_items(ProbDev* const* probs, const CholItem* items) {
  const CholItem it = items[blockIdx.x];
  const ProbDev* pd = probs[it.prob];
  if (!pd->active || warm_cold(pd)) return;
  const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
  const int nb = (n + 15) / 16;
  const int t = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (t >= nb * nb) return;
  const float* L = reinterpret_cast<const float*>(pd->C) + (long long)it.slice * 2 * n * n;
  warm_tile_mfma(L, pd->Z + (long long)it.slice * n * n, const_cast<float*>(L) + (long long)n * n, n,
                 16 * (t % nb), 16 * (t / nb), threadIdx.x & 63);
}

// Dot products over the M rows.  Chunks q < qm - 1 hold M rows in every lane,
// chunk qm - 1 in the lanes where lastm is set, later chunks only Z rows (those
// are skipped: the bound is the same for every lane).
template <int R>
__device__ inline float dot32_m(const float (&x)[R], const float (&y)[R], bool lastm, int qm) {
  float d0 = 0.f, d1 = 0.f;
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    if (q < qm) {   // a uniform branch per chunk: the loop stays unrolled over registers
      const int r = 4 * q;
      float p = x[r] * y[r];
      p = fmaf(x[r + 1], y[r + 1], p);
      p = fmaf(x[r + 2], y[r + 2], p);
      p = fmaf(x[r + 3], y[r + 3], p);
      p = (q + 1 < qm || lastm) ? p : 0.f;
      if (q & 1) d1 += p;
      else d0 += p;
    }
  }
  return d0 + d1;
}

template <int R>
__device__ inline double dot64_m(const float (&x)[R], const float (&y)[R], bool lastm, int qm) {
  double d0 = 0.0, d1 = 0.0;
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    if (q < qm) {
      const int r = 4 * q;
      double p = (double)x[r] * (double)y[r];
      p = fma((double)x[r + 1], (double)y[r + 1], p);
      p = fma((double)x[r + 2], (double)y[r + 2], p);
      p = fma((double)x[r + 3], (double)y[r + 3], p);
      p = (q + 1 < qm || lastm) ? p : 0.0;
      if (q & 1) d1 += p;
      else d0 += p;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return d0 + d1;
}

// One slice of the warm-started Jacobi.
struct WarmJob {
  const float* M;           // n x n, column-major: L Z, or L when cold
  float* Z;                 // n x n, column-major: read unless cold, rewritten
  float* out;               // kept columns, scaled
  int32_t* rank;
  int32_t* sweeps;
  unsigned long long* sweep_total;
  unsigned long long* rot_total;
  unsigned int* hits;
  double* nuc;              // sum of (sigma_i - tau) over the kept columns (may be null)
  double tau, tol;
  int n, max_sweeps, cold;
};

template <int G, int R>
__device__ __attribute__((always_inline)) inline void jacobi_warm_body(const WarmJob& a, int nbuf, int ldw,
                                                                       unsigned char* smem) {
  constexpr int Q = R / 4;
  const int n = a.n;
  const int npad = (n + 3) / 4 * 4;
  const int npairs = (n + 1) >> 1;
  const int npos = exch_positions(npairs);
  const int tps = npairs * G;
  const int tid = threadIdx.x;
  const bool active = tid < tps;
  const int t2 = active ? tid : 0;   // idle lanes alias lane 0 and never write
  const int g = t2 / G, l = t2 - (t2 / G) * G;
  int* wg_ctl = reinterpret_cast<int*>(smem);
  float* bufA = reinterpret_cast<float*>(smem + kWgCtlBytes);
  float* bufB = (nbuf == 2) ? bufA + (size_t)npos * ldw : bufA;
  int* ctl = reinterpret_cast<int*>(bufA + (size_t)nbuf * npos * ldw);
  const float* __restrict__ Ms = a.M;
  float* Zs = a.Z;

  const int qm = (npad + 4 * G - 1) / (4 * G);   // chunks that hold M rows in some lane
  const bool lastm = 4 * (l + G * (qm - 1)) < npad;   // chunk qm - 1 holds M rows in this lane

  // ---- load: slot g holds columns g (top) and 2 npairs - 1 - g (bottom) ----
  float av[R], bv[R];
  int ida = g, idb = 2 * npairs - 1 - g;   // idb == n: the zero column of odd n
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 4 * (l + G * q) + e;
      float x = 0.f, y = 0.f;
      if (active) {
        if (row < npad) {
          if (row < n) {
            x = Ms[(long long)ida * n + row];
            y = idb < n ? Ms[(long long)idb * n + row] : 0.f;
          }
        } else if (row - npad < n) {
          const int zr = row - npad;
          if (a.cold) {
            x = zr == ida ? 1.f : 0.f;
            y = zr == idb ? 1.f : 0.f;
          } else {
            x = Zs[(long long)ida * n + zr];
            y = idb < n ? Zs[(long long)idb * n + zr] : 0.f;
          }
        }
      }
      av[4 * q + e] = x;
      bv[4 * q + e] = y;
    }
  if (tid == 0) {
    wg_ctl[0] = 0;
    wg_ctl[1] = 0;
  }
  __syncthreads();

  double tol = a.tol;
  const bool dot32 = decode_tol(tol);
  // loop-invariant and uniform: held in scalar registers (frees vector
  // registers the round loop would otherwise spill)
  const double tol2 = uniform_d(tol * tol);
  const double big2 = uniform_d(big_rotation2(tol));
  double na = 0.0, nb = 0.0;
  int sweep = 0, my_sweeps = 0;
  bool converged = false;
  long long rotations = 0;
  for (;;) {
    na = group_sum<G>(dot64_m<R>(av, av, lastm, qm));
    nb = group_sum<G>(dot64_m<R>(bv, bv, lastm, qm));
    unsigned my_rot = 0;
    int c = npairs;
    bool ring = (c & 1) == 0;
    int s0 = 0, i = g, r = 0;
    const int nrounds = 2 * npairs - 1;
    for (int k = 0; k < nrounds; ++k) {
      // the rotation of the slot's pair, on the whole column (identity, c = 1
      // and s = 0, on lanes without one)
      float cf = 1.f, sf = 0.f;
      double t = 0.0;
      double d = 0.0, pa = 0.0, pb = 0.0;
      bool rot = false;
      if (active) {
        d = dot32 ? (double)group_sumf<G>(dot32_m<R>(av, bv, lastm, qm)) : group_sum<G>(dot64_m<R>(av, bv, lastm, qm));
        pa = fmax(na, 0.0);
        pb = fmax(nb, 0.0);
        rot = d != 0.0 && d * d > tol2 * (pa * pb);
        if (rot) {
          jacobi_angle(d, pa, pb, t, cf, sf);
        }
      }
      // waves without a rotation skip the update (most of them in the late
      // sweeps of a warm start)
      if (__builtin_amdgcn_ballot_w64(rot) != 0) rotate_in_place<R>(av, bv, cf, sf);
      if (rot) {
        na = fma(-t, d, pa);
        nb = fma(t, d, pb);
        my_rot += (l == 0) ? 1u + (d * d > big2 * (pa * pb) ? kBigOne : 0u) : 0u;
      }
      if (k + 1 == nrounds) break;
      if (ring && r + 1 < c) {
        if (nbuf == 2) {
          const int nxt = s0 + (i + 1 == c ? 0 : i + 1);
          float* buf = (r & 1) ? bufB : bufA;
          if (active) put_col<G, R>(buf, ldw, g, l, bv, Q, nb, idb);
          __syncthreads();
          if (active) get_col<G, R>(buf, ldw, nxt, l, bv, Q, nb, idb);
        } else {
          // one buffer, one barrier: in round r of the phase slot i writes
          // position (i + r) mod c of its range and reads (i + 1 + r) mod c,
          // slot i+1's; the position it writes next round is the one only it
          // read this round, so no second barrier is needed
          const int wpos = i + r < c ? i + r : i + r - c;
          const int rpos = wpos + 1 == c ? 0 : wpos + 1;
          if (active) put_col<G, R>(bufA, ldw, s0 + wpos, l, bv, Q, nb, idb);
          __syncthreads();
          if (active) get_col<G, R>(bufA, ldw, s0 + rpos, l, bv, Q, nb, idb);
        }
        ++r;
      } else if (ring) {
        const int h = c >> 1;
        const bool first = i < h;
        // the ring rounds' last reads may still be in flight (single buffer)
        if (nbuf == 1 && r > 0) __syncthreads();
        if (active) {
          if (first) put_col<G, R>(bufB, ldw, g, l, bv, Q, nb, idb);
          else put_col<G, R>(bufB, ldw, g, l, av, Q, na, ida);
        }
        __syncthreads();
        if (active) {
          if (first) get_col<G, R>(bufB, ldw, g + h, l, bv, Q, nb, idb);
          else get_col<G, R>(bufB, ldw, g - h, l, av, Q, na, ida);
        }
        if (nbuf == 1) __syncthreads();
        c = h;
        ring = (c & 1) == 0;
        s0 = (g / c) * c;
        i = g - s0;
        r = 0;
      } else {
        const int pos0 = s0 + s0 / c;
        if (active) {
          put_col<G, R>(bufA, ldw, pos0 + i, l, av, Q, na, ida);
          if (i == 0) put_col<G, R>(bufA, ldw, pos0 + c, l, bv, Q, nb, idb);
        }
        __syncthreads();
        if (active && i != 0) {
          get_col<G, R>(bufA, ldw, pos0 + (i == 1 ? c : i - 1), l, av, Q, na, ida);
          put_col<G, R>(bufA, ldw, pos0 + i - 1, l, bv, Q, nb, idb);
        }
        __syncthreads();
        if (active) get_col<G, R>(bufA, ldw, pos0 + i, l, bv, Q, nb, idb);
        ++r;
      }
    }
    // one slice per workgroup: the workgroup's counters are the slice's
    if (my_rot) atomicAdd(reinterpret_cast<unsigned*>(&wg_ctl[sweep & 1]), my_rot);
    __syncthreads();
    const unsigned any = static_cast<unsigned>(wg_ctl[sweep & 1]);
    if (tid == 0) wg_ctl[(sweep + 1) & 1] = 0;
    __syncthreads();
    ++sweep;
    rotations += any & 0xFFFFu;
    my_sweeps = sweep;
    converged = (any >> 16) == 0;
    if (converged || sweep >= a.max_sweeps) break;
  }

  // ---- output: the accumulated Z, then the kept columns as jacobi_body ------
  if (active) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int zr = 4 * (l + G * q) + e - npad;
        if (zr >= 0 && zr < n) {
          if (ida < n) Zs[(long long)ida * n + zr] = av[4 * q + e];
          if (idb < n) Zs[(long long)idb * n + zr] = bv[4 * q + e];
        }
      }
  }
  na = group_sum<G>(dot64_m<R>(av, av, lastm, qm));
  nb = group_sum<G>(dot64_m<R>(bv, bv, lastm, qm));
  const double sa = sqrt(na), sb = sqrt(nb);
  const bool ka = active && ida < n && sa > a.tau;
  const bool kb = active && idb < n && sb > a.tau;
  // the exchange buffer is free once the last sweep's barriers have passed
  double* nucs = reinterpret_cast<double*>(bufA);
  if (active && l == 0) {
    ctl[3 + g] = (int)ka + (int)kb;
    nucs[g] = (ka ? sa - a.tau : 0.0) + (kb ? sb - a.tau : 0.0);
  }
  __syncthreads();
  if (active && t2 == 0) {
    int acc = 0;
    double nsum = 0.0;
    for (int p = 0; p < npairs; ++p) {
      const int cnt = ctl[3 + p];
      ctl[3 + p] = acc;
      acc += cnt;
      nsum += nucs[p];
    }
    ctl[2] = acc;
    if (a.nuc) *a.nuc = nsum;
  }
  __syncthreads();
  float* out = a.out;
  const int j0 = active ? ctl[3 + g] : 0;
  const double sca = ka ? sqrt(1.0 - a.tau / sa) / sa : 0.0;
  const double scb = kb ? sqrt(1.0 - a.tau / sb) / sb : 0.0;
  const int da = ka ? j0 : -1;
  const int db = kb ? j0 + (int)ka : -1;
  // the LDS columns' first n rows are the M rows
  if (active) put_col<G, R>(bufA, ldw, g, l, av, Q, sca, da);
  __syncthreads();
  if (active) stage_out(out, bufA, ldw, n, npairs, t2, tps);
  __syncthreads();
  if (active) put_col<G, R>(bufA, ldw, g, l, bv, Q, scb, db);
  __syncthreads();
  if (active) stage_out(out, bufA, ldw, n, npairs, t2, tps);
  if (active && t2 == 0) {
    if (a.rank) *a.rank = ctl[2];
    if (a.sweeps) *a.sweeps = my_sweeps;
    if (a.sweep_total) atomicAdd(a.sweep_total, (unsigned long long)my_sweeps);
    if (a.rot_total) atomicAdd(a.rot_total, (unsigned long long)rotations);
    if (!converged && a.hits) atomicAdd(a.hits, 1u);
  }
}

template <int G, int R, int LB>
__global__ __launch_bounds__(LB) void k_jacobi_warm(WarmArgs a, int nbuf, int ldw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const long long s = blockIdx.x;
  WarmJob j;
  j.M = a.M + s * a.m_stride;
  j.Z = a.Z + s * a.n * a.n;
  j.out = a.bk + s * a.bk_stride;
  j.rank = a.rank ? a.rank + s : nullptr;
  j.sweeps = a.sweeps ? a.sweeps + s : nullptr;
  j.sweep_total = a.sweep_total;
  j.rot_total = a.rot_total;
  j.hits = a.hits;
  j.nuc = a.nuc ? a.nuc + s : nullptr;
  j.tau = a.tau;
  j.tol = a.tol;
  j.n = a.n;
  j.max_sweeps = a.max_sweeps;
  j.cold = a.cold;
  jacobi_warm_body<G, R>(j, nbuf, ldw, smem);
}

// Batch: one workgroup per slice of the warm-started problems.
template <int G, int R, int LB>
__global__ __launch_bounds__(LB) void k_jacobi_warm_items(ProbDev* const* probs, const CholItem* items, double tol,
                                                         int max_sweeps, int nbuf, int ldw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const CholItem it = items[blockIdx.x];
  ProbDev* pd = probs[it.prob];
  if (!pd->active) return;
  const int n = pd->I1 < pd->I2 ? pd->I1 : pd->I2;
  const bool cold = warm_cold(pd);
  const float* L = reinterpret_cast<const float*>(pd->C) + (long long)it.slice * 2 * n * n;
  WarmJob j;
  j.M = cold ? L : L + (long long)n * n;
  j.Z = pd->Z + (long long)it.slice * n * n;
  j.out = pd->Bk + (long long)it.slice * pd->N;
  j.rank = pd->rank + it.slice;
  j.sweeps = pd->sweeps + it.slice;
  j.sweep_total = &pd->sweep_total;
  j.rot_total = &pd->rot_total;
  j.hits = &pd->maxsweep_hits;
  j.nuc = pd->nuc + it.slice;
  j.tau = pd->tau;
  j.tol = tol;
  j.n = n;
  j.max_sweeps = max_sweeps;
  j.cold = cold ? 1 : 0;
  jacobi_warm_body<G, R>(j, nbuf, ldw, smem);
}

// ---- rebuild D_W = Bk (Bk^T W) ------------------------------------------------
constexpr int RB_TN = 16;   // working columns per workgroup
constexpr int RB_TK = 32;   // rows per LDS chunk
constexpr int RB_RMAX = 256;       // kept columns of the register-resident kernel's slices
constexpr int RB_RMAX_BLK = 512;   // kept columns of the blocked kernel's slices

__device__ inline float w_at(const float* W, bool trans, int I1, int row, int col) {
  return trans ? W[(long long)row * I1 + col] : W[(long long)col * I1 + row];
}

// Working columns j0 .. j0+15 of one slice: Z = Bk^T W(:, j0..) (r x 16), then
// D_W(:, j0..) = Bk Z.  W and D may alias: the tile is read in full before any
// of it is written, and no other workgroup touches these entries.  The kept
// columns' LDS (a chunk of Bk and Z) is sized by the launch for rcap >= r
// columns (dynamic), so small slices keep more workgroups per CU.
__host__ __device__ inline size_t rebuild_lds_bytes(int rcap) {
  return ((size_t)RB_TK * (rcap + 1) + (size_t)rcap * (RB_TN + 1)) * sizeof(float);
}

__host__ __device__ inline int rebuild_rcap(int kmax) { return ((kmax + 15) / 16) * 16; }

template <int RMAX>
__device__ void rebuild_body(const float* W, float* D, const float* Bk, int r, int I1, int I2, int j0,
                             bool flip, int rcap) {
  __shared__ float Ws[RB_TK][RB_TN + 1];
  extern __shared__ float rb_dyn[];
  const int ldb = rcap + 1;
  float* Bs = rb_dyn;                    // RB_TK x ldb: a chunk of rows of Bk
  float* Z = rb_dyn + RB_TK * ldb;       // rcap x (RB_TN + 1)
  // flip: the working matrix is W^T (n x m), so the same two products give
  // D_W^T = B (B^T W^T), i.e. D_W = (W B) B^T with B n x r
  const bool trans = (I1 < I2) != flip;
  const int m = flip ? (I1 < I2 ? I1 : I2) : (I1 < I2 ? I2 : I1);
  const int n = flip ? (I1 < I2 ? I2 : I1) : (I1 < I2 ? I1 : I2);
  const int nq = (r + 15) >> 4;
  const int rpad = nq << 4;
  const int tid = threadIdx.x;
  const int jj = tid & 15, hi = tid >> 4;

  // phase A: Z[i][jj] = sum_k Bk[k][i] W[k][j0 + jj]
  float zacc[RMAX / 16];
#pragma unroll
  for (int q = 0; q < RMAX / 16; ++q) zacc[q] = 0.f;
  if (r > 0) {
    for (int k0 = 0; k0 < m; k0 += RB_TK) {
      for (int idx = tid; idx < RB_TK * RB_TN; idx += 256) {
        int kk, c;
        if (trans) { c = idx % RB_TN; kk = idx / RB_TN; } else { kk = idx % RB_TK; c = idx / RB_TK; }
        const int row = k0 + kk, col = j0 + c;
        Ws[kk][c] = (row < m && col < n) ? w_at(W, trans, I1, row, col) : 0.f;
      }
      for (int idx = tid; idx < RB_TK * rpad; idx += 256) {
        const int kk = idx % RB_TK, i = idx / RB_TK;
        const int row = k0 + kk;
        Bs[kk * ldb + i] = (row < m && i < r) ? Bk[(long long)i * m + row] : 0.f;
      }
      __syncthreads();
      for (int kk = 0; kk < RB_TK; ++kk) {
        const float w = Ws[kk][jj];
#pragma unroll
        for (int q = 0; q < RMAX / 16; ++q)
          if (q < nq) zacc[q] = fmaf(Bs[kk * ldb + hi + 16 * q], w, zacc[q]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < RMAX / 16; ++q)
    if (q < nq) Z[(hi + 16 * q) * (RB_TN + 1) + jj] = zacc[q];
  __syncthreads();

  // phase B: D_W[k][j0 + jj] = sum_i Bk[k][i] Z[i][jj].  Consecutive lanes
  // store consecutive addresses: along the columns when D_W's rows are
  // contiguous (trans), else along the rows.
  const int bc = trans ? jj : hi;   // this lane's output column in the block
  const int br = trans ? hi : jj;   // and its row offset in the chunk (+ 16 h)
  for (int k0 = 0; k0 < m; k0 += RB_TK) {
    for (int idx = tid; idx < RB_TK * rpad; idx += 256) {
      const int kk = idx % RB_TK, i = idx / RB_TK;
      const int row = k0 + kk;
      Bs[kk * ldb + i] = (row < m && i < r) ? Bk[(long long)i * m + row] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = br + 16 * h;
      float acc = 0.f;
      for (int i = 0; i < r; ++i) acc = fmaf(Bs[kk * ldb + i], Z[i * (RB_TN + 1) + bc], acc);
      const int row = k0 + kk, col = j0 + bc;
      if (row < m && col < n) {
        if (trans) D[(long long)row * I1 + col] = acc;
        else D[(long long)col * I1 + row] = acc;
      }
    }
    __syncthreads();
  }
}

// The same rebuild for working matrices of at most MMAX rows (256, or 384 for
// the complex slices' interleaved rows): the block's 16 columns of W are staged
// once (all m rows), and the kept columns are taken sixteen at a time (a chunk
// of Bk staged, Z = Bk^T W for the chunk, then D_W += Bk Z), so a slice of low
// rank costs two staging passes and four barriers instead of a pass per 32
// rows.  LDS: the block, one chunk of Bk and Z, each padded to an odd pitch.
constexpr int RBS_MMAX = 256;
constexpr int RBS_MMAX_CX = 384;

// Index (row, c) of entry e = row + m c (or c + 16 row when rows are the long
// dimension) stepped by 256 entries without a division per step.
struct RbIdx {
  int a, b;          // a: the fast index, b: the slow one
  int qa, qb, lim;   // 256 = qb lim + qa
  __device__ RbIdx(int e, int lim_) : lim(lim_) {
    b = e / lim_;
    a = e - b * lim_;
    qb = 256 / lim_;
    qa = 256 - qb * lim_;
  }
  __device__ void step() {
    a += qa;
    b += qb;
    if (a >= lim) {
      a -= lim;
      ++b;
    }
  }
};

template <int MMAX>
__device__ void rebuild_body_small(const float* W, float* D, const float* Bk, int r, int I1, int I2, int j0,
                                   bool flip) {
  __shared__ float Xs[RB_TN][MMAX + 1];  // W(:, j0 + c) at Xs[c][row]
  __shared__ float Bs[RB_TN][MMAX + 1];  // Bk(:, i0 + i) at Bs[i][row]
  __shared__ float Zs[RB_TN][RB_TN + 1]; // Z(i0 + i, c)
  const bool trans = (I1 < I2) != flip;
  const int m = flip ? (I1 < I2 ? I1 : I2) : (I1 < I2 ? I2 : I1);
  const int n = flip ? (I1 < I2 ? I2 : I1) : (I1 < I2 ? I1 : I2);
  const int tid = threadIdx.x;
  const int nout = RB_TN * m;
  // the block, coalesced along whichever dimension W keeps contiguous
  // (trans: entry e = c + 16 row, else e = row + m c)
  {
    RbIdx x(tid, trans ? RB_TN : m);
    for (int idx = tid; idx < nout; idx += 256, x.step()) {
      const int row = trans ? x.b : x.a, c = trans ? x.a : x.b;
      const int col = j0 + c;
      Xs[c][row] = col < n ? w_at(W, trans, I1, row, col) : 0.f;
    }
  }
  // output ownership: consecutive lanes store consecutive addresses
  float acc[(RB_TN * MMAX + 255) / 256];
#pragma unroll
  for (int u = 0; u < (RB_TN * MMAX + 255) / 256; ++u) acc[u] = 0.f;
  for (int i0 = 0; i0 < r; i0 += RB_TN) {
    const int nc = r - i0 < RB_TN ? r - i0 : RB_TN;
    {
      RbIdx x(tid, m);
      for (int idx = tid; idx < nout; idx += 256, x.step())
        Bs[x.b][x.a] = x.b < nc ? Bk[(long long)(i0 + x.b) * m + x.a] : 0.f;
    }
    __syncthreads();
    {   // Z(i, c) = sum_row Bk(row, i0 + i) W(row, j0 + c), one entry per lane
        // (four interleaved partial sums: a shorter dependent chain)
      const int i = tid >> 4, c = tid & 15;
      float z0 = 0.f, z1 = 0.f, z2 = 0.f, z3 = 0.f;
      int row = 0;
      for (; row + 4 <= m; row += 4) {
        z0 = fmaf(Bs[i][row], Xs[c][row], z0);
        z1 = fmaf(Bs[i][row + 1], Xs[c][row + 1], z1);
        z2 = fmaf(Bs[i][row + 2], Xs[c][row + 2], z2);
        z3 = fmaf(Bs[i][row + 3], Xs[c][row + 3], z3);
      }
      for (; row < m; ++row) z0 = fmaf(Bs[i][row], Xs[c][row], z0);
      Zs[i][c] = (z0 + z1) + (z2 + z3);
    }
    __syncthreads();
    RbIdx x(tid, trans ? RB_TN : m);
#pragma unroll
    for (int u = 0; u < (RB_TN * MMAX + 255) / 256; ++u, x.step()) {
      if (tid + 256 * u < nout) {
        const int row = trans ? x.b : x.a, c = trans ? x.a : x.b;
        float v = acc[u];
        for (int i = 0; i < nc; ++i) v = fmaf(Bs[i][row], Zs[i][c], v);
        acc[u] = v;
      }
    }
    __syncthreads();
  }
  RbIdx x(tid, trans ? RB_TN : m);
#pragma unroll
  for (int u = 0; u < (RB_TN * MMAX + 255) / 256; ++u, x.step()) {
    if (tid + 256 * u < nout) {
      const int row = trans ? x.b : x.a, c = trans ? x.a : x.b;
      const int col = j0 + c;
      if (col < n) {
        if (trans) D[(long long)row * I1 + col] = acc[u];
        else D[(long long)col * I1 + row] = acc[u];
      }
    }
  }
}

template <int MMAX>
__global__ __launch_bounds__(256) void k_rebuild_small(RebuildArgs a) {
  const int s = blockIdx.y;
  const int n = a.flip ? (a.I1 < a.I2 ? a.I2 : a.I1) : (a.I1 < a.I2 ? a.I1 : a.I2);
  const int j0 = blockIdx.x * RB_TN;
  if (j0 >= n) return;
  const long long off = (long long)s * a.slice_stride;
  const float* bk = a.bk + (long long)s * (a.bk_stride ? a.bk_stride : a.slice_stride);
  rebuild_body_small<MMAX>(a.W + off, a.D + off, bk, a.rank[s], a.I1, a.I2, j0, a.flip != 0);
}

template <int RMAX>
__global__ __launch_bounds__(256) void k_rebuild(RebuildArgs a) {
  const int s = blockIdx.y;
  const int n = a.flip ? (a.I1 < a.I2 ? a.I2 : a.I1) : (a.I1 < a.I2 ? a.I1 : a.I2);
  const int j0 = blockIdx.x * RB_TN;
  if (j0 >= n) return;
  const long long off = (long long)s * a.slice_stride;
  const float* bk = a.bk + (long long)s * (a.bk_stride ? a.bk_stride : a.slice_stride);
  rebuild_body<RMAX>(a.W + off, a.D + off, bk, a.rank[s], a.I1, a.I2, j0, a.flip != 0, a.rcap);
}

template <int RMAX>
__global__ __launch_bounds__(256) void k_rebuild_tiles(ProbDev* const* probs, const RebuildTile* tiles,
                                                       int rcap) {
  const RebuildTile t = tiles[blockIdx.x];
  const ProbDev* pd = probs[t.prob];
  if (!pd->active) return;
  const long long off = (long long)t.slice * pd->N;
  const int m = pd->precond ? (pd->I1 < pd->I2 ? pd->I1 : pd->I2) : (pd->I1 < pd->I2 ? pd->I2 : pd->I1);
  if (m <= RBS_MMAX)
    rebuild_body_small<RBS_MMAX>(pd->Gh + off, pd->Gh + off, pd->Bk + off, pd->rank[t.slice], pd->I1, pd->I2,
                                 t.j0, pd->precond != 0);
  else
    rebuild_body<RMAX>(pd->Gh + off, pd->Gh + off, pd->Bk + off, pd->rank[t.slice], pd->I1, pd->I2, t.j0,
                       pd->precond != 0, rcap);
}

// ---- lsvd: sort, normalise, V = W^T U / sigma, orthonormalise ---------------
constexpr int LS_NMAX = 256;
constexpr int LS_MMAX = 2048;

__device__ inline double block_sum256(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Orthonormalise the n columns of Q (len x n, ld len) in order by classical
// Gram-Schmidt with one re-orthogonalisation pass.  Column k is replaced by a
// canonical basis vector (the first that survives the projection) when ok[k]
// is false or when it is numerically dependent on the columns before it.
__device__ void cgs2_columns(float* Q, int len, int n, const int* ok, double* v, double* c,
                             double* red) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    for (int cand = -1; cand < len; ++cand) {
      if (cand < 0 && !ok[k]) continue;
      for (int row = tid; row < len; row += 256)
        v[row] = cand < 0 ? (double)Q[(long long)k * len + row] : (row == cand ? 1.0 : 0.0);
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int j = tid; j < k; j += 256) {
          double acc = 0.0;
          for (int row = 0; row < len; ++row) acc += (double)Q[(long long)j * len + row] * v[row];
          c[j] = acc;
        }
        __syncthreads();
        for (int row = tid; row < len; row += 256) {
          double acc = v[row];
          for (int j = 0; j < k; ++j) acc -= c[j] * (double)Q[(long long)j * len + row];
          v[row] = acc;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int row = tid; row < len; row += 256) part += v[row] * v[row];
      const double nrm = sqrt(block_sum256(part, red));
      if (nrm > 0.5) {   // existing columns start at norm ~1; candidates at 1
        for (int row = tid; row < len; row += 256) Q[(long long)k * len + row] = (float)(v[row] / nrm);
        __syncthreads();
        break;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_lsvd_finalize(LsvdArgs a) {
  __shared__ int perm[LS_NMAX];
  __shared__ int ok[LS_NMAX];
  __shared__ double sg[LS_NMAX];
  __shared__ double cbuf[LS_NMAX];
  __shared__ double vbuf[LS_MMAX];
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int I1 = a.I1, I2 = a.I2;
  const bool trans = I1 < I2;
  const int m = trans ? I2 : I1;
  const int n = trans ? I1 : I2;
  const int tid = threadIdx.x;
  const double* sig = a.sigma + (long long)s * n;
  for (int i = tid; i < n; i += 256) {
    const double si = sig[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = sig[j];
      rk += (sj > si) || (sj == si && j < i);
    }
    perm[rk] = i;
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256) sg[k] = sig[perm[k]];
  __syncthreads();
  const double smax = n > 0 ? sg[0] : 0.0;
  const double cut = smax * 1e-6;
  for (int k = tid; k < n; k += 256) ok[k] = sg[k] > cut;
  const float* W = a.W + (long long)s * a.slice_stride;
  const float* cols = a.cols + (long long)s * a.slice_stride;
  // Uw (m x n) and Vw (n x n) live in the output factors:
  //   I1 >= I2: U = Uw (I1 x n), V = Vw (I2 x n);  I1 < I2: U = Vw (I1 x n), V = Uw (I2 x n).
  float* Uw = trans ? a.V + (long long)s * I2 * n : a.U + (long long)s * I1 * n;
  float* Vw = trans ? a.U + (long long)s * I1 * n : a.V + (long long)s * I2 * n;
  __syncthreads();
  for (int idx = tid; idx < m * n; idx += 256) {
    const int k = idx / m, row = idx - k * m;
    const double sk = sg[k];
    Uw[(long long)k * m + row] = sk > cut ? (float)((double)cols[(long long)perm[k] * m + row] / sk) : 0.f;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += 256) {
    const int k = idx / n, j = idx - k * n;
    const double sk = sg[k];
    double acc = 0.0;
    if (sk > cut) {
      for (int row = 0; row < m; ++row)
        acc += (double)w_at(W, trans, I1, row, j) * (double)Uw[(long long)k * m + row];
      acc /= sk;
    }
    Vw[(long long)k * n + j] = (float)acc;
  }
  __syncthreads();
  // W^T u / sigma loses orthogonality like eps sigma_max / sigma; re-orthogonalising
  // in decreasing-sigma order changes U S V^T by at most ~eps sigma_max
  cgs2_columns(Uw, m, n, ok, vbuf, cbuf, red);
  cgs2_columns(Vw, n, n, ok, vbuf, cbuf, red);
  float* S = a.S + (long long)s * n * n;
  for (int idx = tid; idx < n * n; idx += 256) {
    const int k = idx / n, j = idx - k * n;
    S[idx] = (j == k) ? (float)sg[k] : 0.f;
  }
  if (a.sig_out)
    for (int k = tid; k < n; k += 256) a.sig_out[(long long)s * n + k] = (float)sg[k];
}

// cgs2_columns for complex columns held as interleaved (Re, Im) rows (2 len
// floats per column): c_j = q_j^H v, v -= sum_j c_j q_j, twice, then
// normalise; v and c hold interleaved FP64 pairs.
__device__ void cgs2_columns_cx(float* Q, int len, int n, const int* ok, double* v, double* c, double* red) {
  const int tid = threadIdx.x;
  const long long cs = 2LL * len;
  for (int k = 0; k < n; ++k) {
    for (int cand = -1; cand < len; ++cand) {
      if (cand < 0 && !ok[k]) continue;
      for (int row = tid; row < len; row += 256) {
        v[2 * row] = cand < 0 ? (double)Q[k * cs + 2 * row] : (row == cand ? 1.0 : 0.0);
        v[2 * row + 1] = cand < 0 ? (double)Q[k * cs + 2 * row + 1] : 0.0;
      }
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        for (int j = tid; j < k; j += 256) {
          double cr = 0.0, ci = 0.0;
          for (int row = 0; row < len; ++row) {
            const double qr = Q[j * cs + 2 * row], qi = Q[j * cs + 2 * row + 1];
            cr += qr * v[2 * row] + qi * v[2 * row + 1];
            ci += qr * v[2 * row + 1] - qi * v[2 * row];
          }
          c[2 * j] = cr;
          c[2 * j + 1] = ci;
        }
        __syncthreads();
        for (int row = tid; row < len; row += 256) {
          double ar = v[2 * row], ai = v[2 * row + 1];
          for (int j = 0; j < k; ++j) {
            const double qr = Q[j * cs + 2 * row], qi = Q[j * cs + 2 * row + 1];
            ar -= c[2 * j] * qr - c[2 * j + 1] * qi;
            ai -= c[2 * j] * qi + c[2 * j + 1] * qr;
          }
          v[2 * row] = ar;
          v[2 * row + 1] = ai;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int row = tid; row < len; row += 256) part += v[2 * row] * v[2 * row] + v[2 * row + 1] * v[2 * row + 1];
      const double nrm = sqrt(block_sum256(part, red));
      if (nrm > 0.5) {
        for (int row = tid; row < len; row += 256) {
          Q[k * cs + 2 * row] = (float)(v[2 * row] / nrm);
          Q[k * cs + 2 * row + 1] = (float)(v[2 * row + 1] / nrm);
        }
        __syncthreads();
        break;
      }
    }
  }
}

// Economy factors of complex slices (Fourier modes), one workgroup per
// conjugate-pair representative t: the singular values sorted descending,
// Uw = cols / sigma, Vw = W^H Uw / sigma, both re-orthonormalised (complex
// CGS2, in the scratch), then the factors of slice rep[t] (I1 >= I2: U = Uw,
// V = Vw; I1 < I2, W the plain transpose: U = conj(Vw), V = conj(Uw)) and the
// conjugates for its partner into real and imaginary planes.  A self-conjugate
// slice (real data) gets zero imaginary parts.
__global__ __launch_bounds__(256) void k_lsvd_finalize_cx(LsvdCxArgs a) {
  __shared__ int perm[LS_NMAX];
  __shared__ int ok[LS_NMAX];
  __shared__ double sg[LS_NMAX];
  __shared__ double cbuf[2 * LS_NMAX];
  __shared__ double vbuf[LS_MMAX];
  __shared__ double red[256];
  const int t = blockIdx.x;
  const int p = a.rep[t], q = a.partner[t];
  const int I1 = a.I1, I2 = a.I2;
  const bool trans = I1 < I2;
  const int m = trans ? I2 : I1;
  const int n = trans ? I1 : I2;
  const int tid = threadIdx.x;
  const double* sig = a.sigma + (long long)t * n;
  for (int i = tid; i < n; i += 256) {
    const double si = sig[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = sig[j];
      rk += (sj > si) || (sj == si && j < i);
    }
    perm[rk] = i;
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256) sg[k] = sig[perm[k]];
  __syncthreads();
  const double cut = (n > 0 ? sg[0] : 0.0) * 1e-6;
  for (int k = tid; k < n; k += 256) ok[k] = sg[k] > cut;
  const float* W = a.W + (long long)t * a.w_stride;
  const float* cols = a.cols + (long long)t * a.w_stride;
  float* Uw = a.scratch + (long long)t * a.scratch_stride;   // 2m x n
  float* Vw = Uw + 2LL * m * n;                              // 2n x n
  __syncthreads();
  for (int idx = tid; idx < 2 * m * n; idx += 256) {
    const int k = idx / (2 * m), r = idx - k * 2 * m;
    const double sk = sg[k];
    Uw[idx] = sk > cut ? (float)((double)cols[(long long)perm[k] * 2 * m + r] / sk) : 0.f;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += 256) {
    const int k = idx / n, j = idx - k * n;
    const double sk = sg[k];
    double ar = 0.0, ai = 0.0;
    if (sk > cut) {
      const float* wj = W + (long long)j * 2 * m;
      const float* uk = Uw + (long long)k * 2 * m;
      for (int row = 0; row < m; ++row) {   // conj(w) u
        const double wr = wj[2 * row], wi = wj[2 * row + 1], ur = uk[2 * row], ui = uk[2 * row + 1];
        ar += wr * ur + wi * ui;
        ai += wr * ui - wi * ur;
      }
      ar /= sk;
      ai /= sk;
    }
    Vw[(long long)k * 2 * n + 2 * j] = (float)ar;
    Vw[(long long)k * 2 * n + 2 * j + 1] = (float)ai;
  }
  __syncthreads();
  cgs2_columns_cx(Uw, m, n, ok, vbuf, cbuf, red);
  cgs2_columns_cx(Vw, n, n, ok, vbuf, cbuf, red);
  // U (I1 x n) and V (I2 x n) of slice p; Uw has m rows, Vw n rows
  const float* Us = trans ? Vw : Uw;
  const float* Vs = trans ? Uw : Vw;
  const float sgn = trans ? -1.f : 1.f;   // conjugated when transposed
  const long long pu = (long long)a.P * I1 * n, pv = (long long)a.P * I2 * n, ps = (long long)a.P * n * n;
  for (int idx = tid; idx < I1 * n; idx += 256) {
    const float re = Us[2 * idx], im = sgn * Us[2 * idx + 1];
    a.U[(long long)p * I1 * n + idx] = re;
    a.U[pu + (long long)p * I1 * n + idx] = q == p ? 0.f : im;
    if (q != p) {
      a.U[(long long)q * I1 * n + idx] = re;
      a.U[pu + (long long)q * I1 * n + idx] = -im;
    }
  }
  for (int idx = tid; idx < I2 * n; idx += 256) {
    const float re = Vs[2 * idx], im = sgn * Vs[2 * idx + 1];
    a.V[(long long)p * I2 * n + idx] = re;
    a.V[pv + (long long)p * I2 * n + idx] = q == p ? 0.f : im;
    if (q != p) {
      a.V[(long long)q * I2 * n + idx] = re;
      a.V[pv + (long long)q * I2 * n + idx] = -im;
    }
  }
  for (int idx = tid; idx < n * n; idx += 256) {
    const int k = idx / n, j = idx - k * n;
    const float v = (j == k) ? (float)sg[k] : 0.f;
    a.S[(long long)p * n * n + idx] = v;
    a.S[ps + (long long)p * n * n + idx] = 0.f;
    a.S[(long long)q * n * n + idx] = v;
    a.S[ps + (long long)q * n * n + idx] = 0.f;
  }
  if (a.sig_out)
    for (int k = tid; k < n; k += 256) {
      a.sig_out[(long long)p * n + k] = (float)sg[k];
      a.sig_out[(long long)q * n + k] = (float)sg[k];
    }
}

template <int G, int R, int LB>
hipError_t launch_one(const JacobiArgs& a, const JacobiConfig& c, hipStream_t s) {
  const int ldw = G * R + 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<G, R, LB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi<G, R, LB>), dim3(a.nslices), dim3(c.threads), c.lds, s, a, c.nbuf,
                     ldw);
  return hipGetLastError();
}

template <int G, int R>
hipError_t launch_gr(const JacobiArgs& a, const JacobiConfig& c, hipStream_t s) {
  // workgroups of <= 768 lanes run at most 3 waves per SIMD: 168 VGPRs per lane
  if (c.threads <= 768) return launch_one<G, R, 768>(a, c, s);
  return launch_one<G, R, 1024>(a, c, s);
}

template <int G>
hipError_t launch_g(const JacobiArgs& a, const JacobiConfig& c, hipStream_t s) {
  switch (c.R) {
    case 4: return launch_gr<G, 4>(a, c, s);
    case 8: return launch_gr<G, 8>(a, c, s);
    case 12: return launch_gr<G, 12>(a, c, s);
    case 16: return launch_gr<G, 16>(a, c, s);
    case 20: return launch_gr<G, 20>(a, c, s);
    case 24: return launch_gr<G, 24>(a, c, s);
    case 28: return launch_gr<G, 28>(a, c, s);
    case 32: return launch_gr<G, 32>(a, c, s);
    default: return hipErrorInvalidValue;
  }
}

template <int G, int R, int LB>
hipError_t launch_items_one(ProbDev* const* probs, const SvtItem* items, int nitems,
                            const JacobiBatchConfig& c, double tol, int max_sweeps, hipStream_t s) {
  const int ldw = G * R + 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_items<G, R, LB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi_items<G, R, LB>), dim3(nitems), dim3(c.threads), c.lds, s, probs,
                     items, tol, max_sweeps, c.nbuf, ldw);
  return hipGetLastError();
}

template <int G>
hipError_t launch_items_g(ProbDev* const* probs, const SvtItem* items, int nitems,
                          const JacobiBatchConfig& c, double tol, int max_sweeps, hipStream_t s) {
#define LT_ITEMS_CASE(RR)                                                                  \
  case RR:                                                                                 \
    return c.threads <= 768 ? launch_items_one<G, RR, 768>(probs, items, nitems, c, tol, max_sweeps, s) \
                            : launch_items_one<G, RR, 1024>(probs, items, nitems, c, tol, max_sweeps, s);
  switch (c.RMAX) {
    LT_ITEMS_CASE(4)
    LT_ITEMS_CASE(8)
    LT_ITEMS_CASE(12)
    LT_ITEMS_CASE(16)
    LT_ITEMS_CASE(20)
    LT_ITEMS_CASE(24)
    LT_ITEMS_CASE(28)
    LT_ITEMS_CASE(32)
    default: return hipErrorInvalidValue;
  }
#undef LT_ITEMS_CASE
}

template <int G, int R>
hipError_t launch_blk_one(const JacobiArgs& a, const JacobiBlkConfig& c, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_blk<G, R>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi_blk<G, R>), dim3(a.nslices), dim3(c.threads), c.lds, s, a);
  return hipGetLastError();
}

template <int G, int R>
hipError_t launch_blk_items_one(ProbDev* const* probs, const CholItem* items, int nitems, int threads,
                                size_t lds, double tol, int max_sweeps, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_blk_items<G, R>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi_blk_items<G, R>), dim3(nitems), dim3(threads), lds, s, probs, items, tol,
                     max_sweeps);
  return hipGetLastError();
}

size_t jacobi_lds_bytes(int npairs, int ldw, int nbuf) {
  return kWgCtlBytes + slice_lds_bytes(npairs, ldw, nbuf);
}

// ---- wide blocked Jacobi: one workgroup per block pair ----------------------
//
// The blocked layout above (working buffer of nblk blocks of b columns, the
// round-robin tournament over the blocks, the first block round of a sweep
// rotating every pair inside the two blocks as well), but every block round is
// one launch in which each block pair of each slice is a workgroup of its own:
// a slice spreads over nblk / 2 compute units instead of one, which is what
// slices with many columns and few of them per tensor need (the 1080 x 1920
// and 2160 x 3840 frames).  The block pairs of one round are disjoint, so the
// workgroups of a launch touch disjoint columns.  Per-slice state on the
// device (WideState) carries the sweep's rotation counts between launches; a
// sweep-end launch decides convergence (a sweep whose rotations were all small,
// as for the other kernels), and launches skip converged slices.

struct WideState {
  int done;                     // 0 running, 1 converged, 2 stopped at max_sweeps
  int sweeps;                   // sweeps done
  unsigned rot, big;            // this sweep's rotations and large rotations
  unsigned long long rot_total;
  unsigned long long pad;
};
static_assert(sizeof(WideState) == kWideStateBytes, "wide state size");

__device__ inline WideState* wide_state(const WideArgs& a, int s) {
  return reinterpret_cast<WideState*>(static_cast<char*>(a.state) + (size_t)s * kWideStateBytes);
}

// Working matrix W (m x n, the slice or its transpose) into the working buffer
// (ncols columns of mpad rows, zero beyond W): 32 x 32 tiles through LDS, read
// along the slice's contiguous dimension, written along the buffer's.
__global__ __launch_bounds__(256) void k_wide_copy_in(WideArgs a, int mpad, int ncols) {
  __shared__ float tile[32][33];
  const int s = blockIdx.z;
  const bool trans = a.I1 < a.I2;
  const int m = trans ? a.I2 : a.I1;
  const int n = trans ? a.I1 : a.I2;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const float* A = a.src + (long long)s * a.slice_stride;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int rr = trans ? ty + 8 * k : tx, cc = trans ? tx : ty + 8 * k;
    const int row = r0 + rr, col = c0 + cc;
    float v = 0.f;
    if (row < m && col < n) v = trans ? A[(long long)row * a.I1 + col] : A[(long long)col * a.I1 + row];
    tile[rr][cc] = v;
  }
  __syncthreads();
  float* Wk = a.work + (long long)s * a.work_stride;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int row = r0 + tx, col = c0 + ty + 8 * k;
    if (row < mpad && col < ncols) Wk[(long long)col * mpad + row] = tile[tx][ty + 8 * k];
  }
}

// Workgroup size of the wide kernels: 1024 lanes hold 16 rows per lane in 128
// registers; more rows per lane take 512-lane workgroups (256 registers).
template <int R>
constexpr int wide_lanes() { return R <= 16 ? 1024 : 512; }

// One block round: workgroup (pi, s) rotates block pair pi of round br of slice s.
template <int G, int R>
__global__ __launch_bounds__(wide_lanes<R>()) void k_wide_round(WideArgs a, int b, int nblk, int qeff, int nbuf, int br) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.y;
  WideState* st = wide_state(a, s);
  if (st->done) return;   // the whole workgroup returns
  const int mpad = 4 * G * qeff, ldw = mpad + 4;
  const int tps = b * G;
  const int tid = threadIdx.x;
  const bool active = tid < tps;
  const int g = active ? tid / G : 0, l = tid % G;
  int* wg_ctl = reinterpret_cast<int*>(smem);
  float* buf = reinterpret_cast<float*>(smem + kWgCtlBytes);
  float* bufB = nbuf == 2 ? buf + (size_t)exch_positions(b) * ldw : buf;
  float* Wk = a.work + (long long)s * a.work_stride;
  double tol = a.tol;
  const bool dot32 = decode_tol(tol);
  const int pi = blockIdx.x;
  const int A = blk_at(pi, br, nblk), B = blk_at(nblk - 1 - pi, br, nblk);
  int ida = A * b + g, idb = B * b + g;
  float av[R], bv[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    av[e] = 0.f;
    bv[e] = 0.f;
  }
  if (tid == 0) {
    wg_ctl[0] = 0;
    wg_ctl[1] = 0;
  }
  if (active) {
    load_work_col<G, R>(Wk, mpad, ida, l, av, qeff);
    load_work_col<G, R>(Wk, mpad, idb, l, bv, qeff);
  }
  __syncthreads();
  double na = group_sum<G>(dot64<R>(av, av));
  double nb = group_sum<G>(dot64<R>(bv, bv));
  const unsigned my_rot = sweep_rounds<G, R>(av, bv, na, nb, ida, idb, active, dot32, tol, b, g, l, qeff, buf,
                                             bufB, nbuf, ldw, br > 0);
  if (active) {
    store_work_col<G, R>(Wk, mpad, ida, l, av, qeff);
    store_work_col<G, R>(Wk, mpad, idb, l, bv, qeff);
  }
  if (my_rot & 0xFFFFu) atomicAdd(&wg_ctl[0], (int)(my_rot & 0xFFFFu));
  if (my_rot >> 16) atomicAdd(&wg_ctl[1], (int)(my_rot >> 16));
  __syncthreads();
  if (tid == 0) {
    if (wg_ctl[0]) atomicAdd(&st->rot, (unsigned)wg_ctl[0]);
    if (wg_ctl[1]) atomicAdd(&st->big, (unsigned)wg_ctl[1]);
  }
}

// End of a sweep (one thread per slice): count it, stop a slice whose
// rotations were all small (or at the sweep limit), clear the counters, and
// count the slices still running into *active (cleared by the host before).
__global__ void k_wide_sweep_end(WideArgs a, int* active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.nslices) return;
  WideState* st = wide_state(a, s);
  if (st->done == 0) {
    st->sweeps += 1;
    st->rot_total += st->rot;
    if (st->big == 0) st->done = 1;
    else if (st->sweeps >= a.max_sweeps) st->done = 2;
    st->rot = 0;
    st->big = 0;
    if (st->done == 0) atomicAdd(active, 1);
  }
}

// Output of a slice (one workgroup): kept columns, scaled, in column order,
// and the slice's counts, as the blocked kernel writes them.
template <int G, int R>
__global__ __launch_bounds__(wide_lanes<R>()) void k_wide_out(WideArgs a, int b, int nblk, int qeff) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.x;
  const WideState* st = wide_state(a, s);
  const bool trans = a.I1 < a.I2;
  const int m = trans ? a.I2 : a.I1;
  const int n = trans ? a.I1 : a.I2;
  const int mpad = 4 * G * qeff, ldw = mpad + 4;
  const int ncols = nblk * b;
  const int tps = b * G;
  const int tid = threadIdx.x;
  const bool active = tid < tps;
  const int g = active ? tid / G : 0, l = tid % G;
  float* buf = reinterpret_cast<float*>(smem + kWgCtlBytes);
  int* ctl = reinterpret_cast<int*>(buf + (size_t)exch_positions(b) * ldw);
  const float* Wk = a.work + (long long)s * a.work_stride;
  float* out = a.bk + (long long)s * a.bk_stride;
  float av[R];
#pragma unroll
  for (int e = 0; e < R; ++e) av[e] = 0.f;
  if (tid == 0) ctl[2] = 0;
  __syncthreads();
  double nsum = 0.0;
  double* nucs = reinterpret_cast<double*>(buf);
  for (int c0 = 0; c0 < ncols; c0 += b) {
    const int id = c0 + g;
    if (active) load_work_col<G, R>(Wk, mpad, id, l, av, qeff);
    const double sa = sqrt(group_sum<G>(dot64<R>(av, av)));
    const bool ka = active && id < n && sa > a.tau;
    if (active && l == 0) {
      ctl[3 + g] = ka ? 1 : 0;
      nucs[g] = ka ? sa - a.tau : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      int acc = ctl[2];
      for (int i = 0; i < b; ++i) {
        const int c = ctl[3 + i];
        ctl[3 + i] = acc;
        acc += c;
        nsum += nucs[i];
      }
      ctl[2] = acc;
    }
    __syncthreads();
    const int d = ka ? ctl[3 + g] : -1;
    const double sc = ka ? sqrt(1.0 - a.tau / sa) / sa : 0.0;
    if (active) put_col<G, R>(buf, ldw, g, l, av, qeff, sc, d);
    __syncthreads();
    if (active) stage_out(out, buf, ldw, m, b, tid, tps);
    __syncthreads();
  }
  if (tid == 0) {
    if (a.rank) a.rank[s] = ctl[2];
    if (a.nuc) a.nuc[s] = nsum;
    if (a.sweeps) a.sweeps[s] = st->sweeps;
    if (a.sweep_total) atomicAdd(a.sweep_total, (unsigned long long)st->sweeps);
    if (a.rot_total) atomicAdd(a.rot_total, st->rot_total);
    if (st->done == 2 && a.hits) atomicAdd(a.hits, 1u);
  }
}

template <int G, int R>
hipError_t launch_wide_sweep_one(const WideArgs& a, const JacobiWideConfig& c, int* active, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_wide_round<G, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)c.lds);
  if (e != hipSuccess) return e;
  for (int br = 0; br < c.nblk - 1; ++br) {
    hipLaunchKernelGGL((k_wide_round<G, R>), dim3(c.nblk / 2, a.nslices), dim3(c.threads), c.lds, s, a, c.b,
                       c.nblk, c.qeff, c.nbuf, br);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_fill_zero(active, sizeof(int), s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_wide_sweep_end, dim3((a.nslices + 255) / 256), dim3(256), 0, s, a, active);
  return hipGetLastError();
}

template <int G, int R>
hipError_t launch_wide_out_one(const WideArgs& a, const JacobiWideConfig& c, hipStream_t s) {
  const size_t lds = blk_lds_bytes(c.b, 4 * G * c.qeff + 4, 1);
  hipError_t e = hipFuncSetAttribute((const void*)k_wide_out<G, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_wide_out<G, R>), dim3(a.nslices), dim3(c.threads), lds, s, a, c.b, c.nblk, c.qeff);
  return hipGetLastError();
}

}  // namespace

int jacobi_pick_config(int m, int n, int max_lds, JacobiConfig* cfg, int force_G) {
  // n <= 256 also bounds the kept-column count of the rebuild kernel's LDS arrays
  if (m < 1 || n < 1 || m < n || n > RB_RMAX) return -1;
  const int npairs = (n + 1) / 2;
  const int Gs[5] = {64, 32, 16, 8, 4};
  int bestG = 0;
  int fallbackG = 0;
  for (int i = 0; i < 5; ++i) {
    const int G = Gs[i];
    if (force_G && G != force_G) continue;
    const int threads = ((npairs * G + 63) / 64) * 64;
    int R = (m + G - 1) / G;
    R = ((R + 3) / 4) * 4;
    if (threads > 1024 || R > 32) continue;
    const int ldw = G * R + 4;
    if (jacobi_lds_bytes(npairs, ldw, 1) > (size_t)max_lds) continue;
    if (R >= 8 && !bestG) bestG = G;
    fallbackG = G;   // ends as the smallest feasible G
  }
  const int G = bestG ? bestG : fallbackG;
  if (!G) return -1;
  int R = (m + G - 1) / G;
  R = ((R + 3) / 4) * 4;
  cfg->G = G;
  cfg->R = R;
  cfg->threads = ((npairs * G + 63) / 64) * 64;
  const int ldw = G * R + 4;
  if (jacobi_lds_bytes(npairs, ldw, 2) <= (size_t)max_lds) {
    cfg->nbuf = 2;
  } else {
    cfg->nbuf = 1;
  }
  cfg->lds = jacobi_lds_bytes(npairs, ldw, cfg->nbuf);
  return 0;
}

hipError_t launch_jacobi(const JacobiArgs& a0, const JacobiConfig& c, hipStream_t s) {
  if (a0.nslices <= 0) return hipSuccess;
  JacobiArgs a = a0;
  a.qeff = c.R / 4;
  switch (c.G) {
    case 4: return launch_g<4>(a, c, s);
    case 8: return launch_g<8>(a, c, s);
    case 16: return launch_g<16>(a, c, s);
    case 32: return launch_g<32>(a, c, s);
    case 64: return launch_g<64>(a, c, s);
    default: return hipErrorInvalidValue;
  }
}

// Complex slices: the stacked working matrix has ms = 2 m interleaved rows and
// n complex columns.  One 768-lane bound (up to 168 VGPRs per lane, for up to
// 48 rows per lane), G = 16 or 8 lanes per pair, R from a short list.
template <int G, int R>
static hipError_t launch_cx_one(const JacobiArgs& a, const JacobiConfig& c, hipStream_t s) {
  const int ldw = G * R + 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<G, R, 768, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi<G, R, 768, true>), dim3(a.nslices), dim3(c.threads), c.lds, s, a, c.nbuf, ldw);
  return hipGetLastError();
}

// Rows per lane instantiated (a count rounds up to the next): G = 16 serves
// columns of more than 128 rows only (more than 8 per lane), and G = 8 takes
// columns of more than 128 rows only when 16 lanes per pair would exceed the
// workgroup (n > 96, so more than 192 rows: more than 24 per lane).
static int cx_round_r(int G, int r) {
  static const int r8[] = {8, 16, 32, 36, 40, 44, 48};
  static const int r16[] = {16, 24, 32, 40, 48};
  const int* v = G == 8 ? r8 : r16;
  const int nv = G == 8 ? 7 : 5;
  for (int i = 0; i < nv; ++i)
    if (r <= v[i]) return v[i];
  return 0;
}

int jacobi_cx_config(int ms, int n, int max_lds, JacobiConfig* cfg) {
  if (ms < 2 || (ms & 1) || n < 1 || ms < n || 2 * n > RB_RMAX_BLK) return -1;
  const int npairs = (n + 1) / 2;
  const int Gs[2] = {16, 8};
  for (int gi = 0; gi < 2; ++gi) {
    const int G = Gs[gi];
    if (G == 16 && ms <= 128) continue;   // short columns: 8 lanes already hold them in <= 16 rows each
    const int threads = ((npairs * G + 63) / 64) * 64;
    if (threads > 768) continue;
    const int R = cx_round_r(G, (ms + G - 1) / G);
    if (!R) continue;
    const int ldw = G * R + 4;
    int nbuf = 2;
    if (jacobi_lds_bytes(npairs, ldw, 2) > (size_t)max_lds) nbuf = 1;
    if (jacobi_lds_bytes(npairs, ldw, nbuf) > (size_t)max_lds) continue;
    cfg->G = G;
    cfg->R = R;
    cfg->threads = threads;
    cfg->nbuf = nbuf;
    cfg->lds = jacobi_lds_bytes(npairs, ldw, nbuf);
    return 0;
  }
  return -1;
}

hipError_t launch_jacobi_cx(const JacobiArgs& a0, const JacobiConfig& c, hipStream_t s) {
  if (a0.nslices <= 0) return hipSuccess;
  if ((a0.mode != 0 && a0.mode != 1) || (a0.I1 & 1) || a0.I1 < a0.I2 || a0.tol < 0.0) return hipErrorInvalidValue;
  JacobiArgs a = a0;
  a.qeff = c.R / 4;
  if (c.G == 8) {
    switch (c.R) {
      case 8: return launch_cx_one<8, 8>(a, c, s);
      case 16: return launch_cx_one<8, 16>(a, c, s);
      case 32: return launch_cx_one<8, 32>(a, c, s);
      case 36: return launch_cx_one<8, 36>(a, c, s);
      case 40: return launch_cx_one<8, 40>(a, c, s);
      case 44: return launch_cx_one<8, 44>(a, c, s);
      case 48: return launch_cx_one<8, 48>(a, c, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (c.G == 16) {
    switch (c.R) {
      case 16: return launch_cx_one<16, 16>(a, c, s);
      case 24: return launch_cx_one<16, 24>(a, c, s);
      case 32: return launch_cx_one<16, 32>(a, c, s);
      case 40: return launch_cx_one<16, 40>(a, c, s);
      case 48: return launch_cx_one<16, 48>(a, c, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

template <int G, int R, int LB>
static hipError_t launch_warm_one(const WarmArgs& a, const JacobiConfig& c, hipStream_t s) {
  const int ldw = G * R + 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_warm<G, R, LB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi_warm<G, R, LB>), dim3(a.nslices), dim3(c.threads), c.lds, s, a, c.nbuf, ldw);
  return hipGetLastError();
}

template <int G>
static hipError_t launch_warm_g(const WarmArgs& a, const JacobiConfig& c, hipStream_t s) {
#define LT_WARM_CASE(RR)                                                                      \
  case RR:                                                                                    \
    return c.threads <= 768 ? launch_warm_one<G, RR, 768>(a, c, s) : launch_warm_one<G, RR, 1024>(a, c, s);
  switch (c.R) {
    LT_WARM_CASE(4)
    LT_WARM_CASE(8)
    LT_WARM_CASE(12)
    LT_WARM_CASE(16)
    LT_WARM_CASE(20)
    LT_WARM_CASE(24)
    LT_WARM_CASE(28)
    LT_WARM_CASE(32)
    LT_WARM_CASE(36)
    default: return hipErrorInvalidValue;
  }
#undef LT_WARM_CASE
}

// The warm kernel's columns hold 2 npad rows (M, then Z), at most 36 per lane.
int jacobi_warm_config(int n, int max_lds, JacobiConfig* cfg, int force_G) {
  if (n < 2 || n > RB_RMAX) return -1;
  const int npairs = (n + 1) / 2;
  const int rows = 2 * ((n + 3) / 4) * 4;
  const int Gs[3] = {16, 8, 4};
  int pick = 0, fallback = 0, forced = 0;
  for (int i = 0; i < 3; ++i) {
    const int G = Gs[i];
    const int threads = ((npairs * G + 63) / 64) * 64;
    int R = (rows + G - 1) / G;
    R = ((R + 3) / 4) * 4;
    if (threads > 1024 || R > 36) continue;
    if (jacobi_lds_bytes(npairs, G * R + 4, 1) > (size_t)max_lds) continue;
    if (R >= 8 && !pick) pick = G;
    fallback = G;
    if (G == force_G) forced = G;
  }
  // a requested lane count (autotuner) when it holds the factor, else the
  // fewest-lanes choice with at least 8 rows per lane
  const int G = forced ? forced : (pick ? pick : fallback);
  if (!G) return -1;
  int R = (rows + G - 1) / G;
  R = ((R + 3) / 4) * 4;
  cfg->G = G;
  cfg->R = R;
  cfg->threads = ((npairs * G + 63) / 64) * 64;
  cfg->nbuf = jacobi_lds_bytes(npairs, G * R + 4, 2) <= (size_t)max_lds ? 2 : 1;
  cfg->lds = jacobi_lds_bytes(npairs, G * R + 4, cfg->nbuf);
  return 0;
}

hipError_t launch_jacobi_warm(const WarmArgs& a, const JacobiConfig& c, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  switch (c.G) {
    case 4: return launch_warm_g<4>(a, c, s);
    case 8: return launch_warm_g<8>(a, c, s);
    case 16: return launch_warm_g<16>(a, c, s);
    default: return hipErrorInvalidValue;
  }
}

template <int G, int R, int LB>
static hipError_t launch_warm_items_one(ProbDev* const* probs, const CholItem* items, int nitems,
                                        const JacobiConfig& c, double tol, int max_sweeps, hipStream_t s) {
  const int ldw = G * R + 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_warm_items<G, R, LB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jacobi_warm_items<G, R, LB>), dim3(nitems), dim3(c.threads), c.lds, s, probs, items, tol,
                     max_sweeps, c.nbuf, ldw);
  return hipGetLastError();
}

template <int G>
static hipError_t launch_warm_items_g(ProbDev* const* probs, const CholItem* items, int nitems,
                                      const JacobiConfig& c, double tol, int max_sweeps, hipStream_t s) {
#define LT_WARM_ITEMS_CASE(RR)                                                                      \
  case RR:                                                                                          \
    return c.threads <= 768 ? launch_warm_items_one<G, RR, 768>(probs, items, nitems, c, tol, max_sweeps, s) \
                            : launch_warm_items_one<G, RR, 1024>(probs, items, nitems, c, tol, max_sweeps, s);
  switch (c.R) {
    LT_WARM_ITEMS_CASE(4)
    LT_WARM_ITEMS_CASE(8)
    LT_WARM_ITEMS_CASE(12)
    LT_WARM_ITEMS_CASE(16)
    LT_WARM_ITEMS_CASE(20)
    LT_WARM_ITEMS_CASE(24)
    LT_WARM_ITEMS_CASE(28)
    LT_WARM_ITEMS_CASE(32)
    LT_WARM_ITEMS_CASE(36)
    default: return hipErrorInvalidValue;
  }
#undef LT_WARM_ITEMS_CASE
}

hipError_t launch_jacobi_warm_items(ProbDev* const* probs, const CholItem* items, int nitems, const JacobiConfig& c,
                                    double tol, int max_sweeps, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  switch (c.G) {
    case 4: return launch_warm_items_g<4>(probs, items, nitems, c, tol, max_sweeps, s);
    case 8: return launch_warm_items_g<8>(probs, items, nitems, c, tol, max_sweeps, s);
    case 16: return launch_warm_items_g<16>(probs, items, nitems, c, tol, max_sweeps, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_warm_product_items(ProbDev* const* probs, const CholItem* items, int nitems, int nmax,
                                     hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const int nb = (nmax + 15) / 16;
  if (nmax < 1 || (nb * nb + 3) / 4 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_warm_product_items, dim3((unsigned)nitems, (unsigned)((nb * nb + 3) / 4)), dim3(256), 0, s,
                     probs, items);
  return hipGetLastError();
}

hipError_t launch_warm_product(const float* L, long long l_stride, const float* Z, float* M,
                               long long m_stride, int n, int nslices, hipStream_t s) {
  if (nslices <= 0) return hipSuccess;
  const int nb = (n + 15) / 16;
  const long long jobs = (long long)nslices * nb * nb;
  hipLaunchKernelGGL(k_warm_product_mfma, dim3((unsigned)((jobs + 3) / 4)), dim3(256), 0, s, L, l_stride, Z, M,
                     m_stride, n, nb, nslices);
  return hipGetLastError();
}

int jacobi_batch_config(const int* m, const int* n, int count, int max_lds, int force_G,
                        JacobiBatchConfig* cfg, int* nsub_out, int* qeff_out) {
  if (count <= 0) return -1;
  const int Gs[5] = {8, 16, 4, 32, 64};
  for (int gi = 0; gi < 5; ++gi) {
    const int G = Gs[gi];
    if (force_G && G != force_G) continue;
    int RMAX = 0, T = 0;
    bool ok = true;
    for (int i = 0; i < count && ok; ++i) {
      if (m[i] < n[i] || n[i] < 1 || n[i] > RB_RMAX) { ok = false; break; }
      const int npairs = (n[i] + 1) / 2;
      int R = (m[i] + G - 1) / G;
      R = ((R + 3) / 4) * 4;
      const int t = ((npairs * G + 63) / 64) * 64;
      if (R > 32 || t > 1024) ok = false;
      RMAX = R > RMAX ? R : RMAX;
      T = t > T ? t : T;
    }
    if (!ok) continue;
    const int ldw = G * RMAX + 4;
    int nbuf = 2;
    for (int i = 0; i < count; ++i)
      if (jacobi_lds_bytes((n[i] + 1) / 2, ldw, 2) > (size_t)max_lds) nbuf = 1;
    size_t lds = 0;
    for (int i = 0; i < count && ok; ++i) {
      const int npairs = (n[i] + 1) / 2;
      const size_t sb = slice_lds_bytes(npairs, ldw, nbuf);
      if (kWgCtlBytes + sb > (size_t)max_lds) { ok = false; break; }
      int nsub = T / (npairs * G);
      const int fit = (int)(((size_t)max_lds - kWgCtlBytes) / sb);
      if (nsub > fit) nsub = fit;
      if (nsub < 1) nsub = 1;
      int R = (m[i] + G - 1) / G;
      R = ((R + 3) / 4) * 4;
      nsub_out[i] = nsub;
      qeff_out[i] = R / 4;
      const size_t need = kWgCtlBytes + (size_t)nsub * sb;
      lds = need > lds ? need : lds;
    }
    if (!ok) continue;
    cfg->G = G;
    cfg->RMAX = RMAX;
    cfg->threads = T;
    cfg->nbuf = nbuf;
    cfg->lds = lds;
    return 0;
  }
  return -1;
}

hipError_t launch_jacobi_items(ProbDev* const* probs, const SvtItem* items, int nitems,
                               const JacobiBatchConfig& c, double tol, int max_sweeps,
                               hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  switch (c.G) {
    case 4: return launch_items_g<4>(probs, items, nitems, c, tol, max_sweeps, s);
    case 8: return launch_items_g<8>(probs, items, nitems, c, tol, max_sweeps, s);
    case 16: return launch_items_g<16>(probs, items, nitems, c, tol, max_sweeps, s);
    case 32: return launch_items_g<32>(probs, items, nitems, c, tol, max_sweeps, s);
    case 64: return launch_items_g<64>(probs, items, nitems, c, tol, max_sweeps, s);
    default: return hipErrorInvalidValue;
  }
}

bool jacobi_reg_shape(int m, int n) {
  if (m < 1 || n < 1 || m < n || n > RB_RMAX) return false;
  const int npairs = (n + 1) / 2;
  for (int G = 4; G <= 64; G *= 2) {
    const int threads = ((npairs * G + 63) / 64) * 64;
    int R = (m + G - 1) / G;
    R = ((R + 3) / 4) * 4;
    if (threads <= 1024 && R <= 32) return true;
  }
  return false;
}

const int kBlkVariants[kBlkNumVariants][2] = {{16, 16}, {32, 16}, {64, 16}, {64, 32}};

int jacobi_blk_pick_config(int m, int n, int max_lds, JacobiBlkConfig* cfg) {
  if (m < 2 || n < 2 || m < n || n > RB_RMAX_BLK) return -1;
  // (lanes per pair, rows per lane) in order of preference: the fewest lanes
  // that hold the column (widest blocks) at 16 rows per lane, then 32 rows
  for (int vi = 0; vi < kBlkNumVariants; ++vi) {
    const int G = kBlkVariants[vi][0], R = kBlkVariants[vi][1];
    const int qeff = (m + 4 * G - 1) / (4 * G);
    if (qeff > R / 4) continue;
    const int mpad = 4 * G * qeff, ldw = mpad + 4;
    int bmax = (1024 / G) & ~1;
    while (bmax >= 2 && blk_lds_bytes(bmax, ldw, 1) > (size_t)max_lds) bmax -= 2;
    if (bmax < 2) continue;
    int nblk = (n + bmax - 1) / bmax;
    nblk += nblk & 1;
    if (nblk < 2) nblk = 2;
    for (; nblk <= n + 1; nblk += 2) {
      int b = (n + nblk - 1) / nblk;
      b += b & 1;
      if (b < 2) b = 2;
      if (b > bmax || blk_lds_bytes(b, ldw, 1) > (size_t)max_lds) continue;
      const int nbuf = blk_lds_bytes(b, ldw, 2) <= (size_t)max_lds ? 2 : 1;
      cfg->G = G;
      cfg->R = R;
      cfg->variant = vi;
      cfg->b = b;
      cfg->nblk = nblk;
      cfg->qeff = qeff;
      cfg->threads = ((b * G + 63) / 64) * 64;
      cfg->nbuf = nbuf;
      cfg->lds = blk_lds_bytes(b, ldw, nbuf);
      cfg->work_floats = (long long)nblk * b * mpad;
      return 0;
    }
  }
  return -1;
}

hipError_t launch_jacobi_blk(const JacobiArgs& a0, const JacobiBlkConfig& c, hipStream_t s) {
  if (a0.nslices <= 0) return hipSuccess;
  if (a0.mode != 0 || !a0.work) return hipErrorInvalidValue;
  JacobiArgs a = a0;
  a.qeff = c.qeff;
  a.blk_b = c.b;
  a.blk_n = c.nblk;
  a.blk_nbuf = c.nbuf;
  a.work_stride = c.work_floats;
  switch (c.variant) {
    case 0: return launch_blk_one<16, 16>(a, c, s);
    case 1: return launch_blk_one<32, 16>(a, c, s);
    case 2: return launch_blk_one<64, 16>(a, c, s);
    case 3: return launch_blk_one<64, 32>(a, c, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_jacobi_blk_items(ProbDev* const* probs, const CholItem* items, int nitems, int variant,
                                   int threads, size_t lds, double tol, int max_sweeps, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  switch (variant) {
    case 0: return launch_blk_items_one<16, 16>(probs, items, nitems, threads, lds, tol, max_sweeps, s);
    case 1: return launch_blk_items_one<32, 16>(probs, items, nitems, threads, lds, tol, max_sweeps, s);
    case 2: return launch_blk_items_one<64, 16>(probs, items, nitems, threads, lds, tol, max_sweeps, s);
    case 3: return launch_blk_items_one<64, 32>(probs, items, nitems, threads, lds, tol, max_sweeps, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rebuild_tiles(ProbDev* const* probs, const RebuildTile* tiles, int ntiles, int wide,
                                int kmax, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int rcap = rebuild_rcap(kmax);
  if (kmax < 1 || rcap > (wide ? RB_RMAX_BLK : RB_RMAX)) return hipErrorInvalidValue;
  const size_t lds = rebuild_lds_bytes(rcap);
  if (wide) {
    hipError_t e = hipFuncSetAttribute((const void*)k_rebuild_tiles<RB_RMAX_BLK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rebuild_tiles<RB_RMAX_BLK>, dim3(ntiles), dim3(256), lds, s, probs, tiles, rcap);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_rebuild_tiles<RB_RMAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rebuild_tiles<RB_RMAX>, dim3(ntiles), dim3(256), lds, s, probs, tiles, rcap);
  }
  return hipGetLastError();
}

hipError_t launch_rebuild(const RebuildArgs& a, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  const int n = a.flip ? (a.I1 < a.I2 ? a.I2 : a.I1) : (a.I1 < a.I2 ? a.I1 : a.I2);
  // kept columns are at most min(I1, I2), or the caller's bound
  const int kmax = a.kmax ? a.kmax : (a.I1 < a.I2 ? a.I1 : a.I2);
  if (kmax > RB_RMAX_BLK) return hipErrorInvalidValue;
  dim3 grid((n + RB_TN - 1) / RB_TN, a.nslices);
  const int m = a.flip ? (a.I1 < a.I2 ? a.I1 : a.I2) : (a.I1 < a.I2 ? a.I2 : a.I1);
  if (m <= RBS_MMAX) {
    hipLaunchKernelGGL(k_rebuild_small<RBS_MMAX>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (m <= RBS_MMAX_CX) {   // e.g. the complex slices' interleaved rows
    hipLaunchKernelGGL(k_rebuild_small<RBS_MMAX_CX>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  RebuildArgs b = a;
  b.rcap = rebuild_rcap(kmax);
  const size_t lds = rebuild_lds_bytes(b.rcap);
  if (kmax > RB_RMAX) {
    hipError_t e = hipFuncSetAttribute((const void*)k_rebuild<RB_RMAX_BLK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rebuild<RB_RMAX_BLK>, grid, dim3(256), lds, s, b);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_rebuild<RB_RMAX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rebuild<RB_RMAX>, grid, dim3(256), lds, s, b);
  }
  return hipGetLastError();
}

// Wide blocked Jacobi variants (lanes per pair G, rows per lane R): the fewest
// lanes that hold the column at up to R rows per lane.
constexpr int kWideNumVariants = 5;
const int kWideVariants[kWideNumVariants][2] = {{16, 16}, {32, 16}, {64, 16}, {64, 24}, {64, 36}};

int jacobi_wide_pick_config(int m, int n, int max_lds, JacobiWideConfig* cfg) {
  if (m < 2 || n < 2 || m < n) return -1;
  for (int vi = 0; vi < kWideNumVariants; ++vi) {
    const int G = kWideVariants[vi][0], R = kWideVariants[vi][1];
    const int qeff = (m + 4 * G - 1) / (4 * G);
    if (qeff > R / 4) continue;
    const int mpad = 4 * G * qeff, ldw = mpad + 4;
    int b = ((R <= 16 ? 1024 : 512) / G) & ~1;   // wide_lanes<R>() lanes at most
    while (b >= 2 && blk_lds_bytes(b, ldw, 1) > (size_t)max_lds) b -= 2;
    if (b < 2) continue;
    int nblk = (n + b - 1) / b;
    nblk += nblk & 1;
    if (nblk < 2) nblk = 2;
    int bb = (n + nblk - 1) / nblk;   // balance the blocks
    bb += bb & 1;
    if (bb < 2) bb = 2;
    cfg->G = G;
    cfg->R = R;
    cfg->variant = vi;
    cfg->b = bb;
    cfg->nblk = nblk;
    cfg->qeff = qeff;
    cfg->threads = ((bb * G + 63) / 64) * 64;
    cfg->nbuf = blk_lds_bytes(bb, ldw, 2) <= (size_t)max_lds ? 2 : 1;
    cfg->lds = blk_lds_bytes(bb, ldw, cfg->nbuf);
    cfg->work_floats = (long long)nblk * bb * mpad;
    return 0;
  }
  return -1;
}

hipError_t launch_wide_copy_in(const WideArgs& a, const JacobiWideConfig& c, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  const int mpad = 4 * c.G * c.qeff, ncols = c.nblk * c.b;
  dim3 grid((unsigned)((ncols + 31) / 32), (unsigned)((mpad + 31) / 32), (unsigned)a.nslices);
  hipLaunchKernelGGL(k_wide_copy_in, grid, dim3(256), 0, s, a, mpad, ncols);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fill_zero(a.state, (size_t)a.nslices * kWideStateBytes, s);
}

hipError_t launch_wide_sweep(const WideArgs& a, const JacobiWideConfig& c, int* active, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  switch (c.variant) {
    case 0: return launch_wide_sweep_one<16, 16>(a, c, active, s);
    case 1: return launch_wide_sweep_one<32, 16>(a, c, active, s);
    case 2: return launch_wide_sweep_one<64, 16>(a, c, active, s);
    case 3: return launch_wide_sweep_one<64, 24>(a, c, active, s);
    case 4: return launch_wide_sweep_one<64, 36>(a, c, active, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wide_out(const WideArgs& a, const JacobiWideConfig& c, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  switch (c.variant) {
    case 0: return launch_wide_out_one<16, 16>(a, c, s);
    case 1: return launch_wide_out_one<32, 16>(a, c, s);
    case 2: return launch_wide_out_one<64, 16>(a, c, s);
    case 3: return launch_wide_out_one<64, 24>(a, c, s);
    case 4: return launch_wide_out_one<64, 36>(a, c, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lsvd_finalize_cx(const LsvdCxArgs& a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  const int m = a.I1 > a.I2 ? a.I1 : a.I2, n = a.I1 > a.I2 ? a.I2 : a.I1;
  if (n > LS_NMAX || 2 * m > LS_MMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lsvd_finalize_cx, dim3(a.npairs), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lsvd_finalize(const LsvdArgs& a, hipStream_t s) {
  if (a.nslices <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lsvd_finalize, dim3(a.nslices), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace lt
