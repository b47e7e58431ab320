// Host runtime of liblt.so: the C-ABI declared in include/lt.h.
//
// Every operation is a short sequence of kernel launches on the handle's
// stream; the only host work is argument checking, workspace carving, building
// the data-independent PGA schedule (Alg. 5: t_k and mu_k), and, for custom
// mode matrices, their FP64 inversion before upload.
#include "lt_internal.h"
#include "../../include/lt.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstddef>
#include <mutex>
#include <new>
#include <string>
#include <vector>

constexpr size_t kPinnedDoubles = 128;   // host staging: scalars and one problem record

// Workspace of lt_svt_prox_noalloc: a file-scope device array, one copy per
// GPU, kept until the process ends.  Host code never passes `scratch` itself to
// a kernel (on the host it only names the symbol): lt_create resolves each
// device's copy to its device address with hipGetSymbolAddress, with that
// device current, and the entry point uses that address.
constexpr size_t kNoallocScratchBytes = LT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch copy (dev: the current device).
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct lt_handle {
  hipStream_t stream = nullptr;
  int device = 0;
  void* scratch = nullptr;             // this device's copy of `scratch` (device address)
  hipError_t scratch_rc = hipSuccess;  // why it is null, if it is
  int max_lds = 65536;
  std::string err;
  double* pinned = nullptr;   // small host staging for readbacks (kPinnedDoubles)
  // kernel timing (lt_profile_begin / lt_profile_end)
  bool prof_on = false;
  std::vector<hipEvent_t> events;          // pool, used in start/stop pairs
  size_t ev_next = 0;
  std::vector<std::pair<int, size_t>> recs;  // (class, index of the start event)
  int64_t dropped = 0;
};

namespace {

constexpr int kMaxP = 4096;
constexpr size_t kEventPool = 8192;

// Records a HIP event pair around the launches made during its lifetime.
struct ProfScope {
  lt_handle* h;
  int cls;
  long long idx = -1;
  ProfScope(lt_handle* hh, int c) : h(hh), cls(c) {
    if (!h || !h->prof_on) return;
    if (h->ev_next + 2 > h->events.size()) {
      ++h->dropped;
      return;
    }
    idx = (long long)h->ev_next;
    h->ev_next += 2;
    (void)hipEventRecord(h->events[idx], h->stream);
  }
  ~ProfScope() {
    if (idx < 0) return;
    (void)hipEventRecord(h->events[idx + 1], h->stream);
    h->recs.emplace_back(cls, (size_t)idx);
  }
};

int fail(lt_handle* h, int code, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return code;
}

#define HIP_TRY(h, expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((h), LT_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

struct Shape {
  int order = 0;
  long long I1 = 0, I2 = 0, P = 1, N = 0, nel = 0;
  int nmodes = 0;
  int n[LT_MAX_ORDER] = {0};
  int kind[LT_MAX_ORDER] = {0};
  const double* custom[LT_MAX_ORDER] = {nullptr};
  bool any_custom = false;
  bool any_dft = false;   // Fourier modes: complex transform-domain slices
};

int parse(lt_handle* h, const lt_desc* d, Shape* s) {
  if (!d) return fail(h, LT_ERR_ARG, "descriptor is NULL");
  if (d->order < 2 || d->order > LT_MAX_ORDER)
    return fail(h, LT_ERR_SHAPE, "order %d outside 2..%d", d->order, LT_MAX_ORDER);
  s->order = d->order;
  for (int i = 0; i < d->order; ++i)
    if (d->dims[i] < 1 || d->dims[i] > (1LL << 30))
      return fail(h, LT_ERR_SHAPE, "dims[%d] = %lld out of range", i, (long long)d->dims[i]);
  s->I1 = d->dims[0];
  s->I2 = d->dims[1];
  s->P = 1;
  s->nmodes = d->order - 2;
  for (int i = 2; i < d->order; ++i) {
    const int k = d->kind[i];
    if (k != LT_DCT && k != LT_DFT && k != LT_IDENTITY && k != LT_CUSTOM)
      return fail(h, LT_ERR_ARG, "mode %d: unknown kind %d", i + 1, k);
    if (k == LT_CUSTOM && !d->custom[i])
      return fail(h, LT_ERR_ARG, "mode %d: LT_CUSTOM without a matrix", i + 1);
    s->n[i - 2] = (int)d->dims[i];
    s->kind[i - 2] = k;
    s->custom[i - 2] = d->custom[i];
    s->any_custom |= (k == LT_CUSTOM);
    s->any_dft |= (k == LT_DFT);
    s->P *= d->dims[i];
    if (s->P > kMaxP) return fail(h, LT_ERR_SHAPE, "more than %d frontal slices", kMaxP);
  }
  s->N = s->I1 * s->I2;
  s->nel = s->N * s->P;
  return LT_OK;
}

// ---- workspace carving -------------------------------------------------------
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct TransformWs {
  float* K = nullptr;
  float* Kinv = nullptr;
  uint16_t *Khi = nullptr, *Klo = nullptr, *Kihi = nullptr, *Kilo = nullptr;
  double* custom = nullptr;   // per custom mode: M then M^{-1}
};

void carve_transform(Carver& c, const Shape& s, int precision, TransformWs* t) {
  const size_t P2 = (size_t)s.P * s.P;
  // Fourier modes: the stacked real forms, 2P x P and P x 2P (FP32 only)
  t->K = c.take<float>(s.any_dft ? 2 * P2 : P2);
  t->Kinv = c.take<float>(s.any_dft ? 2 * P2 : P2);
  if (precision == LT_PREC_BF16X3 && !s.any_dft) {
    t->Khi = c.take<uint16_t>(P2);
    t->Klo = c.take<uint16_t>(P2);
    t->Kihi = c.take<uint16_t>(P2);
    t->Kilo = c.take<uint16_t>(P2);
  }
  size_t nc = 0;
  for (int i = 0; i < s.nmodes; ++i)
    if (s.kind[i] == LT_CUSTOM) nc += 2 * (size_t)s.n[i] * s.n[i];
  if (nc) t->custom = c.take<double>(nc);
}

// Gauss-Jordan inverse with partial pivoting, FP64, row-major n x n.
bool invert(const double* M, int n, std::vector<double>& inv) {
  std::vector<double> a(M, M + (size_t)n * n);
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(a[(size_t)r * n + col]) > fabs(a[(size_t)piv * n + col])) piv = r;
    if (a[(size_t)piv * n + col] == 0.0) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)piv * n + k], a[(size_t)col * n + k]);
        std::swap(inv[(size_t)piv * n + k], inv[(size_t)col * n + k]);
      }
    const double d = a[(size_t)col * n + col];
    for (int k = 0; k < n; ++k) {
      a[(size_t)col * n + k] /= d;
      inv[(size_t)col * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = a[(size_t)r * n + col];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)col * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
      }
    }
  }
  return true;
}

int build_transform(lt_handle* h, const Shape& s, int precision, const TransformWs& t) {
  lt::KronDesc fwd{}, inv{};
  fwd.nmodes = inv.nmodes = s.nmodes;
  double* dst = t.custom;
  for (int i = 0; i < s.nmodes; ++i) {
    fwd.n[i] = inv.n[i] = s.n[i];
    fwd.kind[i] = inv.kind[i] = s.kind[i];
    if (s.kind[i] == LT_CUSTOM) {
      const int n = s.n[i];
      std::vector<double> Mi;
      if (!invert(s.custom[i], n, Mi))
        return fail(h, LT_ERR_ARG, "mode %d: custom matrix is singular", i + 3);
      const size_t bytes = (size_t)n * n * sizeof(double);
      HIP_TRY(h, hipMemcpyAsync(dst, s.custom[i], bytes, hipMemcpyHostToDevice, h->stream));
      HIP_TRY(h, hipMemcpyAsync(dst + (size_t)n * n, Mi.data(), bytes, hipMemcpyHostToDevice,
                                h->stream));
      // the pageable source must stay valid until the copy has been consumed
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      fwd.custom[i] = dst;
      inv.custom[i] = dst + (size_t)n * n;
      dst += 2 * (size_t)n * n;
    }
  }
  ProfScope ps(h, LT_PROF_OTHER);
  if (s.any_dft) {
    HIP_TRY(h, lt::launch_build_kron_dft(fwd, (int)s.P, 0, t.K, h->stream));
    HIP_TRY(h, lt::launch_build_kron_dft(inv, (int)s.P, 1, t.Kinv, h->stream));
    return LT_OK;
  }
  HIP_TRY(h, lt::launch_build_kron(fwd, (int)s.P, 0, t.K, t.Khi, t.Klo, h->stream));
  HIP_TRY(h, lt::launch_build_kron(inv, (int)s.P, 1, t.Kinv, t.Kihi, t.Kilo, h->stream));
  (void)precision;
  return LT_OK;
}

lt::GemmArgs gemm_plain(const TransformWs& t, bool inverse, int P, long long N, const float* in,
                        float* out, bool dft = false) {
  lt::GemmArgs g{};
  g.K = inverse ? t.Kinv : t.K;
  g.Khi = inverse ? t.Kihi : t.Khi;
  g.Klo = inverse ? t.Kilo : t.Klo;
  g.P = P;
  g.N = N;
  g.B = in;
  g.out = out;
  if (dft) {   // real and imaginary planes: 2P rows out of the forward, into the inverse
    if (inverse) g.Kd = 2 * P;
    else g.Mo = 2 * P;
  }
  return g;
}

int gemm(lt_handle* h, const lt::GemmArgs& g, int prec, int pro, int epi, int cls,
         int* n_partials = nullptr) {
  ProfScope ps(h, cls);
  HIP_TRY(h, lt::launch_transform_gemm(g, prec, pro, epi, h->stream, n_partials));
  return LT_OK;
}

// Default Jacobi tolerance: 1e-7.  With 1e-6 the 256 x 256 noisy completion
// (300 iterations) ended 1.7e-4 from the FP64 oracle: its clustered noise
// singular values let the early stop (all rotations of a sweep small) fire with
// columns still 2.5e-4 from orthogonal; 1e-7 gives 3.0e-5 there for 1% more
// sweeps (1.5e-6 on the video workload, 5% slower).
constexpr double kJacobiTolDefault = 1e-7;

void resolve_opts(const lt_svd_opts* o, double* tol, int* max_sweeps, int* prec) {
  *tol = (o && o->jacobi_tol > 0) ? o->jacobi_tol : kJacobiTolDefault;
  // the kernels take FP32 pair dot products when handed the tolerance negated
  if (o && o->fp32_dots) *tol = -*tol;
  *max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : 40;
  *prec = o ? o->precision : LT_PREC_F32;
}

int check_prec(lt_handle* h, int prec) {
  if (prec != LT_PREC_F32 && prec != LT_PREC_BF16X3)
    return fail(h, LT_ERR_ARG, "unknown precision %d", prec);
  return LT_OK;
}

int jacobi_config(lt_handle* h, const Shape& s, lt::JacobiConfig* cfg) {
  const int m = (int)(s.I1 > s.I2 ? s.I1 : s.I2);
  const int n = (int)(s.I1 > s.I2 ? s.I2 : s.I1);
  const char* env = getenv("LT_JACOBI_G");
  const int forceG = env ? atoi(env) : 0;
  if (lt::jacobi_pick_config(m, n, h->max_lds, cfg, forceG) != 0)
    return fail(h, LT_ERR_SHAPE,
                "slice %lld x %lld exceeds the register-resident Jacobi kernel "
                "(needs ceil(n/2)*G <= 1024 and ceil(m/G) <= 32)",
                (long long)s.I1, (long long)s.I2);
  return LT_OK;
}

// The SVT buffers of slices of one shape (the Jacobi's kept columns, counters,
// Gram / Cholesky blocks, blocked-kernel working buffers).
struct SvtCore {
  float* Bk = nullptr;
  int32_t* rank = nullptr;
  int32_t* sweeps = nullptr;
  double* C = nullptr;   // preconditioning: per-slice Gram matrix, then its Cholesky factor
  float* work = nullptr;  // blocked Jacobi: per-slice working buffers
  double* nuc = nullptr;  // per slice: sum of (sigma_i - tau) over the kept singular values
  // wide path: FP32 factors (precond), rebuild scratch, per-slice state, counter
  float* L32 = nullptr;
  float* T = nullptr;
  void* wstate = nullptr;
  int* active = nullptr;
  double* thr = nullptr;
};

// Fourier modes: the transform-domain slices are complex, in two planes (real
// then imaginary, P x N each).  For real data slice q = conj(p) of its partner
// (negated frequency indices along the Fourier modes), so one slice per pair is
// thresholded, through the real embedding [[X, -Y], [Y, X]] (2 I1 x 2 I2): its
// singular values are those of X + iY, each twice, and its SVT is the
// embedding of the complex SVT (of which the left block column is [Re; Im]).
struct DftWs {
  float* E = nullptr;         // embeddings of the representatives, npairs x 4N
  int32_t* rep = nullptr;     // representative slice of each pair (p <= its partner)
  int32_t* partner = nullptr;
  int npairs = 0;
  SvtCore inner;              // SVT buffers of the embeddings
  float* Lc = nullptr;        // complex path: Cholesky factors (2n interleaved rows x n), npairs of them
  double* thr = nullptr;      // complex path: the multi-launch Cholesky's per-slice pivot floor
};

struct SvtWs {
  TransformWs t;
  float* Gh = nullptr;
  float* Bk = nullptr;
  int32_t* rank = nullptr;
  int32_t* sweeps = nullptr;
  double* C = nullptr;   // preconditioning: per-slice Gram matrix, then its Cholesky factor
  float* work = nullptr;  // blocked Jacobi: per-slice working buffers
  double* nuc = nullptr;  // per slice: sum of (sigma_i - tau) over the kept singular values
  float* L32 = nullptr;   // wide path (see SvtCore)
  float* T = nullptr;
  void* wstate = nullptr;
  int* active = nullptr;
  double* thr = nullptr;
  DftWs dft;              // Fourier modes only
};

// Representatives and partners of the conjugate pairs of slices (slice index:
// first trailing mode fastest; partner: Fourier indices negated modulo I_i).
void dft_pairs(const Shape& s, std::vector<int>* rep, std::vector<int>* partner) {
  rep->clear();
  partner->clear();
  for (long long p = 0; p < s.P; ++p) {
    long long rem = p, q = 0, stride = 1;
    for (int m = 0; m < s.nmodes; ++m) {
      const long long d = s.n[m], k = rem % d;
      rem /= d;
      q += (s.kind[m] == LT_DFT ? (d - k) % d : k) * stride;
      stride *= d;
    }
    if (p <= q) {
      rep->push_back((int)p);
      partner->push_back((int)q);
    }
  }
}

Shape embed_shape(const Shape& s, int npairs) {
  Shape e;
  e.order = 3;
  e.I1 = 2 * s.I1;
  e.I2 = 2 * s.I2;
  e.P = npairs;
  e.N = e.I1 * e.I2;
  e.nel = e.N * e.P;
  e.nmodes = 1;
  e.n[0] = npairs;
  e.kind[0] = LT_IDENTITY;
  return e;
}

// The one-workgroup preconditioned SVT paths take slices with
// 2 <= n <= LT_PRECOND_MAX_N (the Cholesky of the n x n Gram matrix runs in LDS
// up to n = 200, in global memory beyond); the wide path preconditions wider
// slices with its own multi-launch Cholesky (svt_plan).
static_assert(LT_PRECOND_MAX_N == 512, "the Cholesky kernels take n <= 512");

bool precond_shape(const Shape& s) {
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  return n >= 2 && n <= LT_PRECOND_MAX_N;
}

long long precond_n(const Shape& s) { return s.I1 < s.I2 ? s.I1 : s.I2; }

// Slices the register-resident Jacobi kernel cannot hold (more than 256
// columns, or columns too long for the lanes a pair can have) run the blocked
// kernel.  Its layout is fixed by the shape and a 160 KiB LDS budget (MI355X),
// so workspace sizes do not depend on the device; the launch checks the
// device's LDS.
constexpr int kBlkLdsBudget = 160 * 1024;
constexpr int kCholLdsMaxN = 200;   // the LDS Cholesky kernel's limit

// How the SVT of a slice shape runs: the Jacobi on the slice itself or on its
// n x n Cholesky factor (precond), by the register-resident or the blocked
// kernel; jm x jn is the Jacobi's working matrix.
struct SvtPlan {
  bool precond = false;
  bool blocked = false;
  bool wide = false;      // the wide blocked Jacobi (one workgroup per block pair)
  int jm = 0, jn = 0;
  lt::JacobiBlkConfig bcfg{};
  lt::JacobiWideConfig wcfg{};
};

// Slices beyond the single-workgroup blocked kernel (more than 512 columns or,
// unpreconditioned, 2048 rows) take the wide blocked Jacobi: on the n x n
// Cholesky factor up to n = kWideMaxN when preconditioning is requested, else on
// the slice itself up to kWideMaxN rows.
constexpr int kWideMaxN = 2304;

// Preconditioning applies when requested for 2 <= n <= 200 (Cholesky in LDS),
// and for n <= 512 when the register kernel cannot hold the slice itself: on
// square slices of 256 columns the sweeps it saves (about one in eight on the
// completion iterates measured) do not pay for the global-memory Cholesky,
// while a slice that needs the blocked kernel gains both fewer sweeps and, when
// tall, a shorter working matrix.  False if no kernel takes the shape.
// batch: the batch engine's choice (its ticks are captured as graphs: the
// one-workgroup blocked kernel up to 512 columns, never the wide kernel, which
// synchronises the host once per sweep); otherwise (lt_svt_prox,
// lt_complete_pga, ...) every shape beyond the register-resident kernel takes
// the wide kernel, which spreads a slice over nblk / 2 workgroups (measured:
// the 512 x 512 x 3 x 64 request 10.0 -> 12.4 iterations/s, the Fourier video's
// 288 x 288 factors 28 -> 63); LT_WIDE=0 in the environment restores the
// one-workgroup kernel there.
bool svt_plan(const Shape& s, bool precond_req, SvtPlan* p, bool batch = false) {
  const long long m64 = s.I1 > s.I2 ? s.I1 : s.I2;
  const long long n64 = s.I1 > s.I2 ? s.I2 : s.I1;
  if (n64 > kWideMaxN || m64 > (1LL << 20)) return false;
  const int m = (int)m64, n = (int)n64;
  p->precond = precond_req && precond_shape(s) && (n <= kCholLdsMaxN || !lt::jacobi_reg_shape(m, n));
  p->jm = p->precond ? n : m;
  p->jn = n;
  p->blocked = false;
  p->wide = false;
  if (lt::jacobi_reg_shape(p->jm, p->jn)) return true;
  const char* env = getenv("LT_WIDE");
  const bool prefer_wide = !batch && !(env && atoi(env) == 0);
  if (!prefer_wide && lt::jacobi_blk_pick_config(p->jm, p->jn, kBlkLdsBudget, &p->bcfg) == 0) {
    p->blocked = true;
    return true;
  }
  p->precond = precond_req && n >= 2;
  p->jm = p->precond ? n : m;
  if (p->jm > kWideMaxN || lt::jacobi_wide_pick_config(p->jm, p->jn, kBlkLdsBudget, &p->wcfg) != 0) return false;
  p->blocked = true;
  p->wide = true;
  return true;
}

// Working-buffer floats per slice the blocked kernel may need for this shape
// (with or without preconditioning).
long long blocked_work_floats(const Shape& s) {
  long long wf = 0;
  for (int pc = 0; pc < 2; ++pc) {
    SvtPlan p;
    if (!svt_plan(s, pc != 0, &p) || !p.blocked) continue;
    const long long f = p.wide ? p.wcfg.work_floats : p.bcfg.work_floats;
    if (f > wf) wf = f;
  }
  return wf;
}

int check_blk_lds(lt_handle* h, const Shape& s, const lt::JacobiBlkConfig& c) {
  if (c.lds > (size_t)h->max_lds)
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld: the blocked Jacobi kernel needs %zu bytes of LDS",
                s.I1, s.I2, c.lds);
  return LT_OK;
}

void carve_svt_core(Carver& c, const Shape& s, SvtCore* w) {
  w->Bk = c.take<float>((size_t)s.nel);
  w->rank = c.take<int32_t>((size_t)s.P);
  w->sweeps = c.take<int32_t>((size_t)s.P);
  w->nuc = c.take<double>((size_t)s.P);
  SvtPlan pp;
  if (svt_plan(s, true, &pp) && pp.precond) w->C = c.take<double>((size_t)(s.P * precond_n(s) * precond_n(s)));
  const long long wf = blocked_work_floats(s);
  if (wf) w->work = c.take<float>((size_t)s.P * (size_t)wf);
  SvtPlan pw;
  const bool wide = (svt_plan(s, true, &pp) && pp.wide) || (svt_plan(s, false, &pw) && pw.wide);
  if (wide) {
    if (pp.wide && pp.precond) {
      w->L32 = c.take<float>((size_t)(s.P * precond_n(s) * precond_n(s)));
      w->thr = c.take<double>((size_t)s.P);
    }
    w->T = c.take<float>((size_t)s.nel);
    w->wstate = c.take<char>((size_t)s.P * lt::kWideStateBytes);
    w->active = c.take<int>(1);
  }
}

void carve_svt(Carver& c, const Shape& s, int prec, SvtWs* w) {
  carve_transform(c, s, prec, &w->t);
  if (!s.any_dft) {
    w->Gh = c.take<float>((size_t)s.nel);
    SvtCore core;
    carve_svt_core(c, s, &core);
    w->Bk = core.Bk;
    w->rank = core.rank;
    w->sweeps = core.sweeps;
    w->C = core.C;
    w->work = core.work;
    w->nuc = core.nuc;
    w->L32 = core.L32;
    w->T = core.T;
    w->wstate = core.wstate;
    w->active = core.active;
    w->thr = core.thr;
    return;
  }
  w->Gh = c.take<float>(2 * (size_t)s.nel);   // real plane, then imaginary plane
  w->rank = c.take<int32_t>((size_t)s.P);
  w->sweeps = c.take<int32_t>((size_t)s.P);
  w->nuc = c.take<double>((size_t)s.P);
  std::vector<int> rep, partner;
  dft_pairs(s, &rep, &partner);
  DftWs& d = w->dft;
  d.npairs = (int)rep.size();
  d.rep = c.take<int32_t>(rep.size());
  d.partner = c.take<int32_t>(rep.size());
  const Shape se = embed_shape(s, d.npairs);
  d.E = c.take<float>((size_t)se.nel);
  carve_svt_core(c, se, &d.inner);
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  d.Lc = c.take<float>((size_t)(d.npairs * 2 * n * n));
  d.thr = c.take<double>((size_t)d.npairs);
}

// Upload the pair tables of a Fourier workspace (once per call).
int dft_prepare(lt_handle* h, const Shape& s, const SvtWs& w) {
  if (!s.any_dft) return LT_OK;
  std::vector<int> rep, partner;
  dft_pairs(s, &rep, &partner);
  HIP_TRY(h, hipMemcpyAsync(w.dft.rep, rep.data(), rep.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(w.dft.partner, partner.data(), partner.size() * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));   // the host vectors go out of scope
  return LT_OK;
}

// Warm start of the completion's SVT (real transforms, preconditioned slices
// on the register-resident kernel): per slice the rotations Z (n x n)
// accumulated since the last cold start.
constexpr int kWarmRestartDefault = 256;

bool warm_shape(const Shape& s) {
  if (s.any_dft) return false;
  SvtPlan pl;
  if (!svt_plan(s, true, &pl) || !pl.precond || pl.blocked) return false;
  const int n = (int)precond_n(s);
  lt::JacobiConfig cfg;
  return lt::jacobi_warm_config(n, kBlkLdsBudget, &cfg) == 0;
}

struct WarmState {
  float* Z = nullptr;       // P x n x n
  bool cold = true;
};

struct PgaWs {
  SvtWs svt;
  float* Z = nullptr;       // warm start (warm_shape only)
  float* Xb = nullptr;
  double* partials = nullptr;
  double* norms = nullptr;
  double* nucsum = nullptr;
  unsigned long long* sweep_total = nullptr;
  unsigned long long* slowest_total = nullptr;   // per-iteration largest slice sweep count, summed
  unsigned long long* rot_total = nullptr;
  unsigned int* maxsweep_hits = nullptr;
  unsigned int* nonfinite = nullptr;
};

long long n_partials(const Shape& s) {
  return ((s.N + 63) / 64) * ((s.P + 63) / 64);
}

void carve_pga(Carver& c, const Shape& s, int prec, PgaWs* w) {
  carve_svt(c, s, prec, &w->svt);
  if (warm_shape(s)) w->Z = c.take<float>((size_t)(s.P * precond_n(s) * precond_n(s)));
  w->Xb = c.take<float>((size_t)s.nel);
  w->partials = c.take<double>(2 * (size_t)n_partials(s));
  w->norms = c.take<double>(2);
  w->nucsum = c.take<double>(1);
  w->sweep_total = c.take<unsigned long long>(1);
  w->slowest_total = c.take<unsigned long long>(1);
  w->rot_total = c.take<unsigned long long>(1);
  w->maxsweep_hits = c.take<unsigned int>(1);
  w->nonfinite = c.take<unsigned int>(1);
}

struct LprodWs {
  TransformWs t;
  float *Ah = nullptr, *Bh = nullptr, *Ch = nullptr;
};

struct LsvdWs {
  TransformWs t;
  float* Ah = nullptr;
  float* cols = nullptr;
  double* sigma = nullptr;
  float *Uh = nullptr, *Sh = nullptr, *Vh = nullptr;
  int32_t* sweeps = nullptr;
  // full factors (Alg. 3 shapes): U I1 x I1, S I1 x I2, V I2 x I2 per slice, and
  // the Householder reflectors (FP64, m x n per slice) completing the longer side
  float *Uf = nullptr, *Sf = nullptr, *Vf = nullptr;
  double* H = nullptr;
  double* beta = nullptr;
  double* mr = nullptr;   // multirank: mean and maximum
};

void carve_lsvd(Carver& c, const Shape& s, int prec, LsvdWs* w, bool full = false) {
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  const long long m = s.I1 < s.I2 ? s.I2 : s.I1;
  carve_transform(c, s, prec, &w->t);
  w->Ah = c.take<float>((size_t)s.nel);
  w->cols = c.take<float>((size_t)s.nel);
  w->sigma = c.take<double>((size_t)(s.P * n));
  w->Uh = c.take<float>((size_t)(s.P * s.I1 * n));
  w->Sh = c.take<float>((size_t)(s.P * n * n));
  w->Vh = c.take<float>((size_t)(s.P * s.I2 * n));
  w->sweeps = c.take<int32_t>((size_t)s.P);
  w->mr = c.take<double>(2);
  if (full) {
    w->Uf = c.take<float>((size_t)(s.P * s.I1 * s.I1));
    w->Sf = c.take<float>((size_t)(s.P * s.I1 * s.I2));
    w->Vf = c.take<float>((size_t)(s.P * s.I2 * s.I2));
    if (m > n) {
      w->H = c.take<double>((size_t)(s.P * m * n));
      w->beta = c.take<double>((size_t)(s.P * n));
    }
  }
}

// lt_lsvd under Fourier modes (economy factors): the transform's two planes,
// the representatives' complex working matrices and the complex Jacobi's
// columns (2 N floats each), their norms, the finalisation's scratch, and the
// transform-domain factors in two planes each.
struct LsvdDftWs {
  TransformWs t;
  float* Ah = nullptr;
  float* E = nullptr;
  float* cols = nullptr;
  double* sigma = nullptr;
  int32_t* sweeps = nullptr;
  int32_t* rep = nullptr;
  int32_t* partner = nullptr;
  float* scratch = nullptr;
  float *Uh = nullptr, *Sh = nullptr, *Vh = nullptr;
  double* sigP = nullptr;   // multirank: the norms of every slice (P x n)
  double* mr = nullptr;     // multirank: mean and maximum
  float* Bk = nullptr;      // truncation: the first k columns with their i-twins (4 N floats per representative)
  int32_t* kept = nullptr;  // truncation: 2 k per representative
  int npairs = 0;
};

void carve_lsvd_dft(Carver& c, const Shape& s, int prec, LsvdDftWs* w, bool truncate = false) {
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  const long long m = s.I1 < s.I2 ? s.I2 : s.I1;
  std::vector<int> rep, partner;
  dft_pairs(s, &rep, &partner);
  w->npairs = (int)rep.size();
  const size_t np = rep.size();
  carve_transform(c, s, prec, &w->t);
  w->Ah = c.take<float>(2 * (size_t)s.nel);
  w->E = c.take<float>(np * 2 * (size_t)s.N);
  w->cols = c.take<float>(np * 2 * (size_t)s.N);
  w->sigma = c.take<double>(np * (size_t)n);
  w->sweeps = c.take<int32_t>(np);
  w->rep = c.take<int32_t>(np);
  w->partner = c.take<int32_t>(np);
  w->scratch = c.take<float>(np * (size_t)(2 * m * n + 2 * n * n));
  w->Uh = c.take<float>(2 * (size_t)(s.P * s.I1 * n));
  w->Sh = c.take<float>(2 * (size_t)(s.P * n * n));
  w->Vh = c.take<float>(2 * (size_t)(s.P * s.I2 * n));
  w->sigP = c.take<double>((size_t)(s.P * n));
  w->mr = c.take<double>(2);
  if (truncate) {
    w->Bk = c.take<float>(np * 4 * (size_t)s.N);
    w->kept = c.take<int32_t>(np);
  }
}

int check_ws(lt_handle* h, void* ws, size_t have, size_t need) {
  if (!ws) return fail(h, LT_ERR_WORKSPACE, "workspace is NULL");
  if (have < need)
    return fail(h, LT_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", have, need);
  return LT_OK;
}

// D = the SVT of the slices from the Jacobi's kept columns: D_W = Bk (Bk^T W),
// or (W B) B^T on the preconditioned path.
int rebuild_svt(lt_handle* h, const Shape& s, const float* Gh, float* Dh, const SvtCore& w, int32_t* rank,
                bool precond) {
  lt::RebuildArgs r{};
  r.W = Gh;
  r.D = Dh;
  r.bk = w.Bk;
  r.rank = rank;
  r.slice_stride = s.N;
  r.I1 = (int)s.I1;
  r.I2 = (int)s.I2;
  r.nslices = (int)s.P;
  r.flip = precond ? 1 : 0;
  ProfScope ps(h, LT_PROF_REBUILD);
  HIP_TRY(h, lt::launch_rebuild(r, h->stream));
  return LT_OK;
}

// The wide blocked Jacobi SVT (many columns, few slices): Gram matrix and
// Cholesky (multi-launch) when preconditioned, then the block rounds launched
// sweep by sweep until every slice has converged (one host synchronisation per
// sweep reads the number still running), then the kept columns and the rebuild
// as two batched GEMMs (any kept count).
int run_wide_svt(lt_handle* h, const Shape& s, const float* Gh, float* Dh, const SvtCore& w, const SvtPlan& pl,
                 double tau, double tol, int max_sweeps, int32_t* rank, int32_t* sweeps,
                 unsigned long long* sweep_total, unsigned long long* rot_total, unsigned int* hits) {
  if (!w.work || !w.T || !w.wstate || !w.active || (pl.precond && (!w.L32 || !w.C || !w.thr)))
    return fail(h, LT_ERR_WORKSPACE, "no wide-Jacobi buffers in the workspace");
  const lt::JacobiWideConfig& c = pl.wcfg;
  if (c.lds > (size_t)h->max_lds)
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld: the wide Jacobi needs %zu bytes of LDS", s.I1, s.I2, c.lds);
  lt::WideArgs a{};
  const int n = (int)precond_n(s);
  if (pl.precond) {
    const long long cst = (long long)n * n;
    ProfScope ps(h, LT_PROF_PRECOND);
    lt::GramArgs g{Gh, s.N, w.C, cst, (int)s.I1, (int)s.I2, (int)s.P};
    HIP_TRY(h, lt::launch_gram(g, h->stream));
    HIP_TRY(h, lt::launch_chol_big(w.C, cst, n, (int)s.P, w.L32, cst, w.thr, h->stream));
    a.src = w.L32;
    a.slice_stride = cst;
    a.I1 = n;
    a.I2 = n;
  } else {
    a.src = Gh;
    a.slice_stride = s.N;
    a.I1 = (int)s.I1;
    a.I2 = (int)s.I2;
  }
  a.nslices = (int)s.P;
  a.work = w.work;
  a.work_stride = c.work_floats;
  a.state = w.wstate;
  a.tau = tau;
  a.tol = tol;
  a.max_sweeps = max_sweeps;
  a.bk = w.Bk;
  a.bk_stride = s.N;
  a.rank = rank;
  a.sweeps = sweeps;
  a.nuc = w.nuc;
  a.sweep_total = sweep_total;
  a.rot_total = rot_total;
  a.hits = hits;
  {
    ProfScope ps(h, LT_PROF_JACOBI);
    HIP_TRY(h, lt::launch_wide_copy_in(a, c, h->stream));
    for (int sw = 0; sw < max_sweeps; ++sw) {
      HIP_TRY(h, lt::launch_wide_sweep(a, c, w.active, h->stream));
      HIP_TRY(h, hipMemcpyAsync(h->pinned, w.active, sizeof(int), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      if (*reinterpret_cast<int*>(h->pinned) == 0) break;
    }
    HIP_TRY(h, lt::launch_wide_out(a, c, h->stream));
  }
  lt::RebuildArgs r{};
  r.W = Gh;
  r.D = Dh;
  r.bk = w.Bk;
  r.rank = rank;
  r.slice_stride = s.N;
  r.I1 = (int)s.I1;
  r.I2 = (int)s.I2;
  r.nslices = (int)s.P;
  r.flip = pl.precond ? 1 : 0;
  ProfScope ps(h, LT_PROF_REBUILD);
  HIP_TRY(h, lt::launch_rebuild_gemm(r, w.T, h->stream));
  return LT_OK;
}

int run_jacobi_svt(lt_handle* h, const Shape& s, const float* Gh, float* Dh, const SvtCore& w,
                   double tau, double tol, int max_sweeps, int32_t* rank, int32_t* sweeps,
                   unsigned long long* sweep_total, unsigned long long* rot_total,
                   unsigned int* hits, bool precond, const WarmState* warm = nullptr) {
  SvtPlan pl;
  if (!svt_plan(s, precond && w.C, &pl))
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld exceeds the Jacobi kernels", s.I1, s.I2);
  if (pl.wide)
    return run_wide_svt(h, s, Gh, Dh, w, pl, tau, tol, max_sweeps, rank, sweeps, sweep_total, rot_total, hits);
  precond = pl.precond;
  lt::JacobiArgs j{};
  lt::JacobiConfig cfg;
  const lt::JacobiBlkConfig& bcfg = pl.bcfg;
  const bool blocked = pl.blocked;
  int rc;
  if (blocked) {
    if ((rc = check_blk_lds(h, s, bcfg))) return rc;
    if (!w.work) return fail(h, LT_ERR_WORKSPACE, "no blocked-Jacobi working buffer in the workspace");
    j.work = w.work;
  }
  if (precond) {
    // Jacobi on L = R^T (n x n), C = W^T W = R^T R: its kept columns are the
    // scaled right singular vectors B, and D_W = (W B) B^T
    const int n = (int)precond_n(s);
    const long long cst = (long long)n * n;
    if (n <= lt::kGramCholMaxN) {
      ProfScope ps(h, LT_PROF_PRECOND);
      lt::GramArgs g{Gh, s.N, w.C, cst, (int)s.I1, (int)s.I2, (int)s.P};
      HIP_TRY(h, lt::launch_gram_chol(g, h->stream));
    } else {
      {
        ProfScope ps(h, LT_PROF_PRECOND);
        lt::GramArgs g{Gh, s.N, w.C, cst, (int)s.I1, (int)s.I2, (int)s.P};
        HIP_TRY(h, lt::launch_gram(g, h->stream));
      }
      {
        ProfScope ps(h, LT_PROF_PRECOND);
        lt::CholArgs c{w.C, cst, n, (int)s.P};
        HIP_TRY(h, lt::launch_chol(c, h->stream));
      }
    }
    Shape sq = s;
    sq.I1 = n;
    sq.I2 = n;
    if (!blocked && (rc = jacobi_config(h, sq, &cfg))) return rc;
    j.src = reinterpret_cast<const float*>(w.C);
    j.slice_stride = 2 * cst;   // L slice s occupies the first half of the slice's FP64 block
    j.I1 = n;
    j.I2 = n;
    j.bk_stride = s.N;
    if (warm && warm->Z && !blocked) {
      // warm start: the Jacobi runs on M = L Z (written over the second half of
      // each slice's block), carrying Z along
      lt::JacobiConfig wc;
      if (lt::jacobi_warm_config(n, h->max_lds, &wc) != 0)
        return fail(h, LT_ERR_SHAPE, "slice %lld x %lld: no warm-start Jacobi configuration", s.I1, s.I2);
      lt::WarmArgs wa{};
      wa.M = j.src;
      wa.m_stride = 2 * cst;
      if (!warm->cold) {
        float* Mw = reinterpret_cast<float*>(w.C) + cst;
        ProfScope ps(h, LT_PROF_PRECOND);
        HIP_TRY(h, lt::launch_warm_product(reinterpret_cast<const float*>(w.C), 2 * cst, warm->Z, Mw, 2 * cst,
                                           n, (int)s.P, h->stream));
        wa.M = Mw;
      }
      wa.Z = warm->Z;
      wa.bk = w.Bk;
      wa.bk_stride = s.N;
      wa.rank = rank;
      wa.sweeps = sweeps;
      wa.sweep_total = sweep_total;
      wa.rot_total = rot_total;
      wa.hits = hits;
      wa.nuc = w.nuc;
      wa.tau = tau;
      wa.tol = tol;
      wa.n = n;
      wa.nslices = (int)s.P;
      wa.max_sweeps = max_sweeps;
      wa.cold = warm->cold ? 1 : 0;
      {
        ProfScope ps(h, LT_PROF_JACOBI);
        HIP_TRY(h, lt::launch_jacobi_warm(wa, wc, h->stream));
      }
      return rebuild_svt(h, s, Gh, Dh, w, rank, true);
    }
  } else {
    if (!blocked && (rc = jacobi_config(h, s, &cfg))) return rc;
    j.src = Gh;
    j.slice_stride = s.N;
    j.I1 = (int)s.I1;
    j.I2 = (int)s.I2;
  }
  j.nslices = (int)s.P;
  j.tau = tau;
  j.tol = tol;
  j.max_sweeps = max_sweeps;
  j.mode = 0;
  j.bk = w.Bk;
  j.rank = rank;
  j.sweeps = sweeps;
  j.sweep_total = sweep_total;
  j.rot_total = rot_total;
  j.maxsweep_hits = hits;
  j.nuc = w.nuc;
  {
    ProfScope ps(h, LT_PROF_JACOBI);
    if (blocked) HIP_TRY(h, lt::launch_jacobi_blk(j, bcfg, h->stream));
    else HIP_TRY(h, lt::launch_jacobi(j, cfg, h->stream));
  }
  return rebuild_svt(h, s, Gh, Dh, w, rank, precond);
}

SvtCore core_of(const SvtWs& w) {
  SvtCore c;
  c.Bk = w.Bk;
  c.rank = w.rank;
  c.sweeps = w.sweeps;
  c.C = w.C;
  c.work = w.work;
  c.nuc = w.nuc;
  c.L32 = w.L32;
  c.T = w.T;
  c.wstate = w.wstate;
  c.active = w.active;
  c.thr = w.thr;
  return c;
}

// Preconditioning of the complex path: Cholesky-QR of the complex slice W = QR
// through its real form T = [w_1, i w_1, w_2, i w_2, ...] (interleaved rows):
// T^T T is the real form of W^H W, and its real Cholesky factor, unique with a
// positive diagonal, is the real form of the complex one (L = R^H lower), so
// the even columns of the real factor are L's columns.  The complex Jacobi then
// runs on L (2 n interleaved rows), whose kept columns are the scaled right
// singular vectors B: D = (W B) B^H, formed as (T B') B'^T with B' = [b, i b],
// of whose columns the even ones are D's.  It applies when requested for
// 2 <= n with 2 n <= LT_PRECOND_MAX_N, using the Gram blocks carve_svt_core
// gives the embeddings when their own plan preconditions.
bool dft_complex_precond(const Shape& s, bool precond_req, int max_lds, lt::JacobiConfig* cc) {
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  if (!precond_req || n < 2 || 2 * n > LT_PRECOND_MAX_N) return false;
  std::vector<int> rep, partner;
  dft_pairs(s, &rep, &partner);
  SvtPlan pe;
  if (!svt_plan(embed_shape(s, (int)rep.size()), true, &pe) || !pe.precond) return false;
  return lt::jacobi_cx_config(2 * (int)n, (int)n, max_lds, cc) == 0;
}

// Fourier slices take the complex Hermitian Jacobi when its register-resident
// kernel holds the Jacobi's working matrix: the complex Cholesky factor (2 n
// interleaved rows, preconditioned, above) or else the representative itself
// (2 max(I1, I2) rows by min(I1, I2) columns).  Otherwise, or with
// LT_DFT_EMBED=1 in the environment, the real embedding.  *pc: preconditioned.
bool dft_complex(const Shape& s, bool precond_req, int max_lds, lt::JacobiConfig* cc, bool* pc) {
  *pc = false;
  if (!s.any_dft) return false;
  const char* env = getenv("LT_DFT_EMBED");
  if (env && atoi(env) == 1) return false;
  if (dft_complex_precond(s, precond_req, max_lds, cc)) {
    *pc = true;
    return true;
  }
  const long long m = s.I1 > s.I2 ? s.I1 : s.I2, n = s.I1 > s.I2 ? s.I2 : s.I1;
  if (m > 4096) return false;
  return lt::jacobi_cx_config(2 * (int)m, (int)n, max_lds, cc) == 0;
}

// The complex path: the representatives' working matrices (2 N floats each,
// or their twinned real forms, 4 N, when preconditioned) into the embedding
// buffer, the preconditioner (above), the Hermitian Jacobi (each kept column
// written with its product by i: up to 2 n columns, 4 N floats per
// representative in the embedding's Bk), the real rebuild over the interleaved
// rows in place, and the results back to the planes.
int run_cx_svt(lt_handle* h, const Shape& s, const SvtWs& w, const lt::JacobiConfig& cc, bool pc, double tau,
               double tol, int max_sweeps, int32_t* rank, int32_t* sweeps, unsigned long long* sweep_total,
               unsigned long long* rot_total, unsigned int* hits) {
  const DftWs& d = w.dft;
  const int m = (int)(s.I1 > s.I2 ? s.I1 : s.I2), n = (int)(s.I1 > s.I2 ? s.I2 : s.I1);
  const long long N = s.N;
  float* Re = w.Gh;
  float* Im = w.Gh + s.nel;
  if (pc && !d.inner.C) return fail(h, LT_ERR_WORKSPACE, "no Gram blocks for the complex preconditioner");
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_dft_stack(Re, Im, d.rep, d.npairs, (int)s.I1, (int)s.I2, d.E, h->stream, pc));
  }
  lt::JacobiArgs a{};
  if (pc) {
    // T (2m x 2n, 4N floats per representative): real Gram and Cholesky, then
    // L's columns (the even ones of the real factor) into Lc.  Up to 192
    // columns the one-kernel Cholesky (FP32 factor over the first half of
    // each FP64 block), beyond it the multi-launch one, which converts the
    // even columns itself
    const int n2 = 2 * n;
    const long long cst = (long long)n2 * n2;
    const long long lcs = (long long)n2 * n;
    lt::GramArgs g{d.E, 4 * N, d.inner.C, cst, 2 * m, n2, d.npairs};
    ProfScope ps(h, LT_PROF_PRECOND);
    if (n2 <= lt::kGramCholMaxN) {
      HIP_TRY(h, lt::launch_gram_chol(g, h->stream));
    } else {   // from the complex columns (T's even ones, 4m floats apart): half the work of T's Gram
      HIP_TRY(h, lt::launch_gram_cx(d.E, 4 * N, 4LL * m, m, n, d.inner.C, cst, d.npairs, h->stream));
    }
    if (n2 <= 192) {
      if (n2 > lt::kGramCholMaxN) {
        lt::CholArgs c{d.inner.C, cst, n2, d.npairs};
        HIP_TRY(h, lt::launch_chol(c, h->stream));
      }
      HIP_TRY(h, lt::launch_even_columns(reinterpret_cast<const float*>(d.inner.C), 2 * cst, d.Lc, lcs, n2, n,
                                         d.npairs, h->stream));
    } else {
      HIP_TRY(h, lt::launch_chol_big(d.inner.C, cst, n2, d.npairs, d.Lc, lcs, d.thr, h->stream, 2));
    }
    a.src = d.Lc;
    a.slice_stride = lcs;
    a.I1 = n2;
    a.I2 = n;
  } else {
    a.src = d.E;
    a.slice_stride = 2 * N;
    a.I1 = 2 * m;
    a.I2 = n;
  }
  a.nslices = d.npairs;
  a.tau = tau;
  a.tol = fabs(tol);
  a.max_sweeps = max_sweeps;
  a.mode = 0;
  a.bk = d.inner.Bk;
  a.bk_stride = 4 * N;
  a.rank = d.inner.rank;
  a.sweeps = d.inner.sweeps;
  a.sweep_total = sweep_total;
  a.rot_total = rot_total;
  a.maxsweep_hits = hits;
  a.nuc = d.inner.nuc;
  {
    ProfScope ps(h, LT_PROF_JACOBI);
    HIP_TRY(h, lt::launch_jacobi_cx(a, cc, h->stream));
  }
  lt::RebuildArgs r{};
  r.W = d.E;
  r.D = d.E;
  r.bk = d.inner.Bk;
  r.rank = d.inner.rank;
  r.slice_stride = pc ? 4 * N : 2 * N;
  r.bk_stride = 4 * N;
  r.kmax = 2 * n;
  r.I1 = 2 * m;
  r.I2 = pc ? 2 * n : n;
  r.nslices = d.npairs;
  r.flip = pc ? 1 : 0;
  {
    ProfScope ps(h, LT_PROF_REBUILD);
    HIP_TRY(h, lt::launch_rebuild(r, h->stream));
  }
  ProfScope ps(h, LT_PROF_OTHER);
  HIP_TRY(h, lt::launch_dft_unstack(d.E, d.rep, d.partner, d.npairs, (int)s.I1, (int)s.I2, Re, Im, d.inner.rank,
                                    rank, d.inner.sweeps, sweeps, d.inner.nuc, w.nuc, h->stream, pc));
  return LT_OK;
}

// SVT of the transform-domain slices of w.Gh in place: real slices directly,
// complex ones (Fourier modes) one slice per conjugate pair, by the complex
// Jacobi or through the real embeddings.  rank / sweeps: per slice (P entries).
int run_svt(lt_handle* h, const Shape& s, const SvtWs& w, double tau, double tol, int max_sweeps,
            int32_t* rank, int32_t* sweeps, unsigned long long* sweep_total, unsigned long long* rot_total,
            unsigned int* hits, bool precond, const WarmState* warm = nullptr) {
  if (!s.any_dft)
    return run_jacobi_svt(h, s, w.Gh, w.Gh, core_of(w), tau, tol, max_sweeps, rank, sweeps, sweep_total,
                          rot_total, hits, precond, warm);
  lt::JacobiConfig cc;
  bool pc;
  if (dft_complex(s, precond, h->max_lds, &cc, &pc))
    return run_cx_svt(h, s, w, cc, pc, tau, tol, max_sweeps, rank, sweeps, sweep_total, rot_total, hits);
  const DftWs& d = w.dft;
  const Shape se = embed_shape(s, d.npairs);
  float* Re = w.Gh;
  float* Im = w.Gh + s.nel;
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_dft_embed(Re, Im, d.rep, d.npairs, (int)s.I1, (int)s.I2, d.E, h->stream));
  }
  int rc = run_jacobi_svt(h, se, d.E, d.E, d.inner, tau, tol, max_sweeps, d.inner.rank, d.inner.sweeps,
                          sweep_total, rot_total, hits, precond);
  if (rc) return rc;
  ProfScope ps(h, LT_PROF_OTHER);
  HIP_TRY(h, lt::launch_dft_extract(d.E, d.rep, d.partner, d.npairs, (int)s.I1, (int)s.I2, Re, Im,
                                    d.inner.rank, rank, d.inner.sweeps, sweeps, d.inner.nuc, w.nuc,
                                    h->stream));
  return LT_OK;
}

// Operations that take Fourier modes: the product, the SVT, the completion, the
// economy *_L-SVD, the truncation and the multirank, FP32 only.
int check_dft(lt_handle* h, const Shape& s, int prec, bool op_supports) {
  if (!s.any_dft) return LT_OK;
  if (!op_supports)
    return fail(h, LT_ERR_UNSUPPORTED, "Fourier modes are not supported by this operation");
  if (prec != LT_PREC_F32)
    return fail(h, LT_ERR_UNSUPPORTED, "Fourier modes take the FP32 transform only");
  return LT_OK;
}

bool precond_requested(const lt_svd_opts* o) { return !(o && o->no_precondition); }

// alpha of Section 3.2 (||L(A)||_F^2 = alpha ||A||_F^2) for the DCT, identity
// and Fourier modes (alpha_i^2 = 1, 1 and I_i): the tensor nuclear norm of
// Theorem 21 is the sum of the transform-domain singular values over alpha.
// 0 when a custom mode matrix is present (not known to be a scaled unitary).
double nuclear_alpha(const Shape& s) {
  double a = 1.0;
  for (int i = 0; i < s.nmodes; ++i) {
    if (s.kind[i] == LT_CUSTOM) return 0.0;
    if (s.kind[i] == LT_DFT) a *= (double)s.n[i];
  }
  return a;
}

// The SVT of this shape is supported by one of the Jacobi kernels svt_plan
// chooses (register-resident, blocked or wide; on the slice itself or on its
// Cholesky-QR factor) and fits the device's LDS.
int check_svt_shape(lt_handle* h, const Shape& s0, bool precond) {
  Shape s = s0;
  lt::JacobiConfig cc;
  bool pc;
  if (dft_complex(s0, precond, h->max_lds, &cc, &pc)) return LT_OK;
  if (s0.any_dft) {
    std::vector<int> rep, partner;
    dft_pairs(s0, &rep, &partner);
    s = embed_shape(s0, (int)rep.size());
  }
  SvtPlan p;
  if (!svt_plan(s, precond, &p))
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld exceeds the Jacobi kernels (n <= %d; without "
                "preconditioning m <= %d)", s.I1, s.I2, kWideMaxN, kWideMaxN);
  if (p.wide) {
    if (p.wcfg.lds > (size_t)h->max_lds)
      return fail(h, LT_ERR_SHAPE, "slice %lld x %lld: the wide Jacobi needs %zu bytes of LDS", s.I1, s.I2,
                  p.wcfg.lds);
    return LT_OK;
  }
  if (p.blocked) return check_blk_lds(h, s, p.bcfg);
  lt::JacobiConfig probe;
  Shape sq = s;
  sq.I1 = p.jm;
  sq.I2 = p.jn;
  return jacobi_config(h, sq, &probe);
}


// ---- batch engine: per-problem workspace ------------------------------------
struct ProblemWs {
  lt::ProbDev* st = nullptr;
  TransformWs t;
  float* Xb = nullptr;
  float* Gh = nullptr;
  float* Bk = nullptr;
  int32_t* rank = nullptr;
  int32_t* sweeps = nullptr;
  double* nuc = nullptr;  // per slice: the last prox's sum of (sigma_i - mu_k)
  double* betas = nullptr;
  double* mus = nullptr;
  double* partials = nullptr;
  unsigned int* scratch = nullptr;
  double* C = nullptr;   // preconditioning: Gram matrices / Cholesky factors
  float* work = nullptr;  // blocked Jacobi: per-slice working buffers
  float* Z = nullptr;     // warm-started Jacobi: per-slice accumulated rotations
  int n_partials = 0;
};

// A problem of the batch engine runs the preconditioned SVT when its options
// ask for it (the default) and its slices allow it.
bool problem_precond(const Shape& s, const lt_pga_params* p) {
  SvtPlan pl;
  return svt_plan(s, precond_requested(&p->svd), &pl, true) && pl.precond;
}

// A batch problem warm-starts its Jacobi as lt_complete_pga does (same shapes,
// same cold-start period); 0: never.
int problem_warm_period(const Shape& s, const lt_pga_params* p) {
  if (!problem_precond(s, p) || p->svd.warm_restart < 0 || !warm_shape(s)) return 0;
  return p->svd.warm_restart == 0 ? kWarmRestartDefault : p->svd.warm_restart;
}

void carve_problem(Carver& c, const Shape& s, int prec, int max_iter, bool precond, bool warm, ProblemWs* w) {
  w->st = c.take<lt::ProbDev>(1);
  carve_transform(c, s, prec, &w->t);
  w->Xb = c.take<float>((size_t)s.nel);
  w->Gh = c.take<float>((size_t)s.nel);
  w->Bk = c.take<float>((size_t)s.nel);
  w->rank = c.take<int32_t>((size_t)s.P);
  w->sweeps = c.take<int32_t>((size_t)s.P);
  w->nuc = c.take<double>((size_t)s.P + 1);   // + the sum for lt_problem_status
  w->betas = c.take<double>((size_t)max_iter);
  w->mus = c.take<double>((size_t)max_iter);
  w->n_partials = (int)n_partials(s);
  w->partials = c.take<double>(2 * (size_t)w->n_partials);
  w->scratch = c.take<unsigned int>(4);
  if (precond) w->C = c.take<double>((size_t)(s.P * precond_n(s) * precond_n(s)));
  SvtPlan pl;
  if (svt_plan(s, precond, &pl, true) && pl.blocked) w->work = c.take<float>((size_t)s.P * (size_t)pl.bcfg.work_floats);
  if (warm) w->Z = c.take<float>((size_t)(s.P * precond_n(s) * precond_n(s)));
}

int check_pga_params(lt_handle* h, const lt_pga_params* p) {
  if (!p) return fail(h, LT_ERR_ARG, "params is NULL");
  if (!(p->mu0 > 0) || !(p->nu > 0 && p->nu <= 1) || !(p->mu_bar > 0 && p->mu_bar <= p->mu0) ||
      p->max_iter < 1 || !isfinite(p->mu0))
    return fail(h, LT_ERR_ARG, "invalid PGA parameters (need mu0 > 0, 0 < nu <= 1, "
                               "0 < mu_bar <= mu0, max_iter >= 1)");
  return LT_OK;
}

// Alg. 5 scalars that depend on no data: beta_k = (t_{k-1} - 1) / t_k with
// t_0 = t_1 = 1, t_{k+1} = (1 + sqrt(4 t_k^2 + 1)) / 2; mu_1 = mu0,
// mu_{k+1} = max(nu mu_k, mu_bar) (or mu0 throughout when fixed_mu).
void pga_schedule(const lt_pga_params* p, std::vector<double>& betas, std::vector<double>& mus) {
  betas.resize(p->max_iter);
  mus.resize(p->max_iter);
  double t_prev = 1.0, t = 1.0, mu = p->mu0;
  for (int k = 0; k < p->max_iter; ++k) {
    betas[k] = (t_prev - 1.0) / t;
    mus[k] = p->fixed_mu ? p->mu0 : mu;
    t_prev = t;
    t = (1.0 + sqrt(4.0 * t * t + 1.0)) / 2.0;
    mu = fmax(p->nu * mu, p->mu_bar);
  }
}

struct BatchTables {
  std::vector<lt::ProbDev*> ptrs;
  std::vector<lt::GemmTile> gemm;
  std::vector<lt::SvtItem> items;
  std::vector<lt::RebuildTile> rebuild;
  std::vector<lt::GramTile> gram;
  std::vector<lt::CholItem> chol;    // Cholesky in LDS (n <= 200)
  int chol_nmax = 0;
  std::vector<lt::CholItem> cholg;   // Cholesky in global memory (n > 200)
  int cholg_nmax = 0;
  // blocked Jacobi: items grouped by lanes per pair (16, 32, 64), each group's
  // launch shape; rebuild tiles of slices with more than 256 columns
  std::vector<lt::CholItem> blk;
  int blk_count[lt::kBlkNumVariants] = {};
  int blk_threads[lt::kBlkNumVariants] = {};
  size_t blk_lds[lt::kBlkNumVariants] = {};
  std::vector<lt::RebuildTile> rebuild_wide;
  int rebuild_kmax = 0, rebuild_wide_kmax = 0;   // largest min(I1, I2) of each tile list
  // warm-started Jacobi: items grouped by configuration (G, R, nbuf), each
  // group's launch shape; the products M = L Z over the same slices
  std::vector<lt::CholItem> warm;
  std::vector<lt::JacobiConfig> warm_cfg;
  std::vector<int> warm_count;
  int warm_nmax = 0;
  bool any_reg = false;
  lt::JacobiBatchConfig cfg{};
  int prec = 0, max_sweeps = 40;
  double tol = kJacobiTolDefault;
  size_t rebuild_slices = 0;   // total frontal slices of the batch
};

int build_tables(lt_handle* h, int n, const lt_problem* probs, int force_G, BatchTables* T) {
  if (n <= 0 || !probs) return fail(h, LT_ERR_ARG, "empty batch");
  if (force_G == 0) {
    const char* env = getenv("LT_JACOBI_G");
    force_G = env ? atoi(env) : 0;
  }
  std::vector<Shape> shapes(n);
  std::vector<int> ms(n), ns(n), nsub(n, 1), qeff(n, 1);
  std::vector<int> blocked(n, 0);
  std::vector<lt::JacobiBlkConfig> bcfg(n);
  std::vector<int> warm(n, 0);
  std::vector<lt::JacobiConfig> wcfg(n);
  for (int i = 0; i < n; ++i) {
    int rc = parse(h, probs[i].desc, &shapes[i]);
    if (rc) return rc;
    if ((rc = check_dft(h, shapes[i], LT_PREC_F32, false))) return rc;
    double tol;
    int max_sweeps, prec;
    resolve_opts(&probs[i].params.svd, &tol, &max_sweeps, &prec);
    if (i == 0) {
      T->tol = tol;
      T->max_sweeps = max_sweeps;
      T->prec = prec;
    } else if (tol != T->tol || max_sweeps != T->max_sweeps || prec != T->prec) {
      return fail(h, LT_ERR_ARG, "problems of one batch must share precision and Jacobi options");
    }
    ms[i] = (int)(shapes[i].I1 > shapes[i].I2 ? shapes[i].I1 : shapes[i].I2);
    ns[i] = (int)(shapes[i].I1 > shapes[i].I2 ? shapes[i].I2 : shapes[i].I1);
    SvtPlan pl;
    if (!svt_plan(shapes[i], problem_precond(shapes[i], &probs[i].params), &pl, true))
      return fail(h, LT_ERR_SHAPE, "slice %lld x %lld exceeds the Jacobi kernels", shapes[i].I1, shapes[i].I2);
    if (pl.wide)
      return fail(h, LT_ERR_SHAPE, "slice %lld x %lld: the batch engine takes slices up to 512 columns",
                  shapes[i].I1, shapes[i].I2);
    ms[i] = pl.jm;   // n for the Jacobi on the n x n factor
    // the lane count asked for (autotuner) applies to the warm-started items
    // too when their kernel takes it (4, 8 or 16 lanes per pair)
    if (problem_warm_period(shapes[i], &probs[i].params) > 0 &&
        lt::jacobi_warm_config(ns[i], h->max_lds, &wcfg[i], force_G) == 0)
      warm[i] = 1;
    if (pl.blocked) {
      int rc2 = check_blk_lds(h, shapes[i], pl.bcfg);
      if (rc2) return rc2;
      blocked[i] = 1;
      bcfg[i] = pl.bcfg;
    }
  }
  // the register-resident kernel's configuration covers the other problems
  std::vector<int> rm, rn, ridx;
  for (int i = 0; i < n; ++i)
    if (!blocked[i]) {
      rm.push_back(ms[i]);
      rn.push_back(ns[i]);
      ridx.push_back(i);
    }
  T->any_reg = !ridx.empty();
  if (T->any_reg) {
    std::vector<int> rsub(ridx.size()), rq(ridx.size());
    if (lt::jacobi_batch_config(rm.data(), rn.data(), (int)ridx.size(), h->max_lds, force_G, &T->cfg,
                                rsub.data(), rq.data()) != 0)
      return fail(h, LT_ERR_SHAPE, "a slice shape of the batch exceeds the register-resident Jacobi kernel");
    for (size_t k = 0; k < ridx.size(); ++k) {
      nsub[ridx[k]] = rsub[k];
      qeff[ridx[k]] = rq[k];
    }
  }
  T->ptrs.resize(n);
  std::vector<std::pair<double, lt::SvtItem>> costed;
  for (int i = 0; i < n; ++i) {
    Carver c(probs[i].ws);
    ProblemWs w;
    const bool pc = problem_precond(shapes[i], &probs[i].params);
    carve_problem(c, shapes[i], T->prec, probs[i].params.max_iter, pc,
                  problem_warm_period(shapes[i], &probs[i].params) > 0, &w);
    T->ptrs[i] = w.st;
    const Shape& s = shapes[i];
    const int ntx = (int)((s.N + 63) / 64), nty = (int)((s.P + 63) / 64);
    for (int ty = 0; ty < nty; ++ty)
      for (int tx = 0; tx < ntx; ++tx) T->gemm.push_back(lt::GemmTile{i, tx, ty, ty * ntx + tx});
    if (!blocked[i] && !warm[i]) {
      const int rounds = 2 * ((ns[i] + 1) / 2) - 1;
      for (int s0 = 0; s0 < (int)s.P; s0 += nsub[i]) {
        const int k = (int)(s.P - s0) < nsub[i] ? (int)(s.P - s0) : nsub[i];
        costed.push_back({(double)rounds * qeff[i], lt::SvtItem{i, s0, k, qeff[i]}});
      }
    }
    // rebuild tiles over the working matrix's columns: W's n columns, or W^T's
    // m columns when the preconditioned SVT rebuilds (W B) B^T
    const int mw = (int)(s.I1 > s.I2 ? s.I1 : s.I2);
    const int ncols = pc ? mw : ns[i];
    std::vector<lt::RebuildTile>& rt = ns[i] > 256 ? T->rebuild_wide : T->rebuild;
    int& kmax = ns[i] > 256 ? T->rebuild_wide_kmax : T->rebuild_kmax;
    kmax = ns[i] > kmax ? ns[i] : kmax;
    for (int sl = 0; sl < (int)s.P; ++sl)
      for (int j0 = 0; j0 < ncols; j0 += 16) rt.push_back(lt::RebuildTile{i, sl, j0, 0});
    T->rebuild_slices += (size_t)s.P;
    if (pc) {
      const int tg = (ns[i] + 31) / 32;
      const bool lds = ns[i] <= kCholLdsMaxN;
      for (int sl = 0; sl < (int)s.P; ++sl) {
        for (int t = 0; t < tg * (tg + 1) / 2; ++t) T->gram.push_back(lt::GramTile{i, sl, t, 0});
        (lds ? T->chol : T->cholg).push_back(lt::CholItem{i, sl});
      }
      int& nmax = lds ? T->chol_nmax : T->cholg_nmax;
      nmax = ns[i] > nmax ? ns[i] : nmax;
    }
  }
  // blocked items, grouped by kernel variant
  for (int gi = 0; gi < lt::kBlkNumVariants; ++gi) {
    for (int i = 0; i < n; ++i) {
      if (!blocked[i] || bcfg[i].variant != gi) continue;
      for (int sl = 0; sl < (int)shapes[i].P; ++sl) T->blk.push_back(lt::CholItem{i, sl});
      T->blk_count[gi] += (int)shapes[i].P;
      T->blk_threads[gi] = bcfg[i].threads > T->blk_threads[gi] ? bcfg[i].threads : T->blk_threads[gi];
      T->blk_lds[gi] = bcfg[i].lds > T->blk_lds[gi] ? bcfg[i].lds : T->blk_lds[gi];
    }
  }
  // warm-started items, grouped by configuration
  for (int i = 0; i < n; ++i) {
    if (!warm[i]) continue;
    size_t gi = 0;
    while (gi < T->warm_cfg.size() &&
           !(T->warm_cfg[gi].G == wcfg[i].G && T->warm_cfg[gi].R == wcfg[i].R && T->warm_cfg[gi].nbuf == wcfg[i].nbuf))
      ++gi;
    if (gi == T->warm_cfg.size()) {
      T->warm_cfg.push_back(wcfg[i]);
      T->warm_count.push_back(0);
    }
    lt::JacobiConfig& g = T->warm_cfg[gi];
    g.threads = wcfg[i].threads > g.threads ? wcfg[i].threads : g.threads;
    g.lds = wcfg[i].lds > g.lds ? wcfg[i].lds : g.lds;
    T->warm_nmax = ns[i] > T->warm_nmax ? ns[i] : T->warm_nmax;
  }
  for (size_t gi = 0; gi < T->warm_cfg.size(); ++gi) {
    const lt::JacobiConfig& g = T->warm_cfg[gi];
    for (int i = 0; i < n; ++i) {
      if (!warm[i] || wcfg[i].G != g.G || wcfg[i].R != g.R || wcfg[i].nbuf != g.nbuf) continue;
      for (int sl = 0; sl < (int)shapes[i].P; ++sl) T->warm.push_back(lt::CholItem{i, sl});
      T->warm_count[gi] += (int)shapes[i].P;
    }
  }
  // longest first, ties by problem then slice (deterministic)
  std::stable_sort(costed.begin(), costed.end(),
                   [](const std::pair<double, lt::SvtItem>& a, const std::pair<double, lt::SvtItem>& b) {
                     return a.first > b.first;
                   });
  for (auto& c : costed) T->items.push_back(c.second);
  return LT_OK;
}

struct BatchWs {
  lt::ProbDev** ptrs = nullptr;
  lt::GemmTile* gemm = nullptr;
  lt::SvtItem* items = nullptr;
  lt::RebuildTile* rebuild = nullptr;
  lt::GramTile* gram = nullptr;
  lt::CholItem* chol = nullptr;
  lt::CholItem* cholg = nullptr;
  lt::CholItem* blk = nullptr;
  lt::RebuildTile* rebuild_wide = nullptr;
  lt::CholItem* warm = nullptr;
};

// The item count depends on how many slices a workgroup packs (device LDS);
// the table is sized for one item per slice so the size does not.
void carve_batch(Carver& c, const BatchTables& T, BatchWs* w) {
  w->ptrs = c.take<lt::ProbDev*>(T.ptrs.size());
  w->gemm = c.take<lt::GemmTile>(T.gemm.size());
  w->items = c.take<lt::SvtItem>(T.rebuild_slices);
  w->rebuild = c.take<lt::RebuildTile>(T.rebuild.size());
  w->gram = c.take<lt::GramTile>(T.gram.size());
  w->chol = c.take<lt::CholItem>(T.chol.size());
  w->cholg = c.take<lt::CholItem>(T.cholg.size());
  w->blk = c.take<lt::CholItem>(T.blk.size());
  w->rebuild_wide = c.take<lt::RebuildTile>(T.rebuild_wide.size());
  w->warm = c.take<lt::CholItem>(T.warm.size());
}

// The *_L-SVD under Fourier modes (Section 2's t-SVD): one complex SVD per
// conjugate pair by the complex Jacobi in its all-columns mode.  The core
// transforms A, stacks the representatives' working matrices and runs the
// Jacobi (columns and norms); `finalize` adds the economy factors
// (k_lsvd_finalize_cx: the representative's and, conjugated, its partner's, in
// two planes; Uw sorted and orthonormal in the scratch).
int lsvd_fourier_core(lt_handle* h, const Shape& s, const float* A, double tol, int max_sweeps, int prec,
                      const LsvdDftWs& w, float* sigma_out, bool finalize) {
  int rc;
  const int m = (int)(s.I1 > s.I2 ? s.I1 : s.I2), n = (int)(s.I1 > s.I2 ? s.I2 : s.I1);
  lt::JacobiConfig cc;
  if (n > 256 || 2 * m > 2048 || lt::jacobi_cx_config(2 * m, n, h->max_lds, &cc) != 0)
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld exceeds the complex Jacobi kernel", s.I1, s.I2);
  if ((rc = build_transform(h, s, prec, w.t))) return rc;
  const int P = (int)s.P;
  if ((rc = gemm(h, gemm_plain(w.t, false, P, s.N, A, w.Ah, true), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                 LT_PROF_FORWARD)))
    return rc;
  std::vector<int> rep, partner;
  dft_pairs(s, &rep, &partner);
  HIP_TRY(h, hipMemcpyAsync(w.rep, rep.data(), rep.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(w.partner, partner.data(), partner.size() * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));   // the host vectors go out of scope
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_dft_stack(w.Ah, w.Ah + s.nel, w.rep, w.npairs, (int)s.I1, (int)s.I2, w.E, h->stream));
  }
  lt::JacobiArgs j{};
  j.src = w.E;
  j.slice_stride = 2 * s.N;
  j.I1 = 2 * m;
  j.I2 = n;
  j.nslices = w.npairs;
  j.tau = 0.0;
  j.tol = fabs(tol);
  j.max_sweeps = max_sweeps;
  j.mode = 1;
  j.bk = w.cols;
  j.bk_stride = 2 * s.N;
  j.sweeps = w.sweeps;
  j.sigma = w.sigma;
  {
    ProfScope ps(h, LT_PROF_JACOBI);
    HIP_TRY(h, lt::launch_jacobi_cx(j, cc, h->stream));
  }
  if (!finalize) return LT_OK;
  lt::LsvdCxArgs f{};
  f.W = w.E;
  f.cols = w.cols;
  f.sigma = w.sigma;
  f.w_stride = 2 * s.N;
  f.rep = w.rep;
  f.partner = w.partner;
  f.npairs = w.npairs;
  f.P = P;
  f.I1 = (int)s.I1;
  f.I2 = (int)s.I2;
  f.U = w.Uh;
  f.S = w.Sh;
  f.V = w.Vh;
  f.sig_out = sigma_out;
  f.scratch = w.scratch;
  f.scratch_stride = 2LL * m * n + 2LL * n * n;
  ProfScope ps(h, LT_PROF_OTHER);
  HIP_TRY(h, lt::launch_lsvd_finalize_cx(f, h->stream));
  return LT_OK;
}

int lsvd_fourier(lt_handle* h, const lt_desc* a, const Shape& s, const float* A, float* U, float* S, float* V,
                 float* sigma, int economy, int transform_domain, double tol, int max_sweeps, int prec, void* ws,
                 size_t ws_bytes) {
  int rc;
  if ((rc = check_dft(h, s, prec, true))) return rc;
  if (!economy || transform_domain)
    return fail(h, LT_ERR_UNSUPPORTED, "Fourier modes: lt_lsvd returns economy factors in the spatial domain only");
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_LSVD, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LsvdDftWs w;
  carve_lsvd_dft(c, s, prec, &w);
  if ((rc = lsvd_fourier_core(h, s, A, tol, max_sweeps, prec, w, sigma, true))) return rc;
  const int P = (int)s.P;
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  if ((rc = gemm(h, gemm_plain(w.t, true, P, s.I1 * n, w.Uh, U, true), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                 LT_PROF_INVERSE)))
    return rc;
  if ((rc = gemm(h, gemm_plain(w.t, true, P, n * n, w.Sh, S, true), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                 LT_PROF_INVERSE)))
    return rc;
  return gemm(h, gemm_plain(w.t, true, P, s.I2 * n, w.Vh, V, true), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
              LT_PROF_INVERSE);
}

// Multirank under Fourier modes: the complex Jacobi's norms of each
// representative count for both slices of its pair.
int multirank_fourier(lt_handle* h, const lt_desc* a, const Shape& s, const float* A, double rtol, int32_t* rank,
                      double* avg, int32_t* tubal, double tol, int max_sweeps, int prec, void* ws,
                      size_t ws_bytes) {
  int rc;
  if ((rc = check_dft(h, s, prec, true))) return rc;
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_LSVD, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LsvdDftWs w;
  carve_lsvd_dft(c, s, prec, &w);
  if ((rc = lsvd_fourier_core(h, s, A, tol, max_sweeps, prec, w, nullptr, false))) return rc;
  const int n = (int)(s.I1 < s.I2 ? s.I1 : s.I2);
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_expand_pairs(w.sigma, w.rep, w.partner, w.npairs, n, w.sigP, h->stream));
    HIP_TRY(h, lt::launch_multirank(w.sigP, (int)s.P, n, rtol, rank, w.mr, h->stream));
  }
  if (avg || tubal) {
    HIP_TRY(h, hipMemcpyAsync(h->pinned, w.mr, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (avg) *avg = h->pinned[0];
    if (tubal) *tubal = (int32_t)h->pinned[1];
  }
  return LT_OK;
}

// Rank-k truncation under Fourier modes: A_k's complex slice in working
// orientation is U_k U_k^H W (U_k: the first k sorted, orthonormal left
// singular vectors from the finalisation), formed by the real rebuild over the
// interleaved rows from each column and its product by i, then the results back
// to the planes (partners conjugated) and the inverse transform.
int truncate_fourier(lt_handle* h, const lt_desc* a, const Shape& s, const float* A, int32_t k, float* Ak,
                     double tol, int max_sweeps, int prec, void* ws, size_t ws_bytes) {
  int rc;
  if ((rc = check_dft(h, s, prec, true))) return rc;
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_TRUNCATE, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LsvdDftWs w;
  carve_lsvd_dft(c, s, prec, &w, true);
  if ((rc = lsvd_fourier_core(h, s, A, tol, max_sweeps, prec, w, nullptr, true))) return rc;
  const int m = (int)(s.I1 > s.I2 ? s.I1 : s.I2), n = (int)(s.I1 > s.I2 ? s.I2 : s.I1);
  const int kk = k <= 0 ? 0 : (k < n ? (int)k : n);
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_twin_columns(w.scratch, 2LL * m * n + 2LL * n * n, 2 * m, kk, w.Bk, 4 * s.N, w.npairs,
                                       h->stream));
    HIP_TRY(h, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(w.kept), 2 * kk, (size_t)w.npairs, h->stream));
  }
  lt::RebuildArgs r{};
  r.W = w.E;
  r.D = w.E;
  r.bk = w.Bk;
  r.rank = w.kept;
  r.slice_stride = 2 * s.N;
  r.bk_stride = 4 * s.N;
  r.kmax = 2 * n;
  r.I1 = 2 * m;
  r.I2 = n;
  r.nslices = w.npairs;
  r.flip = 0;
  {
    ProfScope ps(h, LT_PROF_REBUILD);
    HIP_TRY(h, lt::launch_rebuild(r, h->stream));
  }
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_dft_unstack(w.E, w.rep, w.partner, w.npairs, (int)s.I1, (int)s.I2, w.Ah, w.Ah + s.nel,
                                      nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, h->stream));
  }
  return gemm(h, gemm_plain(w.t, true, (int)s.P, s.N, w.Ah, Ak, true), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
              LT_PROF_INVERSE);
}

}  // namespace

struct lt_batch {
  lt_handle* h = nullptr;
  int n = 0;
  BatchTables T;
  BatchWs w;
  int use_graph = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* lt_status_string(int status) {
  switch (status) {
    case LT_OK: return "ok";
    case LT_ERR_ARG: return "invalid argument";
    case LT_ERR_SHAPE: return "invalid or unsupported shape";
    case LT_ERR_UNSUPPORTED: return "unsupported on this library";
    case LT_ERR_NONFINITE: return "non-finite input";
    case LT_ERR_HIP: return "HIP runtime error";
    case LT_ERR_WORKSPACE: return "workspace missing or too small";
    case LT_WARN_MAXSWEEPS: return "warning: Jacobi sweep limit reached";
    case LT_WARN_NOT_CONVERGED: return "warning: PGA iteration limit reached";
    default: return "unknown status";
  }
}

int lt_create(lt_handle** out, void* stream) {
  if (!out) return LT_ERR_ARG;
  lt_handle* h = new (std::nothrow) lt_handle();
  if (!h) return LT_ERR_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return LT_ERR_HIP;
  }
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) ==
          hipSuccess &&
      lds > 0)
    h->max_lds = lds;
  // the handle's device is current here: resolve its scratch copy once
  h->scratch_rc = scratch_address(h->device, &h->scratch);
  if (hipHostMalloc((void**)&h->pinned, kPinnedDoubles * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    delete h;
    return LT_ERR_HIP;
  }
  *out = h;
  return LT_OK;
}

int lt_destroy(lt_handle* h) {
  if (!h) return LT_ERR_ARG;
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  if (h->pinned) (void)hipHostFree(h->pinned);
  delete h;
  return LT_OK;
}

int lt_set_stream(lt_handle* h, void* stream) {
  if (!h) return LT_ERR_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  return LT_OK;
}

const char* lt_last_error(const lt_handle* h) { return h ? h->err.c_str() : "null handle"; }

int lt_profile_begin(lt_handle* h) {
  if (!h) return LT_ERR_ARG;
  if (h->events.empty()) {
    h->events.resize(kEventPool);
    for (size_t i = 0; i < kEventPool; ++i)
      if (hipEventCreate(&h->events[i]) != hipSuccess) {
        h->events.resize(i);
        return fail(h, LT_ERR_HIP, "hipEventCreate failed");
      }
  }
  h->ev_next = 0;
  h->recs.clear();
  h->dropped = 0;
  h->prof_on = true;
  return LT_OK;
}

int lt_profile_end(lt_handle* h, lt_profile* out) {
  if (!h || !out) return LT_ERR_ARG;
  h->prof_on = false;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  memset(out, 0, sizeof(*out));
  for (const auto& r : h->recs) {
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, h->events[r.second], h->events[r.second + 1]));
    out->calls[r.first] += 1;
    out->ms[r.first] += ms;
  }
  out->dropped = h->dropped;
  h->recs.clear();
  h->ev_next = 0;
  return LT_OK;
}

size_t lt_workspace_bytes(const lt_desc* a, const lt_desc* b, int op, int precision) {
  Shape s;
  if (parse(nullptr, a, &s) != LT_OK) return 0;
  if (precision != LT_PREC_F32 && precision != LT_PREC_BF16X3) return 0;
  if (s.any_dft && (precision != LT_PREC_F32 || (op != LT_OP_SVT && op != LT_OP_PGA && op != LT_OP_LPRODUCT &&
                                                 op != LT_OP_LSVD && op != LT_OP_TRUNCATE)))
    return 0;
  Carver c(nullptr);
  switch (op) {
    case LT_OP_SVT: {
      SvtWs w;
      carve_svt(c, s, precision, &w);
      break;
    }
    case LT_OP_PGA: {
      PgaWs w;
      carve_pga(c, s, precision, &w);
      break;
    }
    case LT_OP_LPRODUCT: {
      Shape sb;
      if (!b || parse(nullptr, b, &sb) != LT_OK) return 0;
      LprodWs w;
      carve_transform(c, s, precision, &w.t);
      const size_t planes = s.any_dft ? 2 : 1;   // Fourier modes: real and imaginary planes
      w.Ah = c.take<float>(planes * (size_t)s.nel);
      w.Bh = c.take<float>(planes * (size_t)sb.nel);
      w.Ch = c.take<float>(planes * (size_t)(s.I1 * sb.I2 * s.P));
      break;
    }
    case LT_OP_LSVD: {
      if (s.any_dft) {
        LsvdDftWs w;
        carve_lsvd_dft(c, s, precision, &w);
        break;
      }
      LsvdWs w;
      carve_lsvd(c, s, precision, &w);
      break;
    }
    case LT_OP_LSVD_FULL: {
      LsvdWs w;
      carve_lsvd(c, s, precision, &w, true);
      break;
    }
    case LT_OP_TRUNCATE: {
      if (s.any_dft) {
        LsvdDftWs w;
        carve_lsvd_dft(c, s, precision, &w, true);
        break;
      }
      LsvdWs w;
      carve_lsvd(c, s, precision, &w);
      (void)c.take<int32_t>((size_t)s.P);   // kept count per slice
      break;
    }
    default: return 0;
  }
  return c.off + 256;
}

int lt_svt_path(const lt_desc* a, const lt_svd_opts* opts) {
  Shape s;
  int rc = parse(nullptr, a, &s);
  if (rc) return rc;
  lt::JacobiConfig cc;
  bool pc;
  if (dft_complex(s, precond_requested(opts), kBlkLdsBudget, &cc, &pc))
    return LT_SVT_COMPLEX | (pc ? LT_SVT_PRECOND : 0);
  if (s.any_dft) {   // the Jacobi runs on the real embeddings of the complex slices
    std::vector<int> rep, partner;
    dft_pairs(s, &rep, &partner);
    s = embed_shape(s, (int)rep.size());
  }
  SvtPlan p;
  if (!svt_plan(s, precond_requested(opts), &p)) return LT_ERR_SHAPE;
  return (p.precond ? LT_SVT_PRECOND : 0) | (p.blocked ? LT_SVT_BLOCKED : 0) | (p.wide ? LT_SVT_WIDE : 0);
}

int lt_pga_warm(const lt_desc* a, const lt_svd_opts* opts) {
  Shape s;
  int rc = parse(nullptr, a, &s);
  if (rc) return rc;
  if (!precond_requested(opts) || (opts && opts->warm_restart < 0)) return 0;
  return warm_shape(s) ? 1 : 0;
}

int lt_svt_prox(lt_handle* h, const lt_desc* a, const float* A, double tau, float* D,
                int32_t* rank_out, int32_t* sweeps_out, const lt_svd_opts* opts, void* ws,
                size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, a, &s);
  if (rc) return rc;
  if (!A || !D) return fail(h, LT_ERR_ARG, "A or D is NULL");
  if (!(tau >= 0.0) || !isfinite(tau)) return fail(h, LT_ERR_ARG, "tau must be finite and >= 0");
  double tol;
  int max_sweeps, prec;
  resolve_opts(opts, &tol, &max_sweeps, &prec);
  if ((rc = check_prec(h, prec))) return rc;
  if ((rc = check_dft(h, s, prec, true))) return rc;
  if ((rc = check_svt_shape(h, s, precond_requested(opts)))) return rc;
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_SVT, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  SvtWs w;
  carve_svt(c, s, prec, &w);
  if ((rc = dft_prepare(h, s, w))) return rc;
  if ((rc = build_transform(h, s, prec, w.t))) return rc;
  if ((rc = gemm(h, gemm_plain(w.t, false, (int)s.P, s.N, A, w.Gh, s.any_dft), prec, lt::PRO_PLAIN,
                 lt::EPI_PLAIN, LT_PROF_FORWARD)))
    return rc;
  rc = run_svt(h, s, w, tau, tol, max_sweeps, rank_out ? rank_out : w.rank, sweeps_out ? sweeps_out : w.sweeps,
               nullptr, nullptr, nullptr, precond_requested(opts));
  if (rc) return rc;
  return gemm(h, gemm_plain(w.t, true, (int)s.P, s.N, w.Gh, D, s.any_dft), prec, lt::PRO_PLAIN,
              lt::EPI_PLAIN, LT_PROF_INVERSE);
}

int lt_svt_prox_noalloc(lt_handle* h, const lt_desc* a, const float* A, double tau, float* D,
                        int32_t* rank_out, int32_t* sweeps_out, const lt_svd_opts* opts) {
  if (!h) return LT_ERR_ARG;
  if (!h->scratch)
    return fail(h, LT_ERR_HIP, "no device address for the static scratch on device %d: %s", h->device,
                hipGetErrorString(h->scratch_rc));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
    return fail(h, LT_ERR_ARG, "the handle belongs to device %d, the current device is %d", h->device, dev);
  double tol;
  int max_sweeps, prec;
  resolve_opts(opts, &tol, &max_sweeps, &prec);
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_SVT, prec);
  if (need > kNoallocScratchBytes)
    return fail(h, LT_ERR_WORKSPACE,
                "this SVT needs %zu bytes of workspace; the static scratch holds %zu (LT_NOALLOC_SCRATCH_BYTES)",
                need, kNoallocScratchBytes);
  // need == 0 (invalid descriptor or options): lt_svt_prox reports the reason
  return lt_svt_prox(h, a, A, tau, D, rank_out, sweeps_out, opts, h->scratch, kNoallocScratchBytes);
}

int lt_lproduct(lt_handle* h, const lt_desc* a, const float* A, const lt_desc* b,
                const float* B, float* C, int precision, void* ws, size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  Shape sa, sb;
  int rc = parse(h, a, &sa);
  if (rc) return rc;
  if ((rc = parse(h, b, &sb))) return rc;
  if (!A || !B || !C) return fail(h, LT_ERR_ARG, "A, B or C is NULL");
  if ((rc = check_prec(h, precision))) return rc;
  if ((rc = check_dft(h, sa, precision, true))) return rc;
  if (sa.order != sb.order || sa.I2 != sb.I1)
    return fail(h, LT_ERR_SHAPE, "inner dimensions differ (%lld vs %lld)", sa.I2, sb.I1);
  for (int i = 2; i < sa.order; ++i)
    if (a->dims[i] != b->dims[i] || a->kind[i] != b->kind[i] ||
        (a->kind[i] == LT_CUSTOM && a->custom[i] != b->custom[i]))
      return fail(h, LT_ERR_SHAPE, "mode %d differs between A and B", i + 1);
  const size_t need = lt_workspace_bytes(a, b, LT_OP_LPRODUCT, precision);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LprodWs w;
  carve_transform(c, sa, precision, &w.t);
  const bool dft = sa.any_dft;   // complex transform-domain slices, in real and imaginary planes
  const size_t planes = dft ? 2 : 1;
  w.Ah = c.take<float>(planes * (size_t)sa.nel);
  w.Bh = c.take<float>(planes * (size_t)sb.nel);
  w.Ch = c.take<float>(planes * (size_t)(sa.I1 * sb.I2 * sa.P));
  if ((rc = build_transform(h, sa, precision, w.t))) return rc;
  const int P = (int)sa.P;
  if ((rc = gemm(h, gemm_plain(w.t, false, P, sa.N, A, w.Ah, dft), precision, lt::PRO_PLAIN,
                 lt::EPI_PLAIN, LT_PROF_FORWARD)))
    return rc;
  if ((rc = gemm(h, gemm_plain(w.t, false, P, sb.N, B, w.Bh, dft), precision, lt::PRO_PLAIN,
                 lt::EPI_PLAIN, LT_PROF_FORWARD)))
    return rc;
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_facewise(w.Ah, w.Bh, w.Ch, (int)sa.I1, (int)sa.I2, (int)sb.I2, P,
                                   h->stream, dft));
  }
  return gemm(h, gemm_plain(w.t, true, P, sa.I1 * sb.I2, w.Ch, C, dft), precision, lt::PRO_PLAIN,
              lt::EPI_PLAIN, LT_PROF_INVERSE);
}

// Transform-domain singular values of every slice (the Jacobi in its
// all-columns mode), unsorted, into w.sigma; w.Ah holds L(A) and w.cols the
// final columns.
int lsvd_core(lt_handle* h, const Shape& s, const float* A, int prec, double tol, int max_sweeps,
              const LsvdWs& w) {
  lt::JacobiConfig cfg;
  int rc;
  if ((rc = jacobi_config(h, s, &cfg))) return rc;
  if ((rc = build_transform(h, s, prec, w.t))) return rc;
  const int P = (int)s.P;
  if ((rc = gemm(h, gemm_plain(w.t, false, P, s.N, A, w.Ah), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                 LT_PROF_FORWARD)))
    return rc;
  lt::JacobiArgs j{};
  j.src = w.Ah;
  j.slice_stride = s.N;
  j.I1 = (int)s.I1;
  j.I2 = (int)s.I2;
  j.nslices = P;
  j.tau = 0.0;
  j.tol = tol;
  j.max_sweeps = max_sweeps;
  j.mode = 1;
  j.bk = w.cols;
  j.rank = nullptr;
  j.sweeps = w.sweeps;
  j.sigma = w.sigma;
  ProfScope ps(h, LT_PROF_JACOBI);
  HIP_TRY(h, lt::launch_jacobi(j, cfg, h->stream));
  return LT_OK;
}

int lt_multirank(lt_handle* h, const lt_desc* a, const float* A, double rtol, int32_t* rank, double* avg,
                 int32_t* tubal, const lt_svd_opts* opts, void* ws, size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, a, &s);
  if (rc) return rc;
  if (!A || !rank) return fail(h, LT_ERR_ARG, "A or rank is NULL");
  if (!(rtol >= 0.0) || !isfinite(rtol)) return fail(h, LT_ERR_ARG, "rtol must be finite and >= 0");
  double tol;
  int max_sweeps, prec;
  resolve_opts(opts, &tol, &max_sweeps, &prec);
  if ((rc = check_prec(h, prec))) return rc;
  if (s.any_dft)
    return multirank_fourier(h, a, s, A, rtol, rank, avg, tubal, tol, max_sweeps, prec, ws, ws_bytes);
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  const long long mrows = s.I1 < s.I2 ? s.I2 : s.I1;
  if (n > 256 || mrows > 2048)
    return fail(h, LT_ERR_SHAPE, "multirank supports min(I1, I2) <= 256 and max(I1, I2) <= 2048");
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_LSVD, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LsvdWs w;
  carve_lsvd(c, s, prec, &w);
  if ((rc = lsvd_core(h, s, A, prec, tol, max_sweeps, w))) return rc;
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_multirank(w.sigma, (int)s.P, (int)n, rtol, rank, w.mr, h->stream));
  }
  if (avg || tubal) {
    HIP_TRY(h, hipMemcpyAsync(h->pinned, w.mr, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (avg) *avg = h->pinned[0];
    if (tubal) *tubal = (int32_t)h->pinned[1];
  }
  return LT_OK;
}

int lt_lsvd(lt_handle* h, const lt_desc* a, const float* A, float* U, float* S, float* V,
            float* sigma, int economy, int transform_domain, const lt_svd_opts* opts, void* ws,
            size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, a, &s);
  if (rc) return rc;
  if (!A || !U || !S || !V) return fail(h, LT_ERR_ARG, "A, U, S or V is NULL");
  double tol;
  int max_sweeps, prec;
  resolve_opts(opts, &tol, &max_sweeps, &prec);
  if ((rc = check_prec(h, prec))) return rc;
  if (s.any_dft)
    return lsvd_fourier(h, a, s, A, U, S, V, sigma, economy, transform_domain, tol, max_sweeps, prec, ws,
                        ws_bytes);
  lt::JacobiConfig cfg;
  if ((rc = jacobi_config(h, s, &cfg))) return rc;
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  const long long mrows = s.I1 < s.I2 ? s.I2 : s.I1;
  if (n > 256 || mrows > 2048)
    return fail(h, LT_ERR_SHAPE, "lsvd supports min(I1, I2) <= 256 and max(I1, I2) <= 2048");
  const bool full = economy == 0;
  const size_t need = lt_workspace_bytes(a, nullptr, full ? LT_OP_LSVD_FULL : LT_OP_LSVD, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LsvdWs w;
  carve_lsvd(c, s, prec, &w, full);
  if ((rc = lsvd_core(h, s, A, prec, tol, max_sweeps, w))) return rc;
  const int P = (int)s.P;
  lt::LsvdArgs f{};
  f.W = w.Ah;
  f.cols = w.cols;
  f.sigma = w.sigma;
  f.slice_stride = s.N;
  f.I1 = (int)s.I1;
  f.I2 = (int)s.I2;
  f.nslices = P;
  const bool direct = transform_domain && !full;   // economy factors straight into the outputs
  f.U = direct ? U : w.Uh;
  f.S = direct ? S : w.Sh;
  f.V = direct ? V : w.Vh;
  f.sig_out = sigma;
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_lsvd_finalize(f, h->stream));
  }
  if (full) {
    // Alg. 3's shapes: the economy factors padded, the longer side's factor
    // completed to an orthonormal basis, S padded with zeros
    const int I1 = (int)s.I1, I2 = (int)s.I2, nn = (int)n;
    float* Uf = transform_domain ? U : w.Uf;
    float* Sf = transform_domain ? S : w.Sf;
    float* Vf = transform_domain ? V : w.Vf;
    {
      ProfScope ps(h, LT_PROF_OTHER);
      HIP_TRY(h, lt::launch_pad_copy(w.Uh, Uf, I1, nn, I1, I1, P, h->stream));
      HIP_TRY(h, lt::launch_pad_copy(w.Sh, Sf, nn, nn, I1, I2, P, h->stream));
      HIP_TRY(h, lt::launch_pad_copy(w.Vh, Vf, I2, nn, I2, I2, P, h->stream));
      if (I1 > nn) HIP_TRY(h, lt::launch_complete_basis(Uf, w.H, w.beta, I1, nn, P, h->stream));
      if (I2 > nn) HIP_TRY(h, lt::launch_complete_basis(Vf, w.H, w.beta, I2, nn, P, h->stream));
    }
    if (!transform_domain) {
      if ((rc = gemm(h, gemm_plain(w.t, true, P, s.I1 * s.I1, Uf, U), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                     LT_PROF_INVERSE)))
        return rc;
      if ((rc = gemm(h, gemm_plain(w.t, true, P, s.I1 * s.I2, Sf, S), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                     LT_PROF_INVERSE)))
        return rc;
      if ((rc = gemm(h, gemm_plain(w.t, true, P, s.I2 * s.I2, Vf, V), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                     LT_PROF_INVERSE)))
        return rc;
    }
    return LT_OK;
  }
  if (!transform_domain) {
    if ((rc = gemm(h, gemm_plain(w.t, true, P, s.I1 * n, w.Uh, U), prec, lt::PRO_PLAIN,
                   lt::EPI_PLAIN, LT_PROF_INVERSE)))
      return rc;
    if ((rc = gemm(h, gemm_plain(w.t, true, P, n * n, w.Sh, S), prec, lt::PRO_PLAIN,
                   lt::EPI_PLAIN, LT_PROF_INVERSE)))
      return rc;
    if ((rc = gemm(h, gemm_plain(w.t, true, P, s.I2 * n, w.Vh, V), prec, lt::PRO_PLAIN,
                   lt::EPI_PLAIN, LT_PROF_INVERSE)))
      return rc;
  }
  return LT_OK;
}

int lt_ltruncate(lt_handle* h, const lt_desc* a, const float* A, int32_t k, float* Ak,
                 const lt_svd_opts* opts, void* ws, size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, a, &s);
  if (rc) return rc;
  if (!A || !Ak) return fail(h, LT_ERR_ARG, "A or Ak is NULL");
  double tol;
  int max_sweeps, prec;
  resolve_opts(opts, &tol, &max_sweeps, &prec);
  if ((rc = check_prec(h, prec))) return rc;
  if (s.any_dft) return truncate_fourier(h, a, s, A, k, Ak, tol, max_sweeps, prec, ws, ws_bytes);
  lt::JacobiConfig cfg;
  if ((rc = jacobi_config(h, s, &cfg))) return rc;
  const long long n = s.I1 < s.I2 ? s.I1 : s.I2;
  const long long mrows = s.I1 < s.I2 ? s.I2 : s.I1;
  if (n > 256 || mrows > 2048)
    return fail(h, LT_ERR_SHAPE, "truncation supports min(I1, I2) <= 256 and max(I1, I2) <= 2048");
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_TRUNCATE, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  LsvdWs w;
  carve_lsvd(c, s, prec, &w);
  int32_t* kept = c.take<int32_t>((size_t)s.P);
  if ((rc = build_transform(h, s, prec, w.t))) return rc;
  const int P = (int)s.P;
  if ((rc = gemm(h, gemm_plain(w.t, false, P, s.N, A, w.Ah), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
                 LT_PROF_FORWARD)))
    return rc;
  // per slice: all singular triplets (Jacobi, then sorted and normalised),
  // transform domain
  lt::JacobiArgs j{};
  j.src = w.Ah;
  j.slice_stride = s.N;
  j.I1 = (int)s.I1;
  j.I2 = (int)s.I2;
  j.nslices = P;
  j.tau = 0.0;
  j.tol = tol;
  j.max_sweeps = max_sweeps;
  j.mode = 1;
  j.bk = w.cols;
  j.sweeps = w.sweeps;
  j.sigma = w.sigma;
  {
    ProfScope ps(h, LT_PROF_JACOBI);
    HIP_TRY(h, lt::launch_jacobi(j, cfg, h->stream));
  }
  lt::LsvdArgs f{};
  f.W = w.Ah;
  f.cols = w.cols;
  f.sigma = w.sigma;
  f.slice_stride = s.N;
  f.I1 = (int)s.I1;
  f.I2 = (int)s.I2;
  f.nslices = P;
  f.U = w.Uh;
  f.S = w.Sh;
  f.V = w.Vh;
  {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_lsvd_finalize(f, h->stream));
  }
  // A_k's slice in working orientation: U_k U_k^T W = U_k S_k V_k^T, with U_k
  // the first k left singular vectors of the working matrix (m x n, slice
  // stride m n = I1 I2)
  const int kk = k <= 0 ? 0 : (k < n ? (int)k : (int)n);
  HIP_TRY(h, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(kept), kk, (size_t)P, h->stream));
  lt::RebuildArgs r{};
  r.W = w.Ah;
  r.D = w.Ah;
  r.bk = s.I1 < s.I2 ? w.Vh : w.Uh;
  r.rank = kept;
  r.slice_stride = s.N;
  r.I1 = (int)s.I1;
  r.I2 = (int)s.I2;
  r.nslices = P;
  r.flip = 0;
  {
    ProfScope ps(h, LT_PROF_REBUILD);
    HIP_TRY(h, lt::launch_rebuild(r, h->stream));
  }
  return gemm(h, gemm_plain(w.t, true, P, s.N, w.Ah, Ak), prec, lt::PRO_PLAIN, lt::EPI_PLAIN,
              LT_PROF_INVERSE);
}

int lt_complete_pga(lt_handle* h, const lt_desc* a, const float* M, const uint8_t* mask,
                    const lt_pga_params* p, float* X, lt_pga_report* rep, void* ws,
                    size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, a, &s);
  if (rc) return rc;
  if (!M || !mask || !X || !p) return fail(h, LT_ERR_ARG, "M, mask, X or params is NULL");
  if (!(p->mu0 > 0) || !(p->nu > 0 && p->nu <= 1) || !(p->mu_bar > 0 && p->mu_bar <= p->mu0) ||
      p->max_iter < 1 || !isfinite(p->mu0) || p->start_iter < 0)
    return fail(h, LT_ERR_ARG, "invalid PGA parameters (need mu0 > 0, 0 < nu <= 1, "
                               "0 < mu_bar <= mu0, max_iter >= 1, start_iter >= 0)");
  double tol;
  int max_sweeps, prec;
  resolve_opts(&p->svd, &tol, &max_sweeps, &prec);
  if ((rc = check_prec(h, prec))) return rc;
  if ((rc = check_dft(h, s, prec, true))) return rc;
  if ((rc = check_svt_shape(h, s, precond_requested(&p->svd)))) return rc;
  const size_t need = lt_workspace_bytes(a, nullptr, LT_OP_PGA, prec);
  if ((rc = check_ws(h, ws, ws_bytes, need))) return rc;
  Carver c(ws);
  PgaWs w;
  carve_pga(c, s, prec, &w);
  if ((rc = dft_prepare(h, s, w.svt))) return rc;
  hipStream_t st = h->stream;

  // NaN / Inf among the observed entries: one host sync before any iteration
  HIP_TRY(h, hipMemsetAsync(w.nonfinite, 0, sizeof(unsigned int) * 1, st));
  HIP_TRY(h, lt::launch_count_nonfinite(M, mask, s.nel, w.nonfinite, st));
  HIP_TRY(h, hipMemcpyAsync(h->pinned, w.nonfinite, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipStreamSynchronize(st));
  if (*reinterpret_cast<unsigned int*>(h->pinned) != 0)
    return fail(h, LT_ERR_NONFINITE, "%u non-finite observed entries in M",
                *reinterpret_cast<unsigned int*>(h->pinned));

  if ((rc = build_transform(h, s, prec, w.svt.t))) return rc;
  const size_t bytes = (size_t)s.nel * sizeof(float);
  float* Xcur = X;        // X^k
  float* Xprev = w.Xb;    // X^{k-1}
  const int k0 = p->start_iter;
  if (k0 == 0) {
    HIP_TRY(h, hipMemsetAsync(Xcur, 0, bytes, st));
    HIP_TRY(h, hipMemsetAsync(Xprev, 0, bytes, st));
  }
  HIP_TRY(h, hipMemsetAsync(w.sweep_total, 0, sizeof(unsigned long long), st));
  HIP_TRY(h, hipMemsetAsync(w.slowest_total, 0, sizeof(unsigned long long), st));
  HIP_TRY(h, hipMemsetAsync(w.rot_total, 0, sizeof(unsigned long long), st));
  HIP_TRY(h, hipMemsetAsync(w.maxsweep_hits, 0, sizeof(unsigned int), st));
  const int nsvd = (int)(s.any_dft ? w.svt.dft.npairs : s.P);   // slice SVDs per iteration

  const int check_every = p->check_every > 0 ? p->check_every : 1;
  const int restart = p->svd.warm_restart == 0 ? kWarmRestartDefault : p->svd.warm_restart;
  double t_prev = 1.0, t = 1.0, mu = p->mu0;   // t_0 = t_1 = 1, mu_1 = mu0
  for (int k = 0; k < k0; ++k) {                // the schedule at a continued run's start
    t_prev = t;
    t = (1.0 + sqrt(4.0 * t * t + 1.0)) / 2.0;
    mu = fmax(p->nu * mu, p->mu_bar);
  }
  int iters = 0;
  bool converged = false;
  double crit = NAN;
  for (int k = k0; k < k0 + p->max_iter; ++k) {
    const double beta = (t_prev - 1.0) / t;   // eq. (52)
    const double mu_k = p->fixed_mu ? p->mu0 : mu;

    lt::GemmArgs f = gemm_plain(w.svt.t, false, (int)s.P, s.N, nullptr, w.svt.Gh, s.any_dft);
    f.X = Xcur;
    f.Xp = Xprev;
    f.M = M;
    f.mask = mask;
    f.beta = (float)beta;
    if ((rc = gemm(h, f, prec, lt::PRO_PGA, lt::EPI_PLAIN, LT_PROF_FORWARD))) return rc;
    WarmState warm;
    if (w.Z && restart > 0) {
      warm.Z = w.Z;
      warm.cold = k % restart == 0;
    }
    rc = run_svt(h, s, w.svt, mu_k, tol, max_sweeps, w.svt.rank, w.svt.sweeps, w.sweep_total, w.rot_total,
                 w.maxsweep_hits, precond_requested(&p->svd), warm.Z ? &warm : nullptr);
    if (rc) return rc;
    lt::GemmArgs b = gemm_plain(w.svt.t, true, (int)s.P, s.N, w.svt.Gh, Xprev, s.any_dft);
    b.X = Xcur;
    b.Xp = Xprev;
    b.beta = (float)beta;
    b.partials = w.partials;
    int np = 0;
    if ((rc = gemm(h, b, prec, lt::PRO_PLAIN, lt::EPI_PGA, LT_PROF_INVERSE, &np))) return rc;
    {
      ProfScope ps(h, LT_PROF_OTHER);
      HIP_TRY(h, lt::launch_reduce_partials(w.partials, np, w.norms, st, w.svt.sweeps, nsvd, w.slowest_total));
    }
    float* tmp = Xcur;   // X^{k+1} now lives in the old X^{k-1} buffer
    Xcur = Xprev;
    Xprev = tmp;
    iters = k + 1 - k0;

    t_prev = t;
    t = (1.0 + sqrt(4.0 * t * t + 1.0)) / 2.0;
    const bool at_floor = p->fixed_mu || mu_k <= p->mu_bar;
    mu = fmax(p->nu * mu, p->mu_bar);

    if (p->tol > 0 && (iters % check_every == 0 || iters == p->max_iter)) {
      HIP_TRY(h, hipMemcpyAsync(h->pinned, w.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(h, hipStreamSynchronize(st));
      const double num = h->pinned[0], den = h->pinned[1];
      crit = den > 0 ? sqrt(num) / sqrt(den) : INFINITY;   // 0/0 counts as not converged
      if (crit <= p->tol && (at_floor || !p->gate_until_floor)) {
        converged = true;
        break;
      }
    }
  }
  if (Xcur != X) {
    // X gets the last iterate and the workspace the one before it (for a
    // continued run); the transform-domain buffer is free to hold one of them
    HIP_TRY(h, hipMemcpyAsync(w.svt.Gh, X, bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(X, Xcur, bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(w.Xb, w.svt.Gh, bytes, hipMemcpyDeviceToDevice, st));
  }
  // nuclear norm of the last iterate (Theorem 21): its transform-domain
  // singular values are the last prox's sigma_i - mu_k
  const double alpha = nuclear_alpha(s);
  if (alpha > 0) {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, lt::launch_sum_scaled(w.svt.nuc, (int)s.P, 1.0 / alpha, w.nucsum, st));
    HIP_TRY(h, hipMemcpyAsync(h->pinned + 5, w.nucsum, sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(h, hipMemcpyAsync(h->pinned, w.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipMemcpyAsync(h->pinned + 2, w.sweep_total, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipMemcpyAsync(h->pinned + 3, w.maxsweep_hits, sizeof(unsigned int),
                            hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipMemcpyAsync(h->pinned + 4, w.rot_total, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipMemcpyAsync(h->pinned + 6, w.slowest_total, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipStreamSynchronize(st));
  const double num = h->pinned[0], den = h->pinned[1];
  crit = den > 0 ? sqrt(num) / sqrt(den) : INFINITY;
  unsigned long long sweeps_total;
  memcpy(&sweeps_total, h->pinned + 2, sizeof(sweeps_total));
  unsigned int hits;
  memcpy(&hits, h->pinned + 3, sizeof(hits));
  unsigned long long rots;
  memcpy(&rots, h->pinned + 4, sizeof(rots));
  unsigned long long slowest;
  memcpy(&slowest, h->pinned + 6, sizeof(slowest));
  if (rep) {
    rep->iters = iters;
    rep->converged = converged ? 1 : 0;
    rep->max_sweeps_hit = (int32_t)hits;
    rep->slowest_sweeps = (int32_t)(slowest > 0x7fffffffULL ? 0x7fffffffULL : slowest);
    rep->last_crit = crit;
    rep->total_sweeps = (int64_t)sweeps_total;
    // slice SVDs performed: one per conjugate pair under Fourier modes
    rep->total_slices = (int64_t)iters * nsvd;
    rep->total_rotations = (int64_t)rots;
    rep->nuclear_norm = alpha > 0 ? h->pinned[5] : NAN;
  }
  if (p->tol > 0 && !converged) return LT_WARN_NOT_CONVERGED;
  if (hits) return LT_WARN_MAXSWEEPS;
  return LT_OK;
}

size_t lt_problem_workspace_bytes(const lt_desc* a, const lt_pga_params* p) {
  Shape s;
  if (parse(nullptr, a, &s) != LT_OK || !p || p->max_iter < 1) return 0;
  if (p->svd.precision != LT_PREC_F32 && p->svd.precision != LT_PREC_BF16X3) return 0;
  if (s.any_dft) return 0;   // the batch engine runs real transforms only
  SvtPlan pl;
  if (!svt_plan(s, problem_precond(s, p), &pl, true) || pl.wide) return 0;   // nor the wide Jacobi
  Carver c(nullptr);
  ProblemWs w;
  carve_problem(c, s, p->svd.precision, p->max_iter, problem_precond(s, p), problem_warm_period(s, p) > 0, &w);
  return c.off + 256;
}

}  // extern "C"

namespace {

// Device record and schedule of one batch problem.  svt_only: a single SVT
// D = D_tau(M) as one tick (mask NULL: every entry observed, so the forward
// pass reads M; X^k = X^{k-1} = X, the output; threshold tau, momentum 0).
int init_problem(lt_handle* h, const lt_problem* p, bool svt_only, double tau) {
  if (!h || !p) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, p->desc, &s);
  if (rc) return rc;
  if (!p->M || (!p->mask && !svt_only) || !p->X) return fail(h, LT_ERR_ARG, "M, mask or X is NULL");
  if (!svt_only && (rc = check_pga_params(h, &p->params))) return rc;
  double tol;
  int max_sweeps, prec;
  resolve_opts(&p->params.svd, &tol, &max_sweeps, &prec);
  if ((rc = check_prec(h, prec))) return rc;
  if ((rc = check_dft(h, s, prec, false))) return rc;
  SvtPlan plan;
  if (!svt_plan(s, problem_precond(s, &p->params), &plan, true))
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld exceeds the Jacobi kernels", s.I1, s.I2);
  if (plan.wide)
    return fail(h, LT_ERR_SHAPE, "slice %lld x %lld: the batch engine takes slices up to 512 columns "
                "(wider ones run through lt_svt_prox / lt_complete_pga)", s.I1, s.I2);
  const lt::JacobiBlkConfig& bcfg = plan.bcfg;
  const bool blk = plan.blocked;
  if (blk) {
    if ((rc = check_blk_lds(h, s, bcfg))) return rc;
  } else {
    int m = plan.jm, n = plan.jn;
    lt::JacobiBatchConfig cfg;
    int ns, qe;
    if (lt::jacobi_batch_config(&m, &n, 1, h->max_lds, 0, &cfg, &ns, &qe) != 0)
      return fail(h, LT_ERR_SHAPE, "slice %lld x %lld exceeds the Jacobi kernels", s.I1, s.I2);
  }
  const size_t need = lt_problem_workspace_bytes(p->desc, &p->params);
  if ((rc = check_ws(h, p->ws, p->ws_bytes, need))) return rc;
  Carver c(p->ws);
  ProblemWs w;
  const bool pc = problem_precond(s, &p->params);
  const int wp = problem_warm_period(s, &p->params);
  carve_problem(c, s, prec, p->params.max_iter, pc, wp > 0, &w);
  hipStream_t st = h->stream;
  if (!svt_only) {
    HIP_TRY(h, lt::launch_fill_zero(w.scratch, 16, st));
    HIP_TRY(h, lt::launch_count_nonfinite(p->M, p->mask, s.nel, w.scratch, st));
    HIP_TRY(h, hipMemcpyAsync(h->pinned, w.scratch, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    if (*reinterpret_cast<unsigned int*>(h->pinned) != 0)
      return fail(h, LT_ERR_NONFINITE, "%u non-finite observed entries in M",
                  *reinterpret_cast<unsigned int*>(h->pinned));
  }
  if ((rc = build_transform(h, s, prec, w.t))) return rc;
  std::vector<double> betas, mus;
  if (svt_only) {
    betas.assign(1, 0.0);
    mus.assign(1, tau);
  } else {
    pga_schedule(&p->params, betas, mus);
  }
  HIP_TRY(h, hipMemcpyAsync(w.betas, betas.data(), betas.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(h, hipMemcpyAsync(w.mus, mus.data(), mus.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (!svt_only) {
    HIP_TRY(h, lt::launch_fill_zero(p->X, (size_t)s.nel * sizeof(float), st));
    HIP_TRY(h, lt::launch_fill_zero(w.Xb, (size_t)s.nel * sizeof(float), st));
  }
  lt::ProbDev d{};
  d.I1 = (int)s.I1;
  d.I2 = (int)s.I2;
  d.P = (int)s.P;
  d.N = s.N;
  d.nel = s.nel;
  d.M = p->M;
  d.mask = p->mask;
  d.Xa = p->X;
  d.Xb = svt_only ? p->X : w.Xb;
  d.Gh = w.Gh;
  d.Bk = w.Bk;
  d.rank = w.rank;
  d.sweeps = w.sweeps;
  d.nuc = w.nuc;
  d.K = w.t.K;
  d.Kinv = w.t.Kinv;
  d.Khi = w.t.Khi;
  d.Klo = w.t.Klo;
  d.Kihi = w.t.Kihi;
  d.Kilo = w.t.Kilo;
  d.betas = w.betas;
  d.mus = w.mus;
  d.partials = w.partials;
  d.n_partials = w.n_partials;
  d.max_iter = p->params.max_iter;
  d.tol = p->params.tol;
  d.mu_bar = p->params.fixed_mu ? p->params.mu0 : p->params.mu_bar;
  d.gate_until_floor = p->params.gate_until_floor;
  d.enabled = 1;
  d.C = w.C;
  d.precond = pc ? 1 : 0;
  d.Z = w.Z;
  d.warm_period = wp;
  if (blk) {
    d.work = w.work;
    d.work_stride = bcfg.work_floats;
    d.blk_b = bcfg.b;
    d.blk_n = bcfg.nblk;
    d.blk_q = bcfg.qeff;
    d.blk_variant = bcfg.variant;
    d.blk_nbuf = bcfg.nbuf;
  }
  d.crit = NAN;
  HIP_TRY(h, hipMemcpyAsync(w.st, &d, sizeof(d), hipMemcpyHostToDevice, st));
  HIP_TRY(h, hipStreamSynchronize(st));   // host vectors and d go out of scope
  return LT_OK;
}

}  // namespace

extern "C" {

int lt_problem_init(lt_handle* h, const lt_problem* p) { return init_problem(h, p, false, 0.0); }

int lt_problem_status(lt_handle* h, const lt_problem* p, lt_pga_report* rep, int32_t* done) {
  if (!h || !p) return LT_ERR_ARG;
  Shape s;
  int rc = parse(h, p->desc, &s);
  if (rc) return rc;
  double tol;
  int max_sweeps, prec;
  resolve_opts(&p->params.svd, &tol, &max_sweeps, &prec);
  Carver c(p->ws);
  ProblemWs w;
  const bool pc = problem_precond(s, &p->params);
  carve_problem(c, s, prec, p->params.max_iter, pc, problem_warm_period(s, &p->params) > 0, &w);
  // on the handle's stream only: work of other streams (other lanes of a
  // server) is not waited for
  static_assert(sizeof(lt::ProbDev) <= kPinnedDoubles * sizeof(double), "staging too small");
  lt::ProbDev d;
  HIP_TRY(h, hipMemcpyAsync(h->pinned, w.st, sizeof(d), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  memcpy(&d, h->pinned, sizeof(d));
  if (d.done && d.parity) {
    // the last iterate is in the second buffer: move it to X and record that
    HIP_TRY(h, hipMemcpyAsync(p->X, w.Xb, (size_t)s.nel * sizeof(float), hipMemcpyDeviceToDevice,
                              h->stream));
    int zero = 0;
    HIP_TRY(h, hipMemcpyAsync(reinterpret_cast<char*>(w.st) + offsetof(lt::ProbDev, parity), &zero,
                              sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  }
  if (done) *done = d.done;
  if (rep) {
    rep->iters = d.iter;
    rep->converged = d.done == 1;
    rep->max_sweeps_hit = (int32_t)d.maxsweep_hits;
    rep->slowest_sweeps = 0;
    rep->last_crit = d.iter > 0 ? d.crit : NAN;
    rep->total_sweeps = (int64_t)d.sweep_total;
    rep->total_slices = (int64_t)d.iter * s.P;
    rep->total_rotations = (int64_t)d.rot_total;
    rep->nuclear_norm = NAN;
    const double alpha = nuclear_alpha(s);
    if (d.iter > 0 && alpha > 0) {
      HIP_TRY(h, lt::launch_sum_scaled(w.nuc, (int)s.P, 1.0 / alpha, w.nuc + s.P, h->stream));
      HIP_TRY(h, hipMemcpyAsync(h->pinned, w.nuc + s.P, sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      rep->nuclear_norm = h->pinned[0];
    }
  }
  return LT_OK;
}

size_t lt_batch_workspace_bytes(int n, const lt_problem* probs) {
  lt_handle tmp;
  tmp.max_lds = 163840;
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
    tmp.max_lds = lds;
  BatchTables T;
  if (build_tables(&tmp, n, probs, 0, &T) != LT_OK) return 0;
  Carver c(nullptr);
  BatchWs w;
  carve_batch(c, T, &w);
  return c.off + 256;
}

int lt_batch_create(lt_handle* h, int n, const lt_problem* probs, void* bws, size_t bws_bytes,
                    int use_graph, int jacobi_lanes, lt_batch** out) {
  if (!h || !out) return LT_ERR_ARG;
  lt_batch* b = new (std::nothrow) lt_batch();
  if (!b) return LT_ERR_ARG;
  b->h = h;
  b->n = n;
  b->use_graph = use_graph;
  if (jacobi_lanes != 0 && jacobi_lanes != 4 && jacobi_lanes != 8 && jacobi_lanes != 16 &&
      jacobi_lanes != 32 && jacobi_lanes != 64) {
    delete b;
    return fail(h, LT_ERR_ARG, "jacobi_lanes must be 0, 4, 8, 16, 32 or 64");
  }
  int rc = build_tables(h, n, probs, jacobi_lanes, &b->T);
  if (rc) {
    delete b;
    return rc;
  }
  Carver c0(nullptr);
  BatchWs tmp;
  carve_batch(c0, b->T, &tmp);
  if ((rc = check_ws(h, bws, bws_bytes, c0.off + 256))) {
    delete b;
    return rc;
  }
  Carver c(bws);
  carve_batch(c, b->T, &b->w);
  hipStream_t st = h->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  hipError_t e = up(b->w.ptrs, b->T.ptrs.data(), b->T.ptrs.size() * sizeof(lt::ProbDev*));
  if (e == hipSuccess) e = up(b->w.gemm, b->T.gemm.data(), b->T.gemm.size() * sizeof(lt::GemmTile));
  if (e == hipSuccess) e = up(b->w.items, b->T.items.data(), b->T.items.size() * sizeof(lt::SvtItem));
  if (e == hipSuccess)
    e = up(b->w.rebuild, b->T.rebuild.data(), b->T.rebuild.size() * sizeof(lt::RebuildTile));
  if (e == hipSuccess) e = up(b->w.gram, b->T.gram.data(), b->T.gram.size() * sizeof(lt::GramTile));
  if (e == hipSuccess) e = up(b->w.chol, b->T.chol.data(), b->T.chol.size() * sizeof(lt::CholItem));
  if (e == hipSuccess) e = up(b->w.cholg, b->T.cholg.data(), b->T.cholg.size() * sizeof(lt::CholItem));
  if (e == hipSuccess) e = up(b->w.blk, b->T.blk.data(), b->T.blk.size() * sizeof(lt::CholItem));
  if (e == hipSuccess)
    e = up(b->w.rebuild_wide, b->T.rebuild_wide.data(), b->T.rebuild_wide.size() * sizeof(lt::RebuildTile));
  if (e == hipSuccess) e = up(b->w.warm, b->T.warm.data(), b->T.warm.size() * sizeof(lt::CholItem));
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && use_graph) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return fail(h, LT_ERR_HIP, "batch setup failed: %s", hipGetErrorString(e));
  }
  *out = b;
  return LT_OK;
}

static hipError_t enqueue_tick(lt_batch* b, hipStream_t s, bool prof) {
  lt_handle* h = b->h;
  const int n = b->n;
  const BatchTables& T = b->T;
  hipError_t e;
  {
    ProfScope ps(prof ? h : nullptr, LT_PROF_OTHER);
    if ((e = lt::launch_batch_begin(b->w.ptrs, n, s)) != hipSuccess) return e;
  }
  {
    ProfScope ps(prof ? h : nullptr, LT_PROF_FORWARD);
    if ((e = lt::launch_gemm_grouped(b->w.ptrs, b->w.gemm, (int)T.gemm.size(), T.prec, 0, s)) != hipSuccess)
      return e;
  }
  if (!T.gram.empty()) {
    ProfScope ps(prof ? h : nullptr, LT_PROF_PRECOND);
    if ((e = lt::launch_gram_tiles(b->w.ptrs, b->w.gram, (int)T.gram.size(), s)) != hipSuccess) return e;
    if ((e = lt::launch_chol_items(b->w.ptrs, b->w.chol, (int)T.chol.size(), T.chol_nmax, s)) != hipSuccess)
      return e;
    if ((e = lt::launch_chol_items(b->w.ptrs, b->w.cholg, (int)T.cholg.size(), T.cholg_nmax, s)) !=
        hipSuccess)
      return e;
    if ((e = lt::launch_warm_product_items(b->w.ptrs, b->w.warm, (int)T.warm.size(), T.warm_nmax, s)) !=
        hipSuccess)
      return e;
  }
  if (!T.blk.empty()) {
    // the long blocked slices first, so the register-resident items fill in behind them
    ProfScope ps(prof ? h : nullptr, LT_PROF_JACOBI);
    int off = 0;
    for (int gi = 0; gi < lt::kBlkNumVariants; ++gi) {
      if (T.blk_count[gi] &&
          (e = lt::launch_jacobi_blk_items(b->w.ptrs, b->w.blk + off, T.blk_count[gi], gi,
                                           T.blk_threads[gi], T.blk_lds[gi], T.tol, T.max_sweeps, s)) !=
              hipSuccess)
        return e;
      off += T.blk_count[gi];
    }
  }
  if (!T.warm.empty()) {
    ProfScope ps(prof ? h : nullptr, LT_PROF_JACOBI);
    int off = 0;
    for (size_t gi = 0; gi < T.warm_cfg.size(); ++gi) {
      if ((e = lt::launch_jacobi_warm_items(b->w.ptrs, b->w.warm + off, T.warm_count[gi], T.warm_cfg[gi], T.tol,
                                            T.max_sweeps, s)) != hipSuccess)
        return e;
      off += T.warm_count[gi];
    }
  }
  if (T.any_reg && !T.items.empty()) {
    ProfScope ps(prof ? h : nullptr, LT_PROF_JACOBI);
    if ((e = lt::launch_jacobi_items(b->w.ptrs, b->w.items, (int)T.items.size(), T.cfg, T.tol,
                                     T.max_sweeps, s)) != hipSuccess)
      return e;
  }
  {
    ProfScope ps(prof ? h : nullptr, LT_PROF_REBUILD);
    if ((e = lt::launch_rebuild_tiles(b->w.ptrs, b->w.rebuild, (int)T.rebuild.size(), 0, T.rebuild_kmax, s)) !=
        hipSuccess)
      return e;
    if ((e = lt::launch_rebuild_tiles(b->w.ptrs, b->w.rebuild_wide, (int)T.rebuild_wide.size(), 1,
                                      T.rebuild_wide_kmax, s)) != hipSuccess)
      return e;
  }
  {
    ProfScope ps(prof ? h : nullptr, LT_PROF_INVERSE);
    if ((e = lt::launch_gemm_grouped(b->w.ptrs, b->w.gemm, (int)T.gemm.size(), T.prec, 1, s)) != hipSuccess)
      return e;
  }
  {
    ProfScope ps(prof ? h : nullptr, LT_PROF_OTHER);
    if ((e = lt::launch_batch_end(b->w.ptrs, n, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

int lt_batch_step(lt_batch* b, int ticks) {
  if (!b || ticks < 0) return LT_ERR_ARG;
  lt_handle* h = b->h;
  if (!b->use_graph) {
    for (int t = 0; t < ticks; ++t) {
      hipError_t e = enqueue_tick(b, h->stream, true);
      if (e != hipSuccess) return fail(h, LT_ERR_HIP, "tick launch failed: %s", hipGetErrorString(e));
    }
    return LT_OK;
  }
  if (!b->exec) {
    HIP_TRY(h, hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    hipError_t e = enqueue_tick(b, b->cap, false);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(h, LT_ERR_HIP, "tick capture failed: %s / %s", hipGetErrorString(e),
                  hipGetErrorString(e2));
    }
    b->graph = g;
    HIP_TRY(h, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  for (int t = 0; t < ticks; ++t) {
    ProfScope ps(h, LT_PROF_OTHER);
    HIP_TRY(h, hipGraphLaunch(b->exec, h->stream));
  }
  return LT_OK;
}

int lt_batch_destroy(lt_batch* b) {
  if (!b) return LT_ERR_ARG;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return LT_OK;
}

// ---- batched SVT: D_i = D_{tau_i}(A_i) for n tensors through one batch tick ----
// Each tensor is a one-iteration problem of the batch engine (every entry
// observed, threshold tau_i, no momentum), so the forward transforms of all
// tensors run as one grouped GEMM, the Jacobi SVDs of all their slices as one
// launch per kernel family, then one rebuild and one grouped inverse GEMM.

}  // extern "C"

namespace {

void svt_batch_problem(const lt_desc* d, const float* A, float* D, double tau, const lt_svd_opts* o,
                       lt_problem* p) {
  memset(p, 0, sizeof(*p));
  p->desc = d;
  p->M = A;
  p->mask = nullptr;
  p->X = D;
  p->params.mu0 = tau;
  p->params.nu = 1.0;
  p->params.mu_bar = tau;
  p->params.max_iter = 1;
  p->params.check_every = 1;
  p->params.fixed_mu = 1;
  if (o) p->params.svd = *o;
  p->params.svd.warm_restart = -1;   // a single SVT: no rotations to carry
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

size_t lt_svt_batched_workspace_bytes(int n, const lt_desc* const* a, const lt_svd_opts* opts) {
  if (n <= 0 || !a) return 0;
  std::vector<lt_problem> probs((size_t)n);
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    svt_batch_problem(a[i], nullptr, nullptr, 1.0, opts, &probs[i]);
    const size_t b = lt_problem_workspace_bytes(a[i], &probs[i].params);
    if (b == 0) return 0;
    total += align256(b);
  }
  const size_t tb = lt_batch_workspace_bytes(n, probs.data());
  if (tb == 0) return 0;
  return total + align256(tb);
}

int lt_svt_prox_batched(lt_handle* h, int n, const lt_desc* const* a, const float* const* A, const double* tau,
                        float* const* D, int32_t* const* rank_out, const lt_svd_opts* opts, void* ws,
                        size_t ws_bytes) {
  if (!h) return LT_ERR_ARG;
  if (n <= 0 || !a || !A || !tau || !D) return fail(h, LT_ERR_ARG, "empty batch or NULL array");
  for (int i = 0; i < n; ++i) {
    if (!a[i] || !A[i] || !D[i]) return fail(h, LT_ERR_ARG, "tensor %d: NULL descriptor or pointer", i);
    if (!(tau[i] >= 0.0) || !isfinite(tau[i])) return fail(h, LT_ERR_ARG, "tau[%d] must be finite and >= 0", i);
    Shape s;
    int rc = parse(h, a[i], &s);
    if (rc) return rc;
    if ((rc = check_dft(h, s, LT_PREC_F32, false))) return rc;
  }
  const size_t need = lt_svt_batched_workspace_bytes(n, a, opts);
  if (need == 0) return fail(h, LT_ERR_SHAPE, "a tensor of the batch is not supported by the batch engine");
  int rc = check_ws(h, ws, ws_bytes, need);
  if (rc) return rc;
  std::vector<lt_problem> probs((size_t)n);
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    svt_batch_problem(a[i], A[i], D[i], tau[i], opts, &probs[i]);
    const size_t b = lt_problem_workspace_bytes(a[i], &probs[i].params);
    probs[i].ws = base + off;
    probs[i].ws_bytes = b;
    off += align256(b);
    if ((rc = init_problem(h, &probs[i], true, tau[i]))) return rc;
  }
  lt_batch b;
  b.h = h;
  b.n = n;
  if ((rc = build_tables(h, n, probs.data(), 0, &b.T))) return rc;
  Carver c(base + off);
  carve_batch(c, b.T, &b.w);
  hipStream_t st = h->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  const BatchTables& T = b.T;
  hipError_t e = up(b.w.ptrs, T.ptrs.data(), T.ptrs.size() * sizeof(lt::ProbDev*));
  if (e == hipSuccess) e = up(b.w.gemm, T.gemm.data(), T.gemm.size() * sizeof(lt::GemmTile));
  if (e == hipSuccess) e = up(b.w.items, T.items.data(), T.items.size() * sizeof(lt::SvtItem));
  if (e == hipSuccess) e = up(b.w.rebuild, T.rebuild.data(), T.rebuild.size() * sizeof(lt::RebuildTile));
  if (e == hipSuccess) e = up(b.w.gram, T.gram.data(), T.gram.size() * sizeof(lt::GramTile));
  if (e == hipSuccess) e = up(b.w.chol, T.chol.data(), T.chol.size() * sizeof(lt::CholItem));
  if (e == hipSuccess) e = up(b.w.cholg, T.cholg.data(), T.cholg.size() * sizeof(lt::CholItem));
  if (e == hipSuccess) e = up(b.w.blk, T.blk.data(), T.blk.size() * sizeof(lt::CholItem));
  if (e == hipSuccess)
    e = up(b.w.rebuild_wide, T.rebuild_wide.data(), T.rebuild_wide.size() * sizeof(lt::RebuildTile));
  if (e == hipSuccess) e = up(b.w.warm, T.warm.data(), T.warm.size() * sizeof(lt::CholItem));
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host tables go out of scope
  if (e == hipSuccess) e = enqueue_tick(&b, st, true);
  if (e != hipSuccess) return fail(h, LT_ERR_HIP, "batched SVT launch failed: %s", hipGetErrorString(e));
  for (int i = 0; rank_out && i < n; ++i) {
    if (!rank_out[i]) continue;
    Shape s;
    (void)parse(h, a[i], &s);
    Carver pc(probs[i].ws);
    ProblemWs pw;
    carve_problem(pc, s, T.prec, 1, problem_precond(s, &probs[i].params), false, &pw);
    HIP_TRY(h, hipMemcpyAsync(rank_out[i], pw.rank, (size_t)s.P * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  }
  return LT_OK;
}

}  // extern "C"
