// C-ABI entry points of libthzspec: argument checking, plan selection and
// caching, and launch of the hot-path kernels on the caller's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "thzspec.h"

namespace tz {
namespace {

thread_local std::string g_err;

tz_status fail(tz_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

tz_status hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? TZ_ENOMEM : TZ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define TZ_HIP(call, what)                       \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// ---------------------------------------------------------------------------
// device-side plan storage
// ---------------------------------------------------------------------------
struct DevMem {
  void *p = nullptr;
  DevMem() = default;
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    return dev_malloc(&p, bytes ? bytes : 16);
  }
  template <class T>
  T *as() const { return (T *)p; }
};

// Device scratch of a plan, one buffer per stream: work on one stream is
// ordered, and calls on different streams never share a buffer.
struct Workspace {
  std::map<hipStream_t, std::pair<std::unique_ptr<DevMem>, size_t>> per;
  tz_status get(hipStream_t s, size_t bytes, void **out) {
    auto &e = per[s];
    if (!e.first) e.first.reset(new DevMem());
    if (bytes > e.second) {
      TZ_HIP(hipStreamSynchronize(s), "workspace");  // the old buffer may still be read
      TZ_HIP(e.first->alloc(bytes), "workspace");
      e.second = bytes;
    }
    *out = e.first->p;
    return TZ_OK;
  }
};

// Traces per four-step chunk: the chunk's L-point intermediates (written by
// one kernel, read by the next) are kept near this many bytes so that they
// stay in the last-level cache.
constexpr int64_t kLongChunkBytes = (int64_t)128 << 20;

struct BluePlan {
  int64_t N, M, Ns, Mb;
  int nseg, nblk, L;
  int L1 = 0;  // > 0: four-step long path, L = L1 * (L / L1)
  DevMem c_pre, c_post, V, tbig;
  DevMem c_pre1, c_post1;  // twisted tables of the half-length form (allocated when it applies)
  Workspace work;
};

struct ZoomPlan {
  std::shared_ptr<BluePlan> blue;
  int64_t N, LD, K, D;
  int T;
  DevMem g, ph;
  Workspace u;
};

struct PadPlan {
  int64_t N, Nfft;
  int F, P;
  int realF = 0, realP = 0;  // whole-spectrum real-input kernel (N_fft = 2 realP realF)
  bool mixed = false;        // 7-smooth N_fft: mixed-radix FFT of the zero-padded row
  MixPlan mix{};
  int subF = 0, subP = 0;    // N_fft = subP subF: subP sub-transforms of subF points (mix)
  int subPairs = 0;          // ... as conjugate pairs (real rows, subP = 16 or 32)
  std::shared_ptr<BluePlan> blue;  // Nfft with no fast factorisation
};


struct Device {
  // shared: an explicit plan (tz_plan_create) keeps the tables it uses alive
  // past tz_release_plans()
  std::map<int64_t, std::shared_ptr<DevMem>> twiddles;  // L -> e^{-j 2 pi m/L}
  std::map<int64_t, std::shared_ptr<DevMem>> roots;     // Nfft -> e^{-j 2 pi m/Nfft}
  std::map<int64_t, std::shared_ptr<DevMem>> mixtw;     // L -> per-pass twiddles of the mixed-radix FFT
  std::map<std::string, std::shared_ptr<BluePlan>> blue;
  std::map<std::string, std::shared_ptr<ZoomPlan>> zoom;
  std::map<std::string, std::shared_ptr<PadPlan>> pad;
  Workspace nd_t, nd_u;  // intermediates of the multi-dimensional transforms
};

std::mutex g_mu;
std::map<int, std::unique_ptr<Device>> g_dev;

Device &device_state(int dev) {
  auto &d = g_dev[dev];
  if (!d) d.reset(new Device());
  return *d;
}

std::string phase_key(const PhaseParams &p) {
  char buf[200];
  if (p.rational)
    snprintf(buf, sizeof buf, "r%lld/%lld/%lld", (long long)p.pa, (long long)p.pw, (long long)p.q);
  else if (p.ma != 0.0 || p.mw != 0.0)
    snprintf(buf, sizeof buf, "s%a/%a/%a/%a", p.a, p.w, p.ma, p.mw);
  else
    snprintf(buf, sizeof buf, "f%a/%a", p.a, p.w);
  std::string key = buf;
  if (p.out_scale != 1.0) {
    snprintf(buf, sizeof buf, "x%a", p.out_scale);
    key += buf;
  }
  return key;
}

// tables held by an explicit plan beside its Bluestein / zoom / pad plans
using Keep = std::vector<std::shared_ptr<DevMem>>;

tz_status get_twiddles(Device &d, int64_t L, hipStream_t s, const float2 **out, Keep *keep = nullptr) {
  auto &slot = d.twiddles[L];
  if (!slot) {
    auto m = std::make_shared<DevMem>();
    TZ_HIP(m->alloc(sizeof(float2) * L), "twiddle table");
    TZ_HIP(build_twiddles(m->as<float2>(), L, s), "twiddle build");
    TZ_HIP(hipStreamSynchronize(s), "twiddle build");
    slot = m;
  }
  *out = slot->as<float2>();
  if (keep) keep->push_back(slot);
  return TZ_OK;
}

tz_status get_roots(Device &d, int64_t Nfft, hipStream_t s, const float2 **out, Keep *keep = nullptr) {
  auto &slot = d.roots[Nfft];
  if (!slot) {
    auto m = std::make_shared<DevMem>();
    TZ_HIP(m->alloc(sizeof(float2) * Nfft), "root table");
    TZ_HIP(build_root_table(m->as<float2>(), Nfft, Nfft, s), "root build");
    TZ_HIP(hipStreamSynchronize(s), "root build");
    slot = m;
  }
  *out = slot->as<float2>();
  if (keep) keep->push_back(slot);
  return TZ_OK;
}

// per-pass twiddle tables of a mixed-radix length, cached like the other tables
tz_status get_mix_twiddles(Device &d, const MixPlan &pl, hipStream_t s, const float2 **out, Keep *keep) {
  auto &slot = d.mixtw[pl.L];
  if (!slot) {
    auto m = std::make_shared<DevMem>();
    TZ_HIP(m->alloc(sizeof(float2) * (size_t)std::max(pl.ntw, 1)), "mixed-radix twiddles");
    TZ_HIP(build_mix_twiddles(m->as<float2>(), pl, s), "mixed-radix twiddles");
    TZ_HIP(hipStreamSynchronize(s), "mixed-radix twiddles");
    slot = m;
  }
  *out = slot->as<float2>();
  if (keep) keep->push_back(slot);
  return TZ_OK;
}

// Shape of a Bluestein plan: 1 = single-pass workgroup FFTs (with bin blocks
// and input segments when N + M - 1 > 16384), 0 = four-step long path of
// length *Llong, -1 = too long for either.  The long path is taken when the
// blocks x segments of the single-pass form would transform more points than
// one long FFT pair.
int blue_shape(int64_t N, int64_t M, int *L, int64_t *Ns, int *nseg, int64_t *Mb, int *nblk, int *L1,
               int64_t *Llong, bool fast = false) {
  const bool seg_ok = czt_shape(N, M, L, Ns, nseg, Mb, nblk, fast);
  if (seg_ok && *nseg == 1 && *nblk == 1) return 1;
  // smallest four-step length: a power of two (>= 2^17) or 5 * 2^a
  int64_t Lb = next_pow2(N + M - 1);
  if (Lb < ((int64_t)1 << 17)) Lb = (int64_t)1 << 17;
  int l1p = 0, l15 = 0;
  bool long_ok = long_shape(Lb, &l1p);
  *L1 = l1p;
  for (int64_t L5 = (int64_t)320 * 256; L5 <= (int64_t)320 * kMaxL; L5 *= 2)
    if (L5 >= N + M - 1) {
      if (long_shape(L5, &l15) && (!long_ok || L5 < Lb)) {
        Lb = L5;
        *L1 = l15;
        long_ok = true;
      }
      break;
    }
  if (long_ok && (!seg_ok || (int64_t)*nseg * *nblk * *L > Lb)) {
    *Llong = Lb;
    return 0;
  }
  return seg_ok ? 1 : -1;
}

// fast: bin blocks on a shorter FFT where they run faster (FP32 unit-circle
// callers); otherwise one block whenever N + M - 1 fits one FFT
tz_status get_blue(Device &d, int64_t N, int64_t M, const PhaseParams &p, hipStream_t s,
                   std::shared_ptr<BluePlan> *out, bool fast = false) {
  char kb[96];
  snprintf(kb, sizeof kb, "%lld/%lld/%c/", (long long)N, (long long)M, fast ? 'f' : 'o');
  std::string key = std::string(kb) + phase_key(p);
  auto it = d.blue.find(key);
  if (it != d.blue.end()) {
    *out = it->second;
    return TZ_OK;
  }
  auto pl = std::make_shared<BluePlan>();
  pl->N = N;
  pl->M = M;
  int L1 = 0;
  int64_t Llong = 0;
  const int seg = blue_shape(N, M, &pl->L, &pl->Ns, &pl->nseg, &pl->Mb, &pl->nblk, &L1, &Llong, fast);
  if (seg < 0)
    return fail(TZ_EUNSUPPORTED, "N=%lld, M=%lld: N + M - 1 exceeds the longest FFT (2^24)", (long long)N,
                (long long)M);
  if (seg == 0)
    tz_log("czt plan N=%lld M=%lld: four-step L=%lld = %d x %lld", (long long)N, (long long)M, (long long)Llong,
           L1, (long long)(Llong / L1));
  else
    tz_log("czt plan N=%lld M=%lld: single-pass L=%d, %d segment(s) of %lld samples, %d block(s) of %lld bins",
           (long long)N, (long long)M, pl->L, pl->nseg, (long long)pl->Ns, pl->nblk, (long long)pl->Mb);
  if (seg == 0) {
    pl->L = (int)Llong;
    pl->L1 = L1;
    pl->Ns = N;
    pl->Mb = M;
    pl->nseg = pl->nblk = 1;
    TZ_HIP(pl->tbig.alloc(sizeof(float2) * (2048 + Llong / 2048)), "twiddle table");
    TZ_HIP(build_root_table(pl->tbig.as<float2>(), 2048, Llong, s), "twiddle table");
    TZ_HIP(build_root_table(pl->tbig.as<float2>() + 2048, Llong / 2048, Llong / 2048, s), "twiddle table");
  }
  TZ_HIP(pl->c_pre.alloc(sizeof(float2) * pl->Ns * pl->nblk), "chirp table");
  TZ_HIP(pl->c_post.alloc(sizeof(float2) * pl->Mb * pl->nblk * pl->nseg), "chirp table");
  TZ_HIP(pl->V.alloc(sizeof(float2) * pl->L), "chirp spectrum");
  TZ_HIP(build_bluestein_tables(p, pl->Ns, pl->nseg, pl->Mb, pl->nblk, pl->L, pl->L1, pl->c_pre.as<float2>(),
                                pl->c_post.as<float2>(), pl->V.as<float2>(), s),
         "chirp tables");
  if (!pl->L1 && czt_half_supported(pl->L, pl->nseg, pl->Ns, pl->Mb)) {
    TZ_HIP(pl->c_pre1.alloc(sizeof(float2) * pl->Ns * pl->nblk), "chirp table");
    TZ_HIP(pl->c_post1.alloc(sizeof(float2) * pl->Mb * pl->nblk), "chirp table");
    TZ_HIP(build_half_tables(p, pl->Ns, pl->Mb, pl->nblk, pl->L, pl->c_pre1.as<float2>(),
                             pl->c_post1.as<float2>(), s),
           "chirp tables");
  }
  TZ_HIP(hipStreamSynchronize(s), "chirp tables");
  d.blue[key] = pl;
  *out = pl;
  return TZ_OK;
}

struct Common {
  int64_t B, xs, os;
  int in_kind;
  int precision, flags;
  hipStream_t stream;
};

tz_status check_common(const void *x, int64_t N, void *X, const tz_opts *o, int64_t bins, Common *c) {
  tz_opts def;
  tz_opts_init(&def);
  if (!o) o = &def;
  if (!x || !X) return fail(TZ_EINVAL, "x and X must be device pointers, got NULL");
  if (N < 1) return fail(TZ_EINVAL, "N must be >= 1 (got %lld)", (long long)N);
  c->B = o->batch == 0 ? 1 : o->batch;
  if (c->B < 1) return fail(TZ_EINVAL, "batch must be >= 1 (got %lld)", (long long)o->batch);
  c->xs = o->in_stride == 0 ? N : o->in_stride;
  if (c->xs < N && c->B > 1) return fail(TZ_EINVAL, "in_stride %lld < N %lld", (long long)c->xs, (long long)N);
  c->os = o->out_stride == 0 ? bins : o->out_stride;
  if (c->os < bins && c->B > 1)
    return fail(TZ_EINVAL, "out_stride %lld < bins %lld", (long long)c->os, (long long)bins);
  if (o->in_dtype != TZ_F32 && o->in_dtype != TZ_F64)
    return fail(TZ_EINVAL, "in_dtype must be TZ_F32 or TZ_F64");
  c->in_kind = o->in_dtype == TZ_F64 ? 1 : 0;
  c->precision = o->precision;
  if (c->precision != TZ_FP32 && c->precision != TZ_SPLIT_FP16 && c->precision != TZ_SPLIT_BF16 &&
      c->precision != TZ_FP64)
    return fail(TZ_EINVAL, "unknown precision %d", c->precision);
  c->flags = o->flags;
  c->stream = (hipStream_t)o->stream;
  if (c->B * (c->xs > c->os ? c->xs : c->os) > ((int64_t)1 << 46))
    return fail(TZ_EINVAL, "batch too large");
  return TZ_OK;
}

bool unit(tz_c64 z) { return fabs(hypot(z.re, z.im) - 1.0) <= 1e-12; }
bool finite_nonzero(tz_c64 z) { return isfinite(z.re) && isfinite(z.im) && (z.re != 0.0 || z.im != 0.0); }

double frac01(double v) { return v - floor(v); }

// Off-unit-circle contour (|A| = e^ma, |W| = e^mw): the log magnitudes of
// the premultiply, f(n) = -n ma + n^2 mw / 2 (n < N), and of the conjugate
// chirp, h(m) = -m^2 mw / 2 (-N < m < M), are parabolas; their maxima alpha
// and beta are divided out so that no FFT operand exceeds |x|, and the
// postmultiply carries e^{k^2 mw / 2 + alpha + beta}.  An FFT convolution's
// rounding is set by its largest operands, so outputs that depend on the
// small end of these magnitudes lose relative accuracy roughly as e^{S/2},
// S the sum of the two spreads (max - min of f and of h): the GPU path takes
// contours with S <= 6 (every table magnitude then lies within e^{+-18}).
// Spirals need one bin block and one input segment (single-pass or
// four-step plan).
constexpr double kSpiralSpread = 6.0;

tz_status spiral_scaling(int64_t N, int64_t M, double ma, double mw, PhaseParams *p) {
  if (!isfinite(ma) || !isfinite(mw)) return fail(TZ_EINVAL, "|A| and |W| must be finite and non-zero");
  int L, nseg, nblk, l1;
  int64_t Ns, Mb, Ll;
  if (blue_shape(N, M, &L, &Ns, &nseg, &Mb, &nblk, &l1, &Ll) == 1 && (nseg != 1 || nblk != 1))
    return fail(TZ_EUNSUPPORTED, "spiral contours need N + M - 1 within one FFT pair (no bin blocks)");
  auto f = [&](double n) { return -n * ma + 0.5 * n * n * mw; };
  const double nl = (double)(N - 1);
  double fmax = std::max(f(0.0), f(nl)), fmin = std::min(f(0.0), f(nl));
  if (mw != 0.0) {
    const double nv = std::min(std::max(ma / mw, 0.0), nl);  // vertex of f
    for (double n : {floor(nv), ceil(nv)}) {
      fmax = std::max(fmax, f(n));
      fmin = std::min(fmin, f(n));
    }
  }
  const double mmax = (double)std::max(N - 1, M - 1);
  const double hend = -0.5 * mmax * mmax * mw;  // h at the widest lag; h(0) = 0
  const double hmax = std::max(0.0, hend), hmin = std::min(0.0, hend);
  const double spread = (fmax - fmin) + (hmax - hmin);
  if (spread > kSpiralSpread)
    return fail(TZ_EUNSUPPORTED,
                "spiral contour too steep for FP32 tables: chirp magnitudes spread over e^%.1f (limit e^%.0f)",
                spread, kSpiralSpread);
  p->ma = ma;
  p->mw = mw;
  p->alpha = fmax;
  p->beta = hmax;
  return TZ_OK;
}

// Everything a Bluestein launch needs beyond x and X, resolved through the
// device's table caches (which may allocate and synchronise); exec_blue then
// only launches kernels.  The four-step path runs chunks of traces through a
// workspace of ws bytes.
struct BlueExec {
  std::shared_ptr<BluePlan> pl;
  const float2 *tw = nullptr, *tw_col = nullptr, *tw_row = nullptr;
  const float2 *tw_half = nullptr;  // twiddles of L/2 points (half-length form)
  int64_t chunk = 0;
  size_t ws = 0;
};

tz_status prepare_blue(Device &d, const std::shared_ptr<BluePlan> &pl, int in_kind, const Common &c,
                       hipStream_t s, BlueExec *e, Keep *keep = nullptr) {
  e->pl = pl;
  if (c.precision == TZ_FP64) return fail(TZ_EUNSUPPORTED, "TZ_FP64 evaluates czt() only");
  if (pl->L1) {
    const int L2 = pl->L / pl->L1;
    if (c.precision != TZ_FP32 && !long_rows_mfma_supported(pl->L1, L2))
      return fail(TZ_EUNSUPPORTED, "split precision on the four-step path needs rows of L2 in {1024, 2048, "
                                   "4096, 8192, 16384}; N=%lld, M=%lld has L=%d = %d x %d",
                  (long long)pl->N, (long long)pl->M, pl->L, pl->L1, L2);
    tz_status st = get_twiddles(d, pl->L1, s, &e->tw_col, keep);
    if (st) return st;
    if ((st = get_twiddles(d, L2, s, &e->tw_row, keep))) return st;
    e->chunk = kLongChunkBytes / ((int64_t)pl->L * 8);
    if (e->chunk < 1) e->chunk = 1;
    if (e->chunk > c.B) e->chunk = c.B;
    e->ws = sizeof(float2) * (size_t)pl->L * (size_t)e->chunk;
    return TZ_OK;
  }
  if (c.precision != TZ_FP32 && !czt_mfma_supported(pl->L, pl->nseg, pl->nblk, in_kind))
    return fail(TZ_EUNSUPPORTED, "split precision needs L in {4096, 8192, 16384} with one bin block "
                                 "(N + M - 1 <= 16384) and real input; this plan has L=%d",
                pl->L);
  if (pl->c_pre1.p) {
    tz_status st = get_twiddles(d, pl->L / 2, s, &e->tw_half, keep);
    if (st) return st;
  }
  return get_twiddles(d, pl->L, s, &e->tw, keep);
}

// launches only; M (<= the plan's M) bins per trace, ws of e.ws bytes
tz_status exec_blue(const BlueExec &e, const void *x, int in_kind, void *X, const Common &c, int64_t M, void *ws,
                    hipStream_t s) {
  const BluePlan &pl = *e.pl;
  if (pl.L1) {
    LongLaunch a;
    a.L1 = pl.L1;
    a.L2 = pl.L / pl.L1;
    a.precision = c.precision;
    a.tw_col = e.tw_col;
    a.tw_row = e.tw_row;
    a.chunk = e.chunk;
    a.work = (float2 *)ws;
    a.x = x;
    a.in_kind = in_kind;
    a.xs = c.xs;
    a.N = pl.N;
    a.c_pre = pl.c_pre.as<float2>();
    a.c_post = pl.c_post.as<float2>();
    a.Vt = pl.V.as<float2>();
    a.tbig = pl.tbig.as<float2>();
    a.X = (float2 *)X;
    a.os = c.os;
    a.M = M;
    a.B = c.B;
    TZ_HIP(launch_czt_long(a, s), "czt (four-step) launch");
    return TZ_OK;
  }
  CztLaunch a;
  a.x = x;
  a.in_kind = in_kind;
  a.xs = c.xs;
  a.N = pl.N;
  a.Ns = pl.Ns;
  a.nseg = pl.nseg;
  a.c_pre = pl.c_pre.as<float2>();
  a.c_post = pl.c_post.as<float2>();
  a.V = pl.V.as<float2>();
  a.tw = e.tw;
  a.X = (float2 *)X;
  a.os = c.os;
  a.M = M;
  a.Mb = pl.Mb;
  a.nblk = pl.nblk;
  a.L = pl.L;
  a.B = c.B;
  a.precision = c.precision;
  if (e.tw_half) {
    a.c_pre1 = pl.c_pre1.as<float2>();
    a.c_post1 = pl.c_post1.as<float2>();
    a.tw_half = e.tw_half;
  }
  if (c.precision != TZ_FP32) {
    TZ_HIP(launch_czt_mfma(a, s), "czt (split precision) launch");
  } else {
    TZ_HIP(launch_czt(a, s), "czt launch");
  }
  return TZ_OK;
}

// one-shot form: the four-step workspace is the plan's per-stream buffer;
// M_out < pl.M evaluates only the first M_out bins (0 = all)
tz_status run_blue(Device &d, std::shared_ptr<BluePlan> pl, const void *x, int in_kind, void *X, const Common &c,
                   hipStream_t s, int64_t M_out = 0) {
  BlueExec e;
  tz_status st = prepare_blue(d, pl, in_kind, c, s, &e);
  if (st) return st;
  void *ws = nullptr;
  if (e.ws && (st = pl->work.get(s, e.ws, &ws))) return st;
  return exec_blue(e, x, in_kind, X, c, M_out > 0 ? M_out : pl->M, ws, s);
}

// zoom arguments shared by zoom_fft and zoom_fft_nd; K = round(M fs / (D (f2 - f1)))
tz_status check_zoom(double fs, double f1, double f2, int64_t M, int64_t D, int T, double fc, int64_t *K) {
  if (M < 1 || D < 1) return fail(TZ_EINVAL, "M and D must be >= 1");
  if (!isfinite(fs) || !isfinite(f1) || !isfinite(f2) || fs <= 0.0 || f2 <= f1)
    return fail(TZ_EINVAL, "need finite fs > 0 and f2 > f1");
  if (T < 1) return fail(TZ_EINVAL, "fir_taps must be >= 1");
  if (!(fc > 0.0) || !isfinite(fc)) return fail(TZ_EINVAL, "fir_cutoff_hz must be > 0");
  *K = zoom_short_length(fs, f1, f2, M, D);
  if (*K < 1) return fail(TZ_EINVAL, "short-DFT length K = round(M fs / (D (f2 - f1))) is < 1");
  return TZ_OK;
}

// zoom plan: FIR taps modulated to the band centre, mixing phasors, and the
// short DFT as a CZT of the decimated sequence
tz_status get_zoom(Device &d, int64_t N, double fs, double f1, double f2, int64_t M, int64_t D, int T, double fc,
                   int64_t K, hipStream_t s, std::shared_ptr<ZoomPlan> *out) {
  const int64_t LD = (N + D - 1) / D;
  const double nuN = 0.5 * (f1 + f2) / fs;
  char kb[200];
  snprintf(kb, sizeof kb, "%lld/%lld/%lld/%d/%a/%a/%lld", (long long)N, (long long)M, (long long)D, T,
           nuN - floor(nuN), fc / fs, (long long)K);
  auto &zp = d.zoom[kb];
  if (!zp) {
    auto pl = std::make_shared<ZoomPlan>();
    pl->N = N;
    pl->LD = LD;
    pl->K = K;
    pl->D = D;
    pl->T = T;
    // short DFT: X[k] = sum_m u[m] e^{-j 2 pi (k - floor(M/2)) m / K}: a CZT with
    // W = e^{-j 2 pi / K} and A = e^{-j 2 pi floor(M/2) / K} (rational, q = K)
    const PhaseParams p = zoom_phase(K, M);
    tz_status st = get_blue(d, LD, M, p, s, &pl->blue, true);
    if (st) return st;
    TZ_HIP(pl->g.alloc(sizeof(double2) * T), "zoom taps");
    TZ_HIP(pl->ph.alloc(sizeof(double2) * LD), "zoom phasors");
    TZ_HIP(build_zoom_tables(pl->g.as<double2>(), T, fc / fs, nuN - floor(nuN), pl->ph.as<double2>(), LD, D, s),
           "zoom tables");
    TZ_HIP(hipStreamSynchronize(s), "zoom tables");
    zp = pl;
  }
  *out = zp;
  return TZ_OK;
}

// the zoom's front end writes the decimated rows u (u_bytes), the short DFT
// reads them; both resolved like BlueExec
struct ZoomExec {
  std::shared_ptr<ZoomPlan> z;
  BlueExec b;
  size_t u_bytes = 0;
};

tz_status prepare_zoom(Device &d, const std::shared_ptr<ZoomPlan> &z, const Common &c, hipStream_t s,
                       ZoomExec *e, Keep *keep = nullptr) {
  e->z = z;
  e->u_bytes = (sizeof(float2) * (size_t)z->LD * (size_t)c.B + 255) & ~(size_t)255;
  Common c2 = c;
  c2.xs = z->LD;
  return prepare_blue(d, z->blue, 2, c2, s, &e->b, keep);
}

// front end (mix, FIR, decimate) into u, then the short DFT into X; x holds
// c.B rows c.xs elements apart
tz_status exec_zoom(const ZoomExec &e, const void *x, int in_kind, void *X, const Common &c, void *u, void *ws,
                    hipStream_t s) {
  const ZoomPlan &z = *e.z;
  ZoomFrontLaunch f;
  f.x = x;
  f.in_kind = in_kind;
  f.xs = c.xs;
  f.N = z.N;
  f.D = z.D;
  f.LD = z.LD;
  f.T = z.T;
  f.g = z.g.as<double2>();
  f.ph = z.ph.as<double2>();
  f.u = (float2 *)u;
  f.B = c.B;
  TZ_HIP(launch_zoom_front(f, s), "zoom front-end launch");
  Common c2 = c;
  c2.xs = z.LD;
  return exec_blue(e.b, u, 2, X, c2, z.blue->M, ws, s);
}

// one-shot form: u and the four-step workspace are the plans' per-stream buffers
tz_status run_zoom(Device &d, const std::shared_ptr<ZoomPlan> &zp, const void *x, int in_kind, void *X,
                   const Common &c) {
  ZoomExec e;
  tz_status st = prepare_zoom(d, zp, c, c.stream, &e);
  if (st) return st;
  void *u = nullptr, *ws = nullptr;
  if ((st = zp->u.get(c.stream, e.u_bytes, &u))) return st;
  if (e.b.ws && (st = zp->blue->work.get(c.stream, e.b.ws, &ws))) return st;
  return exec_zoom(e, x, in_kind, X, c, u, ws, c.stream);
}

// ---------------------------------------------------------------------------
// Multi-dimensional transforms.  Pass p applies the 1-D transform of axis
// d-1-p along the contiguous last axis of the current layout and a batched
// transpose then moves the new last axis to the front:
//   [..., N_a] -> transform -> [..., M_a] -> transpose -> [M_a, ...],
// so after d passes the layout is [M_0, ..., M_{d-1}].  Arrays run in chunks
// whose two intermediates stay near kNdChunkBytes each, so that a pass's
// output and its transposed copy are read back from the last-level cache.
// ---------------------------------------------------------------------------
constexpr int64_t kNdChunkBytes = (int64_t)64 << 20;

// run(axis, in, in_kind, rows, in_row_stride, out, out_row_stride)
using AxisRun = std::function<tz_status(int, const void *, int, int64_t, int64_t, float2 *, int64_t)>;

tz_status run_nd(Device &d, int ndim, const int64_t *Ns, const int64_t *Ms, const void *x, void *X,
                 const Common &c, const AxisRun &run) {
  const int64_t esz = c.in_kind == 1 ? 8 : 4;
  if (ndim == 1) return run(0, x, c.in_kind, c.B, c.xs, (float2 *)X, c.os);
  int64_t NN = 1, maxsz = 0, sh[TZ_MAX_DIMS];
  for (int i = 0; i < ndim; ++i) NN *= Ns[i];
  for (int i = 0; i < ndim; ++i) sh[i] = Ns[i];
  for (int p = 0; p < ndim; ++p) {
    const int a = ndim - 1 - p;
    int64_t R = 1;
    for (int i = 0; i < ndim - 1; ++i) R *= sh[i];
    maxsz = std::max(maxsz, R * Ms[a]);
    for (int i = ndim - 1; i > 0; --i) sh[i] = sh[i - 1];
    sh[0] = Ms[a];
  }
  int64_t nb = kNdChunkBytes / (8 * maxsz);
  nb = std::max<int64_t>(1, std::min(nb, c.B));
  // transpose workgroups: nb ceil(R/64) ceil(C/64) <= nb (R C / 4096 + (R + C) / 64 + 1), R C <= maxsz
  if (nb * (maxsz / 4096 + maxsz / 32 + 1) >= ((int64_t)1 << 32))
    return fail(TZ_EUNSUPPORTED, "multi-dimensional intermediate of %lld elements is too large", (long long)maxsz);
  void *tp = nullptr, *up = nullptr;
  tz_status st = d.nd_t.get(c.stream, sizeof(float2) * (size_t)(nb * maxsz), &tp);
  if (st) return st;
  if ((st = d.nd_u.get(c.stream, sizeof(float2) * (size_t)(nb * maxsz), &up))) return st;
  float2 *T = (float2 *)tp, *U = (float2 *)up;
  for (int64_t b0 = 0; b0 < c.B; b0 += nb) {
    const int64_t n = std::min(nb, c.B - b0);
    for (int i = 0; i < ndim; ++i) sh[i] = Ns[i];
    const void *in = (const char *)x + b0 * c.xs * esz;
    int kind = c.in_kind;
    for (int p = 0; p < ndim; ++p) {
      const int a = ndim - 1 - p;
      const int64_t Na = sh[ndim - 1];
      int64_t R = 1;
      for (int i = 0; i < ndim - 1; ++i) R *= sh[i];
      if (p == 0 && c.xs != NN && n > 1) {
        // arrays not packed: each array's lines are uniform on their own
        for (int64_t i = 0; i < n; ++i)
          if ((st = run(a, (const char *)x + (b0 + i) * c.xs * esz, kind, R, Na, T + i * R * Ms[a], Ms[a])))
            return st;
      } else if ((st = run(a, in, kind, n * R, Na, T, Ms[a]))) {
        return st;
      }
      const bool last = p == ndim - 1;
      TransposeLaunch t;
      t.y = T;
      t.ys = R * Ms[a];
      t.R = R;
      t.C = Ms[a];
      t.out = last ? (float2 *)X + b0 * c.os : U;
      t.os = last ? c.os : R * Ms[a];
      t.nb = n;
      TZ_HIP(launch_transpose(t, c.stream), "transpose launch");
      in = U;
      kind = 2;
      for (int i = ndim - 1; i > 0; --i) sh[i] = sh[i - 1];
      sh[0] = Ms[a];
    }
  }
  return TZ_OK;
}

int current_device() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return dev;
}

// reduce n/d (d > 0) and return via num/den
void reduce(__int128 &n, __int128 &d) {
  __int128 a = n < 0 ? -n : n, b = d;
  while (b) {
    __int128 t = a % b;
    a = b;
    b = t;
  }
  if (a > 1) {
    n /= a;
    d /= a;
  }
}

}  // namespace

void set_last_error(const char *msg) { g_err = msg; }

bool fault_injected(const char *what) {
  const char *f = getenv("TZ_FAULT");
  return f && strstr(f, what);
}

hipError_t dev_malloc(void **p, size_t bytes) {
  if (fault_injected("alloc")) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s) {
  if (fault_injected("alloc")) return hipErrorOutOfMemory;
  return hipMallocAsync(p, bytes, s);
}

void tz_log(const char *fmt, ...) {
  if (!getenv("TZ_LOG")) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fprintf(stderr, "thzspec: %s\n", buf);
}

PhaseParams band_phase(int64_t fs_hz, int64_t f1_hz, int64_t f2_hz, int64_t M) {
  __int128 na = f1_hz % fs_hz, da = fs_hz;
  __int128 nw = f2_hz - f1_hz, dw = (__int128)M * fs_hz;
  reduce(na, da);
  reduce(nw, dw);
  __int128 g = da, h = dw;
  while (h) {
    __int128 t = g % h;
    g = h;
    h = t;
  }
  const __int128 q = da / g * dw;
  PhaseParams p{};
  if (q < ((__int128)1 << 61)) {
    p.rational = 1;
    p.q = (int64_t)q;
    p.pa = (int64_t)(na * (q / da) % q);
    p.pw = (int64_t)(nw * (q / dw) % q);
  }
  p.a = frac01((double)f1_hz / (double)fs_hz);
  p.w = frac01((double)(f2_hz - f1_hz) / ((double)M * (double)fs_hz));
  return p;
}

// inverse DFT of N points: W = e^{+j 2 pi / N} = e^{-j 2 pi (N-1)/N}, A = 1,
// outputs scaled by 1/N
PhaseParams idft_phase(int64_t N) {
  PhaseParams p{};
  p.rational = 1;
  p.q = N;
  p.pw = (N - 1) % N;
  p.pa = 0;
  p.w = (double)p.pw / (double)N;
  p.a = 0.0;
  p.out_scale = 1.0 / (double)N;
  return p;
}

PhaseParams zoom_phase(int64_t K, int64_t M) {
  PhaseParams p{};
  p.rational = 1;
  p.q = K;
  p.pw = 1 % K;
  p.pa = (K - (M / 2) % K) % K;
  p.w = 1.0 / (double)K;
  p.a = (double)p.pa / (double)K;
  return p;
}

// ---------------------------------------------------------------------------
// zero-padded FFT: plan lookup, resolution of its tables, launches
// ---------------------------------------------------------------------------
tz_status get_pad(Device &d, int64_t N, int64_t nfft, hipStream_t s, std::shared_ptr<PadPlan> *out) {
  char kb[64];
  snprintf(kb, sizeof kb, "%lld/%lld", (long long)N, (long long)nfft);
  auto &pp = d.pad[kb];
  if (!pp) {
    auto pl = std::make_shared<PadPlan>();
    pl->N = N;
    pl->Nfft = nfft;
    pl->F = 0;
    if (nfft % 2 == 0) {
      const int64_t nh = nfft / 2;
      for (int64_t F = 1024; F <= 2048; F <<= 1)
        if (2 * F >= N && nh % F == 0 && fftpad_real_supported((int)F, (int)(nh / F))) {
          pl->realF = (int)F;
          pl->realP = (int)(nh / F);
          break;
        }
    }
    for (int64_t F = kMinL; F <= kMaxL; F <<= 1)
      if (F >= N && nfft % F == 0) {
        pl->F = (int)F;
        pl->P = (int)(nfft / F);
        break;
      }
    // sub-transforms of a short 7-smooth F (whole 128-byte runs of bins per
    // workgroup) before the power-of-two FFTs of F >= N, whose P workgroups
    // per trace each write every P-th bin
    if (!pl->realF && nfft < ((int64_t)1 << 28)) {
      const int sp = sub_plan(N, nfft, &pl->subF, &pl->subP, &pl->mix);
      if (sp) {
        pl->F = 0;
        pl->subPairs = sp == 2;
      }
    }
    if (!pl->realF && !pl->subF && !pl->F) pl->mixed = mix_plan(nfft, &pl->mix);
    if (pl->realF)
      tz_log("fft_zeropad plan N=%lld N_fft=%lld: real-input kernel, %d FFTs of %d", (long long)N, (long long)nfft,
             pl->realP, pl->realF);
    else if (pl->subF)
      tz_log("fft_zeropad plan N=%lld N_fft=%lld: %d sub-transforms of %d (mixed radix, %d passes%s)", (long long)N,
             (long long)nfft, pl->subP, pl->subF, pl->mix.npass, pl->subPairs ? ", conjugate pairs" : "");
    else if (pl->F)
      tz_log("fft_zeropad plan N=%lld N_fft=%lld: %d FFTs of %d", (long long)N, (long long)nfft, pl->P, pl->F);
    else if (pl->mixed)
      tz_log("fft_zeropad plan N=%lld N_fft=%lld: mixed radix, %d passes", (long long)N, (long long)nfft,
             pl->mix.npass);
    else
      tz_log("fft_zeropad plan N=%lld N_fft=%lld: Bluestein", (long long)N, (long long)nfft);
    if (!pl->F && !pl->subF && !pl->mixed) {  // no fast factorisation: evaluate the same bins as a CZT
      PhaseParams p{};
      p.rational = 1;
      p.q = nfft;
      p.pa = 0;
      p.pw = 1;
      p.a = 0.0;
      p.w = 1.0 / (double)nfft;
      tz_status st = get_blue(d, N, nfft, p, s, &pl->blue, true);
      if (st) return st;
    }
    pp = pl;
  }
  *out = pp;
  return TZ_OK;
}

struct PadExec {
  std::shared_ptr<PadPlan> pp;
  BlueExec b;  // N_fft without a fast factorisation
  const float2 *tw = nullptr, *root = nullptr, *rh = nullptr, *rf = nullptr;
  int64_t nout = 0;
  int half = 0;
};

tz_status prepare_pad(Device &d, const std::shared_ptr<PadPlan> &pp, int in_kind, bool half, const Common &c,
                      hipStream_t s, PadExec *e, Keep *keep = nullptr) {
  e->pp = pp;
  e->half = half ? 1 : 0;
  e->nout = half ? pp->Nfft / 2 + 1 : pp->Nfft;
  if (pp->blue) return prepare_blue(d, pp->blue, in_kind, c, s, &e->b, keep);
  tz_status st;
  if (pp->mixed) {
    if (c.B > INT32_MAX) return fail(TZ_EUNSUPPORTED, "more than 2^31 - 1 traces for N_fft = %lld", (long long)pp->Nfft);
    return get_mix_twiddles(d, pp->mix, s, &e->root, keep);
  }
  if (pp->subF) {
    if (c.B * (pp->subPairs ? 1 : pp->subP / 8) > INT32_MAX)
      return fail(TZ_EUNSUPPORTED, "too many traces for N_fft = %lld in one launch", (long long)pp->Nfft);
    if ((st = get_mix_twiddles(d, pp->mix, s, &e->tw, keep))) return st;
    return get_roots(d, pp->Nfft, s, &e->root, keep);
  }
  if (pp->realF) {
    if ((st = get_twiddles(d, pp->realF, s, &e->tw, keep))) return st;
    if ((st = get_roots(d, pp->Nfft / 2, s, &e->rh, keep))) return st;
    return get_roots(d, pp->Nfft, s, &e->rf, keep);
  }
  if ((st = get_twiddles(d, pp->F, s, &e->tw, keep))) return st;
  if (pp->P > 1 && (st = get_roots(d, pp->Nfft, s, &e->root, keep))) return st;
  return TZ_OK;
}

tz_status exec_pad(const PadExec &e, const void *x, int in_kind, void *X, const Common &c, void *ws, hipStream_t s) {
  const PadPlan &pp = *e.pp;
  // a Bluestein plan evaluates all Nfft bins; with TZ_HALF only the first nout
  if (pp.blue) return exec_blue(e.b, x, in_kind, X, c, e.nout, ws, s);
  if (pp.mixed) {
    MixLaunch a;
    a.mode = in_kind;
    a.x = x;
    a.xs = c.xs;
    a.N = pp.N;
    a.X = (float2 *)X;
    a.os = c.os;
    a.nout = e.nout;
    a.plan = pp.mix;
    a.tw = e.root;
    a.scale = 1.0f;
    a.B = c.B;
    TZ_HIP(launch_fft_mixed(a, s), "fft_zeropad (mixed radix) launch");
    return TZ_OK;
  }
  if (pp.subF) {
    SubLaunch a;
    a.in_kind = in_kind;
    a.pairs = pp.subPairs;
    a.x = x;
    a.xs = c.xs;
    a.N = pp.N;
    a.P = pp.subP;
    a.X = (float2 *)X;
    a.os = c.os;
    a.nout = e.nout;
    a.plan = pp.mix;
    a.tw = e.tw;
    a.root = e.root;
    a.B = c.B;
    TZ_HIP(launch_fftpad_sub(a, s), "fft_zeropad (sub-transforms) launch");
    return TZ_OK;
  }
  if (pp.realF) {
    PadRealLaunch a;
    a.x = x;
    a.in_kind = in_kind;
    a.xs = c.xs;
    a.N = pp.N;
    a.F = pp.realF;
    a.P = pp.realP;
    a.tw = e.tw;
    a.root_h = e.rh;
    a.root_f = e.rf;
    a.X = (float2 *)X;
    a.os = c.os;
    a.half = e.half;
    a.B = c.B;
    TZ_HIP(launch_fftpad_real(a, s), "fft_zeropad launch");
    return TZ_OK;
  }
  PadLaunch a;
  a.x = x;
  a.in_kind = in_kind;
  a.xs = c.xs;
  a.N = pp.N;
  a.F = pp.F;
  a.P = pp.P;
  a.tw = e.tw;
  a.root = e.root;
  a.X = (float2 *)X;
  a.os = c.os;
  a.nout = e.nout;
  a.B = c.B;
  TZ_HIP(launch_fftpad(a, s), "fft_zeropad launch");
  return TZ_OK;
}

tz_status exec_direct(DirectLaunch a, const void *x, void *X, hipStream_t s) {
  a.x = x;
  a.X = (double2 *)X;
  TZ_HIP(launch_czt_direct64(a, s), "czt (FP64 direct) launch");
  return TZ_OK;
}

// launch parameters of the FP64 direct CZT: the contour's logarithms, and a
// check that every term's magnitude |A^{-n} W^{nk}| = e^{-n ln|A| + n k ln|W|}
// (extreme at the corners n in {0, N-1}, k in {0, M-1}) stays in FP64's range
tz_status direct_params(int64_t N, int64_t M, tz_c64 W, tz_c64 A, const Common &c, DirectLaunch *a) {
  if (N > ((int64_t)1 << 28)) return fail(TZ_EUNSUPPORTED, "TZ_FP64 czt takes N up to 2^28");
  if ((M + 255) / 256 * c.B > INT32_MAX) return fail(TZ_EUNSUPPORTED, "too many bins x traces for one launch");
  const double ma = log(hypot(A.re, A.im)), mw = log(hypot(W.re, W.im));
  const double n1 = (double)(N - 1), k1 = (double)(M - 1);
  for (double v : {-n1 * ma, -n1 * ma + n1 * k1 * mw})
    if (!(fabs(v) < 700.0))
      return fail(TZ_EUNSUPPORTED, "contour terms reach e^%.0f, outside FP64's range", v);
  a->in_kind = c.in_kind;
  a->xs = c.xs;
  a->N = N;
  a->os = c.os;
  a->M = M;
  a->B = c.B;
  a->ma = ma;
  a->ta = atan2(A.im, A.re);
  a->mw = mw;
  a->tw = atan2(W.im, W.re);
  return TZ_OK;
}

}  // namespace tz

using namespace tz;

// ===========================================================================
extern "C" {

void tz_opts_init(tz_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->batch = 1;
  o->in_dtype = TZ_F32;
  o->precision = TZ_FP32;
}

const char *tz_last_error(void) { return g_err.c_str(); }
const char *tz_version(void) { return "thzspec 0.2 gfx950"; }

tz_status czt(const void *x, int64_t N, int64_t M, tz_c64 W, tz_c64 A, void *X, const tz_opts *o) {
  if (M < 1) return fail(TZ_EINVAL, "M must be >= 1 (got %lld)", (long long)M);
  if (!finite_nonzero(W) || !finite_nonzero(A)) return fail(TZ_EINVAL, "W and A must be finite and non-zero");
  Common c;
  tz_status st = check_common(x, N, X, o, M, &c);
  if (st) return st;
  if (c.precision == TZ_FP64) {
    DirectLaunch a;
    if ((st = direct_params(N, M, W, A, c, &a))) return st;
    a.x = x;
    a.X = (double2 *)X;
    TZ_HIP(launch_czt_direct64(a, c.stream), "czt (FP64 direct) launch");
    return TZ_OK;
  }
  PhaseParams p{};
  p.rational = 0;
  p.a = frac01(atan2(A.im, A.re) / (2.0 * M_PI));
  p.w = frac01(-atan2(W.im, W.re) / (2.0 * M_PI));
  if (!unit(W) || !unit(A)) {
    if ((st = spiral_scaling(N, M, log(hypot(A.re, A.im)), log(hypot(W.re, W.im)), &p))) return st;
    if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "spiral contours run in FP32 only");
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<BluePlan> pl;
  const bool fast = c.precision == TZ_FP32 && p.ma == 0.0 && p.mw == 0.0;
  if ((st = get_blue(d, N, M, p, c.stream, &pl, fast))) return st;
  return run_blue(d, pl, x, c.in_kind, X, c, c.stream);
}

tz_status czt_transfer(const void *x, int64_t N, int64_t M, tz_c64 W, tz_c64 A, void *H, const tz_opts *o) {
  if (M < 1) return fail(TZ_EINVAL, "M must be >= 1 (got %lld)", (long long)M);
  if (!finite_nonzero(W) || !finite_nonzero(A)) return fail(TZ_EINVAL, "W and A must be finite and non-zero");
  Common c;
  tz_status st = check_common(x, N, H, o, M, &c);
  if (st) return st;
  if (c.B % 2) return fail(TZ_EINVAL, "batch must hold reference/sample pairs (got %lld traces)", (long long)c.B);
  if (!unit(W) || !unit(A))
    return fail(TZ_EUNSUPPORTED, "GPU path evaluates the unit circle only (|A| = |W| = 1)");
  if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "czt_transfer runs in FP32 only");
  PhaseParams p{};
  p.rational = 0;
  p.a = frac01(atan2(A.im, A.re) / (2.0 * M_PI));
  p.w = frac01(-atan2(W.im, W.re) / (2.0 * M_PI));
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<BluePlan> pl;
  if ((st = get_blue(d, N, M, p, c.stream, &pl))) return st;
  if (pl->L1 || pl->nseg != 1 || pl->nblk != 1)
    return fail(TZ_EUNSUPPORTED, "czt_transfer needs N + M - 1 <= 16384 (N=%lld, M=%lld)", (long long)N,
                (long long)M);
  const float2 *tw = nullptr;
  if ((st = get_twiddles(d, pl->L, c.stream, &tw))) return st;
  TransferLaunch a;
  a.x = x;
  a.in_kind = c.in_kind;
  a.xs = c.xs;
  a.N = N;
  a.c_pre = pl->c_pre.as<float2>();
  a.V = pl->V.as<float2>();
  a.tw = tw;
  a.H = (float2 *)H;
  a.os = c.os;
  a.M = M;
  a.L = pl->L;
  a.pairs = c.B / 2;
  if (pl->c_pre1.p) {
    if ((st = get_twiddles(d, pl->L / 2, c.stream, &a.tw_half))) return st;
    a.c_post = pl->c_post.as<float2>();
    a.c_pre1 = pl->c_pre1.as<float2>();
    a.c_post1 = pl->c_post1.as<float2>();
  }
  TZ_HIP(launch_czt_transfer(a, c.stream), "czt_transfer launch");
  return TZ_OK;
}

tz_status czt_band_exact(const void *x, int64_t N, int64_t M, int64_t fs_hz, int64_t f1_hz, int64_t f2_hz,
                         void *X, const tz_opts *o) {
  if (M < 1) return fail(TZ_EINVAL, "M must be >= 1 (got %lld)", (long long)M);
  if (fs_hz < 1 || f1_hz < 0 || f2_hz <= f1_hz) return fail(TZ_EINVAL, "need fs >= 1, f1 >= 0, f2 > f1");
  Common c;
  tz_status st = check_common(x, N, X, o, M, &c);
  if (st) return st;
  const PhaseParams p = band_phase(fs_hz, f1_hz, f2_hz, M);
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<BluePlan> pl;
  if ((st = get_blue(d, N, M, p, c.stream, &pl, c.precision == TZ_FP32))) return st;
  return run_blue(d, pl, x, c.in_kind, X, c, c.stream);
}

tz_status fft_zeropad(const void *x, int64_t N, int64_t n_zeros, void *X, const tz_opts *o) {
  if (n_zeros < 0) return fail(TZ_EINVAL, "n_zeros must be >= 0 (got %lld)", (long long)n_zeros);
  const int64_t nfft = N + n_zeros;
  if (nfft > INT32_MAX) return fail(TZ_EINVAL, "N + n_zeros exceeds 2^31 - 1");
  const bool half = o && (o->flags & TZ_HALF);
  const int64_t nout = half ? nfft / 2 + 1 : nfft;
  Common c;
  tz_status st = check_common(x, N, X, o, nout, &c);
  if (st) return st;
  if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "fft_zeropad runs in FP32 only");
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<PadPlan> pp;
  if ((st = get_pad(d, N, nfft, c.stream, &pp))) return st;
  PadExec e;
  if ((st = prepare_pad(d, pp, c.in_kind, half, c, c.stream, &e))) return st;
  void *ws = nullptr;
  if (e.b.ws && (st = pp->blue->work.get(c.stream, e.b.ws, &ws))) return st;
  return exec_pad(e, x, c.in_kind, X, c, ws, c.stream);
}

}  // extern "C"

namespace {
// the inverse DFT reads complex64 rows and runs in FP32
tz_status check_ifft(Common *c) {
  if (c->in_kind != 0) return fail(TZ_EINVAL, "ifft takes complex64 spectra (in_dtype TZ_F32)");
  if (c->precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "ifft runs in FP32 only");
  c->in_kind = 2;
  return TZ_OK;
}

// the inverse DFT: one FFT per row for power-of-two N up to 16384, else the
// Bluestein form (A = 1, W = e^{+j 2 pi / N}, 1/N in the chirp spectrum)
struct IfftExec {
  int64_t N = 0;
  bool direct = false;  // power of two, k_ifft_pow2
  bool mixed = false;   // 7-smooth, mixed-radix FFT
  bool half = false;    // Hermitian half spectra to real rows (mixed radix, two rows per FFT)
  MixPlan mix{};
  const float2 *tw = nullptr;
  BlueExec b;
};

tz_status prepare_ifft(Device &d, int64_t N, const Common &c, hipStream_t s, IfftExec *e, Keep *keep = nullptr,
                       bool half = false) {
  e->N = N;
  e->half = half;
  if (half) {
    if (c.B > INT32_MAX || !mix_plan(N, &e->mix))
      return fail(TZ_EUNSUPPORTED, "the half-spectrum ifft needs a 7-smooth N from %d to %d (got %lld)", kMixMinL,
                  kMixMaxL, (long long)N);
    e->mixed = true;
    return get_mix_twiddles(d, e->mix, s, &e->tw, keep);
  }
  if (ifft_direct_supported(N) && c.B <= INT32_MAX) {
    e->direct = true;
    return get_twiddles(d, N, s, &e->tw, keep);
  }
  if (c.B <= INT32_MAX && mix_plan(N, &e->mix)) {
    e->mixed = true;
    return get_mix_twiddles(d, e->mix, s, &e->tw, keep);
  }
  std::shared_ptr<BluePlan> pl;
  tz_status st = get_blue(d, N, N, idft_phase(N), s, &pl, true);
  if (st) return st;
  return prepare_blue(d, pl, c.in_kind, c, s, &e->b, keep);
}

tz_status exec_ifft(const IfftExec &e, const void *X, void *x, const Common &c, void *ws, hipStream_t s) {
  if (e.mixed) {
    MixLaunch a;
    a.mode = e.half ? 3 : 2;
    a.x = X;
    a.xs = c.xs;
    a.N = e.N;
    a.X = (float2 *)x;
    a.os = c.os;
    a.nout = e.N;
    a.plan = e.mix;
    a.tw = e.tw;
    a.scale = (float)(1.0 / (double)e.N);
    a.B = c.B;
    TZ_HIP(launch_fft_mixed(a, s), "ifft (mixed radix) launch");
    return TZ_OK;
  }
  if (!e.direct) return exec_blue(e.b, X, c.in_kind, x, c, e.N, ws, s);
  IfftLaunch a;
  a.X = (const float2 *)X;
  a.xs = c.xs;
  a.tw = e.tw;
  a.x = (float2 *)x;
  a.os = c.os;
  a.B = c.B;
  a.L = (int)e.N;
  TZ_HIP(launch_ifft_pow2(a, s), "ifft launch");
  return TZ_OK;
}
}  // namespace

extern "C" {

tz_status ifft(const void *X, int64_t N, void *x, const tz_opts *o) {
  const bool half = o && (o->flags & TZ_HALF);
  Common c;
  // half: input rows of N/2 + 1 bins, output rows of N floats
  tz_status st = check_common(X, half ? N / 2 + 1 : N, x, o, N, &c);
  if (st) return st;
  if (N < 1) return fail(TZ_EINVAL, "N must be >= 1 (got %lld)", (long long)N);
  if ((st = check_ifft(&c))) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  IfftExec e;
  if ((st = prepare_ifft(d, N, c, c.stream, &e, nullptr, half))) return st;
  void *ws = nullptr;
  if (!e.direct && !e.mixed && e.b.ws && (st = e.b.pl->work.get(c.stream, e.b.ws, &ws))) return st;
  return exec_ifft(e, X, x, c, ws, c.stream);
}

tz_status zoom_fft(const void *x, int64_t N, double fs, double f1, double f2, int64_t M, int64_t D, void *X,
                   const tz_opts *o) {
  const int T = (o && o->fir_taps) ? o->fir_taps : 63;
  const double fc = (o && o->fir_cutoff_hz != 0.0) ? o->fir_cutoff_hz : fs / (2.0 * (double)D);
  int64_t K = 0;
  tz_status st = check_zoom(fs, f1, f2, M, D, T, fc, &K);
  if (st) return st;
  Common c;
  if ((st = check_common(x, N, X, o, M, &c))) return st;
  if (c.precision == TZ_FP64) return fail(TZ_EUNSUPPORTED, "TZ_FP64 evaluates czt() only");
  // split precision: the short DFT's four-step rows (prepare_blue refuses
  // the shapes without split kernels); the front end is FP64 either way
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<ZoomPlan> zp;
  if ((st = get_zoom(d, N, fs, f1, f2, M, D, T, fc, K, c.stream, &zp))) return st;
  return run_zoom(d, zp, x, c.in_kind, X, c);
}

tz_status czt_nd(const void *x, int ndim, const tz_czt_axis *axes, void *X, const tz_opts *o) {
  if (ndim < 1 || ndim > TZ_MAX_DIMS) return fail(TZ_EINVAL, "ndim must be 1 .. %d (got %d)", TZ_MAX_DIMS, ndim);
  if (!axes) return fail(TZ_EINVAL, "axes must not be NULL");
  int64_t Ns[TZ_MAX_DIMS], Ms[TZ_MAX_DIMS], NN = 1, MM = 1;
  for (int a = 0; a < ndim; ++a) {
    Ns[a] = axes[a].N;
    Ms[a] = axes[a].M;
    if (Ns[a] < 1 || Ms[a] < 1)
      return fail(TZ_EINVAL, "axis %d: N and M must be >= 1 (got %lld, %lld)", a, (long long)Ns[a],
                  (long long)Ms[a]);
    if (!finite_nonzero(axes[a].W) || !finite_nonzero(axes[a].A))
      return fail(TZ_EINVAL, "axis %d: W and A must be finite and non-zero", a);
    if (Ns[a] > ((int64_t)1 << 31) || Ms[a] > ((int64_t)1 << 31))
      return fail(TZ_EINVAL, "axis %d: N and M must be <= 2^31", a);
    NN *= Ns[a];
    MM *= Ms[a];
    if (NN > ((int64_t)1 << 40) || MM > ((int64_t)1 << 40))
      return fail(TZ_EINVAL, "arrays larger than 2^40 elements");
  }
  Common c;
  tz_status st = check_common(x, NN, X, o, MM, &c);
  if (st) return st;
  if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "multi-dimensional transforms run in FP32 only");
  PhaseParams ps[TZ_MAX_DIMS];
  for (int a = 0; a < ndim; ++a) {
    const tz_c64 W = axes[a].W, A = axes[a].A;
    PhaseParams p{};
    p.a = frac01(atan2(A.im, A.re) / (2.0 * M_PI));
    p.w = frac01(-atan2(W.im, W.re) / (2.0 * M_PI));
    if (!unit(W) || !unit(A))
      if ((st = spiral_scaling(Ns[a], Ms[a], log(hypot(A.re, A.im)), log(hypot(W.re, W.im)), &p))) return st;
    ps[a] = p;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<BluePlan> pl[TZ_MAX_DIMS];
  for (int a = 0; a < ndim; ++a)
    if ((st = get_blue(d, Ns[a], Ms[a], ps[a], c.stream, &pl[a], ps[a].ma == 0.0 && ps[a].mw == 0.0)))
      return st;
  return run_nd(d, ndim, Ns, Ms, x, X, c,
                [&](int a, const void *in, int kind, int64_t rows, int64_t is, float2 *out, int64_t os) {
                  Common ca = c;
                  ca.B = rows;
                  ca.xs = is;
                  ca.os = os;
                  return run_blue(d, pl[a], in, kind, out, ca, c.stream);
                });
}

tz_status zoom_fft_nd(const void *x, int ndim, const tz_zoom_axis *axes, void *X, const tz_opts *o) {
  if (ndim < 1 || ndim > TZ_MAX_DIMS) return fail(TZ_EINVAL, "ndim must be 1 .. %d (got %d)", TZ_MAX_DIMS, ndim);
  if (!axes) return fail(TZ_EINVAL, "axes must not be NULL");
  if (o && o->fir_cutoff_hz != 0.0)
    return fail(TZ_EINVAL, "zoom_fft_nd takes its cut-offs per axis (tz_zoom_axis.fc); fir_cutoff_hz must be 0");
  const int T = (o && o->fir_taps) ? o->fir_taps : 63;
  int64_t Ns[TZ_MAX_DIMS], Ms[TZ_MAX_DIMS], Ks[TZ_MAX_DIMS], NN = 1, MM = 1;
  double fcs[TZ_MAX_DIMS];
  tz_status st;
  for (int a = 0; a < ndim; ++a) {
    const tz_zoom_axis &z = axes[a];
    Ns[a] = z.N;
    Ms[a] = z.M;
    if (z.N < 1) return fail(TZ_EINVAL, "axis %d: N must be >= 1 (got %lld)", a, (long long)z.N);
    fcs[a] = z.fc != 0.0 ? z.fc : z.fs / (2.0 * (double)z.D);
    if ((st = check_zoom(z.fs, z.f1, z.f2, z.M, z.D, T, fcs[a], &Ks[a]))) return st;
    if (Ns[a] > ((int64_t)1 << 31) || Ms[a] > ((int64_t)1 << 31))
      return fail(TZ_EINVAL, "axis %d: N and M must be <= 2^31", a);
    NN *= Ns[a];
    MM *= Ms[a];
    if (NN > ((int64_t)1 << 40) || MM > ((int64_t)1 << 40))
      return fail(TZ_EINVAL, "arrays larger than 2^40 elements");
  }
  Common c;
  if ((st = check_common(x, NN, X, o, MM, &c))) return st;
  if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "multi-dimensional transforms run in FP32 only");
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  std::shared_ptr<ZoomPlan> zp[TZ_MAX_DIMS];
  for (int a = 0; a < ndim; ++a) {
    const tz_zoom_axis &z = axes[a];
    if ((st = get_zoom(d, z.N, z.fs, z.f1, z.f2, z.M, z.D, T, fcs[a], Ks[a], c.stream, &zp[a]))) return st;
  }
  return run_nd(d, ndim, Ns, Ms, x, X, c,
                [&](int a, const void *in, int kind, int64_t rows, int64_t is, float2 *out, int64_t os) {
                  Common ca = c;
                  ca.B = rows;
                  ca.xs = is;
                  ca.os = os;
                  return run_zoom(d, zp[a], in, kind, out, ca);
                });
}

// ---------------------------------------------------------------------------
tz_status czt_band(double fs, double f1, double f2, int64_t M, tz_c64 *W, tz_c64 *A) {
  if (!W || !A) return fail(TZ_EINVAL, "W and A must not be NULL");
  if (M < 1 || !(fs > 0.0) || !isfinite(fs) || !isfinite(f1) || !isfinite(f2) || !(f2 > f1))
    return fail(TZ_EINVAL, "need M >= 1, fs > 0, f2 > f1");
  const double w = (f2 - f1) / ((double)M * fs);
  const double a = f1 / fs;
  W->re = cos(2.0 * M_PI * w);
  W->im = -sin(2.0 * M_PI * w);
  A->re = cos(2.0 * M_PI * a);
  A->im = sin(2.0 * M_PI * a);
  return TZ_OK;
}

int64_t fft_zero_count(double fs, int64_t N_fft, double delta) {
  if (!(fs > 0.0) || N_fft < 1 || !(delta > 0.0) || !isfinite(delta)) return -1;
  const double df = fs / (double)N_fft;
  if (delta >= df) return -1;
  // eq. (5): x = fs N / (fs - delta N) - N
  double xz = fs * (double)N_fft / (fs - delta * (double)N_fft) - (double)N_fft;
  int64_t z = (int64_t)ceil(xz);
  if (z < 0) z = 0;
  // settle rounding at the boundary against eq. (4) itself
  while (z > 0 && df - fs / (double)(N_fft + z - 1) >= delta) --z;
  while (df - fs / (double)(N_fft + z) < delta) ++z;
  return z;
}

int64_t czt_points_for_resolution(double fs, double f1, double f2, int64_t N_fft) {
  if (!(fs > 0.0) || !(f2 > f1) || N_fft < 1) return -1;
  return (int64_t)llround((f2 - f1) / fs * (double)N_fft);
}

int64_t zoom_short_length(double fs, double f1, double f2, int64_t M, int64_t D) {
  if (!(fs > 0.0) || !(f2 > f1) || M < 1 || D < 1 || !isfinite(fs) || !isfinite(f1) || !isfinite(f2))
    return -1;
  return (int64_t)llround((double)M * fs / ((double)D * (f2 - f1)));
}

tz_status czt_plan_shape(int64_t N, int64_t M, int64_t *L, int64_t *blocks) {
  if (N < 1 || M < 1 || !L || !blocks) return fail(TZ_EINVAL, "need N, M >= 1 and non-NULL outputs");
  int l, nseg, nblk, l1;
  int64_t ns, mb, llong;
  const int k = blue_shape(N, M, &l, &ns, &nseg, &mb, &nblk, &l1, &llong, true);
  if (k < 0)
    return fail(TZ_EUNSUPPORTED, "N=%lld, M=%lld: N + M - 1 exceeds the longest FFT (2^24)", (long long)N,
                (long long)M);
  *L = k == 0 ? llong : l;
  *blocks = k == 0 ? 1 : (int64_t)nblk * nseg;
  return TZ_OK;
}

// ---------------------------------------------------------------------------
// explicit plans
// ---------------------------------------------------------------------------
}  // extern "C"

struct tz_plan {
  int kind = 0, dev = 0;
  Common c{};
  int64_t bins = 0;
  BlueExec b;
  ZoomExec z;
  PadExec p;
  IfftExec i;
  bool direct = false;  // czt with TZ_FP64: direct summation
  DirectLaunch dl{};
  Keep keep;            // twiddle / root tables, held past tz_release_plans()
  size_t ws = 0;        // workspace bytes
  size_t u_bytes = 0;   // zoom: the workspace starts with the decimated rows
};

namespace {

// argument checks of the one-shot calls without buffers (the plan gets them
// at execution)
const char kNoBuffer = 0;

tz_status plan_czt_phase(const tz_plan_params &pp, const Common &c, PhaseParams *p) {
  if (pp.M < 1) return fail(TZ_EINVAL, "M must be >= 1 (got %lld)", (long long)pp.M);
  if (!finite_nonzero(pp.W) || !finite_nonzero(pp.A)) return fail(TZ_EINVAL, "W and A must be finite and non-zero");
  *p = PhaseParams{};
  p->rational = 0;
  p->a = frac01(atan2(pp.A.im, pp.A.re) / (2.0 * M_PI));
  p->w = frac01(-atan2(pp.W.im, pp.W.re) / (2.0 * M_PI));
  if (!unit(pp.W) || !unit(pp.A)) {
    tz_status st = spiral_scaling(pp.N, pp.M, log(hypot(pp.A.re, pp.A.im)), log(hypot(pp.W.re, pp.W.im)), p);
    if (st) return st;
    if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "spiral contours run in FP32 only");
  }
  return TZ_OK;
}

}  // namespace

extern "C" {

tz_status tz_plan_create(const tz_plan_params *pp, const tz_opts *o, tz_plan **out) {
  if (!pp || !out) return fail(TZ_EINVAL, "params and plan must not be NULL");
  *out = nullptr;
  std::unique_ptr<tz_plan> P(new tz_plan());
  P->kind = pp->kind;
  Common &c = P->c;
  const void *nb = &kNoBuffer;
  tz_status st = TZ_OK;
  switch (pp->kind) {
    case TZ_PLAN_FFT_ZEROPAD: {
      if (pp->n_zeros < 0) return fail(TZ_EINVAL, "n_zeros must be >= 0 (got %lld)", (long long)pp->n_zeros);
      const int64_t nfft = pp->N + pp->n_zeros;
      if (nfft > INT32_MAX) return fail(TZ_EINVAL, "N + n_zeros exceeds 2^31 - 1");
      const bool half = o && (o->flags & TZ_HALF);
      P->bins = half ? nfft / 2 + 1 : nfft;
      if ((st = check_common(nb, pp->N, (void *)nb, o, P->bins, &c))) return st;
      if (c.precision != TZ_FP32) return fail(TZ_EUNSUPPORTED, "fft_zeropad runs in FP32 only");
      std::lock_guard<std::mutex> lk(g_mu);
      Device &d = device_state(current_device());
      std::shared_ptr<PadPlan> pad;
      if ((st = get_pad(d, pp->N, nfft, c.stream, &pad))) return st;
      if ((st = prepare_pad(d, pad, c.in_kind, half, c, c.stream, &P->p, &P->keep))) return st;
      P->ws = P->p.b.ws;
      break;
    }
    case TZ_PLAN_CZT:
    case TZ_PLAN_CZT_BAND_EXACT: {
      PhaseParams ph{};
      P->bins = pp->M;
      if ((st = check_common(nb, pp->N, (void *)nb, o, pp->M < 1 ? 1 : pp->M, &c))) return st;
      bool fast = c.precision == TZ_FP32;
      if (pp->kind == TZ_PLAN_CZT && c.precision == TZ_FP64) {
        if (pp->M < 1) return fail(TZ_EINVAL, "M must be >= 1 (got %lld)", (long long)pp->M);
        if (!finite_nonzero(pp->W) || !finite_nonzero(pp->A))
          return fail(TZ_EINVAL, "W and A must be finite and non-zero");
        if ((st = direct_params(pp->N, pp->M, pp->W, pp->A, c, &P->dl))) return st;
        P->direct = true;
        break;
      }
      if (pp->kind == TZ_PLAN_CZT) {
        if ((st = plan_czt_phase(*pp, c, &ph))) return st;
        fast = fast && ph.ma == 0.0 && ph.mw == 0.0;
      } else {
        if (pp->M < 1) return fail(TZ_EINVAL, "M must be >= 1 (got %lld)", (long long)pp->M);
        if (pp->fs_hz < 1 || pp->f1_hz < 0 || pp->f2_hz <= pp->f1_hz)
          return fail(TZ_EINVAL, "need fs >= 1, f1 >= 0, f2 > f1");
        ph = band_phase(pp->fs_hz, pp->f1_hz, pp->f2_hz, pp->M);
      }
      std::lock_guard<std::mutex> lk(g_mu);
      Device &d = device_state(current_device());
      std::shared_ptr<BluePlan> pl;
      if ((st = get_blue(d, pp->N, pp->M, ph, c.stream, &pl, fast))) return st;
      if ((st = prepare_blue(d, pl, c.in_kind, c, c.stream, &P->b, &P->keep))) return st;
      P->ws = P->b.ws;
      break;
    }
    case TZ_PLAN_ZOOM: {
      const int T = (o && o->fir_taps) ? o->fir_taps : 63;
      const double fc = (o && o->fir_cutoff_hz != 0.0) ? o->fir_cutoff_hz : pp->fs / (2.0 * (double)pp->D);
      int64_t K = 0;
      if ((st = check_zoom(pp->fs, pp->f1, pp->f2, pp->M, pp->D, T, fc, &K))) return st;
      P->bins = pp->M;
      if ((st = check_common(nb, pp->N, (void *)nb, o, pp->M, &c))) return st;
      if (c.precision == TZ_FP64) return fail(TZ_EUNSUPPORTED, "TZ_FP64 evaluates czt() only");
      std::lock_guard<std::mutex> lk(g_mu);
      Device &d = device_state(current_device());
      std::shared_ptr<ZoomPlan> zp;
      if ((st = get_zoom(d, pp->N, pp->fs, pp->f1, pp->f2, pp->M, pp->D, T, fc, K, c.stream, &zp))) return st;
      if ((st = prepare_zoom(d, zp, c, c.stream, &P->z, &P->keep))) return st;
      P->u_bytes = P->z.u_bytes;
      P->ws = P->z.u_bytes + P->z.b.ws;
      break;
    }
    case TZ_PLAN_IFFT: {
      const bool half = o && (o->flags & TZ_HALF);
      P->bins = pp->N;
      if (pp->N < 1) return fail(TZ_EINVAL, "N must be >= 1 (got %lld)", (long long)pp->N);
      if ((st = check_common(nb, half ? pp->N / 2 + 1 : pp->N, (void *)nb, o, pp->N, &c))) return st;
      if ((st = check_ifft(&c))) return st;
      std::lock_guard<std::mutex> lk(g_mu);
      Device &d = device_state(current_device());
      if ((st = prepare_ifft(d, pp->N, c, c.stream, &P->i, &P->keep, half))) return st;
      P->ws = P->i.direct ? 0 : P->i.b.ws;
      break;
    }
    default:
      return fail(TZ_EINVAL, "unknown plan kind %d", pp->kind);
  }
  P->dev = current_device();
  *out = P.release();
  return TZ_OK;
}

tz_status tz_plan_workspace(const tz_plan *P, size_t *bytes) {
  if (!P || !bytes) return fail(TZ_EINVAL, "plan and bytes must not be NULL");
  *bytes = P->ws;
  return TZ_OK;
}

tz_status tz_plan_execute(const tz_plan *P, const void *x, void *X, void *workspace, void *stream) {
  if (!P) return fail(TZ_EINVAL, "plan must not be NULL");
  if (!x || !X) return fail(TZ_EINVAL, "x and X must be device pointers, got NULL");
  if (P->ws && !workspace) return fail(TZ_EINVAL, "this plan needs a workspace of %zu bytes", P->ws);
  const int dev = current_device();
  if (dev != P->dev) return fail(TZ_EINVAL, "plan built on device %d, current device is %d", P->dev, dev);
  const hipStream_t s = (hipStream_t)stream;
  const Common &c = P->c;
  if (P->direct) return exec_direct(P->dl, x, X, s);
  switch (P->kind) {
    case TZ_PLAN_FFT_ZEROPAD: return exec_pad(P->p, x, c.in_kind, X, c, workspace, s);
    case TZ_PLAN_IFFT: return exec_ifft(P->i, x, X, c, workspace, s);
    case TZ_PLAN_ZOOM:
      return exec_zoom(P->z, x, c.in_kind, X, c, workspace, (char *)workspace + P->u_bytes, s);
    default: return exec_blue(P->b, x, c.in_kind, X, c, P->bins, workspace, s);
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free execution: the workspace is a fixed device array of this
// library, one copy per GPU, shared by every call on that GPU
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TZ_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch;  // device -> address of its copy of `scratch`

// the device address of this GPU's copy, looked up once per device with that
// device current (the array's name is only a host-side stand-in)
tz_status static_scratch(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void *p = nullptr;
    TZ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "static scratch address");
    it = g_scratch.emplace(dev, p).first;
  }
  *out = it->second;
  return TZ_OK;
}

// Fit a Bluestein execution into `bytes` of workspace: single-pass plans
// need none; the four-step path runs fewer traces per chunk (the chunk only
// groups traces, every trace is computed the same way).  False if even one
// trace's intermediates do not fit.
bool fit_blue(BlueExec &e, size_t bytes) {
  if (!e.ws) return true;
  if (!e.pl->L1) return e.ws <= bytes;
  const size_t per = sizeof(float2) * (size_t)e.pl->L;
  const int64_t fit = (int64_t)(bytes / per);
  if (fit < 1) return false;
  if (e.chunk > fit) e.chunk = fit;
  e.ws = per * (size_t)e.chunk;
  return true;
}

}  // namespace

extern "C" {

tz_status tz_plan_execute_static(const tz_plan *P, const void *x, void *X, void *stream) {
  if (!P) return fail(TZ_EINVAL, "plan must not be NULL");
  if (!x || !X) return fail(TZ_EINVAL, "x and X must be device pointers, got NULL");
  const int dev = current_device();
  if (dev != P->dev) return fail(TZ_EINVAL, "plan built on device %d, current device is %d", P->dev, dev);
  const size_t cap = TZ_STATIC_SCRATCH_BYTES;
  const hipStream_t s = (hipStream_t)stream;
  const Common &c = P->c;
  if (P->direct) return exec_direct(P->dl, x, X, s);  // no scratch
  bool fits = true;
  BlueExec b;
  switch (P->kind) {
    case TZ_PLAN_FFT_ZEROPAD: b = P->p.b; break;
    case TZ_PLAN_IFFT: b = P->i.b; break;
    case TZ_PLAN_ZOOM:
      b = P->z.b;
      fits = P->u_bytes <= cap;
      break;
    default: b = P->b; break;
  }
  const size_t rest = fits ? cap - (P->kind == TZ_PLAN_ZOOM ? P->u_bytes : 0) : 0;
  if (!fits || !fit_blue(b, rest))
    return fail(TZ_EINVAL,
                "plan needs more workspace than the static scratch holds (%zu bytes; the plan's own execution "
                "takes %zu): use tz_plan_execute with a workspace",
                cap, P->ws);
  void *ws = nullptr;
  tz_status st = static_scratch(dev, &ws);
  if (st) return st;
  switch (P->kind) {
    case TZ_PLAN_FFT_ZEROPAD: {
      PadExec e = P->p;
      e.b = b;
      return exec_pad(e, x, c.in_kind, X, c, ws, s);
    }
    case TZ_PLAN_IFFT: {
      IfftExec e = P->i;
      e.b = b;
      return exec_ifft(e, x, X, c, ws, s);
    }
    case TZ_PLAN_ZOOM: {
      ZoomExec e = P->z;
      e.b = b;
      return exec_zoom(e, x, c.in_kind, X, c, ws, (char *)ws + P->u_bytes, s);
    }
    default: return exec_blue(b, x, c.in_kind, X, c, P->bins, ws, s);
  }
}

void tz_plan_destroy(tz_plan *P) {
  if (!P) return;
  (void)hipDeviceSynchronize();  // work that reads its tables may be in flight
  std::lock_guard<std::mutex> lk(g_mu);
  delete P;
}

tz_status tz_bin_freqs(const tz_plan_params *pp, const tz_opts *o, double *f) {
  if (!pp || !f) return fail(TZ_EINVAL, "params and f_out must not be NULL");
  switch (pp->kind) {
    case TZ_PLAN_FFT_ZEROPAD: {
      if (pp->N < 1 || pp->n_zeros < 0 || !(pp->fs > 0.0) || !isfinite(pp->fs))
        return fail(TZ_EINVAL, "need N >= 1, n_zeros >= 0 and finite fs > 0");
      const int64_t nfft = pp->N + pp->n_zeros;
      const int64_t nout = (o && (o->flags & TZ_HALF)) ? nfft / 2 + 1 : nfft;
      for (int64_t k = 0; k < nout; ++k) f[k] = (double)k * pp->fs / (double)nfft;
      return TZ_OK;
    }
    case TZ_PLAN_CZT: {
      if (pp->M < 1 || !finite_nonzero(pp->W) || !finite_nonzero(pp->A) || !(pp->fs > 0.0) || !isfinite(pp->fs))
        return fail(TZ_EINVAL, "need M >= 1, finite non-zero W and A, finite fs > 0");
      const double na = atan2(pp->A.im, pp->A.re) / (2.0 * M_PI), nw = -atan2(pp->W.im, pp->W.re) / (2.0 * M_PI);
      for (int64_t k = 0; k < pp->M; ++k) f[k] = pp->fs * (na + (double)k * nw);
      return TZ_OK;
    }
    case TZ_PLAN_CZT_BAND_EXACT: {
      if (pp->M < 1 || pp->fs_hz < 1 || pp->f1_hz < 0 || pp->f2_hz <= pp->f1_hz)
        return fail(TZ_EINVAL, "need M >= 1, fs >= 1, f1 >= 0, f2 > f1");
      const double df = (double)(pp->f2_hz - pp->f1_hz) / (double)pp->M;
      for (int64_t k = 0; k < pp->M; ++k) f[k] = (double)pp->f1_hz + (double)k * df;
      return TZ_OK;
    }
    case TZ_PLAN_ZOOM: {
      const int T = (o && o->fir_taps) ? o->fir_taps : 63;
      const double fc = (o && o->fir_cutoff_hz != 0.0) ? o->fir_cutoff_hz : pp->fs / (2.0 * (double)pp->D);
      int64_t K = 0;
      tz_status st = check_zoom(pp->fs, pp->f1, pp->f2, pp->M, pp->D, T, fc, &K);
      if (st) return st;
      const double fN = 0.5 * (pp->f1 + pp->f2), step = pp->fs / ((double)pp->D * (double)K);
      for (int64_t k = 0; k < pp->M; ++k) f[k] = fN + (double)(k - pp->M / 2) * step;
      return TZ_OK;
    }
    case TZ_PLAN_IFFT:
      return fail(TZ_EINVAL, "ifft writes time samples (t = n / fs), not frequency bins");
    default:
      return fail(TZ_EINVAL, "unknown plan kind %d", pp->kind);
  }
}

tz_status tz_autotune(const tz_opts *o) {
  tz_opts def;
  tz_opts_init(&def);
  if (!o) o = &def;
  hipStream_t s = (hipStream_t)o->stream;
  std::lock_guard<std::mutex> lk(g_mu);
  Device &d = device_state(current_device());
  // one single-block Bluestein pair per length, N = M = L/2, on 2^25 points
  // of zero samples (the time does not depend on the values): best of three
  double ns[15] = {};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TZ_HIP(hipEventCreate(&e0), "autotune events");
  std::unique_ptr<void, void (*)(void *)> g0(e0, [](void *e) { (void)hipEventDestroy((hipEvent_t)e); });
  TZ_HIP(hipEventCreate(&e1), "autotune events");
  std::unique_ptr<void, void (*)(void *)> g1(e1, [](void *e) { (void)hipEventDestroy((hipEvent_t)e); });
  for (int lc = 8; lc <= 14; ++lc) {
    const int64_t L = (int64_t)1 << lc, N = L / 2, M = L / 2, B = ((int64_t)1 << 25) / L;
    const PhaseParams p = band_phase(1000000, 0, 500000, M);
    std::shared_ptr<BluePlan> pl;
    tz_status st = get_blue(d, N, M, p, s, &pl, false);
    if (st) return st;
    if (pl->L != L || pl->nblk != 1 || pl->nseg != 1)
      return fail(TZ_EDEVICE, "autotune: unexpected plan for L=%lld", (long long)L);
    Common c{B, N, M, 0, TZ_FP32, 0, s};
    BlueExec e;
    if ((st = prepare_blue(d, pl, 0, c, s, &e))) return st;
    DevMem x, X;
    TZ_HIP(x.alloc(sizeof(float) * (size_t)(B * N)), "autotune input");
    TZ_HIP(X.alloc(sizeof(float2) * (size_t)(B * M)), "autotune output");
    TZ_HIP(hipMemsetAsync(x.p, 0, sizeof(float) * (size_t)(B * N), s), "autotune input");
    if ((st = exec_blue(e, x.p, 0, X.p, c, M, nullptr, s))) return st;  // warm
    float best = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      TZ_HIP(hipEventRecord(e0, s), "autotune");
      if ((st = exec_blue(e, x.p, 0, X.p, c, M, nullptr, s))) return st;
      TZ_HIP(hipEventRecord(e1, s), "autotune");
      TZ_HIP(hipEventSynchronize(e1), "autotune");
      float ms = 0.f;
      TZ_HIP(hipEventElapsedTime(&ms, e0, e1), "autotune");
      if (rep == 0 || ms < best) best = ms;
    }
    ns[lc] = (double)best * 1e6 / (double)B;
    tz_log("autotune: FFT pair of %lld points: %.1f ns (%lld traces)", (long long)L, ns[lc], (long long)B);
  }
  tune_set_pair_costs(ns);
  // one-shot plans made with the old costs are dropped (explicit plans keep
  // the shape they were created with)
  d.blue.clear();
  d.pad.clear();
  d.zoom.clear();
  return TZ_OK;
}

void tz_release_plans(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  g_dev.clear();
}

}  // extern "C"
