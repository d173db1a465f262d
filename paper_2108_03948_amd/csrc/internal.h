// Internal declarations shared by the HIP sources of libthzspec.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace tz {

// Unit-circle chirp parameters: A = e^{j 2 pi a}, W = e^{-j 2 pi w}.
// rational != 0: a = pa / q and w = pw / q exactly (0 <= pa, pw < q < 2^62).
struct PhaseParams {
  int rational;
  double a, w;
  int64_t pa, pw, q;
  // off the unit circle (|A| = e^ma, |W| = e^mw): tables carry magnitudes,
  // pre scaled by e^-alpha, conjugate chirp by e^-beta, post by e^(alpha+beta)
  double ma, mw, alpha, beta;
  // outputs scaled by this factor, folded into the conjugate-chirp spectrum
  // (the inverse DFT's 1/N)
  double out_scale = 1.0;
};

// largest single-workgroup FFT length
constexpr int kMaxL = 16384;
constexpr int kMinL = 256;

inline int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Relative time of one workgroup FFT pair of length L (a power of two in
// [kMinL, kMaxL]): measured on the device by tz_autotune() or read from the
// tune cache, else a built-in table (tune.hip).
double fft_pair_cost(int64_t L);

// Bin blocks of one segment on an FFT shorter than *L that cost less than
// `cost`: blocks of at least 256 bins (narrower ones re-read the input too
// often), at most 256 of them.  Updates *L, *Mb, *nblk when one is cheaper.
inline void shorter_blocks(int64_t N, int64_t M, double cost, int *L, int64_t *Mb, int *nblk) {
  const int64_t top = *L;
  for (int64_t l = kMinL; l < top; l <<= 1) {
    const int64_t mb = l - N + 1;
    if (mb < 256) continue;
    const int64_t nb = (M + mb - 1) / mb;
    if (nb > 256) continue;
    const double c = (double)nb * fft_pair_cost(l);
    if (c < cost) {
      cost = c;
      *L = (int)l;
      *Mb = mb;
      *nblk = (int)nb;
    }
  }
}

// FFT length, bin blocks and input segments of the Bluestein path.
// One workgroup FFT of length L <= kMaxL must hold Ns samples and Mb bins
// without wrap-around: Ns + Mb - 1 <= L.  Without `fast` the plan has one
// block and one segment whenever N + M - 1 <= kMaxL (what the split-precision
// kernel, spiral contours and the transfer kernel need); with `fast` bin
// blocks on a shorter FFT are taken when fft_pair_cost says they run faster
// (any L >= Ns + Mb - 1 gives the same bins).  Returns false when more than
// 256 block x segment pieces would be needed.
inline bool czt_shape(int64_t N, int64_t M, int *L, int64_t *Ns, int *nseg, int64_t *Mb, int *nblk,
                      bool fast = false) {
  if (N + M - 1 <= kMaxL) {
    *L = (int)(next_pow2(N + M - 1) < kMinL ? kMinL : next_pow2(N + M - 1));
    *Ns = N;
    *nseg = 1;
    *Mb = M;
    *nblk = 1;
    if (fast) shorter_blocks(N, M, fft_pair_cost(*L), L, Mb, nblk);
    return true;
  }
  int64_t best = -1, bNs = 0, bMb = 0;
  for (int64_t ns = 256; ns <= kMaxL - 256; ns += 256) {
    const int64_t ns_eff = ns < N ? ns : N;
    int64_t mb = kMaxL - ns_eff + 1;
    if (mb > M) mb = M;
    const int64_t cost = ((N + ns_eff - 1) / ns_eff) * ((M + mb - 1) / mb);
    if (best < 0 || cost < best) {
      best = cost;
      bNs = ns_eff;
      bMb = mb;
    }
    if (ns >= N) break;
  }
  const bool ok = best >= 0 && best <= 256;
  if (ok) {
    *L = kMaxL;
    *Ns = bNs;
    *nseg = (int)((N + bNs - 1) / bNs);
    *Mb = bMb;
    *nblk = (int)((M + bMb - 1) / bMb);
  }
  if (fast) {
    // segments add their partial sums into the output (a read and a write per
    // bin and extra segment): weigh them 1.3x
    const double cost = ok ? (double)best * fft_pair_cost(kMaxL) * (*nseg > 1 ? 1.3 : 1.0) : 1e300;
    int l = kMaxL;
    int64_t mb = 0;
    int nb = 0;
    shorter_blocks(N, M, cost, &l, &mb, &nb);
    if (l != kMaxL) {
      *L = l;
      *Ns = N;
      *nseg = 1;
      *Mb = mb;
      *nblk = nb;
      return true;
    }
  }
  return ok;
}

// phase parameters of a CZT over [f1, f2) with M bins, integer hertz:
// a = f1/fs, w = (f2 - f1)/(M fs), exact when the common denominator fits
PhaseParams band_phase(int64_t fs_hz, int64_t f1_hz, int64_t f2_hz, int64_t M);
// phase parameters of the zoom short DFT: W = e^{-j 2 pi / K}, A = e^{-j 2 pi floor(M/2) / K}
PhaseParams zoom_phase(int64_t K, int64_t M);

// ---- plan-time table builders (tables.hip) ----
hipError_t build_twiddles(float2 *tw, int64_t L, hipStream_t s);
hipError_t build_root_table(float2 *w, int64_t n, int64_t q, hipStream_t s);
// c_pre [nblk][Ns], c_post [nseg][nblk][Mb], V [L]; with L1 > 0, V is stored
// in four-step order: V[k1 L2 + k2] holds bin k1 + L1 k2 (L = L1 L2)
hipError_t build_bluestein_tables(const PhaseParams &p, int64_t Ns, int nseg, int64_t Mb, int nblk,
                                  int64_t L, int L1, float2 *c_pre, float2 *c_post, float2 *V, hipStream_t s);
// the twisted tables of the half-length form: c_pre1[blk][n] = c_pre[blk][n] W_L^{n},
// c_post1[blk][k'] = c_post[blk][k'] W_L^{-k'} (one segment), phases in FP64
hipError_t build_half_tables(const PhaseParams &p, int64_t Ns, int64_t Mb, int nblk, int64_t L, float2 *c_pre1,
                             float2 *c_post1, hipStream_t s);
hipError_t build_zoom_tables(double2 *g, int T, double nu_c, double nu_N, double2 *ph, int64_t LD,
                             int64_t D, hipStream_t s);

// ---- hot-path launchers (kernels.hip) ----
// Bluestein CZT: x [B][xs] real (f32/f64) or complex f32, X [B][os] complex f32.
struct CztLaunch {
  const void *x;
  int in_kind;  // 0 = f32 real, 1 = f64 real, 2 = complex f32
  int64_t xs, N;
  int64_t Ns;  // samples per input segment
  int nseg;    // segments (1 unless N + M - 1 exceeds the longest FFT)
  const float2 *c_pre, *c_post, *V, *tw;
  // L = 8192 with one segment, N <= L/2 and Mb <= L/2: premultiply and
  // postmultiply tables twisted by W_L^{n} and W_L^{-k'}, and the twiddles
  // of L/2 points; nullptr otherwise (the length-L kernel runs)
  const float2 *c_pre1 = nullptr, *c_post1 = nullptr, *tw_half = nullptr;
  float2 *X;
  int64_t os, M, Mb;
  int nblk;
  int L;
  int64_t B;
  int precision;  // TZ_FP32 / split
};
// whether a single-pass plan takes the half-length form (twisted tables)
bool czt_half_supported(int L, int nseg, int64_t Ns, int64_t Mb);
hipError_t launch_czt(const CztLaunch &a, hipStream_t s);
// split-precision (MFMA) variant: L in {4096, 8192, 16384}, one segment, one
// bin block, real input
bool czt_mfma_supported(int L, int nseg, int nblk, int in_kind);
hipError_t launch_czt_mfma(const CztLaunch &a, hipStream_t s);

// Transfer function of row pairs (2p, 2p+1): single-pass Bluestein plan
// (one segment, one block), H [B/2][os] complex f32.
struct TransferLaunch {
  const void *x;
  int in_kind;  // 0 = f32, 1 = f64
  int64_t xs, N;
  const float2 *c_pre, *V, *tw;
  // half-length form (L = 8192, N and M within L/2): the postmultiply, the
  // twisted tables and the twiddles of L/2 points; nullptr otherwise
  const float2 *c_post = nullptr, *c_pre1 = nullptr, *c_post1 = nullptr, *tw_half = nullptr;
  float2 *H;
  int64_t os, M;
  int L;
  int64_t pairs;
};
hipError_t launch_czt_transfer(const TransferLaunch &a, hipStream_t s);

// Four-step Bluestein CZT for long traces (one segment, one bin block):
// L = L1 L2 with L1 in {512, 1024} and 256 <= L2 <= 16384.  work holds
// chunk * L complex values; traces run chunk at a time.
struct LongLaunch {
  const void *x;
  int in_kind;  // 0 = f32 real, 1 = f64 real, 2 = complex f32
  int64_t xs, N;
  const float2 *c_pre, *c_post, *Vt;  // Vt in four-step order
  const float2 *tw_col, *tw_row;      // FFT twiddles of lengths L1 and L2
  const float2 *tbig;                 // W_L^i (i < 2048), then W_L^{2048 i}
  float2 *work;
  float2 *X;
  int64_t os, M;
  int L1, L2;
  int64_t B, chunk;
  int precision;  // TZ_FP32, or split precision for the row FFTs (L2 >= 4096)
};
// L1 for a four-step length L (a power of two in [2^17, 2^24]); false otherwise
bool long_shape(int64_t L, int *L1);
hipError_t launch_czt_long(const LongLaunch &a, hipStream_t s);

// ---- mixed-radix FFT of 7-smooth length, one row per workgroup (mixed.hip) ----
constexpr int kMixMinL = 8;
constexpr int kMixMaxL = 20480;  // the whole row in 160 KB of LDS
constexpr int kMixMaxPasses = 16;
struct MixPlan {
  int L, npass;
  int R[kMixMaxPasses];   // radix of each pass (2, 3, 4, 5, 7, 8), first pass first
  int NS[kMixMaxPasses];  // product of the earlier radices
  int TO[kMixMaxPasses];  // offset of the pass's twiddle table, (R - 1) NS entries
  uint32_t nsm[kMixMaxPasses];  // ceil(2^32 / NS) for the division j / NS
  int ntw;                // twiddle entries of all passes
};
// radices of a 7-smooth L in [kMixMinL, kMixMaxL]; false otherwise
bool mix_plan(int64_t L, MixPlan *pl);
// the per-pass twiddle tables of pl (pl.ntw float2), built in FP64
hipError_t build_mix_twiddles(float2 *twp, const MixPlan &pl, hipStream_t s);
struct MixLaunch {
  int mode;  // 0: real f32 rows, 1: real f64 rows (zero-padded FFT); 2: complex rows, inverse DFT;
             // 3: Hermitian half spectra (L/2 + 1 bins) to real rows (X then holds floats)
  const void *x;
  int64_t xs, N;  // row stride (elements), samples per row (modes 0, 1)
  float2 *X;
  int64_t os, nout;  // output row stride, outputs written per row
  MixPlan plan;
  const float2 *tw;  // per-pass twiddle tables (build_mix_twiddles)
  float scale;       // mode 2: 1/L
  int64_t B;
};
hipError_t launch_fft_mixed(const MixLaunch &a, hipStream_t s);
// zero-padded FFT as P sub-transforms of F points (N_fft = P F, F >= N,
// 7-smooth F in [64, 1024], P a multiple of the tile's 8 or 16 rows)
struct SubLaunch {
  int in_kind;  // 0: f32 rows, 1: f64 rows
  int pairs;    // conjugate pairs (P = 16 or 32, F <= 640, one workgroup per row)
  const void *x;
  int64_t xs, N;
  int P;
  float2 *X;
  int64_t os, nout;
  MixPlan plan;       // the F-point FFT
  const float2 *tw;   // its per-pass twiddles
  const float2 *root; // W_{N_fft}^m, m < N_fft
  int64_t B;
};
// F and P for N and N_fft, with the plan of F: 2 = conjugate pairs,
// 1 = tiles of independent sub-transforms, 0 = no F fits
int sub_plan(int64_t N, int64_t nfft, int *F, int *P, MixPlan *pl);
hipError_t launch_fftpad_sub(const SubLaunch &a, hipStream_t s);

// ---- FP64 direct-summation CZT for any contour (direct.hip) ----
struct DirectLaunch {
  int in_kind;  // 0: f32 traces, 1: f64
  const void *x;
  int64_t xs, N;
  double2 *X;  // complex128 bins
  int64_t os, M, B;
  double ma, ta;  // ln|A|, arg A
  double mw, tw;  // ln|W|, arg W
};
hipError_t launch_czt_direct64(const DirectLaunch &a, hipStream_t s);

// ---- direct inverse DFT of power-of-two length (ifft.hip) ----
struct IfftLaunch {
  const float2 *X;   // B rows of L complex, xs apart
  int64_t xs;
  const float2 *tw;  // W_L^m, m < L
  float2 *x;         // B rows of L complex, os apart
  int64_t os, B;
  int L;
};
// L = 256 .. 16384, a power of two
bool ifft_direct_supported(int64_t N);
hipError_t launch_ifft_pow2(const IfftLaunch &a, hipStream_t s);
// split-precision row kernel of the four-step path (mfma.hip): L2 in
// {4096, 8192, 16384}, L1 in {320, 512, 1024}
bool long_rows_mfma_supported(int L1, int L2);
hipError_t launch_long_rows_mfma(const LongLaunch &a, int L1, int64_t nb, hipStream_t s);

// Zero-padded FFT, direct (N_fft = F) or split (N_fft = P * F, F >= N).
struct PadLaunch {
  const void *x;
  int in_kind;  // 0 = f32, 1 = f64
  int64_t xs, N;
  int F, P;
  const float2 *tw, *root;  // root = W_{Nfft}^m, m < Nfft (split only)
  float2 *X;
  int64_t os, nout;
  int64_t B;
};
hipError_t launch_fftpad(const PadLaunch &a, hipStream_t s);

// Zero-padded FFT of real traces, whole spectrum per workgroup:
// N_fft = 2 P F, ceil(N/2) <= F.  root_h = W_{N_fft/2}^m, root_f = W_{N_fft}^m.
struct PadRealLaunch {
  const void *x;
  int in_kind;
  int64_t xs, N;
  int F, P;
  const float2 *tw, *root_h, *root_f;
  float2 *X;
  int64_t os;
  int half;
  int64_t B;
};
bool fftpad_real_supported(int F, int P);
hipError_t launch_fftpad_real(const PadRealLaunch &a, hipStream_t s);

// Zoom front end: u[b][m] = ph[m] sum_t g[t] x[b][mD - t], m < LD.
struct ZoomFrontLaunch {
  const void *x;
  int in_kind;  // 0 = f32 real, 1 = f64 real, 2 = complex f32
  int64_t xs, N, D, LD;
  int T;
  const double2 *g, *ph;  // FP64 modulated taps and mixing phasors
  float2 *u;
  int64_t B;
};
hipError_t launch_zoom_front(const ZoomFrontLaunch &a, hipStream_t s);

// Batched complex transpose: out[b][c][r] = y[b][r][c] (r < R, c < C), nb
// matrices ys and os elements apart.  The host keeps nb * ceil(R/64) *
// ceil(C/64) below 2^32.
struct TransposeLaunch {
  const float2 *y;
  int64_t ys, R, C;
  float2 *out;
  int64_t os, nb;
};
hipError_t launch_transpose(const TransposeLaunch &a, hipStream_t s);

bool fft_length_supported(int64_t L);

// the uneven batch's schedule for one job table, as the autotuner left it
struct BatchTune {
  int topology = 0, inner = 0;
  double ms = -1.0;
};
// the schedule persisted for the job table with this signature (tune.hip)
bool tune_batch_lookup(const std::string &sig, BatchTune *out);
void tune_batch_store(const std::string &sig, const BatchTune &t);
// per log2 L (8 .. 14): measured time of one FFT pair, made current and saved
void tune_set_pair_costs(const double ns[15]);

// message returned by tz_last_error() on this thread
void set_last_error(const char *msg);

// Fault injection for tests of the error paths, read from the environment at
// every check: TZ_FAULT containing "alloc" makes each device allocation of
// the library fail as out of memory (before hipMalloc is called), "graph"
// makes the uneven batch's graph instantiation fail.
bool fault_injected(const char *what);
// hipMalloc / hipMallocAsync through the allocation fault check
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s);
// One line on stderr, prefixed "thzspec: ", when TZ_LOG is set (plan shapes,
// kernel paths, the batch's classes and schedule).
void tz_log(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

}  // namespace tz
