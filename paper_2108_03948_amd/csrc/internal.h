// Internal declarations shared by the HIP sources of libthzspec.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tz {

// Unit-circle chirp parameters: A = e^{j 2 pi a}, W = e^{-j 2 pi w}.
// rational != 0: a = pa / q and w = pw / q exactly (0 <= pa, pw < q < 2^62).
struct PhaseParams {
  int rational;
  double a, w;
  int64_t pa, pw, q;
};

// largest single-workgroup FFT length
constexpr int kMaxL = 16384;
constexpr int kMinL = 256;

// ---- plan-time table builders (tables.hip) ----
hipError_t build_twiddles(float2 *tw, int64_t L, hipStream_t s);
hipError_t build_root_table(float2 *w, int64_t n, int64_t q, hipStream_t s);
// c_pre [nblk][Ns], c_post [nseg][nblk][Mb], V [L]
hipError_t build_bluestein_tables(const PhaseParams &p, int64_t Ns, int nseg, int64_t Mb, int nblk,
                                  int64_t L, float2 *c_pre, float2 *c_post, float2 *V, hipStream_t s);
hipError_t build_zoom_tables(float2 *g, int T, double nu_c, double nu_N, float2 *ph, int64_t LD,
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
  float2 *X;
  int64_t os, M, Mb;
  int nblk;
  int L;
  int64_t B;
  int precision;  // TZ_FP32 / split
};
hipError_t launch_czt(const CztLaunch &a, hipStream_t s);

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
  int in_kind;
  int64_t xs, N, D, LD;
  int T;
  const float2 *g, *ph;
  float2 *u;
  int64_t B;
};
hipError_t launch_zoom_front(const ZoomFrontLaunch &a, hipStream_t s);

bool fft_length_supported(int64_t L);

}  // namespace tz
