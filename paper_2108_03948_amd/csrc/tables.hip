// Plan-time tables, computed on the GPU in double precision and rounded once
// to float: FFT twiddles, CZT chirps (eq. (13)) and the spectrum of the
// conjugate chirp (the FFT of eq. (15)'s second factor), zoom FIR taps and
// mixing phasors (eqs. (7), (8), (10)).  None of this runs per batch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.h"
#include "phase.h"

namespace tz {

// c_pre[blk][n] = A^{-n} W^{blk Mb n} W^{n^2/2}: block blk evaluates bins
// blk*Mb + k', i.e. the CZT with start point A W^{-blk Mb}.  With twist = L > 0
// the table is c_pre[blk][n] W_L^{n} (the odd-bin half of a split FFT).
__global__ void k_chirp_pre(float2 *c_pre, int64_t N, int nblk, int64_t Mb, PhaseParams p, int64_t twist) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * nblk) return;
  int64_t blk = i / N, n = i % N;
  double cyc = chirp_cycles(p, n, true);
  if (blk) cyc += shift_cycles(p, blk * Mb, n);
  if (twist) cyc += (double)(n % twist) / (double)twist;  // W_L^n = e^{-j 2 pi n/L}
  if (blk || twist) cyc -= floor(cyc);
  // (spiral contours come with one block and one segment)
  const double dn = (double)n;
  c_pre[i] = spiral(p) ? scaled_cycles(cyc, -dn * p.ma + 0.5 * dn * dn * p.mw - p.alpha) : unit_cycles(cyc);
}

// c_post[s][blk][k'] = W^{k'^2/2} A^{-s Ns} W^{(blk Mb + k') s Ns}; with
// twist = L > 0 (one segment) times W_L^{-k'}
__global__ void k_chirp_post(float2 *c_post, int64_t Ns, int nseg, int64_t Mb, int nblk, PhaseParams p,
                             int64_t twist) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mb * nblk * nseg) return;
  const int64_t k = i % Mb, blk = (i / Mb) % nblk, seg = i / (Mb * nblk);
  double cyc = chirp_cycles(p, k, false);
  if (seg) {
    const int64_t n0 = seg * Ns;
    if (p.rational) {
      const uint64_t q = (uint64_t)p.q;
      uint64_t r = mulmod((uint64_t)p.pa, (uint64_t)n0 % q, q);
      r = (r + mulmod(mulmod((uint64_t)p.pw, (uint64_t)(blk * Mb + k) % q, q), (uint64_t)n0 % q, q)) % q;
      cyc += (double)r / (double)q;
    } else {
      cyc += frac_mul(p.a, (double)n0) + frac_mul(p.w, (double)(blk * Mb + k) * (double)n0);
    }
    cyc -= floor(cyc);
  }
  if (twist) {
    cyc -= (double)(k % twist) / (double)twist;
    cyc -= floor(cyc);
  }
  const double dk = (double)k;
  c_post[i] = spiral(p) ? scaled_cycles(cyc, 0.5 * dk * dk * p.mw + p.alpha + p.beta) : unit_cycles(cyc);
}

// v[l] = W^{-l^2/2} for l < Mb and v[L-l] = W^{-l^2/2} for 1 <= l < N; else 0
__global__ void k_chirp_conj(double2 *v, int64_t L, int64_t N, int64_t Mb, PhaseParams p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L) return;
  int64_t l = -1;
  if (i < Mb) l = i;
  else if (L - i < N) l = L - i;
  if (l < 0) {
    v[i] = make_double2(0.0, 0.0);
    return;
  }
  double cyc = chirp_cycles(p, l, false);  // w l^2/2: W^{+l^2/2} = e^{-j 2 pi cyc}
  double s, c;
  sincospi(2.0 * cyc, &s, &c);                 // conjugate: e^{+j 2 pi cyc}
  // |W^{-l^2/2}| = e^{-mw l^2/2}, scaled by e^{-beta}
  const double m = spiral(p) ? exp(-0.5 * (double)l * (double)l * p.mw - p.beta) : 1.0;
  v[i] = make_double2(m * c, m * s);
}

// FFT twiddles tw[m] = e^{-j 2 pi m / L}
__global__ void k_twiddles(float2 *tw, int64_t L) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= L) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)L, &s, &c);
  tw[m] = make_float2((float)c, (float)s);
}

// ---------------------------------------------------------------------------
// double-precision Stockham FFT through global memory (plan time only)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// one radix-R pass (R = 2, 3, 4 or 5), ns = product of the previous radices
__global__ void k_fft64_pass(const double2 *in, double2 *out, int64_t L, int R, int64_t ns) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L / R) return;
  double2 v[5];
  const int64_t jm = j % ns;
  for (int r = 0; r < R; ++r) {
    double2 a = in[j + r * (L / R)];
    if (r && jm) {
      double s, c;
      sincospi(-2.0 * (double)(jm * r) / (double)(ns * R), &s, &c);
      a = zmul(a, make_double2(c, s));
    }
    v[r] = a;
  }
  double2 y[5];
  for (int k = 0; k < R; ++k) {
    double2 acc = make_double2(0.0, 0.0);
    for (int r = 0; r < R; ++r) {
      double s, c;
      sincospi(-2.0 * (double)((k * r) % R) / (double)R, &s, &c);
      acc.x += v[r].x * c - v[r].y * s;
      acc.y += v[r].x * s + v[r].y * c;
    }
    y[k] = acc;
  }
  const int64_t base = (j / ns) * ns * R + jm;
  for (int k = 0; k < R; ++k) out[base + k * ns] = y[k];
}

// out = in * scale, in natural order (L1 = 0) or four-step order: bin
// i = k1 + L1 k2 goes to out[k1 (L/L1) + k2]
__global__ void k_to_float_scaled(const double2 *in, float2 *out, int64_t L, double scale, int64_t L1) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L) return;
  const int64_t o = L1 > 0 ? (i % L1) * (L / L1) + i / L1 : i;
  out[o] = make_float2((float)(in[i].x * scale), (float)(in[i].y * scale));
}

// ---------------------------------------------------------------------------
// zoom tables
// ---------------------------------------------------------------------------
// Hamming-windowed sinc low-pass, cut-off nu_c cycles/sample, unit DC gain,
// then modulated: g[t] = h[t] e^{+j 2 pi nu_N t} so that the mix-down of eq. (7)
// followed by the filter of eq. (10) is  u[m] = e^{-j 2 pi nu_N m D} sum_t g[t] x[mD-t].
__global__ void k_zoom_taps(double2 *g, int T, double nu_c, double nu_N) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sum = 0.0;
  for (int t = 0; t < T; ++t) {
    double h = 1.0;
    if (T > 1) {
      double c = (double)t - 0.5 * (double)(T - 1);
      double u = 2.0 * nu_c * c;
      double sinc = (u == 0.0) ? 1.0 : sinpi(u) / (M_PI * u);
      double w = 0.54 - 0.46 * cospi(2.0 * (double)t / (double)(T - 1));
      h = w * 2.0 * nu_c * sinc;
    }
    sum += h;
  }
  for (int t = 0; t < T; ++t) {
    double h = 1.0;
    if (T > 1) {
      double c = (double)t - 0.5 * (double)(T - 1);
      double u = 2.0 * nu_c * c;
      double sinc = (u == 0.0) ? 1.0 : sinpi(u) / (M_PI * u);
      double w = 0.54 - 0.46 * cospi(2.0 * (double)t / (double)(T - 1));
      h = w * 2.0 * nu_c * sinc;
    }
    h /= sum;
    double cyc = frac_mul(nu_N, (double)t);
    double s, c;
    sincospi(2.0 * cyc, &s, &c);
    g[t] = make_double2(h * c, h * s);
  }
}

// ph[m] = e^{-j 2 pi nu_N m D}
__global__ void k_zoom_phasors(double2 *ph, int64_t LD, int64_t D, double nu_N) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= LD) return;
  double s, c;
  sincospi(-2.0 * frac_mul(nu_N, (double)(m * D)), &s, &c);
  ph[m] = make_double2(c, s);
}

// W_Nfft^m for the split zero-padded FFT
__global__ void k_root_table(float2 *w, int64_t n, int64_t q) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  w[m] = unit_cycles((double)(m % q) / (double)q);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t build_twiddles(float2 *tw, int64_t L, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3(nblocks(L, 256)), dim3(256), 0, s, tw, L);
  return hipGetLastError();
}

hipError_t build_root_table(float2 *w, int64_t n, int64_t q, hipStream_t s) {
  hipLaunchKernelGGL(k_root_table, dim3(nblocks(n, 256)), dim3(256), 0, s, w, n, q);
  return hipGetLastError();
}

// radix list for the FP64 FFT (L must be 2^a 3^b 5^c)
static int radix_list(int64_t L, int *rs) {
  int n = 0;
  while (L % 4 == 0) { rs[n++] = 4; L /= 4; }
  while (L % 2 == 0) { rs[n++] = 2; L /= 2; }
  while (L % 3 == 0) { rs[n++] = 3; L /= 3; }
  while (L % 5 == 0) { rs[n++] = 5; L /= 5; }
  return L == 1 ? n : -1;
}

hipError_t build_bluestein_tables(const PhaseParams &p, int64_t Ns, int nseg, int64_t Mb, int nblk,
                                  int64_t L, int L1, float2 *c_pre, float2 *c_post, float2 *V, hipStream_t s) {
  hipError_t e;
  const int64_t N = Ns;
  hipLaunchKernelGGL(k_chirp_pre, dim3(nblocks(Ns * nblk, 256)), dim3(256), 0, s, c_pre, Ns, nblk, Mb, p,
                     (int64_t)0);
  hipLaunchKernelGGL(k_chirp_post, dim3(nblocks(Mb * nblk * nseg, 256)), dim3(256), 0, s, c_post, Ns,
                     nseg, Mb, nblk, p, (int64_t)0);
  double2 *a = nullptr, *b = nullptr;
  if ((e = dev_malloc_async((void **)&a, sizeof(double2) * L, s)) != hipSuccess) return e;
  if ((e = dev_malloc_async((void **)&b, sizeof(double2) * L, s)) != hipSuccess) {
    hipFreeAsync(a, s);
    return e;
  }
  hipLaunchKernelGGL(k_chirp_conj, dim3(nblocks(L, 256)), dim3(256), 0, s, a, L, N, Mb, p);
  int rs[64];
  int np = radix_list(L, rs);
  if (np < 0) return hipErrorInvalidValue;
  int64_t ns = 1;
  for (int i = 0; i < np; ++i) {
    hipLaunchKernelGGL(k_fft64_pass, dim3(nblocks(L / rs[i], 256)), dim3(256), 0, s, a, b, L, rs[i], ns);
    ns *= rs[i];
    double2 *t = a; a = b; b = t;
  }
  // V = FFT(v) / L (the 1/L of the inverse FFT folded in), times the output scale
  hipLaunchKernelGGL(k_to_float_scaled, dim3(nblocks(L, 256)), dim3(256), 0, s, a, V, L, p.out_scale / (double)L,
                     (int64_t)L1);
  e = hipGetLastError();
  hipFreeAsync(a, s);
  hipFreeAsync(b, s);
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t build_half_tables(const PhaseParams &p, int64_t Ns, int64_t Mb, int nblk, int64_t L, float2 *c_pre1,
                             float2 *c_post1, hipStream_t s) {
  hipLaunchKernelGGL(k_chirp_pre, dim3(nblocks(Ns * nblk, 256)), dim3(256), 0, s, c_pre1, Ns, nblk, Mb, p, L);
  hipLaunchKernelGGL(k_chirp_post, dim3(nblocks(Mb * nblk, 256)), dim3(256), 0, s, c_post1, Ns, 1, Mb, nblk, p,
                     L);
  return hipGetLastError();
}

hipError_t build_zoom_tables(double2 *g, int T, double nu_c, double nu_N, double2 *ph, int64_t LD,
                             int64_t D, hipStream_t s) {
  hipLaunchKernelGGL(k_zoom_taps, dim3(1), dim3(64), 0, s, g, T, nu_c, nu_N);
  hipLaunchKernelGGL(k_zoom_phasors, dim3(nblocks(LD, 256)), dim3(256), 0, s, ph, LD, D, nu_N);
  return hipGetLastError();
}

}  // namespace tz
