// Hot-path kernels: fused Bluestein chirp-Z transform, zero-padded FFT and
// the Zoom FFT front end.  One workgroup transforms one trace (or one bin
// block of one trace); the FFT core keeps the data in registers and
// exchanges it through LDS between radix passes (fft_core.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"
#include "internal.h"

namespace tz {

template <int KIND>
__device__ __forceinline__ float load_real(const void *__restrict__ x, int64_t i) {
  if constexpr (KIND == 1)
    return (float)((const double *)x)[i];
  else
    return ((const float *)x)[i];
}

// ---------------------------------------------------------------------------
// Chirp-Z transform in Bluestein form (eqs. (12)-(15)).
//
// Workgroup (b, blk) evaluates bins k0 + k', k0 = blk*Mb, k' < Mb, of trace b:
//   X[k0+k'] = sum_s post[s][blk][k'] *
//              IFFT_L( FFT_L( x[s Ns + n'] pre[blk][n'] ) * V )[k']
// pre[blk][n'] = A^{-n'} W^{k0 n'} W^{n'^2/2}            (premultiply)
// V = FFT_L(v)/L,  v[l] = W^{-l^2/2}, l in (-Ns, Mb)       (conjugate chirp)
// post[s][blk][k'] = W^{k'^2/2} A^{-s Ns} W^{(k0+k') s Ns} (postmultiply)
// With one segment and one block this is exactly eq. (15).  The inverse FFT
// is the forward FFT of the conjugate, conjugated (1/L sits in V).
// ---------------------------------------------------------------------------
template <int L, int KIND, bool SEG>
__global__ void __launch_bounds__(Fft<L>::NT)
    k_czt(const void *__restrict__ x, int64_t xs, int64_t N, int64_t Ns, int nseg,
          const float2 *__restrict__ c_pre, const float2 *__restrict__ c_post,
          const float2 *__restrict__ V, const float2 *__restrict__ tw, float2 *__restrict__ X,
          int64_t os, int64_t M, int64_t Mb, int nblk) {
  using F = Fft<L>;
  constexpr int NT = F::NT, E = F::E;
  __shared__ float2 lds[lds_points<L>()];
  const unsigned t = threadIdx.x;
  const int64_t b = blockIdx.x / nblk;
  const int blk = blockIdx.x % nblk;
  const int64_t k0 = (int64_t)blk * Mb;
  // per-trace bases are uniform (scalar registers); lane offsets are 32-bit
  const float2 *pre = c_pre + (int64_t)blk * Ns;
  const int64_t kmax = (M - k0 < Mb) ? (M - k0) : Mb;  // bins of this block

  float2 acc[SEG ? E : 1];
  float2 v[E];
  const int nloop = SEG ? nseg : 1;
  for (int s = 0; s < nloop; ++s) {
    const int64_t n0 = (int64_t)s * Ns;
    const int64_t nmax = (N - n0 < Ns) ? (N - n0) : Ns;  // samples of this segment
    const unsigned nlim = (unsigned)nmax;
    const unsigned z0 = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned n = t + NT * e;
      const unsigned nc = clamp_idx(n, nlim) + z0;
      const float2 c = pre[nc];
      float2 val;
      if constexpr (KIND == 2)
        val = cmul(((const float2 *)x + b * xs + n0)[nc], c);
      else if constexpr (KIND == 1)
        val = cscale(c, (float)((const double *)x + b * xs + n0)[nc]);
      else
        val = cscale(c, ((const float *)x + b * xs + n0)[nc]);
      v[F::in_slot(e)] = (n < nlim) ? val : make_float2(0.f, 0.f);
    }
    F::forward(v, lds, t, tw);
    const unsigned z1 = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t + NT * e;
      v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], V[k + z1]));
    }
    F::out_to_in(v);
    F::forward(v, lds, t, tw);
    const float2 *post = c_post + ((int64_t)s * nblk + blk) * Mb;
    float2 *Xb = X + b * os + k0;
    const unsigned klim = (unsigned)kmax;
    const unsigned z2 = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t + NT * e;
      const float2 r = cmul(cconj(v[F::out_slot(e)]), post[clamp_idx(k, klim) + z2]);
      if constexpr (SEG) {
        acc[e] = (s == 0) ? r : cadd(acc[e], r);
      } else {
        if (k < klim) Xb[k] = r;
      }
    }
  }
  if constexpr (SEG) {
    float2 *Xb = X + b * os + k0;
    const unsigned klim = (unsigned)kmax;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t + NT * e;
      if (k < klim) Xb[k] = acc[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Zero-padded FFT (eqs. (2)-(5)), N_fft = P * F with F >= N:
//   X[P q + r] = sum_{n<N} (x[n] W_{Nfft}^{r n}) W_F^{q n},   r < P, q < F.
// For P = 1 this is one F-point FFT of the zero-padded trace.  Workgroup
// (trace, r) runs one F-point FFT; only the N non-zero samples are read.
// Blocks are numbered so that the P workgroups of one trace land on the same
// XCD (dispatch is round-robin over the 8 XCDs) back to back, letting that
// XCD's L2 merge their interleaved writes into whole lines.
// ---------------------------------------------------------------------------
template <int FL, int KIND>
__global__ void __launch_bounds__(Fft<FL>::NT)
    k_fftpad(const void *__restrict__ x, int64_t xs, int64_t N, int P,
             const float2 *__restrict__ root, const float2 *__restrict__ tw,
             float2 *__restrict__ X, int64_t os, int64_t nout, int64_t B) {
  using F = Fft<FL>;
  constexpr int NT = F::NT, E = F::E;
  __shared__ float2 lds[lds_points<FL>()];
  const unsigned t = threadIdx.x;
  const int64_t g = blockIdx.x;
  const int64_t xcd = g & 7, slot = g >> 3;
  const int64_t b = (slot / P) * 8 + xcd;
  const int r = (int)(slot % P);
  if (b >= B) return;  // whole workgroup leaves before any barrier

  const unsigned nlim = (unsigned)N;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n = t + NT * e;
    const unsigned nc = clamp_idx(n, nlim);
    float xv;
    if constexpr (KIND == 1)
      xv = (float)((const double *)x + b * xs)[nc];
    else
      xv = ((const float *)x + b * xs)[nc];
    const float2 val = (P > 1) ? cscale(root[(unsigned)r * nc], xv) : make_float2(xv, 0.f);
    v[F::in_slot(e)] = (n < nlim) ? val : make_float2(0.f, 0.f);
  }
  F::forward(v, lds, t, tw);
  float2 *Xb = X + b * os + r;
  // bins k = q P + r < nout  <=>  q < qlim
  const unsigned qlim = (unsigned)((nout - r + P - 1) / P);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned q = t + NT * e;
    if (q < qlim) Xb[(size_t)q * P] = v[F::out_slot(e)];
  }
}

// ---------------------------------------------------------------------------
// Zoom front end (eqs. (6), (7), (8), (10)): mix-down, low-pass and
// decimation fused, evaluated only at the kept outputs:
//   u[m] = e^{-j 2 pi nu_N m D} sum_{t<T} g[t] x[mD - t],  g[t] = h[t] e^{j 2 pi nu_N t}
// (the same as filtering y[n] = x[n] e^{-j 2 pi nu_N n} with h and keeping
// every D-th output).
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(256)
    k_zoom_front(const void *__restrict__ x, int64_t xs, int64_t N, int64_t D, int64_t LD, int T,
                 const float2 *__restrict__ g, const float2 *__restrict__ ph,
                 float2 *__restrict__ u, int64_t blocks_per_trace) {
  const int64_t b = blockIdx.x / blocks_per_trace;
  const int64_t m = (blockIdx.x % blocks_per_trace) * 256 + threadIdx.x;
  if (m >= LD) return;
  const int64_t base = m * D;
  float2 acc = make_float2(0.f, 0.f);
  for (int tt = 0; tt < T; ++tt) {
    const int64_t n = base - tt;
    if (n >= 0 && n < N) {
      const float xv = load_real<KIND>(x, b * xs + n);
      const float2 gg = g[tt];
      acc.x = fmaf(gg.x, xv, acc.x);
      acc.y = fmaf(gg.y, xv, acc.y);
    }
  }
  u[b * LD + m] = cmul(ph[m], acc);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
bool fft_length_supported(int64_t L) {
  return L >= kMinL && L <= kMaxL && (L & (L - 1)) == 0;
}

template <int L, int KIND>
static void czt_dispatch_seg(const CztLaunch &a, hipStream_t s) {
  const dim3 grid((unsigned)(a.B * a.nblk)), block(Fft<L>::NT);
  if (a.nseg > 1)
    hipLaunchKernelGGL((k_czt<L, KIND, true>), grid, block, 0, s, a.x, a.xs, a.N, a.Ns, a.nseg,
                       a.c_pre, a.c_post, a.V, a.tw, a.X, a.os, a.M, a.Mb, a.nblk);
  else
    hipLaunchKernelGGL((k_czt<L, KIND, false>), grid, block, 0, s, a.x, a.xs, a.N, a.Ns, a.nseg,
                       a.c_pre, a.c_post, a.V, a.tw, a.X, a.os, a.M, a.Mb, a.nblk);
}

template <int L>
static void czt_dispatch_kind(const CztLaunch &a, hipStream_t s) {
  switch (a.in_kind) {
    case 0: czt_dispatch_seg<L, 0>(a, s); break;
    case 1: czt_dispatch_seg<L, 1>(a, s); break;
    default: czt_dispatch_seg<L, 2>(a, s); break;
  }
}

hipError_t launch_czt(const CztLaunch &a, hipStream_t s) {
  switch (a.L) {
    case 256: czt_dispatch_kind<256>(a, s); break;
    case 512: czt_dispatch_kind<512>(a, s); break;
    case 1024: czt_dispatch_kind<1024>(a, s); break;
    case 2048: czt_dispatch_kind<2048>(a, s); break;
    case 4096: czt_dispatch_kind<4096>(a, s); break;
    case 8192: czt_dispatch_kind<8192>(a, s); break;
    case 16384: czt_dispatch_kind<16384>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int FL>
static void pad_dispatch(const PadLaunch &a, hipStream_t s) {
  const int64_t groups = (a.B + 7) / 8;
  const dim3 grid((unsigned)(groups * 8 * a.P)), block(Fft<FL>::NT);
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_fftpad<FL, 1>), grid, block, 0, s, a.x, a.xs, a.N, a.P, a.root, a.tw, a.X,
                       a.os, a.nout, a.B);
  else
    hipLaunchKernelGGL((k_fftpad<FL, 0>), grid, block, 0, s, a.x, a.xs, a.N, a.P, a.root, a.tw, a.X,
                       a.os, a.nout, a.B);
}

hipError_t launch_fftpad(const PadLaunch &a, hipStream_t s) {
  switch (a.F) {
    case 256: pad_dispatch<256>(a, s); break;
    case 512: pad_dispatch<512>(a, s); break;
    case 1024: pad_dispatch<1024>(a, s); break;
    case 2048: pad_dispatch<2048>(a, s); break;
    case 4096: pad_dispatch<4096>(a, s); break;
    case 8192: pad_dispatch<8192>(a, s); break;
    case 16384: pad_dispatch<16384>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zoom_front(const ZoomFrontLaunch &a, hipStream_t s) {
  const int64_t bpt = (a.LD + 255) / 256;
  const dim3 grid((unsigned)(a.B * bpt)), block(256);
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_zoom_front<1>), grid, block, 0, s, a.x, a.xs, a.N, a.D, a.LD, a.T, a.g, a.ph,
                       a.u, bpt);
  else
    hipLaunchKernelGGL((k_zoom_front<0>), grid, block, 0, s, a.x, a.xs, a.N, a.D, a.LD, a.T, a.g, a.ph,
                       a.u, bpt);
  return hipGetLastError();
}

}  // namespace tz
