// Hot-path kernels: fused Bluestein chirp-Z transform, zero-padded FFT and
// the Zoom FFT front end.  One workgroup transforms one trace (or one bin
// block of one trace); the FFT core keeps the data in registers and
// exchanges it through LDS between radix passes (fft_core.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

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
// Four waves per SIMD (128 VGPRs): L = 8192 runs two workgroups per CU
// instead of one
template <int L, int KIND, bool SEG>
__global__ void __launch_bounds__(Fft<L>::NT, 4)
    k_czt(const void *__restrict__ x, int64_t xs, int64_t N, int64_t Ns, int nseg,
          const float2 *__restrict__ c_pre, const float2 *__restrict__ c_post,
          const float2 *__restrict__ V, const float2 *__restrict__ tw, float2 *__restrict__ X,
          int64_t os, int64_t M, int64_t Mb, int nblk, int64_t nitems) {
  using F = Fft<L>;
  constexpr int NT = F::NT, E = F::E;
  constexpr int XB = KIND == 1 ? 8 : (KIND == 2 ? 8 : 4);  // bytes per input sample
  // two-level twiddle table (a half-circle table measured slower here: its
  // extra loads in flight cost occupancy)
  constexpr bool kHalf = false;
  __shared__ float2 lds[lds_points<L>()];
  __shared__ float2 twl[kHalf ? L / 2 : tw_lds_points<L>()];
  const unsigned t = threadIdx.x;
  // With bin blocks every block of a trace reads the same samples: the grid
  // (padded to a multiple of 8) is numbered so that the blocks of one trace
  // run on one XCD and share its L2 instead of fetching the trace once per
  // block from HBM.  Padding workgroups leave before any barrier.
  const int64_t q = nblk > 1 ? xcd_item(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  if (q >= nitems) return;
  const int64_t b = q / nblk;
  const int blk = (int)(q % nblk);
  const int64_t k0 = (int64_t)blk * Mb;
  // a block wholly past the bins asked for (M below the plan's bin count)
  // has nothing to write: the whole workgroup leaves before any barrier
  if (k0 >= M) return;
  const int64_t kmax = (M - k0 < Mb) ? (M - k0) : Mb;  // bins of this block, >= 1
  const auto twd = [&]() {
    if constexpr (kHalf)
      return load_half_twiddles<L>(twl, tw, t, NT);
    else
      return load_twiddles<L>(twl, tw, t, NT);
  }();
  __syncthreads();
  const Rsrc rV = make_rsrc(V, (uint64_t)L * 8);
  const Rsrc rX = make_rsrc(X + b * os + k0, (uint64_t)kmax * 8);

  float2 v[E];
  const int nloop = SEG ? nseg : 1;
  for (int s = 0; s < nloop; ++s) {
    // with segments every iteration derives its thread offsets afresh, so
    // none of them is loop-invariant and held in registers across iterations;
    // the same removes the spills of the single-pass kernel at L = 16384
    constexpr bool kFresh = SEG || L >= 16384;
    const unsigned t1 = kFresh ? t + opaque_zero() : t;
    const int64_t n0 = (int64_t)s * Ns;
    const int64_t nmax = (N - n0 < Ns) ? (N - n0) : Ns;  // samples of this segment
    // reads past the segment return 0: the zero padding of y up to L
    const Rsrc rx = make_rsrc((const char *)x + (b * xs + n0) * XB, (uint64_t)nmax * XB);
    const Rsrc rp = make_rsrc(c_pre + (int64_t)blk * Ns, (uint64_t)nmax * 8);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned n = t1 + NT * e;
      const float2 c = ld_c64(rp, 8 * n);
      if constexpr (KIND == 2)
        v[F::in_slot(e)] = cmul(ld_c64(rx, 8 * n), c);
      else
        v[F::in_slot(e)] = cscale(c, ld_real<KIND>(rx, n));
    }
    F::forward(v, lds, t1, twd);
    // from L = 8192 up the spectrum's offsets are recomputed too (the V
    // loads otherwise pin the first transform's index registers: spills)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t1 + NT * e;
      v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], ld_c64(rV, 8 * (L >= 8192 ? k + opaque_zero() : k))));
    }
    F::out_to_in(v);
    // from L = 8192 up, a fresh copy of the thread index: the second
    // transform recomputes its LDS addresses instead of keeping those of the
    // first one live (fewer registers; shorter transforms run faster without)
    const unsigned t2 = L >= 8192 ? t + opaque_zero() : t1;
    F::forward(v, lds, (int)t2, twd);
    const Rsrc rq = make_rsrc(c_post + ((int64_t)s * nblk + blk) * Mb, (uint64_t)kmax * 8);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = (kFresh ? t2 : t) + NT * e;
      const float2 r = cmul(cconj(v[F::out_slot(e)]), ld_c64(rq, 8 * k));
      // segments accumulate in X itself: segment s > 0 adds to what this
      // same thread stored for the same bins in segment s - 1 (a register
      // accumulator spilled ~80 registers at L = 16384).  A thread's store
      // and later load of one address stay in program order, as for any
      // store-then-load through a pointer; no other thread touches these
      // bins.  Bins past this block are dropped (and read as 0)
      st_c64((SEG && s > 0) ? cadd(ld_c64(rX, 8 * k), r) : r, rX, 8 * k);
    }
  }
}

// ---------------------------------------------------------------------------
// The same transform when the trace (N <= L/2) and the bin block (Mb <= L/2)
// each fill at most half of the FFT length: the length-L pair splits into
// two L/2-point pairs and drops the radix-2 pass of each FFT.  With y zero
// from n = L/2 on,
//   Y[2k + h] = FFT_{L/2}( y[n] W_L^{h n} )[k],                h = 0, 1,
// and the inverse at outputs n < L/2 is
//   g[n] = conj(a_0[n]) + W_L^{-n} conj(a_1[n]),  a_h = FFT_{L/2}( conj(Y[2k + h] V[2k + h]) ).
// Thread group h (threads h NT' .. h NT' + NT' - 1, NT' of the half-length
// FFT) runs the pair of half h in its own half of LDS.  The twist W_L^{n} sits
// in a second premultiply table, and W_L^{-n} in a second postmultiply one:
//   X[k0 + n] = post[n] conj(a_0[n]) + post1[n] conj(a_1[n]).
// For the combine, group 0 hands a_0 of the upper half of the outputs to
// group 1 through LDS and takes a_1 of the lower half: each thread finishes
// E/2 outputs.
// ---------------------------------------------------------------------------
template <int L, int KIND>
__global__ void __launch_bounds__(Fft<L>::NT, 4)
    k_czt_half(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ c_pre,
               const float2 *__restrict__ c_pre1, const float2 *__restrict__ c_post,
               const float2 *__restrict__ c_post1, const float2 *__restrict__ V, const float2 *__restrict__ tw,
               float2 *__restrict__ X, int64_t os, int64_t M, int64_t Mb, int nblk, int64_t nitems) {
  constexpr int LH = L / 2;
  using F = Fft<LH>;
  constexpr int NT = F::NT, E = F::E;
  static_assert(2 * NT == Fft<L>::NT && E == Fft<L>::E, "two half-length FFTs fill the workgroup");
  constexpr int XB = KIND == 1 ? 8 : (KIND == 2 ? 8 : 4);
  __shared__ float2 lds[2 * lds_points<LH>()];
  __shared__ float2 twl[tw_lds_points<LH>()];
  const unsigned t = threadIdx.x;
  const int64_t q = nblk > 1 ? xcd_item(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  if (q >= nitems) return;
  const int64_t b = q / nblk;
  const int blk = (int)(q % nblk);
  const int64_t k0 = (int64_t)blk * Mb;
  if (k0 >= M) return;
  const int64_t kmax = (M - k0 < Mb) ? (M - k0) : Mb;
  const TwLds twd = load_twiddles<LH>(twl, tw, t, 2 * NT);
  __syncthreads();
  // the half this thread's group transforms (wave-uniform: NT is a multiple of 64)
  const unsigned hh = __builtin_amdgcn_readfirstlane(t / NT);
  const unsigned u = t - hh * NT;
  float2 *lh = lds + hh * lds_points<LH>();
  const Rsrc rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
  const Rsrc rp = make_rsrc((hh ? c_pre1 : c_pre) + (int64_t)blk * N, (uint64_t)N * 8);
  const Rsrc rV = make_rsrc(V, (uint64_t)L * 8);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n = u + NT * e;  // past N: 0 (both the sample and its chirp)
    const float2 c = ld_c64(rp, 8 * n);
    if constexpr (KIND == 2)
      v[F::in_slot(e)] = cmul(ld_c64(rx, 8 * n), c);
    else
      v[F::in_slot(e)] = cscale(c, ld_real<KIND>(rx, n));
  }
  F::forward(v, lh, (int)u, twd);
  // bins 2k + h: times V, conjugated for the inverse
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k = u + opaque_zero() + NT * e;
    v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], ld_c64(rV, 8 * (2 * k + hh))));
  }
  F::out_to_in(v);
  const unsigned u2 = u + opaque_zero();
  F::forward(v, lh, (int)u2, twd);
  // a_h[n] at slot out_slot(e), n = u + NT e.  Group 0 finishes n < LH/2
  // (e < E/2), group 1 the rest; each hands the other its a_h of those n.
  // The group index only selects between two copies of the code below, so
  // that every register index stays a compile-time constant.
  const Rsrc rq0 = make_rsrc(c_post + (int64_t)blk * Mb, (uint64_t)kmax * 8);
  const Rsrc rq1 = make_rsrc(c_post1 + (int64_t)blk * Mb, (uint64_t)kmax * 8);
  const Rsrc rX = make_rsrc(X + b * os + k0, (uint64_t)kmax * 8);
  auto combine = [&](auto half) {
    constexpr int H = decltype(half)::value;
    constexpr int GIVE = H ? 0 : E / 2, KEEP = H ? E / 2 : 0;
    __syncthreads();  // the last pass's LDS reads are done
#pragma unroll
    for (int e = 0; e < E / 2; ++e) lds[u2 + NT * (GIVE + e)] = v[F::out_slot(GIVE + e)];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
      const unsigned n = u2 + NT * (KEEP + e);
      const float2 mine = v[F::out_slot(KEEP + e)], other = lds[n];
      const float2 a0 = H ? other : mine, a1 = H ? mine : other;
      const float2 r = cadd(cmul(cconj(a0), ld_c64(rq0, 8 * n)), cmul(cconj(a1), ld_c64(rq1, 8 * n)));
      st_c64(r, rX, 8 * n);  // bins past this block are dropped
    }
  };
  if (hh)
    combine(std::integral_constant<int, 1>{});
  else
    combine(std::integral_constant<int, 0>{});
}

// ---------------------------------------------------------------------------
// Frequency response of sample/reference pairs (Section 1): workgroup p runs
// the Bluestein transform of row 2p (reference) and keeps its result in
// registers, then that of row 2p+1 (sample), and writes only
//   H[k] = X_s[k] / X_r[k] = conj(g_s[k] / g_r[k]),
// g the conjugated inverse FFT of each trace (the postmultiply W^{k^2/2}
// cancels in the ratio).
// ---------------------------------------------------------------------------
// a / b, both scaled by 1/max(|Re b|, |Im b|) so that |b|^2 neither
// overflows nor underflows
__device__ __forceinline__ float2 cdiv(float2 a, float2 b) {
  const float s = 1.f / fmaxf(fabsf(b.x), fabsf(b.y));
  const float2 as = cscale(a, s), bs = cscale(b, s);
  const float d = 1.f / (bs.x * bs.x + bs.y * bs.y);
  return make_float2((as.x * bs.x + as.y * bs.y) * d, (as.y * bs.x - as.x * bs.y) * d);
}

template <int L, int KIND>
__global__ void __launch_bounds__(Fft<L>::NT)
    k_czt_transfer(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ c_pre,
                   const float2 *__restrict__ V, const float2 *__restrict__ tw, float2 *__restrict__ H,
                   int64_t os, int64_t M) {
  using F = Fft<L>;
  constexpr int NT = F::NT, E = F::E;
  constexpr int XB = KIND == 1 ? 8 : 4;
  __shared__ float2 lds[lds_points<L>()];
  __shared__ float2 twl[tw_lds_points<L>()];
  const unsigned t = threadIdx.x;
  const int64_t p = blockIdx.x;
  const TwLds twd = load_twiddles<L>(twl, tw, t, NT);
  __syncthreads();
  const Rsrc rV = make_rsrc(V, (uint64_t)L * 8);
  const Rsrc rp = make_rsrc(c_pre, (uint64_t)N * 8);
  const Rsrc rH = make_rsrc(H + p * os, (uint64_t)M * 8);  // bins past M are dropped
  // From L = 8192 up the reference's g_r waits in H[k] itself (each thread
  // reads back only its own stores of those bins, which stay in program
  // order with its loads) rather than in 2E registers, and each trace of the
  // pair derives its thread offsets afresh: at 16384, 125-140 registers
  // spilled otherwise, and at 8192 the kernel drops from 163 to 84 VGPRs (two
  // workgroups per CU, 4% faster).  Shorter transforms keep g_r in registers
  // (measured faster there).
  constexpr bool kInH = L >= 8192;
  float2 gr[kInH ? 1 : E], v[E];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const unsigned t1 = kInH ? t + opaque_zero() : t;
    const Rsrc rx = make_rsrc((const char *)x + (2 * p + s) * xs * XB, (uint64_t)N * XB);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned n = t1 + NT * e;  // samples past N read as 0
      v[F::in_slot(e)] = cscale(ld_c64(rp, 8 * n), ld_real<KIND>(rx, n));
    }
    F::forward(v, lds, t1, twd);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t1 + NT * e;
      v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], ld_c64(rV, 8 * (k + opaque_zero()))));
    }
    F::out_to_in(v);
    const unsigned t2 = kInH ? t + opaque_zero() : t;
    F::forward(v, lds, t2, twd);
    if (s == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if constexpr (kInH)
          st_c64(v[F::out_slot(e)], rH, 8 * (t2 + NT * e));
        else
          gr[e] = v[F::out_slot(e)];
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const unsigned k = t2 + NT * e;
        const float2 g = kInH ? ld_c64(rH, 8 * k) : gr[kInH ? 0 : e];
        st_c64(cconj(cdiv(v[F::out_slot(e)], g)), rH, 8 * k);
      }
    }
  }
}

// The transfer kernel in the half-length form of k_czt_half (L = 8192, N and
// M at most L/2): each trace of the pair runs as two 4096-point Bluestein
// pairs, X = post conj(a_0) + post1 conj(a_1) is formed for the bins this
// thread finishes, the reference's X_r is held in registers and the
// sample's X_s gives H = X_s / X_r (the postmultiply cancels in the ratio,
// as in k_czt_transfer).  The group's half selects between two copies of
// the code, so that every register index is a compile-time constant.
template <int L, int KIND>
__global__ void __launch_bounds__(Fft<L>::NT, 4)
    k_czt_transfer_half(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ c_pre,
                        const float2 *__restrict__ c_pre1, const float2 *__restrict__ c_post,
                        const float2 *__restrict__ c_post1, const float2 *__restrict__ V,
                        const float2 *__restrict__ tw, float2 *__restrict__ H, int64_t os, int64_t M) {
  constexpr int LH = L / 2;
  using F = Fft<LH>;
  constexpr int NT = F::NT, E = F::E;
  static_assert(2 * NT == Fft<L>::NT && E == Fft<L>::E, "two half-length FFTs fill the workgroup");
  constexpr int XB = KIND == 1 ? 8 : 4;
  __shared__ float2 lds[2 * lds_points<LH>()];
  __shared__ float2 twl[tw_lds_points<LH>()];
  const unsigned t = threadIdx.x;
  const int64_t pr = blockIdx.x;
  const TwLds twd = load_twiddles<LH>(twl, tw, t, 2 * NT);
  __syncthreads();
  const unsigned hh = __builtin_amdgcn_readfirstlane(t / NT);
  const unsigned u = t - hh * NT;
  float2 *lh = lds + hh * lds_points<LH>();
  const Rsrc rp = make_rsrc(hh ? c_pre1 : c_pre, (uint64_t)N * 8);
  const Rsrc rV = make_rsrc(V, (uint64_t)L * 8);
  const Rsrc rq0 = make_rsrc(c_post, (uint64_t)M * 8);
  const Rsrc rq1 = make_rsrc(c_post1, (uint64_t)M * 8);
  const Rsrc rH = make_rsrc(H + pr * os, (uint64_t)M * 8);  // bins past M are dropped
  auto run = [&](auto half) {
    constexpr int HH = decltype(half)::value;
    constexpr int GIVE = HH ? 0 : E / 2, KEEP = HH ? E / 2 : 0;
    float2 xr[E / 2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const unsigned u1 = u + opaque_zero();
      const Rsrc rx = make_rsrc((const char *)x + (2 * pr + s) * xs * XB, (uint64_t)N * XB);
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const unsigned n = u1 + NT * e;  // past N: 0
        v[F::in_slot(e)] = cscale(ld_c64(rp, 8 * n), ld_real<KIND>(rx, n));
      }
      F::forward(v, lh, (int)u1, twd);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const unsigned k = u1 + opaque_zero() + NT * e;
        v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], ld_c64(rV, 8 * (2 * k + HH))));
      }
      F::out_to_in(v);
      const unsigned u2 = u + opaque_zero();
      F::forward(v, lh, (int)u2, twd);
      __syncthreads();  // the last pass's LDS reads are done
#pragma unroll
      for (int e = 0; e < E / 2; ++e) lds[u2 + NT * (GIVE + e)] = v[F::out_slot(GIVE + e)];
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E / 2; ++e) {
        const unsigned n = u2 + NT * (KEEP + e);
        const float2 mine = v[F::out_slot(KEEP + e)], other = lds[n];
        const float2 a0 = HH ? other : mine, a1 = HH ? mine : other;
        const float2 X = cadd(cmul(cconj(a0), ld_c64(rq0, 8 * n)), cmul(cconj(a1), ld_c64(rq1, 8 * n)));
        if (s == 0)
          xr[e] = X;
        else
          st_c64(cdiv(X, xr[e]), rH, 8 * n);
      }
      __syncthreads();  // the swap slots are read before the next trace's FFT reuses LDS
    }
  };
  if (hh)
    run(std::integral_constant<int, 1>{});
  else
    run(std::integral_constant<int, 0>{});
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
  __shared__ float2 twl[tw_lds_points<FL>()];
  const unsigned t = threadIdx.x;
  const int64_t g = blockIdx.x;
  const int64_t xcd = g & 7, slot = g >> 3;
  const int64_t b = (slot / P) * 8 + xcd;
  const int r = (int)(slot % P);
  if (b >= B) return;  // whole workgroup leaves before any barrier
  const TwLds twd = load_twiddles<FL>(twl, tw, t, NT);
  __syncthreads();

  const Rsrc rx = make_rsrc((const char *)x + b * xs * (KIND == 1 ? 8 : 4), (uint64_t)N * (KIND == 1 ? 8 : 4));
  const Rsrc rr = make_rsrc(root, (uint64_t)(P * (int64_t)N) * 8);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n = t + NT * e;  // samples past N read as 0
    const float xv = ld_real<KIND>(rx, n);
    v[F::in_slot(e)] = (P > 1) ? cscale(ld_c64(rr, 8 * ((unsigned)r * n)), xv) : make_float2(xv, 0.f);
  }
  F::forward(v, lds, t, twd);
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
// Zero-padded FFT of a real trace, whole spectrum per workgroup.
//
// With Nh = N_fft/2 and z[m] = x[2m] + j x[2m+1] (m < ceil(N/2)), the
// Nh-point FFT Z of z gives every bin of the real trace:
//   X[k] = (Z[k] + conj Z[Nh-k])/2 - j W_{Nfft}^k (Z[k] - conj Z[Nh-k])/2
// for every k (indices of Z mod Nh, of W mod N_fft), and X[N_fft - k] =
// conj X[k].  Z itself is P independent F-point FFTs (Nh = P F, F >= N/2):
//   Z[P q + r] = FFT_F( z[m] W_{Nh}^{r m} )[q],
// one per wavefront (wave r), so the whole spectrum of the trace sits in the
// registers of one workgroup with no workgroup barrier during the FFTs.
//
// Z is staged through LDS in two halves that pair k with Nh - k: quarters
// {0, 3}, then quarters {1, 2} plus the three neighbours their bins reach.
// Lane l of a wave forms bins k, k+1 (k even) of a contiguous run of pairs
// and writes them with one aligned 16-byte store; the mirror pair
// (N_fft - k, N_fft - k + 1) = conj (X[k], X[k-1]) is aligned too, with
// X[k-1] taken from lane l-1 (lane 63 of the previous step for lane 0).
//
// Persistent: each workgroup fills its twiddle tables once and then takes
// traces g, g + gridDim.x, ... (g: blockIdx.x renumbered per XCD); stores are never waited for at
// barriers, so the writes of one trace drain while the next is loaded and
// transformed.  (Fetching the next trace during the writes was measured
// slower: its samples push FFT outputs into scratch, and loads and stores
// share one in-order counter, so each reload waits for every store issued
// before it.)
// ---------------------------------------------------------------------------
// Lane l receives v from lane l - 1 and lane 0 receives `first`: one DPP
// whole-wave shift per component (no LDS round trip).
__device__ __forceinline__ float2 lane_up1(float2 v, float2 first) {
  constexpr int kWaveShr1 = 0x138;  // DPP control: wave_shr:1
  return make_float2(
      __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first.x), __float_as_int(v.x), kWaveShr1, 0xf, 0xf, false)),
      __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first.y), __float_as_int(v.y), kWaveShr1, 0xf, 0xf, false)));
}
// v of lane 63, uniform over the wave
__device__ __forceinline__ float2 lane63(float2 v) {
  return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), 63)),
                     __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), 63)));
}

template <int F, int P>
struct PadWaveShape {
  using FF = WaveFft<F>;
  static constexpr int E = FF::E;
  static constexpr int NH = P * F;
  static constexpr int STAGE = NH / 2 + 4;  // half of Z, its neighbours and wrap copies, slots from 1
  static constexpr int LDS_FFT = P * FF::window();
  static constexpr int LDS_STAGE = STAGE + STAGE / 16 + 1;
  static constexpr int LDS = LDS_FFT > LDS_STAGE ? LDS_FFT : LDS_STAGE;
  static_assert(E % 4 == 0, "quarters of Z must align with register slots");
  static_assert((NH / 4) % (64 * P) == 0, "each wave takes whole 64-pair steps of one quarter");
};

template <int F, int P, int KIND>
__global__ void __launch_bounds__(64 * P)
    k_fftpad_real(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ root_h,
                  const float2 *__restrict__ root_f, const float2 *__restrict__ tw, float2 *__restrict__ X,
                  int64_t os, int half, int64_t B) {
  using Sh = PadWaveShape<F, P>;
  using FF = typename Sh::FF;
  constexpr int E = Sh::E, NH = Sh::NH, NTH = 64 * P;
  constexpr unsigned Q4 = NH / 4, NF = 2 * NH;
  constexpr unsigned PPW = Q4 / P;  // pairs per wave and phase
  constexpr int IT = (int)PPW / 64;  // 64-pair steps per wave and phase
  constexpr unsigned NU = NH / 64;   // W_Nh^{64 j} = W_NU^j
  constexpr int XB = KIND == 1 ? 8 : 4;
  __shared__ float2 lds[Sh::LDS];
  __shared__ float2 twl[F / 2];
  __shared__ float2 rtl[tw_lds_points<NH>()];
  __shared__ float2 rul[NU];
  __shared__ float2 rfl[tw_lds_points<2 * NH>()];
  const TwHalf<F> twd = load_half_twiddles<F>(twl, tw, threadIdx.x, NTH);
  const TwLds rtd = load_twiddles<NH>(rtl, root_h, threadIdx.x, NTH);
  const TwLds rfd = load_twiddles<2 * NH>(rfl, root_f, threadIdx.x, NTH);
  // W_NU^j / 2: the 1/2 of the combine below rides on the input twiddle
  for (unsigned i = threadIdx.x; i < NU; i += NTH) rul[i] = cscale(root_h[64 * i], 0.5f);

  // The samples of the next trace are fetched cooperatively (SPT per thread)
  // before the first store of the current one and parked in LDS once the
  // current trace's combine no longer needs it.  Loads and stores retire in
  // issue order on one counter, so a fetch issued after the stores (at the
  // top of the next trace) would wait for all of them to drain before the
  // next FFT could start; issued before them, it lets the next FFT run while
  // they drain.
  constexpr int SPT = 2 * F / NTH;
  static_assert(SPT * NTH == 2 * F, "the trace must split evenly over the threads");
  // trace indices are 32-bit (the launcher refuses B >= 2^31): compares and
  // increments stay on the scalar unit
  const unsigned B32 = (unsigned)B;
  auto prefetch = [&](unsigned tb, unsigned tid_, float (&pre)[SPT]) {
    const Rsrc rx = make_rsrc((const char *)x + (int64_t)tb * xs * XB, tb < B32 ? (uint64_t)N * XB : 0);
#pragma unroll
    for (int j = 0; j < SPT; ++j) pre[j] = ld_real<KIND>(rx, tid_ + NTH * j);  // past N (or B): 0
  };
  auto park = [&](const float (&pre)[SPT], unsigned tid_) {
    float *xl = (float *)lds;  // samples 0 .. 2F-1 in the first F points of LDS
#pragma unroll
    for (int j = 0; j < SPT; ++j) xl[tid_ + NTH * j] = pre[j];
  };
  // traces g, g + G, ... with g numbered so that each XCD takes a contiguous
  // run of traces per round: its workgroups' concurrent stores then stay
  // within a few contiguous MB instead of spreading over the whole round
  // (measured on plain 512 KB row writes: 5.2 TB/s against 4.6 TB/s)
  // (32-bit: the 64-bit form took scalar registers that pushed a value out
  // to scratch, and its reload waited for the stores in flight)
  const unsigned g = __builtin_amdgcn_readfirstlane(
      (gridDim.x & 7u) == 0 ? (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x);
  {
    float pre[SPT];
    prefetch(g, threadIdx.x, pre);
    park(pre, threadIdx.x);
  }
  float2 v[E];

  // the wave's first thread index, pinned in a scalar register (the empty
  // asm) for the whole kernel: no vector register carries a thread index
  // across the trace loop, where it would be spilled and its reload, like
  // any load, would wait for every store still in flight
  unsigned w0 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u);
  asm volatile("" : "+s"(w0));
  for (unsigned bu = g; bu < B32; bu += gridDim.x) {
    const int64_t b = bu;
    __syncthreads();  // tables filled / previous trace's staging reads done
    // thread indices through an opaque zero (the lane from mbcnt): everything
    // derived from them (twiddles, LDS addresses) is formed per trace instead
    // of being hoisted out of the loop and kept live in registers across it
    const unsigned tid = w0 + (__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, opaque_zero())) & 63u);
    // the wave index is wave-uniform: it and what derives from it only need
    // scalar registers
    const unsigned r = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    // (x[2m], x[2m+1]), m = lane + 64 e, from the samples parked in LDS
#pragma unroll
    for (int e = 0; e < E; ++e) v[FF::in_slot(e)] = lds[lane + 64 * e];
    __syncthreads();  // every wave holds its samples before the FFT windows reuse the space
    // z[m] W_Nh^{r m} / 2 with m = lane + 64 e: W_Nh^{r lane} W_NU^{r e} / 2
    {
      const float2 wl = rtd(r * lane);
#pragma unroll
      for (int e = 0; e < E; ++e)
        v[FF::in_slot(e)] = cmul(v[FF::in_slot(e)], cmul(wl, rul[(r * (unsigned)e) & (NU - 1)]));
    }
    FF::forward(v, lds + r * FF::window(), lane, twd);  // Z/2

    float pre[SPT];  // the next trace's samples (fetched in phase 0, parked after phase 1)
    const Rsrc rX = make_rsrc(X + b * os, (uint64_t)(half ? NH + 1 : NF) * 8);
    using U4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(rX, 0, 0, 0));
    auto st2 = [&](unsigned voff, float2 a, float2 c) {
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, make_float4(a.x, a.y, c.x, c.y)), rX,
                                             (int)voff, 0, 0);
    };
    // X[k] = Z[k]/2 + conj Z[Nh-k]/2 - j W^k (Z[k]/2 - conj Z[Nh-k]/2), from the halves a, c
    auto comb = [](float2 a, float2 c, float2 w) {
      const float2 cc = cconj(c);
      return cadd(cadd(a, cc), cmul(w, cmul_mj(csub(a, cc))));
    };
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      // LDS slot of Z[z]: phase 0 holds quarters 0 and 3 with Z[-1], Z[Nh], Z[Nh+1]
      // copied to the ends of their runs; phase 1 holds quarters 1 and 2 with
      // Z[Q4-1], Z[3Q4], Z[3Q4+1]; on each run the slot is z plus a constant
      auto slot = [&](int zz) -> int {
        if (ph == 0) return zz < (int)Q4 ? zz + 2 : zz - NH / 2 + 2;
        return zz - (int)Q4 + 2;
      };
      auto bin = [&](unsigned k) {  // any bin 0 <= k < N_fft whose Z pair is staged
        const int kz = (int)(k & (NH - 1)), mz = (int)((NH - (k & (NH - 1))) & (NH - 1));
        return comb(lds[lds_idx(slot(kz))], lds[lds_idx(slot(mz))], rfd(k));
      };
      __syncthreads();  // FFT windows / previous phase's reads are done
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int quarter = (4 * e) / E;
        const int k = (int)(P * (lane + 64 * e) + r);
        const float2 z = v[FF::out_slot(e)];
        if (ph == 0) {
          if (quarter == 0 || quarter == 3) lds[lds_idx(slot(k))] = z;
          if (e == 0 && lane == 0 && r <= 1) lds[lds_idx(NH / 2 + 2 + k)] = z;     // Z[Nh], Z[Nh+1]
          if (e == E - 1 && lane == 63 && r == P - 1) lds[lds_idx(1)] = z;        // Z[-1]
        } else {
          if (quarter == 1 || quarter == 2 || (quarter == 3 && k <= (int)(3 * Q4 + 1)) ||
              (quarter == 0 && k == (int)Q4 - 1))
            lds[lds_idx(slot(k))] = z;
        }
      }
      __syncthreads();
      if (ph == 1) prefetch(bu + gridDim.x, tid + opaque_zero(), pre);

      // wave r takes pairs (k, k+1), k even, k = k0 + 128 it (it < IT):
      // phase 0: k0 = 2 r PPW + 2 lane (r < P/2), 3Q4 + 2 + 2 (r PPW - Q4/2) + 2 lane;
      // phase 1: k0 = Q4 + 2 r PPW + 2 lane.  The lane index passes through an
      // opaque zero here so that these addresses are formed after the FFT
      // rather than hoisted above it and held in registers across it.
      const unsigned lane_ = lane + opaque_zero();
      const bool upper = ph == 0 && r >= (unsigned)(P / 2);
      const unsigned k0 = ph == 0 ? (upper ? 3 * Q4 + 2 + 2 * (r * PPW - Q4 / 2) : 2 * r * PPW) + 2 * lane_
                                  : Q4 + 2 * r * PPW + 2 * lane_;
      const int ca = ph == 0 ? (upper ? 2 - NH / 2 : 2) : 2 - (int)Q4;  // slot - z on the run of Z[k]
      const int cm = ph == 0 ? (upper ? 2 : 2 - NH / 2) : 2 - (int)Q4;  // ... of Z[Nh-k]
      // a step moves k by 128 slots, i.e. 136 LDS points, on every run
      const float2 *pa = lds + lds_idx((int)k0 + ca);                                    // Z[k], Z[k+1]
      const int mlast = NH - (int)k0 - 128 * (IT - 1) + cm;                              // Z[Nh-k] at the last step
      const float2 *pm0 = lds + lds_idx(mlast), *pm1 = lds + lds_idx(mlast - 1);        // Z[Nh-k], Z[Nh-k-1]
      const float2 *ph_ = rfd.hi + (k0 >> 7);                                            // W^{128 (k0/128 + it)}
      const float2 lo0 = rfd.lo[k0 & 127], lo1 = rfd.lo[(k0 + 1) & 127];
      const unsigned vdir = 8 * k0, vmir = 8 * (NF - k0);
      float2 carry = make_float2(0.f, 0.f);
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const float2 hi = ph_[it];
        const float2 x0 = comb(pa[136 * it], pm0[136 * (IT - 1 - it)], cmul(lo0, hi));
        const float2 x1 = comb(pa[136 * it + 1], pm1[136 * (IT - 1 - it)], cmul(lo1, hi));
        // X[k-1] from lane - 1; lane 0 takes the bin before the run (first
        // step) or lane 63 of the previous step
        const float2 xm = lane_up1(x1, it == 0 ? bin((k0 + NF - 1) & (NF - 1)) : carry);
        carry = lane63(x1);
        // the pair (Nh, Nh+1) is the last of phase 0; in the half spectrum
        // only X[Nh] is written, and its mirror would repeat the direct store;
        // the pair (0, 1) (first of phase 0) has no mirror
        const bool top = ph == 0 && it == IT - 1 && r == (unsigned)(P - 1) && lane == 63;
        const bool bottom = ph == 0 && it == 0 && r == 0 && lane == 0;
        if (half && top) {
          st_c64(x0, rX, 8 * NH);
        } else {
          st2(vdir + 1024 * it, x0, x1);
          // mirror pair conj(X[k], X[k-1]) at N_fft - k
          if (!half && !top && !bottom) st2(vmir - 1024 * it, cconj(x0), cconj(xm));
        }
        // one step's loads in flight at a time: the other quarter of Z is
        // still held in registers for the next phase
        __builtin_amdgcn_sched_barrier(0);
      }
      if (ph == 1 && tid == 0) {
        const unsigned k = 3 * Q4;
        const float2 x0 = bin(k), x1 = bin(k + 1), xm = bin(k - 1);
        st2(8 * k, x0, x1);
        if (!half) st2(8 * (NF - k), cconj(x0), cconj(xm));
      }
    }
    __syncthreads();  // the combine's reads of the staged spectrum are done
    park(pre, tid + opaque_zero());
  }  // traces
}

// ---------------------------------------------------------------------------
// Zoom front end (eqs. (6), (7), (8), (10)): mix-down, low-pass and
// decimation fused, evaluated only at the kept outputs:
//   u[m] = e^{-j 2 pi nu_N m D} sum_{t<T} g[t] x[mD - t],  g[t] = h[t] e^{j 2 pi nu_N t}
// (the same as filtering y[n] = x[n] e^{-j 2 pi nu_N n} with h and keeping
// every D-th output).  Taps and phasors are FP64 and the T-term sums are
// accumulated in FP64: an FP32 accumulator rounds at every step and its error
// grows like sqrt(T) relative to |u|, which a narrow output band magnifies.
//
// Workgroup (b, m0) stages x[m0 D - (T-1) .. (m0 + opb - 1) D] in LDS;
// thread j forms output m0 + j.  The lanes of a wave read samples D apart:
// when D is a multiple of 8 (many lanes on one bank) one pad slot every 64
// samples spreads them over the banks (PAD); otherwise the tile is linear and
// the per-tap offsets fold into the LDS instructions.
// ---------------------------------------------------------------------------
template <bool PAD>
__device__ __forceinline__ int zpad(int i) {
  if constexpr (PAD)
    return i + (i >> 6);
  else
    return i;
}

constexpr int kZoomThreads = 256;

// S = split waves per output: 256/S outputs per workgroup (one per lane of S
// groups); group s sums the taps t = s mod S, so a long filter runs as S
// shorter dependent chains.
template <int KIND, int S, bool PAD>
__global__ void __launch_bounds__(kZoomThreads)
    k_zoom_front(const void *__restrict__ x, int64_t xs, int64_t N, int64_t D, int64_t LD, int T,
                 const double2 *__restrict__ g, const double2 *__restrict__ ph, float2 *__restrict__ u,
                 int64_t bpt, int opb, int vec4) {
  // KIND 0 / 1: real f32 / f64 samples; KIND 2: complex f32 (later axes of
  // a multi-dimensional zoom)
  using XT = typename std::conditional<KIND == 1, double,
                                       typename std::conditional<KIND == 2, float2, float>::type>::type;
  extern __shared__ double2 zsm[];
  double2 *part = zsm;  // [S][256 / S] partial sums
  XT *xl = (XT *)(part + kZoomThreads);
  constexpr int nout = kZoomThreads / S;
  const int64_t b = blockIdx.x / bpt;
  const int64_t m0 = (blockIdx.x % bpt) * opb;
  const int64_t n0 = m0 * D - (T - 1);
  const int span = (opb - 1) * (int)D + T;
  // unconditional buffer loads: n >= N is past the extent, and n < 0 wraps to
  // an offset above 2^31 (the host keeps N * sizeof(XT) below that), so both
  // read as 0 and the loads of a thread can all be in flight at once
  const Rsrc rx = make_rsrc((const XT *)x + b * xs, (uint64_t)N * sizeof(XT));
  bool tiled = false;
  if constexpr (KIND == 0) tiled = vec4 != 0;
  if (tiled) {
    // 16-byte loads of 4 samples from a start floored to a multiple of 4: each
    // load lies wholly before 0, wholly inside [0, N) or wholly past N, except
    // the one holding sample N (when N % 4 != 0), loaded sample by sample
    const int64_t n0a = n0 & ~(int64_t)3;
    const int nq = (int)((n0 + span - n0a + 3) >> 2);
    constexpr int kBatch = 4;  // loads of a thread in flight before any is used
    for (int q0 = threadIdx.x; q0 < nq; q0 += kBatch * kZoomThreads) {
      float4 w[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        // quads past the tile take an offset beyond the extent: they read 0
        // with no memory request
        const int q = q0 + u * kZoomThreads;
        const unsigned off = q < nq ? (unsigned)((n0a + 4 * (int64_t)q) * 4) : 0xFFFFFFF0u;
        w[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rx, (int)off, 0, 0));
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int q = q0 + u * kZoomThreads;
        if (q >= nq) break;
        const int64_t sn = n0a + 4 * (int64_t)q;
        if (sn < N && sn + 3 >= N)  // the quad holding sample N - 1 and the end
          w[u] = make_float4(ld_f32(rx, (unsigned)(sn * 4)), ld_f32(rx, (unsigned)(sn * 4 + 4)),
                             ld_f32(rx, (unsigned)(sn * 4 + 8)), ld_f32(rx, (unsigned)(sn * 4 + 12)));
        const int i0 = (int)(sn - n0);  // tile index of sample sn (may be < 0 for the first load)
        const float e4[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (i0 + c >= 0 && i0 + c < span) {
            if constexpr (KIND == 0) xl[zpad<PAD>(i0 + c)] = e4[c];
          }
      }
    }
  } else {
#pragma unroll 8
    for (int i = threadIdx.x; i < span; i += blockDim.x) {
      const unsigned off = (unsigned)((n0 + i) * (int64_t)sizeof(XT));
      if constexpr (KIND == 1)
        xl[zpad<PAD>(i)] = ld_f64(rx, off);
      else if constexpr (KIND == 2)
        xl[zpad<PAD>(i)] = ld_c64(rx, off);
      else
        xl[zpad<PAD>(i)] = ld_f32(rx, off);
    }
  }
  __syncthreads();
  // thread j of group s: output m0 + j, taps t = s, s + S, ...; the lanes of
  // a wave read stride-D samples, spread over the banks by the pad.  A group
  // spans whole waves (256 / S >= 64 lanes), so the tap index is the same
  // across a wave and the taps come through scalar loads (one read per wave
  // instead of one LDS read per lane)
  const int j = threadIdx.x % nout;
  const int sidx = __builtin_amdgcn_readfirstlane(threadIdx.x / nout);
  const int top = j * (int)D + T - 1;  // tile index of x[(m0 + j) D]
  double ar = 0.0, ai = 0.0;
  if (j < opb) {
#pragma unroll 8
    for (int t = sidx; t < T; t += S) {
      const double2 gt = g[t];
      if constexpr (KIND == 2) {
        const float2 xv = xl[zpad<PAD>(top - t)];
        ar = fma(gt.x, (double)xv.x, fma(-gt.y, (double)xv.y, ar));
        ai = fma(gt.x, (double)xv.y, fma(gt.y, (double)xv.x, ai));
      } else {
        const double xv = (double)xl[zpad<PAD>(top - t)];
        ar = fma(gt.x, xv, ar);
        ai = fma(gt.y, xv, ai);
      }
    }
  }
  part[threadIdx.x] = make_double2(ar, ai);
  __syncthreads();
  const int64_t m = m0 + threadIdx.x;
  if ((int)threadIdx.x >= opb || m >= LD) return;
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    sr += part[q * nout + threadIdx.x].x;
    si += part[q * nout + threadIdx.x].y;
  }
  const double2 p = ph[m];
  u[b * LD + m] = make_float2((float)(p.x * sr - p.y * si), (float)(p.x * si + p.y * sr));
}

// same sums with x and the taps read from global memory (filters too long
// for the LDS tile)
template <int KIND>
__global__ void __launch_bounds__(256)
    k_zoom_front_global(const void *__restrict__ x, int64_t xs, int64_t N, int64_t D, int64_t LD, int T,
                        const double2 *__restrict__ g, const double2 *__restrict__ ph, float2 *__restrict__ u,
                        int64_t bpt) {
  const int64_t b = blockIdx.x / bpt;
  const int64_t m = (blockIdx.x % bpt) * 256 + threadIdx.x;
  if (m >= LD) return;
  const int64_t base = m * D;
  double ar = 0.0, ai = 0.0;
  for (int t = 0; t < T; ++t) {
    const int64_t n = base - t;
    if (n >= 0 && n < N) {
      if constexpr (KIND == 2) {
        const float2 xv = ((const float2 *)x)[b * xs + n];
        ar = fma(g[t].x, (double)xv.x, fma(-g[t].y, (double)xv.y, ar));
        ai = fma(g[t].x, (double)xv.y, fma(g[t].y, (double)xv.x, ai));
      } else {
        const double xv = (double)load_real<KIND>(x, b * xs + n);
        ar = fma(g[t].x, xv, ar);
        ai = fma(g[t].y, xv, ai);
      }
    }
  }
  const double2 p = ph[m];
  u[b * LD + m] = make_float2((float)(p.x * ar - p.y * ai), (float)(p.x * ai + p.y * ar));
}

// Persistent form for real f32 traces on 16-byte boundaries (the long-scan and
// batched workloads).  Each workgroup walks tiles (trace b, outputs r opb ..
// r opb + opb - 1) with a grid-stride loop and fetches the next tile's samples
// into registers (QPT 16-byte loads per thread, all in flight at once) while
// the current tile's sums run from LDS, so the HBM reads of one tile overlap
// the FP64 arithmetic of the previous one.  The tile position advances by
// additions (no integer division in the loop).
//
// The tile starts at n0a = n0 rounded down to a multiple of 4 (n0 = m0 D -
// (T-1), delta = n0 - n0a), so quad q lands on tile words 4q .. 4q+3.  With
// P = 2 (D a multiple of 8) the tile has two pad slots after every D samples:
// sample i sits at word i + 2 floor(i / D).  Output o of the tile at tap t
// reads tile sample i = o D + c, c = T - 1 + delta - t, i.e. word o (D + P) +
// c + P floor(c / D).  The output part o (D + 2) has stride 2 mod 4 across the
// banks, so the paired reads of two neighbouring taps (the compiler merges
// them) hit distinct banks; the tap part is the same in every lane, so within
// a block of D taps it is an immediate offset of the LDS read.
//
// Group s of the S tap groups (whole waves) takes the contiguous taps
// [s tpg, (s+1) tpg); lane j of a group sums outputs j + r nout, r < R, so
// every tap fetched through the scalar unit (the same for the whole wave)
// feeds R outputs per lane before the next wait on the scalar and LDS loads.
// The partial sums of the groups then go through the tile's own LDS.
template <int S, int P, int QPT, int R>
__global__ void __launch_bounds__(kZoomThreads)
    k_zoom_front_pf(const float *__restrict__ x, int64_t xs, int64_t N, int D, int64_t LD, int T,
                    const double2 *__restrict__ g, const double2 *__restrict__ ph, float2 *__restrict__ u,
                    int bpt, int opb, int B, uint32_t dmagic) {
  extern __shared__ double2 zsm[];
  float *xl = (float *)zsm;  // the tile, then the partial sums part[S][opb]
  double2 *part = zsm;
  constexpr int nout = kZoomThreads / S;
  const int tid = threadIdx.x;
  const int span = (opb - 1) * D + T;
  // tile (b, r) = tile index b bpt + r; the grid stride in the same form
  struct Pos {
    int b, r;
  };
  const int G = (int)gridDim.x;
  const int sb = G / bpt, sr = G - (G / bpt) * bpt;
  auto advance = [&](Pos q) {
    q.r += sr;
    q.b += sb;
    if (q.r >= bpt) {
      q.r -= bpt;
      ++q.b;
    }
    return q;
  };
  // first sample n0 of the sums, quad-aligned start n0a, quads of the tile
  auto geom = [&](Pos q, int64_t *n0a, int *delta, int *nq) {
    const int64_t n0 = (int64_t)q.r * opb * D - (T - 1);
    *n0a = n0 & ~(int64_t)3;
    *delta = (int)(n0 - *n0a);
    *nq = (*delta + span + 3) >> 2;
  };
  float4 w[QPT];
  // 16-byte loads of the tile's quads; quads before sample 0 take offsets
  // above 2^31 and quads past the tile an offset past the extent, so both read
  // 0 (the host keeps N * 4 below 2^31); the one quad holding sample N - 1
  // and the end of the trace (N % 4 != 0) is loaded sample by sample.  With
  // live = false every load reads 0 without a memory request: the loads are
  // still issued, so the count of loads in flight is the same on every path
  // and a wait for an older load never waits for these
  auto fetch = [&](Pos q, bool live) {
    int64_t n0a;
    int delta, nq;
    geom(q, &n0a, &delta, &nq);
    if (!live) nq = 0;
    const Rsrc rx = make_rsrc(x + (int64_t)(live ? q.b : 0) * xs, (uint64_t)N * 4);
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      const int qi = tid + k * kZoomThreads;
      const int64_t sn = n0a + 4 * (int64_t)qi;
      const unsigned off = qi < nq ? (unsigned)(sn * 4) : 0xFFFFFFF0u;
      w[k] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rx, (int)off, 0, 0));
      if (qi < nq && sn < N && sn + 3 >= N)
        w[k] = make_float4(ld_f32(rx, (unsigned)(sn * 4)), ld_f32(rx, (unsigned)(sn * 4 + 4)),
                           ld_f32(rx, (unsigned)(sn * 4 + 8)), ld_f32(rx, (unsigned)(sn * 4 + 12)));
    }
  };
  const int sidx = __builtin_amdgcn_readfirstlane(tid / nout);
  const int j = tid % nout;
  const int tpg = (T + S - 1) / S;
  const int t_lo = sidx * tpg < T ? sidx * tpg : T;
  const int t_hi = t_lo + tpg < T ? t_lo + tpg : T;
  const int lb = j * (D + P);
  const int ostride = nout * (D + P);  // tile words between outputs j and j + nout
  Pos cur{(int)blockIdx.x / bpt, (int)blockIdx.x - ((int)blockIdx.x / bpt) * bpt};
  if (cur.b >= B) return;
  fetch(cur, true);
  for (;;) {
    int64_t n0a;
    int delta, nq;
    geom(cur, &n0a, &delta, &nq);
    const int64_t m0 = (int64_t)cur.r * opb;
    // this thread's mixing phasors (outputs tid + 256 i of the tile), requested
    // ahead of the next tile's samples: waiting for them never waits for those
    double2 p[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t m = m0 + tid + kZoomThreads * i;
      p[i] = ph[m < LD ? m : LD - 1];
    }
    // quads into the tile (D is a multiple of 4 when P > 0, so a quad never
    // straddles a pad)
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      const int qi = tid + k * kZoomThreads;
      if (qi < nq) {
        const unsigned i = 4u * (unsigned)qi;
        float *d = xl + i + (P ? P * __umulhi(i, dmagic) : 0u);
        d[0] = w[k].x;
        d[1] = w[k].y;
        d[2] = w[k].z;
        d[3] = w[k].w;
      }
    }
    // the registers are free again: the next tile's loads go out before the
    // barrier and stay in flight through this tile's sums
    const Pos next = advance(cur);
    const bool more = next.b < B;
    fetch(more ? next : cur, more);
    __syncthreads();
    // taps [t_lo, t_hi) of outputs j + r nout: tile samples c = T - 1 + delta - t
    double ar[R], ai[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ar[r] = ai[r] = 0.0;
    {
      const int c_lo = T + delta - t_hi, c_hi = T + delta - t_lo;
      const double2 *gp = g + (T - 1 + delta);  // tap of sample c: gp[-c]
      int c = c_lo;
      int cq = P ? c_lo / D : 0;
      while (c < c_hi) {
        const int e = P ? ((cq + 1) * D < c_hi ? (cq + 1) * D : c_hi) : c_hi;
        const float *row = xl + lb + P * cq;
#pragma unroll 8
        for (; c < e; ++c) {
          const double2 gt = gp[-c];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            // outputs past the tile read words past its samples (inside the
            // allocation) and are never stored
            const double xv = (double)row[c + r * ostride];
            ar[r] = fma(gt.x, xv, ar[r]);
            ai[r] = fma(gt.y, xv, ai[r]);
          }
        }
        ++cq;
      }
    }
    __syncthreads();  // every tile read is done: the partial sums take its place
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (j + r * nout < opb) part[sidx * opb + j + r * nout] = make_double2(ar[r], ai[r]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int o = tid + kZoomThreads * i;
      const int64_t m = m0 + o;
      if (o < opb && m < LD) {
        double sr2 = 0.0, si2 = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
          sr2 += part[q * opb + o].x;
          si2 += part[q * opb + o].y;
        }
        u[(int64_t)cur.b * LD + m] =
            make_float2((float)(p[i].x * sr2 - p[i].y * si2), (float)(p[i].x * si2 + p[i].y * sr2));
      }
    }
    if (!more) break;
    __syncthreads();  // the sums are read before the next tile overwrites them
    cur = next;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
bool czt_half_supported(int L, int nseg, int64_t Ns, int64_t Mb) {
  return L == 8192 && nseg == 1 && Ns <= L / 2 && Mb <= L / 2;
}

bool fft_length_supported(int64_t L) {
  return L >= kMinL && L <= kMaxL && (L & (L - 1)) == 0;
}

template <int L, int KIND>
static void czt_dispatch_seg(const CztLaunch &a, hipStream_t s) {
  const int64_t items = a.B * a.nblk;
  // blocked plans: a multiple of 8 workgroups for the XCD-aware numbering
  const dim3 grid((unsigned)(a.nblk > 1 ? (items + 7) / 8 * 8 : items)), block(Fft<L>::NT);
  if constexpr (L == 8192) {
    if (a.c_pre1) {  // one segment, N and the bin block within L/2 (the plan checked)
      hipLaunchKernelGGL((k_czt_half<L, KIND>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_pre1, a.c_post,
                         a.c_post1, a.V, a.tw_half, a.X, a.os, a.M, a.Mb, a.nblk, items);
      return;
    }
  }
  if (a.nseg > 1)
    hipLaunchKernelGGL((k_czt<L, KIND, true>), grid, block, 0, s, a.x, a.xs, a.N, a.Ns, a.nseg,
                       a.c_pre, a.c_post, a.V, a.tw, a.X, a.os, a.M, a.Mb, a.nblk, items);
  else
    hipLaunchKernelGGL((k_czt<L, KIND, false>), grid, block, 0, s, a.x, a.xs, a.N, a.Ns, a.nseg,
                       a.c_pre, a.c_post, a.V, a.tw, a.X, a.os, a.M, a.Mb, a.nblk, items);
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

template <int L>
static void transfer_dispatch(const TransferLaunch &a, hipStream_t s) {
  const dim3 grid((unsigned)a.pairs), block(Fft<L>::NT);
  if constexpr (L == 8192) {
    if (a.c_pre1) {  // N and M within L/2 (the plan checked)
      if (a.in_kind == 1)
        hipLaunchKernelGGL((k_czt_transfer_half<L, 1>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_pre1,
                           a.c_post, a.c_post1, a.V, a.tw_half, a.H, a.os, a.M);
      else
        hipLaunchKernelGGL((k_czt_transfer_half<L, 0>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_pre1,
                           a.c_post, a.c_post1, a.V, a.tw_half, a.H, a.os, a.M);
      return;
    }
  }
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_czt_transfer<L, 1>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.V, a.tw, a.H,
                       a.os, a.M);
  else
    hipLaunchKernelGGL((k_czt_transfer<L, 0>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.V, a.tw, a.H,
                       a.os, a.M);
}

hipError_t launch_czt_transfer(const TransferLaunch &a, hipStream_t s) {
  switch (a.L) {
    case 256: transfer_dispatch<256>(a, s); break;
    case 512: transfer_dispatch<512>(a, s); break;
    case 1024: transfer_dispatch<1024>(a, s); break;
    case 2048: transfer_dispatch<2048>(a, s); break;
    case 4096: transfer_dispatch<4096>(a, s); break;
    case 8192: transfer_dispatch<8192>(a, s); break;
    case 16384: transfer_dispatch<16384>(a, s); break;
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

// resident workgroups per CU x CUs for a kernel with `shm` bytes of dynamic
// LDS, at most `work` (queried once per device, kernel and LDS size)
static unsigned persistent_grid_shm(const void *kernel, int threads, size_t shm, int64_t work) {
  struct Entry {
    int dev;
    const void *fn;
    size_t shm;
    int slots;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int slots = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (const Entry &e : cache)
      if (e.dev == dev && e.fn == kernel && e.shm == shm) slots = e.slots;
  }
  if (!slots) {
    int ncu = 0, occ = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, shm);
    slots = (ncu > 0 ? ncu : 1) * (occ > 0 ? occ : 1);
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({dev, kernel, shm, slots});
  }
  return (unsigned)(work < slots ? work : slots);
}

template <int F, int P>
static void pad_real_launch(const PadRealLaunch &a, hipStream_t s) {
  const dim3 block(64 * P);
  if (a.in_kind == 1) {
    const dim3 grid(persistent_grid_shm((const void *)k_fftpad_real<F, P, 1>, 64 * P, 0, a.B));
    hipLaunchKernelGGL((k_fftpad_real<F, P, 1>), grid, block, 0, s, a.x, a.xs, a.N, a.root_h, a.root_f, a.tw,
                       a.X, a.os, a.half, a.B);
  } else {
    const dim3 grid(persistent_grid_shm((const void *)k_fftpad_real<F, P, 0>, 64 * P, 0, a.B));
    hipLaunchKernelGGL((k_fftpad_real<F, P, 0>), grid, block, 0, s, a.x, a.xs, a.N, a.root_h, a.root_f, a.tw,
                       a.X, a.os, a.half, a.B);
  }
}

// (F, P) pairs with a compiled whole-spectrum kernel
bool fftpad_real_supported(int F, int P) {
  switch (F * 100 + P) {
    case 102408: case 102416: case 204808: case 204816: return true;
    default: return false;
  }
}

hipError_t launch_fftpad_real(const PadRealLaunch &a, hipStream_t s) {
  if (a.B >= ((int64_t)1 << 31)) return hipErrorInvalidValue;  // 32-bit trace indices in the kernel
  switch (a.F * 100 + a.P) {
    case 102408: pad_real_launch<1024, 8>(a, s); break;   // N_fft 16384, N <= 2048
    case 102416: pad_real_launch<1024, 16>(a, s); break;  // N_fft 32768, N <= 2048
    case 204808: pad_real_launch<2048, 8>(a, s); break;   // N_fft 32768, N <= 4096
    case 204816: pad_real_launch<2048, 16>(a, s); break;  // N_fft 65536, N <= 4096
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// persistent front end for aligned f32 traces; false when the filter is too
// long for its tile (the caller then takes the one-tile-per-workgroup kernel)
static bool zoom_front_pf(const ZoomFrontLaunch &a, int S, hipStream_t s) {
  constexpr int64_t kTileBytes = 40 * 1024;  // four workgroups per CU
  constexpr int kQmax = 9;                   // 16-byte loads per thread and tile
  const int P = a.D % 8 == 0 ? 2 : 0;
  // tile of opb outputs: quads (start rounded down by up to 3) and LDS words;
  // the partial sums S x opb double2 share the allocation
  // lanes whose outputs lie past opb (opb < r2 nout) read up to
  // (r2 nout - opb) (D + P) words past the tile, inside the allocation
  auto shape = [&](int64_t opb, int s2, int r2, int64_t *span4, int64_t *bytes) {
    const int64_t span = (opb - 1) * a.D + a.T;
    *span4 = (span + 3 + 3) / 4 * 4;
    const int64_t idle = std::max<int64_t>(0, (int64_t)r2 * (kZoomThreads / s2) - opb);
    const int64_t words = *span4 + P * (*span4 / a.D) + 1 + idle * (a.D + P);
    *bytes = std::max<int64_t>(4 * words, 16 * s2 * opb);
  };
  auto fits = [&](int64_t opb, int s2, int r2) {
    int64_t span4, bytes;
    shape(opb, s2, r2, &span4, &bytes);
    return bytes <= kTileBytes && span4 / 4 <= kQmax * kZoomThreads &&
           (!P || (uint64_t)span4 * (uint64_t)a.D < ((uint64_t)1 << 32));
  };
  // two outputs per lane with the fewest tap groups whose tile fits, else one
  int R = 0;
  int64_t opb = 0;
  for (int s2 = S; s2 <= 4 && !R; s2 *= 2)
    if (fits(2 * (kZoomThreads / s2), s2, 2)) {
      R = 2;
      S = s2;
      opb = 2 * (kZoomThreads / s2);
    }
  if (!R) {
    R = 1;
    for (opb = kZoomThreads / S; opb >= 16; opb -= opb > 64 ? 16 : 4)
      if (fits(opb, S, 1)) break;
  }
  const int64_t bpt = (a.LD + opb - 1) / opb, ntiles = a.B * bpt;
  if (opb < 16 || a.D > (1 << 30) || ntiles >= ((int64_t)1 << 31)) return false;
  int64_t span4, bytes;
  shape(opb, S, R, &span4, &bytes);
  const int nqt = (int)((span4 / 4 + kZoomThreads - 1) / kZoomThreads);
  const size_t shm = (size_t)bytes;
  const uint32_t dmagic = P ? (uint32_t)((((uint64_t)1 << 32) + a.D - 1) / a.D) : 0u;
  auto go = [&](auto kernel) {
    const dim3 grid(persistent_grid_shm((const void *)kernel, kZoomThreads, shm, ntiles)), block(kZoomThreads);
    hipLaunchKernelGGL(kernel, grid, block, shm, s, (const float *)a.x, a.xs, a.N, (int)a.D, a.LD, a.T, a.g, a.ph,
                       a.u, (int)bpt, (int)opb, (int)a.B, dmagic);
  };
  auto by_q = [&](auto k2, auto k4, auto k9) { nqt <= 2 ? go(k2) : (nqt <= 4 ? go(k4) : go(k9)); };
#define TZ_ZPF(S_, P_, R_) by_q(k_zoom_front_pf<S_, P_, 2, R_>, k_zoom_front_pf<S_, P_, 4, R_>, k_zoom_front_pf<S_, P_, 9, R_>)
#define TZ_ZPF_S(P_, R_) (S == 1 ? TZ_ZPF(1, P_, R_) : (S == 2 ? TZ_ZPF(2, P_, R_) : TZ_ZPF(4, P_, R_)))
  if (R == 2)
    P ? TZ_ZPF_S(2, 2) : TZ_ZPF_S(0, 2);
  else
    P ? TZ_ZPF_S(2, 1) : TZ_ZPF_S(0, 1);
#undef TZ_ZPF_S
#undef TZ_ZPF
  return true;
}

hipError_t launch_zoom_front(const ZoomFrontLaunch &a, hipStream_t s) {
  // LDS tile: the partial sums and the samples of opb outputs, within 64 KB
  constexpr int64_t kTileBytes = 64 * 1024;
  const int64_t xb = a.in_kind == 0 ? 4 : 8;
  const int64_t fixed = 16 * kZoomThreads;
  const int S = a.T < 128 ? 1 : (a.T < 256 ? 2 : 4);
  // persistent kernel for filters of 96+ taps on aligned f32 traces (measured:
  // 255 taps, D = 64: 389 -> 291 us; 127 taps, D = 16: 138 -> 113 us); shorter
  // filters run faster one tile per workgroup (63 taps, D = 6: 79 vs 95 us),
  // their sums being too short to cover the extra barriers and phasor loads
  if (a.in_kind == 0 && a.T >= 96 && ((uintptr_t)a.x & 15) == 0 && ((a.xs * 4) & 15) == 0 &&
      a.N * 4 < ((int64_t)1 << 31) && zoom_front_pf(a, S, s))
    return hipGetLastError();
  int64_t opb = 0;
  if (fixed + xb * (a.T + a.T / 64 + 1) <= kTileBytes && a.N * xb < ((int64_t)1 << 31)) {
    const int64_t xmax = (kTileBytes - fixed) / xb * 64 / 65 - 1;  // samples, pads included
    opb = (xmax - a.T) / a.D + 1;
    if (opb > kZoomThreads / S) opb = kZoomThreads / S;
  }
  if (opb >= 1) {
    const int64_t span = (opb - 1) * a.D + a.T;
    const size_t shm = (size_t)(fixed + xb * (span + span / 64 + 1));
    const int64_t bpt = (a.LD + opb - 1) / opb;
    const dim3 grid((unsigned)(a.B * bpt)), block(kZoomThreads);
    // 16-byte tile loads when every trace starts on a 16-byte boundary
    const int vec4 = (a.in_kind == 0 && ((uintptr_t)a.x & 15) == 0 && ((a.xs * 4) & 15) == 0) ? 1 : 0;
    auto go = [&](auto kernel) {
      hipLaunchKernelGGL(kernel, grid, block, shm, s, a.x, a.xs, a.N, a.D, a.LD, a.T, a.g, a.ph, a.u, bpt,
                         (int)opb, vec4);
    };
    auto by_s = [&](auto k1, auto k2, auto k4) { S == 1 ? go(k1) : (S == 2 ? go(k2) : go(k4)); };
    const bool pad = a.D % 8 == 0;
    if (a.in_kind == 1)
      pad ? by_s(k_zoom_front<1, 1, true>, k_zoom_front<1, 2, true>, k_zoom_front<1, 4, true>)
          : by_s(k_zoom_front<1, 1, false>, k_zoom_front<1, 2, false>, k_zoom_front<1, 4, false>);
    else if (a.in_kind == 2)
      pad ? by_s(k_zoom_front<2, 1, true>, k_zoom_front<2, 2, true>, k_zoom_front<2, 4, true>)
          : by_s(k_zoom_front<2, 1, false>, k_zoom_front<2, 2, false>, k_zoom_front<2, 4, false>);
    else
      pad ? by_s(k_zoom_front<0, 1, true>, k_zoom_front<0, 2, true>, k_zoom_front<0, 4, true>)
          : by_s(k_zoom_front<0, 1, false>, k_zoom_front<0, 2, false>, k_zoom_front<0, 4, false>);
    return hipGetLastError();
  }
  const int64_t bpt = (a.LD + 255) / 256;
  const dim3 grid((unsigned)(a.B * bpt)), block(256);
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_zoom_front_global<1>), grid, block, 0, s, a.x, a.xs, a.N, a.D, a.LD, a.T, a.g, a.ph,
                       a.u, bpt);
  else if (a.in_kind == 2)
    hipLaunchKernelGGL((k_zoom_front_global<2>), grid, block, 0, s, a.x, a.xs, a.N, a.D, a.LD, a.T, a.g, a.ph,
                       a.u, bpt);
  else
    hipLaunchKernelGGL((k_zoom_front_global<0>), grid, block, 0, s, a.x, a.xs, a.N, a.D, a.LD, a.T, a.g, a.ph,
                       a.u, bpt);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched complex transpose: out[b][c][r] = y[b][r][c] for r < R, c < C, the
// matrices ys (input) and os (output) elements apart.  Each workgroup moves
// one 64 x 64 tile through LDS, so that every wave reads and writes 512-byte
// row segments; the pad column spreads the column reads over the banks.
// ---------------------------------------------------------------------------
constexpr int kTile = 64;

__global__ void __launch_bounds__(256)
    k_transpose_c64(const float2 *__restrict__ y, int64_t ys, int64_t R, int64_t C, float2 *__restrict__ out,
                    int64_t os, int64_t tr, int64_t tc) {
  __shared__ float2 tile[kTile][kTile + 1];
  const int64_t per = tr * tc;
  const int64_t b = blockIdx.x / per, rem = blockIdx.x - b * per;
  const int64_t r0 = rem / tc * kTile, c0 = rem % tc * kTile;
  const int lx = threadIdx.x & (kTile - 1), ly = threadIdx.x / kTile;
  const float2 *src = y + b * ys;
#pragma unroll
  for (int i = ly; i < kTile; i += 256 / kTile) {
    const int64_t r = r0 + i, c = c0 + lx;
    if (r < R && c < C) tile[i][lx] = src[r * C + c];
  }
  __syncthreads();
  float2 *dst = out + b * os;
#pragma unroll
  for (int i = ly; i < kTile; i += 256 / kTile) {
    const int64_t c = c0 + i, r = r0 + lx;
    if (c < C && r < R) dst[c * R + r] = tile[lx][i];
  }
}

hipError_t launch_transpose(const TransposeLaunch &a, hipStream_t s) {
  const int64_t tr = (a.R + kTile - 1) / kTile, tc = (a.C + kTile - 1) / kTile;
  const dim3 grid((unsigned)(a.nb * tr * tc)), block(256);
  hipLaunchKernelGGL(k_transpose_c64, grid, block, 0, s, a.y, a.ys, a.R, a.C, a.out, a.os, tr, tc);
  return hipGetLastError();
}

}  // namespace tz
