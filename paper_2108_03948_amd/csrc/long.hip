// Bluestein CZT for long traces (N + M - 1 > 16384): the length-L FFTs of
// eq. (15) are split four-step, L = L1 * L2 (L1 = 320 = 5 * 4^3, 512 or 1024;
// L2 a power of two), and run as three kernels per chunk of traces with one
// L-point workspace per trace.
//
// With n = n1 L2 + n2 and k = k1 + L1 k2 (n1, k1 < L1; n2, k2 < L2),
//   FFT_L(y)[k1 + L1 k2] = sum_n2 W_L2^{n2 k2} W_L^{n2 k1} sum_n1 y[n1 L2 + n2] W_L1^{n1 k1}.
// The inverse FFT takes its input in the same (k1, k2) order, so the spectrum
// never has to be put back in natural order:
//   cols   (k_long_cols_fwd): y = x * pre (eq. (13)), L1-point FFT down each
//          column n2, Z[k1][n2] written row-major;
//   rows   (k_long_rows): for each row k1, times W_L^{k1 n2}, L2-point FFT over
//          n2, times V[k1 + L1 k2] (eq. (15)'s second factor, stored in the
//          same order, 1/L folded in), conjugate, L2-point FFT over k2, times
//          W_L^{k1 n2}: Hc[k1][n2], in place of Z;
//   icols  (k_long_cols_inv): L1-point FFT down each column of Hc gives the
//          conjugate of the inverse FFT at n = n1 L2 + n2; bins n < M are
//          conjugated, post-multiplied (eq. (13)) and stored.
// Every kernel reads and writes whole 128-byte rows of 16 columns; the
// intermediate of a chunk is sized to stay in the last-level cache.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"
#include "internal.h"
#include "thzspec.h"

namespace tz {

constexpr int kCols = 16;  // columns per column-FFT workgroup (128 B of complex per row)

// F-point FFTs down kCols adjacent columns of a row-major tile in LDS.
// Thread t works on column c = t % kCols as virtual thread tv = t / kCols of
// an FftShape<F> transform: same passes as Fft<F>, LDS point (i, c) at
// lds_idx(i kCols + c), i.e. rows of 17 complex (the pad spreads the rows a
// wave touches over all banks).
template <int F>
struct ColFft {
  static constexpr int NTV = FftShape<F>::NT;
  static constexpr int E = F / NTV;
  static constexpr int NT = NTV * kCols;
  using Plan = typename FftShape<F>::Plan;
  static constexpr int P = Plan::count;
  static constexpr int R_first = Plan::list[0];
  static constexpr int R_last = Plan::list[P - 1];

  __device__ __forceinline__ static constexpr int in_slot(int e) { return slot_of<E, R_first>(e); }
  __device__ __forceinline__ static constexpr int out_slot(int e) { return slot_of<E, R_last>(e); }
  __device__ __forceinline__ static int at(int i, int c) { return lds_idx(i * kCols + c); }
  static constexpr int ns_before(int p) {
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= Plan::list[i];
    return ns;
  }

  template <int p>
  __device__ __forceinline__ static void pass(float2 (&v)[E], float2 *lds, int tv, int c, const TwLds &tw) {
    constexpr int R = Plan::list[p];
    constexpr int NS = ns_before(p);
    constexpr int NB = E / R;
    constexpr int TWS = F / (NS * R);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = tv + i * NTV;
      if constexpr (NS > 1) apply_twiddles<R>(&v[i * R], tw, (unsigned)(j % NS) * TWS);
      Dft<R>::template run<1>(&v[i * R]);
    }
    if constexpr (p + 1 < P) {
      constexpr int R2 = Plan::list[p + 1];
      constexpr int NB2 = E / R2;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = tv + i * NTV;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[at(base + r * NS, c)] = v[i * R + r];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NB2; ++i) {
        const int j = tv + i * NTV;
#pragma unroll
        for (int r = 0; r < R2; ++r) v[i * R2 + r] = lds[at(j + r * (F / R2), c)];
      }
    }
  }

  template <int... ps>
  __device__ __forceinline__ static void run(float2 (&v)[E], float2 *lds, int tv, int c, const TwLds &tw,
                                             std::integer_sequence<int, ps...>) {
    (pass<ps>(v, lds, tv, c, tw), ...);
  }
  __device__ __forceinline__ static void forward(float2 (&v)[E], float2 *lds, int tv, int c, const TwLds &tw) {
    run(v, lds, tv, c, tw, std::make_integer_sequence<int, P>{});
  }
};

// ---------------------------------------------------------------------------
// cols: Z[b][k1][n2] = sum_n1 x[n1 L2 + n2] pre[n1 L2 + n2] W_L1^{n1 k1}
// ---------------------------------------------------------------------------
template <int L1, int KIND>
__global__ void __launch_bounds__(ColFft<L1>::NT)
    k_long_cols_fwd(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ c_pre,
                    const float2 *__restrict__ tw_col, float2 *__restrict__ Z, int L2) {
  using CF = ColFft<L1>;
  constexpr int E = CF::E, NTV = CF::NTV;
  constexpr int XB = KIND == 0 ? 4 : 8;
  __shared__ float2 lds[lds_points<L1 * kCols>()];
  __shared__ float2 twl[tw_lds_points<L1>()];
  const int t = threadIdx.x, c = t % kCols, tv = t / kCols;
  const int ncg = L2 / kCols;
  const int64_t q = xcd_item(blockIdx.x, gridDim.x);
  const int64_t b = q / ncg;
  const unsigned n2 = (unsigned)((q % ncg) * kCols + c);
  const TwLds twd = load_twiddles<L1>(twl, tw_col, t, CF::NT);
  __syncthreads();
  const Rsrc rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
  const Rsrc rp = make_rsrc(c_pre, (uint64_t)N * 8);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n = (unsigned)(tv + NTV * e) * (unsigned)L2 + n2;  // n >= N reads 0
    const float2 p = ld_c64(rp, 8 * n);
    if constexpr (KIND == 2)
      v[CF::in_slot(e)] = cmul(ld_c64(rx, 8 * n), p);
    else
      v[CF::in_slot(e)] = cscale(p, ld_real<KIND>(rx, n));
  }
  CF::forward(v, lds, tv, c, twd);
  const int64_t L = (int64_t)L1 * L2;
  const Rsrc rz = make_rsrc(Z + b * L, (uint64_t)L * 8);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k1 = (unsigned)(tv + NTV * e);
    st_c64(v[CF::out_slot(e)], rz, 8 * (k1 * (unsigned)L2 + n2));
  }
}

// ---------------------------------------------------------------------------
// rows: Hc[b][k1][n2] = W_L^{k1 n2} FFT_L2( conj( V[k1 + L1 k2] FFT_L2( W_L^{k1 n2} Z[b][k1][.] ) ) )
// ---------------------------------------------------------------------------
template <int L1, int L2>
__global__ void __launch_bounds__(Fft<L2>::NT, 4)
    k_long_rows(float2 *__restrict__ Z, const float2 *__restrict__ Vt, const float2 *__restrict__ tw_row,
                const float2 *__restrict__ tbig, int64_t nb) {
  using F = Fft<L2>;
  constexpr int NT = F::NT, E = F::E;
  constexpr int64_t L = (int64_t)L1 * L2;
  __shared__ float2 lds[lds_points<L2>()];
  __shared__ float2 twl[tw_lds_points<L2>()];
  const unsigned t = threadIdx.x;
  // rows of equal k1 (one V row) for the traces of the chunk run back to back
  const int64_t q = xcd_item(blockIdx.x, gridDim.x);
  const unsigned k1 = (unsigned)(q / nb);
  const int64_t b = q % nb;
  const TwLds twd = load_twiddles<L2>(twl, tw_row, t, NT);
  __syncthreads();
  const Rsrc rz = make_rsrc(Z + b * L + (int64_t)k1 * L2, (uint64_t)L2 * 8);
  const Rsrc rv = make_rsrc(Vt + (int64_t)k1 * L2, (uint64_t)L2 * 8);
  // W_L^{k1 n2} with n2 = t + NT e: a per-thread factor times a per-block one
  const float2 wt = big_twiddle(tbig, k1 * t);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n2 = t + NT * e;
    const float2 w = cmul(wt, big_twiddle(tbig, k1 * (unsigned)(NT * e)));
    v[F::in_slot(e)] = cmul(ld_c64(rz, 8 * n2), w);
  }
  F::forward(v, lds, t, twd);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k2 = t + NT * e;
    v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], ld_c64(rv, 8 * k2)));
  }
  F::out_to_in(v);
  // from L2 = 8192 up the second transform recomputes its LDS addresses
  // (fewer live registers; four waves per SIMD fit)
  F::forward(v, lds, L2 >= 8192 ? (int)(t + opaque_zero()) : (int)t, twd);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n2 = t + NT * e;
    const float2 w = cmul(wt, big_twiddle(tbig, k1 * (unsigned)(NT * e) + opaque_zero()));
    st_c64(cmul(v[F::out_slot(e)], w), rz, 8 * n2);
  }
}

// ---------------------------------------------------------------------------
// icols: X[b][n] = post[n] conj( sum_k1 Hc[b][k1][n2] W_L1^{n1 k1} ),
//        n = n1 L2 + n2 < M
// ---------------------------------------------------------------------------
template <int L1>
__global__ void __launch_bounds__(ColFft<L1>::NT)
    k_long_cols_inv(const float2 *__restrict__ Z, const float2 *__restrict__ c_post,
                    const float2 *__restrict__ tw_col, float2 *__restrict__ X, int64_t os, int64_t M, int L2,
                    int ncg) {
  using CF = ColFft<L1>;
  constexpr int E = CF::E, NTV = CF::NTV;
  __shared__ float2 lds[lds_points<L1 * kCols>()];
  __shared__ float2 twl[tw_lds_points<L1>()];
  const int t = threadIdx.x, c = t % kCols, tv = t / kCols;
  const int64_t q = xcd_item(blockIdx.x, gridDim.x);
  const int64_t b = q / ncg;
  const unsigned n2 = (unsigned)((q % ncg) * kCols + c);
  const TwLds twd = load_twiddles<L1>(twl, tw_col, t, CF::NT);
  __syncthreads();
  const int64_t L = (int64_t)L1 * L2;
  const Rsrc rz = make_rsrc(Z + b * L, (uint64_t)L * 8);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k1 = (unsigned)(tv + NTV * e);
    v[CF::in_slot(e)] = ld_c64(rz, 8 * (k1 * (unsigned)L2 + n2));
  }
  CF::forward(v, lds, tv, c, twd);
  // bins n >= M: post-multiplier reads 0 and the store is dropped
  const Rsrc rq = make_rsrc(c_post, (uint64_t)M * 8);
  const Rsrc rX = make_rsrc(X + b * os, (uint64_t)M * 8);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n = (unsigned)(tv + NTV * e) * (unsigned)L2 + n2;
    st_c64(cmul(cconj(v[CF::out_slot(e)]), ld_c64(rq, 8 * n)), rX, 8 * n);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
bool long_shape(int64_t L, int *L1) {
  auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
  if (L % 320 == 0 && pow2(L / 320) && L / 320 >= 256 && L / 320 <= kMaxL) {
    *L1 = 320;  // L = 5 * 2^a
    return true;
  }
  if (L < (int64_t)512 * 256 || L > (int64_t)1024 * kMaxL || !pow2(L)) return false;
  *L1 = (L <= (int64_t)512 * kMaxL) ? 512 : 1024;
  return true;
}

template <int L1>
static void launch_cols_fwd(const LongLaunch &a, const void *x, int64_t nb, hipStream_t s) {
  const dim3 grid((unsigned)(nb * (a.L2 / kCols))), block(ColFft<L1>::NT);
  switch (a.in_kind) {
    case 1:
      hipLaunchKernelGGL((k_long_cols_fwd<L1, 1>), grid, block, 0, s, x, a.xs, a.N, a.c_pre, a.tw_col, a.work,
                         a.L2);
      break;
    case 2:
      hipLaunchKernelGGL((k_long_cols_fwd<L1, 2>), grid, block, 0, s, x, a.xs, a.N, a.c_pre, a.tw_col, a.work,
                         a.L2);
      break;
    default:
      hipLaunchKernelGGL((k_long_cols_fwd<L1, 0>), grid, block, 0, s, x, a.xs, a.N, a.c_pre, a.tw_col, a.work,
                         a.L2);
  }
}

template <int L1, int L2>
static void launch_rows(const LongLaunch &a, int64_t nb, hipStream_t s) {
  hipLaunchKernelGGL((k_long_rows<L1, L2>), dim3((unsigned)(nb * L1)), dim3(Fft<L2>::NT), 0, s, a.work, a.Vt,
                     a.tw_row, a.tbig, nb);
}

template <int L1>
static bool launch_rows_l2(const LongLaunch &a, int64_t nb, hipStream_t s) {
  switch (a.L2) {
    case 256: launch_rows<L1, 256>(a, nb, s); return true;
    case 512: launch_rows<L1, 512>(a, nb, s); return true;
    case 1024: launch_rows<L1, 1024>(a, nb, s); return true;
    case 2048: launch_rows<L1, 2048>(a, nb, s); return true;
    case 4096: launch_rows<L1, 4096>(a, nb, s); return true;
    case 8192: launch_rows<L1, 8192>(a, nb, s); return true;
    case 16384: launch_rows<L1, 16384>(a, nb, s); return true;
  }
  return false;
}

template <int L1>
static hipError_t run_chunks(const LongLaunch &a, hipStream_t s) {
  const int XB = a.in_kind == 0 ? 4 : 8;
  // column groups holding some bin n < M (only columns n2 < M when M < L2)
  const int64_t live = a.M < a.L2 ? a.M : a.L2;
  const int ncg_out = (int)((live + kCols - 1) / kCols);
  for (int64_t b0 = 0; b0 < a.B; b0 += a.chunk) {
    const int64_t nb = (a.B - b0 < a.chunk) ? (a.B - b0) : a.chunk;
    const void *x = (const char *)a.x + b0 * a.xs * XB;
    launch_cols_fwd<L1>(a, x, nb, s);
    if (a.precision != TZ_FP32) {
      const hipError_t e = launch_long_rows_mfma(a, L1, nb, s);
      if (e != hipSuccess) return e;
    } else if (!launch_rows_l2<L1>(a, nb, s)) {
      return hipErrorInvalidValue;
    }
    // ncg_out * nb workgroups; the XCD numbering needs a multiple of 8
    const int64_t G = nb * ncg_out;
    if (G % 8 == 0) {
      hipLaunchKernelGGL((k_long_cols_inv<L1>), dim3((unsigned)G), dim3(ColFft<L1>::NT), 0, s, a.work, a.c_post,
                         a.tw_col, a.X + b0 * a.os, a.os, a.M, a.L2, ncg_out);
    } else {
      // pad the grid to whole columns groups of the full width (a multiple of 8)
      hipLaunchKernelGGL((k_long_cols_inv<L1>), dim3((unsigned)(nb * (a.L2 / kCols))), dim3(ColFft<L1>::NT), 0,
                         s, a.work, a.c_post, a.tw_col, a.X + b0 * a.os, a.os, a.M, a.L2, a.L2 / kCols);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_czt_long(const LongLaunch &a, hipStream_t s) {
  if (a.L1 == 320 && a.L2 >= 256 && a.L2 <= kMaxL) return run_chunks<320>(a, s);
  if (a.L1 == 512 && a.L2 >= 256 && a.L2 <= kMaxL) return run_chunks<512>(a, s);
  if (a.L1 == 1024 && a.L2 >= 256 && a.L2 <= kMaxL) return run_chunks<1024>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace tz
