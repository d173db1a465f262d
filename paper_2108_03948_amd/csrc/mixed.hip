// Mixed-radix FFT of one row per thread group for any 7-smooth length
// L = 2^a 3^b 5^c 7^d: the zero-padded FFT of eqs. (2)-(5) when N_fft has no
// power-of-two factorisation the dedicated kernels take, and the inverse DFT
// (the IFFT Section 4 times against the FFT) at such lengths, without the
// two longer FFTs of the Bluestein form.
//
// Stockham autosort passes of radix 2, 3, 4, 5, 7 or 8 in the order of the
// plan.  Pass p (radix R, NS = product of the earlier radices) runs the L/R
// butterflies j: inputs j + r L/R (r < R), twiddled by W_{NS R}^{(j mod NS) r},
// a DFT_R in registers, outputs to (j / NS) NS R + j mod NS + r NS.  The first
// pass reads the row straight from global memory and the last writes the
// spectrum straight to it (both coalesced: consecutive j, consecutive
// addresses); the passes between exchange through LDS, each thread holding
// all of its butterflies' inputs in registers between two barriers, so the
// exchange is in place.  Each pass's twiddles sit in a table of their own,
// entry (r - 1) NS + (j mod NS): consecutive butterflies read consecutive
// entries.
//
// Rows are dealt to groups of NT threads, ROWS groups per workgroup, with
// the row length bounded by LMAX: short rows run one wavefront each (wave
// barriers only), long rows a whole workgroup and up to all 160 KB of LDS.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fft_core.h"
#include "internal.h"

namespace tz {

namespace {

// j / NS for j, NS < 2^16: floor(j * ceil(2^32 / NS) / 2^32) is exact there
// (the rounding term j / 2^32 stays below 1 / NS)
__device__ __forceinline__ unsigned div_ns(unsigned j, unsigned m) { return __umulhi(j, m); }

template <int NT>
__device__ __forceinline__ void group_sync() {
  if constexpr (NT == 64)
    wave_sync();
  else
    __syncthreads();
}

template <int NT, int LMAX, int R, int MODE>
__device__ __forceinline__ void mix_pass(int p, const MixPlan &pl, float2 *buf, Rsrc rx, Rsrc rX,
                                         const float2 *twp, float scale, unsigned t) {
  constexpr int NB = (LMAX / R + NT - 1) / NT;  // butterflies per thread at most
  const int L = pl.L, nbf = L / R;
  const unsigned NS = (unsigned)pl.NS[p], nsm = pl.nsm[p];
  const float2 *tw = twp + pl.TO[p];
  const bool first = p == 0, last = p == pl.npass - 1;
  float2 v[NB * R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const unsigned j = t + NT * i;
    if ((int)j < nbf) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const unsigned idx = j + (unsigned)(r * nbf);
        float2 z;
        if (first) {
          if constexpr (MODE == 2) {
            z = cconj(ld_c64(rx, 8 * idx));  // inverse: conjugate, forward FFT, conjugate
          } else {
            z = make_float2(ld_real<MODE>(rx, idx), 0.f);  // samples past N read as 0
          }
        } else {
          z = buf[idx];
        }
        v[i * R + r] = z;
      }
    }
  }
  if (!first) group_sync<NT>();  // every input of this pass is in registers before any output lands
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const unsigned j = t + NT * i;
    if ((int)j < nbf) {
      const unsigned q = NS > 1 ? div_ns(j, nsm) : j;
      const unsigned jm = j - q * NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], tw[(unsigned)(r - 1) * NS + jm]);
      }
      Dft<R>::template run<1>(&v[i * R]);
      const unsigned base = q * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const unsigned pos = base + (unsigned)r * NS;
        if (last) {
          if constexpr (MODE == 2)
            st_c64(cscale(cconj(v[i * R + r]), scale), rX, 8 * pos);
          else
            st_c64(v[i * R + r], rX, 8 * pos);  // bins past nout are dropped
        } else {
          buf[pos] = v[i * R + r];
        }
      }
    }
  }
  if (!last) group_sync<NT>();  // outputs visible to the next pass
}

// MODE 0 / 1: real f32 / f64 rows of N samples zero-padded to L, bins k < nout
// written; MODE 2: complex rows of L points, inverse DFT with scale 1/L.
// TWL: the per-pass twiddle tables (fewer than LMAX entries) are copied to
// LDS once per workgroup and read there; otherwise they are read from global
// memory (L2).
template <int NT, int LMAX, int ROWS, bool TWL, int MODE>
__global__ void __launch_bounds__(NT *ROWS)
    k_fft_mixed(const void *__restrict__ x, int64_t xs, int64_t N, float2 *__restrict__ X, int64_t os,
                int64_t nout, MixPlan pl, const float2 *__restrict__ twg, float scale, int64_t B) {
  static_assert(NT == 64 || ROWS == 1, "workgroup barriers need every group of the workgroup");
  __shared__ float2 lds[ROWS * LMAX + (TWL ? LMAX : 0)];
  const float2 *twp = twg;
  if constexpr (TWL) {
    // every wave of the workgroup takes part before any of them may leave
    float2 *twl = lds + ROWS * LMAX;
    for (int i = threadIdx.x; i < pl.ntw; i += NT * ROWS) twl[i] = twg[i];
    __syncthreads();
    twp = twl;
  }
  const unsigned g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int64_t b = (int64_t)blockIdx.x * ROWS + g;
  // a group past the last row leaves: with NT = 64 it is a wave of its own
  // and has no workgroup barrier to join; larger NT run one row per
  // workgroup, which always exists
  if (b >= B) return;
  constexpr int XB = MODE == 1 ? 8 : (MODE == 2 ? 8 : 4);
  const Rsrc rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)(MODE == 2 ? pl.L : N) * XB);
  const Rsrc rX = make_rsrc(X + b * os, (uint64_t)nout * 8);
  float2 *buf = lds + g * LMAX;
  // the plan lists its radices grouped (8s, one 4 or 2, 3s, 5s, 7s): one loop
  // per radix keeps each pass body's registers to itself
  int p = 0;
  for (; p < pl.npass && pl.R[p] == 8; ++p) mix_pass<NT, LMAX, 8, MODE>(p, pl, buf, rx, rX, twp, scale, t);
  for (; p < pl.npass && pl.R[p] == 4; ++p) mix_pass<NT, LMAX, 4, MODE>(p, pl, buf, rx, rX, twp, scale, t);
  for (; p < pl.npass && pl.R[p] == 2; ++p) mix_pass<NT, LMAX, 2, MODE>(p, pl, buf, rx, rX, twp, scale, t);
  for (; p < pl.npass && pl.R[p] == 3; ++p) mix_pass<NT, LMAX, 3, MODE>(p, pl, buf, rx, rX, twp, scale, t);
  for (; p < pl.npass && pl.R[p] == 5; ++p) mix_pass<NT, LMAX, 5, MODE>(p, pl, buf, rx, rX, twp, scale, t);
  for (; p < pl.npass && pl.R[p] == 7; ++p) mix_pass<NT, LMAX, 7, MODE>(p, pl, buf, rx, rX, twp, scale, t);
}

// per-pass twiddle tables: pass p, entry (r - 1) NS + jm = W_{NS R}^{jm r}
// (FP64 angle from the exact residue jm r mod NS R, rounded once to float)
__global__ void k_mix_twiddles(float2 *twp, MixPlan pl) {
  const int p = blockIdx.y;
  const int R = pl.R[p], NS = pl.NS[p];
  const int n = (R - 1) * NS;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int r = i / NS + 1, jm = i % NS;
    const int64_t q = (int64_t)NS * R, m = ((int64_t)jm * r) % q;
    double s, c;
    sincospi(-2.0 * (double)m / (double)q, &s, &c);
    twp[pl.TO[p] + i] = make_float2((float)c, (float)s);
  }
}

template <int NT, int LMAX, int ROWS, bool TWL, int MODE>
void mix_launch_tier(const MixLaunch &a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.B + ROWS - 1) / ROWS);
  hipLaunchKernelGGL((k_fft_mixed<NT, LMAX, ROWS, TWL, MODE>), dim3(grid), dim3(NT * ROWS), 0, s, a.x, a.xs, a.N,
                     a.X, a.os, a.nout, a.plan, a.tw, a.scale, a.B);
}

// tiers by row length: threads per row, longest row, rows per workgroup,
// twiddles in LDS (LDS (ROWS + TWL) x LMAX x 8 bytes: 40, 20, 40, 80, 160 KB).
// The twiddle copy pays off only where it costs no occupancy (the one-wave
// rows): with one row per workgroup it halves the workgroups per CU.
template <int MODE>
void mix_launch(const MixLaunch &a, hipStream_t s) {
  const int L = a.plan.L;
  if (L <= 1024)
    mix_launch_tier<64, 1024, 4, true, MODE>(a, s);
  else if (L <= 2560)
    mix_launch_tier<256, 2560, 1, false, MODE>(a, s);
  else if (L <= 5120)
    mix_launch_tier<256, 5120, 1, false, MODE>(a, s);
  else if (L <= 10240)
    mix_launch_tier<512, 10240, 1, false, MODE>(a, s);
  else
    mix_launch_tier<1024, kMixMaxL, 1, false, MODE>(a, s);
}

}  // namespace

bool mix_plan(int64_t L, MixPlan *pl) {
  if (L < kMixMinL || L > kMixMaxL) return false;
  int64_t rest = L;
  int n = 0;
  int R[kMixMaxPasses];
  // radix 8 while it divides, then one 4 or 2 for the rest of the power of
  // two, then the odd radices
  while (rest % 8 == 0) R[n++] = 8, rest /= 8;
  if (rest % 4 == 0) R[n++] = 4, rest /= 4;
  if (rest % 2 == 0) R[n++] = 2, rest /= 2;
  for (int f : {3, 5, 7})
    while (rest % f == 0) {
      if (n == kMixMaxPasses) return false;
      R[n++] = f;
      rest /= f;
    }
  if (rest != 1 || n == 0) return false;
  pl->L = (int)L;
  pl->npass = n;
  int64_t ns = 1, off = 0;
  for (int p = 0; p < n; ++p) {
    pl->R[p] = R[p];
    pl->NS[p] = (int)ns;
    pl->TO[p] = (int)off;
    off += (R[p] - 1) * ns;
    pl->nsm[p] = ns > 1 ? (uint32_t)((((uint64_t)1 << 32) + ns - 1) / ns) : 0u;
    ns *= R[p];
  }
  pl->ntw = (int)off;
  return true;
}

hipError_t build_mix_twiddles(float2 *twp, const MixPlan &pl, hipStream_t s) {
  hipLaunchKernelGGL(k_mix_twiddles, dim3(8, (unsigned)pl.npass), dim3(256), 0, s, twp, pl);
  return hipGetLastError();
}

hipError_t launch_fft_mixed(const MixLaunch &a, hipStream_t s) {
  switch (a.mode) {
    case 0: mix_launch<0>(a, s); break;
    case 1: mix_launch<1>(a, s); break;
    case 2: mix_launch<2>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tz
