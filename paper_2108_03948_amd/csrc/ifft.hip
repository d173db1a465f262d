// Inverse DFT of power-of-two length, one workgroup FFT per row:
//   x[n] = (1/L) sum_{k<L} X[k] W_L^{-k n} = (1/L) conj( FFT_L(conj X) )[n],
// the direct form for L = 256 .. 16384: one L-point FFT per row instead of
// the two FFTs of length >= 2L that the Bluestein form of the inverse runs.
// Conjugation and the power-of-two scale are exact, so the result carries
// only the FFT's own rounding.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.h"
#include "internal.h"

namespace tz {

template <int L>
__global__ void __launch_bounds__(Fft<L>::NT, 4)
    k_ifft_pow2(const float2 *__restrict__ X, int64_t xs, const float2 *__restrict__ tw, float2 *__restrict__ x,
                int64_t os) {
  using F = Fft<L>;
  constexpr int NT = F::NT, E = F::E;
  __shared__ float2 lds[lds_points<L>()];
  __shared__ float2 twl[tw_lds_points<L>()];
  const unsigned t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const TwLds twd = load_twiddles<L>(twl, tw, t, NT);
  __syncthreads();
  const Rsrc rX = make_rsrc(X + b * xs, (uint64_t)L * 8);
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[F::in_slot(e)] = cconj(ld_c64(rX, 8 * (t + NT * e)));
  F::forward(v, lds, (int)t, twd);
  const Rsrc rx = make_rsrc(x + b * os, (uint64_t)L * 8);
  constexpr float s = 1.0f / (float)L;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const float2 y = v[F::out_slot(e)];
    st_c64(make_float2(y.x * s, -y.y * s), rx, 8 * (t + NT * e));
  }
}

bool ifft_direct_supported(int64_t N) { return N >= 256 && N <= kMaxL && (N & (N - 1)) == 0; }

template <int L>
static void ifft_launch(const IfftLaunch &a, hipStream_t s) {
  hipLaunchKernelGGL((k_ifft_pow2<L>), dim3((unsigned)a.B), dim3(Fft<L>::NT), 0, s, a.X, a.xs, a.tw, a.x, a.os);
}

hipError_t launch_ifft_pow2(const IfftLaunch &a, hipStream_t s) {
  if (a.B < 1 || a.B > INT32_MAX) return hipErrorInvalidValue;
  switch (a.L) {
    case 256: ifft_launch<256>(a, s); break;
    case 512: ifft_launch<512>(a, s); break;
    case 1024: ifft_launch<1024>(a, s); break;
    case 2048: ifft_launch<2048>(a, s); break;
    case 4096: ifft_launch<4096>(a, s); break;
    case 8192: ifft_launch<8192>(a, s); break;
    case 16384: ifft_launch<16384>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tz
