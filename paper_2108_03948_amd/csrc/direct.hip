// The CZT of eq. (11) by direct summation in FP64 (precision TZ_FP64):
//   X[k] = sum_{n<N} x[n] A^{-n} W^{n k} = sum_n x[n] z_k^n,  z_k = A^{-1} W^k,
// for any contour, including spirals (eqs. (16)-(17)) whose chirp magnitudes
// spread too far for the FP32 Bluestein tables.  One thread per bin k
// carries z_k^n by repeated multiplication (relative rounding ~ n 2^-53);
// z_k comes from the logarithms of A and W (ln z_k = -ln A + k ln W), so its
// angle is -arg A + k arg W reduced by the FP64 sincos.  Workgroups stage 256
// samples at a time in LDS, read by every thread.  The bins are written as
// complex128 (a steep spiral's bins span far more than FP32's range).
// O(N M) work per trace: a reference-quality path, not a fast one.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fft_core.h"
#include "internal.h"

namespace tz {

namespace {

constexpr int kDirectThreads = 256;

template <int KIND>
__global__ void __launch_bounds__(kDirectThreads)
    k_czt_direct64(const void *__restrict__ x, int64_t xs, int64_t N, double2 *__restrict__ X, int64_t os,
                   int64_t M, double ma, double ta, double mw, double tw) {
  __shared__ double xl[kDirectThreads];
  const int64_t nbk = (M + kDirectThreads - 1) / kDirectThreads;  // workgroups per trace
  const int64_t b = blockIdx.x / nbk;
  const int64_t k = (blockIdx.x % nbk) * kDirectThreads + threadIdx.x;
  const double lr = -ma + (double)k * mw, li = -ta + (double)k * tw;
  double sn, cs;
  sincos(li, &sn, &cs);
  const double e = exp(lr);
  const double zr = e * cs, zi = e * sn;
  double pr = 1.0, pi = 0.0, ar = 0.0, ai = 0.0;
  const Rsrc rx = make_rsrc((const char *)x + b * xs * (KIND == 1 ? 8 : 4), (uint64_t)N * (KIND == 1 ? 8 : 4));
  for (int64_t n0 = 0; n0 < N; n0 += kDirectThreads) {
    __syncthreads();  // the previous chunk is read
    const unsigned n = (unsigned)(n0 + threadIdx.x);
    xl[threadIdx.x] = KIND == 1 ? ld_f64(rx, 8 * n) : (double)ld_f32(rx, 4 * n);  // past N: 0
    __syncthreads();
    const int cnt = N - n0 < kDirectThreads ? (int)(N - n0) : kDirectThreads;
    for (int i = 0; i < cnt; ++i) {
      const double xv = xl[i];
      ar = fma(xv, pr, ar);
      ai = fma(xv, pi, ai);
      const double t = fma(pr, zr, -pi * zi);
      pi = fma(pr, zi, pi * zr);
      pr = t;
    }
  }
  // threads past M took part in the staging; only bins k < M are stored
  if (k < M) X[b * os + k] = make_double2(ar, ai);
}

}  // namespace

hipError_t launch_czt_direct64(const DirectLaunch &a, hipStream_t s) {
  const dim3 grid((unsigned)((a.M + kDirectThreads - 1) / kDirectThreads * a.B)), block(kDirectThreads);
  if (a.in_kind == 1)
    hipLaunchKernelGGL(k_czt_direct64<1>, grid, block, 0, s, a.x, a.xs, a.N, a.X, a.os, a.M, a.ma, a.ta, a.mw, a.tw);
  else
    hipLaunchKernelGGL(k_czt_direct64<0>, grid, block, 0, s, a.x, a.xs, a.N, a.X, a.os, a.M, a.ma, a.ta, a.mw, a.tw);
  return hipGetLastError();
}

}  // namespace tz
