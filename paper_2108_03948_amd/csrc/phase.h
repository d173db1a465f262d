// Double-precision phase generation shared by the plan-time table builders.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace tz {

// ---------------------------------------------------------------------------
// phase generation
// ---------------------------------------------------------------------------
// Fractional part of a * m for double a and integer m < 2^53, with the product
// formed exactly as hi + lo (error-free transformation through fma), so the
// result is accurate to ~1e-16 cycles however large a * m is.
static __device__ __forceinline__ double frac_mul(double a, double m) {
  double hi = a * m;
  double lo = fma(a, m, -hi);
  double f = hi - floor(hi);
  f += lo;
  return f - floor(f);
}

// (a * b) mod q for 0 <= a, b < q < 2^63, by doubling and adding (64-bit
// arithmetic only; plan time, so the loop cost does not matter)
static __device__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t r = 0;
  a %= q;
  b %= q;
  while (b) {
    if (b & 1) {
      r += a;
      if (r >= q) r -= q;
    }
    a += a;
    if (a >= q) a -= q;
    b >>= 1;
  }
  return r;
}

// Chirp phase in cycles (the value is e^{-j 2 pi cycles}), with
// A = e^{j 2 pi a} and W = e^{-j 2 pi w}:
//   with_a:  a n + w n^2/2     (A^{-n} W^{n^2/2}, eq. (13) premultiply)
//   else:        w n^2/2       (W^{n^2/2}, eq. (13) postmultiply)
// Rational mode (a = pa/q, w = pw/q): the numerator 2 pa n + pw n^2 is reduced
// modulo 2q exactly in integers before the angle is formed.  Float mode: each
// product is split exactly into hi + lo before its integer part is dropped.
static __device__ double chirp_cycles(const PhaseParams &p, int64_t n, bool with_a) {
  if (p.rational) {
    const uint64_t q2 = 2 * (uint64_t)p.q;
    uint64_t un = (uint64_t)n % q2;
    uint64_t r = mulmod((uint64_t)p.pw, mulmod(un, un, q2), q2);
    if (with_a) r = (r + mulmod(2 * (uint64_t)p.pa % q2, un, q2)) % q2;
    return (double)r / (double)q2;
  }
  double f = frac_mul(0.5 * p.w, (double)n * (double)n);
  if (with_a) f += frac_mul(p.a, (double)n);
  return f - floor(f);
}

// cycles of W^{k0 n} (w k0 n), used to move a bin block to start k0
static __device__ double shift_cycles(const PhaseParams &p, int64_t k0, int64_t n) {
  if (p.rational) {
    const uint64_t q = (uint64_t)p.q;
    uint64_t r = mulmod(mulmod((uint64_t)p.pw, (uint64_t)k0 % q, q), (uint64_t)n % q, q);
    return (double)r / (double)q;
  }
  return frac_mul(p.w, (double)k0 * (double)n);
}

static __device__ __forceinline__ float2 unit_cycles(double cyc) {
  double s, c;
  sincospi(-2.0 * cyc, &s, &c);
  return make_float2((float)c, (float)s);
}

// e^{logmag} e^{-j 2 pi cyc}, formed in double and rounded once
static __device__ __forceinline__ float2 scaled_cycles(double cyc, double logmag) {
  double s, c;
  sincospi(-2.0 * cyc, &s, &c);
  const double m = exp(logmag);
  return make_float2((float)(m * c), (float)(m * s));
}

static __device__ __forceinline__ bool spiral(const PhaseParams &p) { return p.ma != 0.0 || p.mw != 0.0; }

}  // namespace tz
