// Device FFT core for gfx950: one L-point complex FFT per workgroup, data held
// in registers, radix-R butterflies computed in registers, and the data
// exchange between radix passes staged through LDS (Stockham autosort order,
// so the result comes out in natural order with no bit reversal).
//
// Register layout.  A workgroup of NT threads holds L = NT * E points; thread
// t owns the E points t + NT*e (e < E).  Within a pass of radix R a thread
// runs E/R butterflies; butterfly i of thread t has index j = t + i*NT and
// reads inputs j + r*L/R, r < R.  The input of the first pass and the output
// of the last pass therefore both sit at t + NT*e, so global loads and stores
// at both ends are coalesced (consecutive lanes, consecutive addresses), and
// a forward FFT followed by a pointwise product and another FFT needs no LDS
// round trip between the two.
//
// Twiddles come from a table tw[m] = exp(-j 2 pi m / L), m < L, built in
// double precision and rounded once to float.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tz {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -j
__device__ __forceinline__ float2 cmul_mj(float2 a) { return make_float2(a.y, -a.x); }

// ---------------------------------------------------------------------------
// compile-time cos / sin of 2 pi m / R (double, reduced to the first octant)
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// angle 2 pi m / R, exact octant reduction using integer arithmetic on 8m
struct CS {
  double c, s;
};
constexpr CS unit_root(long m, long R) {
  m %= R;
  if (m < 0) m += R;
  // position in units of R/8: work with 8m / R as an exact rational
  long num = 8 * m;  // angle = (num / R) * (pi/4)
  long oct = num / R;
  long rem = num - oct * R;  // angle inside octant = rem/R * pi/4
  double a = (double)rem / (double)R * (kPi / 4.0);
  double c0 = taylor_cos(a), s0 = taylor_sin(a);
  double b = (kPi / 4.0) - a;  // complementary angle for odd octants
  double cb = taylor_cos(b), sb = taylor_sin(b);
  switch (oct) {
    case 0: return CS{c0, s0};
    case 1: return CS{sb, cb};
    case 2: return CS{-s0, c0};
    case 3: return CS{-cb, sb};
    case 4: return CS{-c0, -s0};
    case 5: return CS{-sb, -cb};
    case 6: return CS{s0, -c0};
    default: return CS{cb, -sb};
  }
}

// x * exp(-j 2 pi m / R) with m, R compile-time constants
template <long M, long R>
__device__ __forceinline__ float2 twiddle_const(float2 x) {
  constexpr long mm = ((M % R) + R) % R;
  if constexpr (mm == 0) {
    return x;
  } else if constexpr (4 * mm == R) {  // -j
    return make_float2(x.y, -x.x);
  } else if constexpr (2 * mm == R) {  // -1
    return make_float2(-x.x, -x.y);
  } else if constexpr (4 * mm == 3 * R) {  // +j
    return make_float2(-x.y, x.x);
  } else {
    constexpr CS w = unit_root(mm, R);
    constexpr float c = (float)w.c;
    constexpr float s = (float)(-w.s);  // exp(-j a) = cos a - j sin a
    return make_float2(fmaf(x.x, c, -x.y * s), fmaf(x.x, s, x.y * c));
  }
}

// ---------------------------------------------------------------------------
// in-register DFT of size R (forward, natural order in and out).
// v points at R values spaced S apart in a register array.
// ---------------------------------------------------------------------------
template <int R>
struct Dft;

template <>
struct Dft<1> {
  template <int S>
  __device__ __forceinline__ static void run(float2 *) {}
};

template <>
struct Dft<2> {
  template <int S>
  __device__ __forceinline__ static void run(float2 *v) {
    float2 a = v[0], b = v[S];
    v[0] = cadd(a, b);
    v[S] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  template <int S>
  __device__ __forceinline__ static void run(float2 *v) {
    float2 t0 = cadd(v[0], v[2 * S]);
    float2 t1 = csub(v[0], v[2 * S]);
    float2 t2 = cadd(v[S], v[3 * S]);
    float2 t3 = cmul_mj(csub(v[S], v[3 * S]));
    v[0] = cadd(t0, t2);
    v[2 * S] = csub(t0, t2);
    v[S] = cadd(t1, t3);
    v[3 * S] = csub(t1, t3);
  }
};

// Generic R = R1 * R2 (R1 = 4 when possible, else 2), decimation in time by
// index mapping: X[k1 + R1 k2] = sum_{n2} W_R2^{n2 k2} W_R^{n2 k1}
//                                 sum_{n1} v[R2 n1 + n2] W_R1^{n1 k1}.
template <int R>
struct Dft {
  static constexpr int R1 = (R % 4 == 0 && R > 4) ? 4 : 2;
  static constexpr int R2 = R / R1;

  template <int N2, int K1, int S>
  __device__ __forceinline__ static void tw_one(float2 *a) {
    a[(N2 * R1 + K1) * S] = twiddle_const<(long)N2 * K1, R>(a[(N2 * R1 + K1) * S]);
  }
  template <int N2, int S, int... K1s>
  __device__ __forceinline__ static void tw_row(float2 *a, std::integer_sequence<int, K1s...>) {
    (tw_one<N2, K1s, S>(a), ...);
  }
  template <int S, int... N2s>
  __device__ __forceinline__ static void tw_all(float2 *a, std::integer_sequence<int, N2s...>) {
    (tw_row<N2s, S>(a, std::make_integer_sequence<int, R1>{}), ...);
  }

  template <int S>
  __device__ __forceinline__ static void run(float2 *v) {
    // gather into a[n2][n1] (n2 major), DFT_R1 along n1
    float2 a[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2)
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n2 * R1 + n1] = v[(R2 * n1 + n2) * S];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) Dft<R1>::template run<1>(&a[n2 * R1]);
    // twiddle a[n2][k1] by W_R^{n2 k1}
    tw_all<1>(a, std::make_integer_sequence<int, R2>{});
    // DFT_R2 along n2 for each k1: elements a[n2*R1 + k1], stride R1
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) Dft<R2>::template run<R1>(&a[k1]);
    // output index k1 + R1 k2 holds a[k2*R1 + k1]
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) v[(k1 + R1 * k2) * S] = a[k2 * R1 + k1];
  }
};

// ---------------------------------------------------------------------------
// Radix plans.  A plan lists the radices of the passes, first pass first.
// ---------------------------------------------------------------------------
template <int... Rs>
struct Radices {
  static constexpr int count = sizeof...(Rs);
  static constexpr int list[count] = {Rs...};
  static constexpr int product() {
    int p = 1;
    for (int i = 0; i < count; ++i) p *= list[i];
    return p;
  }
};

template <int L>
struct FftShape;
// L, threads, elements per thread, radices
template <> struct FftShape<256>   { static constexpr int NT = 64;  using Plan = Radices<4, 4, 4, 4>; };
template <> struct FftShape<512>   { static constexpr int NT = 64;  using Plan = Radices<8, 8, 8>; };
template <> struct FftShape<1024>  { static constexpr int NT = 64;  using Plan = Radices<16, 16, 4>; };
template <> struct FftShape<2048>  { static constexpr int NT = 128; using Plan = Radices<16, 16, 8>; };
template <> struct FftShape<4096>  { static constexpr int NT = 256; using Plan = Radices<16, 16, 16>; };
template <> struct FftShape<8192>  { static constexpr int NT = 512; using Plan = Radices<16, 16, 16, 2>; };
template <> struct FftShape<16384> { static constexpr int NT = 1024; using Plan = Radices<16, 16, 16, 4>; };

// A zero the optimiser cannot see through (empty asm on an SGPR).  Adding it
// to a table index keeps the load where it is written: the compiler can
// neither hoist it above this point nor merge it with an identical load of
// an earlier pass (which would keep the values live across passes, or across
// the two FFTs of a Bluestein transform, and exhaust registers).  The pointer
// itself is untouched, so the load stays a global (not flat) access.
__device__ __forceinline__ unsigned opaque_zero() {
  unsigned z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// index clamped into [0, lim) for loads that must not branch (lim >= 1);
// the caller discards the value where a < lim fails
__device__ __forceinline__ unsigned clamp_idx(unsigned a, unsigned lim) { return a < lim ? a : lim - 1; }

// LDS index with one pad slot every 16 points (breaks the power-of-two
// strides of the first passes across banks)
__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 4); }
template <int L>
constexpr int lds_points() { return L + L / 16; }

// register slot of element e (point t + NT*e) in the layout of a radix-R pass
template <int E, int R>
__host__ __device__ constexpr int slot_of(int e) { return (e % (E / R)) * R + e / (E / R); }

template <int L>
struct Fft {
  static constexpr int NT = FftShape<L>::NT;
  static constexpr int E = L / NT;
  using Plan = typename FftShape<L>::Plan;
  static constexpr int P = Plan::count;
  static constexpr int R_first = Plan::list[0];
  static constexpr int R_last = Plan::list[P - 1];
  static_assert(Plan::product() == L, "radix plan must multiply to L");

  // slot holding element e at the input of the first pass / output of the last
  __device__ __forceinline__ static constexpr int in_slot(int e) { return slot_of<E, R_first>(e); }
  __device__ __forceinline__ static constexpr int out_slot(int e) { return slot_of<E, R_last>(e); }

  static constexpr int ns_before(int p) {
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= Plan::list[i];
    return ns;
  }

  // one pass: twiddle + butterfly in registers, then (unless last) exchange
  // through LDS into the layout of the next pass.
  template <int p>
  __device__ __forceinline__ static void pass(float2 (&v)[E], float2 *lds, int t,
                                              const float2 *__restrict__ tw) {
    constexpr int R = Plan::list[p];
    constexpr int NS = ns_before(p);
    constexpr int NB = E / R;
    constexpr int TWS = L / (NS * R);  // table stride of this pass
    const unsigned z = opaque_zero();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if constexpr (NS > 1) {
        const unsigned jm = (unsigned)(j % NS);
#pragma unroll
        for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], tw[jm * r * TWS + z]);
      }
      Dft<R>::template run<1>(&v[i * R]);
    }
    if constexpr (p + 1 < P) {
      constexpr int R2 = Plan::list[p + 1];
      constexpr int NB2 = E / R2;
      __syncthreads();  // previous readers of LDS are done
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + i * NT;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_idx(base + r * NS)] = v[i * R + r];
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NB2; ++i) {
        const int j = t + i * NT;
#pragma unroll
        for (int r = 0; r < R2; ++r) v[i * R2 + r] = lds[lds_idx(j + r * (L / R2))];
      }
    }
  }

  template <int... ps>
  __device__ __forceinline__ static void run_passes(float2 (&v)[E], float2 *lds, int t,
                                                    const float2 *__restrict__ tw,
                                                    std::integer_sequence<int, ps...>) {
    (pass<ps>(v, lds, t, tw), ...);
  }

  // forward FFT in place: v in "in_slot" layout -> v in "out_slot" layout
  __device__ __forceinline__ static void forward(float2 (&v)[E], float2 *lds, int t,
                                                 const float2 *__restrict__ tw) {
    run_passes(v, lds, t, tw, std::make_integer_sequence<int, P>{});
  }

  // re-label registers from the output layout to the input layout
  __device__ __forceinline__ static void out_to_in(float2 (&v)[E]) {
    if constexpr (R_first != R_last) {
      float2 w[E];
#pragma unroll
      for (int e = 0; e < E; ++e) w[in_slot(e)] = v[out_slot(e)];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = w[e];
    }
  }
};

}  // namespace tz
