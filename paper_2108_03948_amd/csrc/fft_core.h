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

#include <utility>

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

// 5-point DFT: with t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4, t4 = x2 - x3,
//   X1,4 = x0 + c1 t1 + c2 t2 -/+ j (s1 t3 + s2 t4),
//   X2,3 = x0 + c2 t1 + c1 t2 -/+ j (s2 t3 - s1 t4),
// c_m = cos(2 pi m/5), s_m = sin(2 pi m/5)
template <>
struct Dft<5> {
  template <int S>
  __device__ __forceinline__ static void run(float2 *v) {
    constexpr CS w1 = unit_root(1, 5), w2 = unit_root(2, 5);
    constexpr float c1 = (float)w1.c, s1 = (float)w1.s, c2 = (float)w2.c, s2 = (float)w2.s;
    const float2 x0 = v[0];
    const float2 t1 = cadd(v[S], v[4 * S]), t2 = cadd(v[2 * S], v[3 * S]);
    const float2 t3 = csub(v[S], v[4 * S]), t4 = csub(v[2 * S], v[3 * S]);
    const float2 a1 = make_float2(fmaf(c2, t2.x, fmaf(c1, t1.x, x0.x)), fmaf(c2, t2.y, fmaf(c1, t1.y, x0.y)));
    const float2 a2 = make_float2(fmaf(c1, t2.x, fmaf(c2, t1.x, x0.x)), fmaf(c1, t2.y, fmaf(c2, t1.y, x0.y)));
    // b1 = s1 t3 + s2 t4, b2 = s2 t3 - s1 t4; -j b = (b.y, -b.x)
    const float2 b1 = make_float2(fmaf(s1, t3.x, s2 * t4.x), fmaf(s1, t3.y, s2 * t4.y));
    const float2 b2 = make_float2(fmaf(s2, t3.x, -s1 * t4.x), fmaf(s2, t3.y, -s1 * t4.y));
    v[0] = cadd(x0, cadd(t1, t2));
    v[S] = cadd(a1, cmul_mj(b1));
    v[4 * S] = csub(a1, cmul_mj(b1));
    v[2 * S] = cadd(a2, cmul_mj(b2));
    v[3 * S] = csub(a2, cmul_mj(b2));
  }
};

// 3-point DFT: with t = x1 + x2, u = x1 - x2,
//   X0 = x0 + t,  X1,2 = x0 - t/2 -/+ j (sqrt(3)/2) u
template <>
struct Dft<3> {
  template <int S>
  __device__ __forceinline__ static void run(float2 *v) {
    constexpr float h = (float)0.86602540378443864676;  // sqrt(3)/2
    const float2 x0 = v[0];
    const float2 t = cadd(v[S], v[2 * S]), u = csub(v[S], v[2 * S]);
    const float2 m = make_float2(fmaf(-0.5f, t.x, x0.x), fmaf(-0.5f, t.y, x0.y));
    // -j h u = (h u.y, -h u.x)
    const float2 b = make_float2(h * u.y, -h * u.x);
    v[0] = cadd(x0, t);
    v[S] = cadd(m, b);
    v[2 * S] = csub(m, b);
  }
};

// 7-point DFT over the symmetric pairs t_m = x_m + x_{7-m}, u_m = x_m - x_{7-m}
// (m = 1, 2, 3):  X_k, X_{7-k} = x0 + sum_m c_{km} t_m -/+ j sum_m s_{km} u_m,
// c_{km} = cos(2 pi k m / 7), s_{km} = sin(2 pi k m / 7)
template <>
struct Dft<7> {
  template <int K, int S>
  __device__ __forceinline__ static void out(float2 *v, float2 x0, const float2 (&t)[3], const float2 (&u)[3]) {
    constexpr CS w1 = unit_root(K * 1, 7), w2 = unit_root(K * 2, 7), w3 = unit_root(K * 3, 7);
    constexpr float c1 = (float)w1.c, c2 = (float)w2.c, c3 = (float)w3.c;
    constexpr float s1 = (float)w1.s, s2 = (float)w2.s, s3 = (float)w3.s;
    const float2 a = make_float2(fmaf(c3, t[2].x, fmaf(c2, t[1].x, fmaf(c1, t[0].x, x0.x))),
                                 fmaf(c3, t[2].y, fmaf(c2, t[1].y, fmaf(c1, t[0].y, x0.y))));
    const float2 bb = make_float2(fmaf(s3, u[2].x, fmaf(s2, u[1].x, s1 * u[0].x)),
                                  fmaf(s3, u[2].y, fmaf(s2, u[1].y, s1 * u[0].y)));
    v[K * S] = cadd(a, cmul_mj(bb));
    v[(7 - K) * S] = csub(a, cmul_mj(bb));
  }
  template <int S>
  __device__ __forceinline__ static void run(float2 *v) {
    const float2 x0 = v[0];
    const float2 t[3] = {cadd(v[S], v[6 * S]), cadd(v[2 * S], v[5 * S]), cadd(v[3 * S], v[4 * S])};
    const float2 u[3] = {csub(v[S], v[6 * S]), csub(v[2 * S], v[5 * S]), csub(v[3 * S], v[4 * S])};
    out<1, S>(v, x0, t, u);
    out<2, S>(v, x0, t, u);
    out<3, S>(v, x0, t, u);
    v[0] = cadd(x0, cadd(t[0], cadd(t[1], t[2])));
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
template <> struct FftShape<320>   { static constexpr int NT = 16;  using Plan = Radices<5, 4, 4, 4>; };
template <> struct FftShape<256>   { static constexpr int NT = 64;  using Plan = Radices<4, 4, 4, 4>; };
template <> struct FftShape<512>   { static constexpr int NT = 64;  using Plan = Radices<8, 8, 8>; };
template <> struct FftShape<1024>  { static constexpr int NT = 64;  using Plan = Radices<16, 16, 4>; };
template <> struct FftShape<2048>  { static constexpr int NT = 128; using Plan = Radices<16, 16, 8>; };
template <> struct FftShape<4096>  { static constexpr int NT = 256; using Plan = Radices<16, 16, 16>; };
template <> struct FftShape<8192>  { static constexpr int NT = 512; using Plan = Radices<16, 2, 16, 16>; };
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

// ---------------------------------------------------------------------------
// Buffer access.  A buffer resource holds a uniform base address and a byte
// extent in scalar registers; each lane supplies a 32-bit byte offset.  Reads
// at or past the extent return 0 and writes there are dropped (the hardware
// range check of raw buffers), which gives zero padding and ragged tails
// without per-lane address arithmetic or branches.
// ---------------------------------------------------------------------------
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc make_rsrc(const void *base, uint64_t bytes) {
  const uint32_t n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, 0x00020000);
}
__device__ __forceinline__ float ld_f32(Rsrc r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double ld_f64(Rsrc r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ float2 ld_c64(Rsrc r, unsigned off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void st_c64(float2 v, Rsrc r, unsigned off) {
  using U2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)off, 0, 0);
}
// real sample n of a float (KIND 0) or double (KIND 1) trace
template <int KIND>
__device__ __forceinline__ float ld_real(Rsrc r, unsigned n) {
  if constexpr (KIND == 1)
    return (float)ld_f64(r, 8 * n);
  else
    return ld_f32(r, 4 * n);
}

// index clamped into [0, lim) for loads that must not branch (lim >= 1);
// the caller discards the value where a < lim fails
__device__ __forceinline__ unsigned clamp_idx(unsigned a, unsigned lim) { return a < lim ? a : lim - 1; }

// Twiddles W_L^m = e^{-j 2 pi m / L} held in LDS as two short tables,
//   W_L^m = lo[m mod 128] * hi[m / 128],   lo[i] = W_L^i, hi[i] = W_L^{128 i},
// filled from the double-precision-built global table at kernel start
// (128 + L/128 entries, <= 2 KB).  Each factor is correctly rounded, so a
// twiddle carries about 1.5 ulp of error, and LDS latency replaces the L2
// latency of a scattered lookup in the full table.
constexpr int kTwLo = 128;
template <int L>
constexpr int tw_lds_points() { return kTwLo + (L + kTwLo - 1) / kTwLo; }

struct TwLds {
  const float2 *lo, *hi;
  __device__ __forceinline__ float2 operator()(unsigned m) const { return cmul(lo[m & (kTwLo - 1)], hi[m >> 7]); }
};

// Twiddles from one half-circle table in LDS: W_L^m = t[m] for m < L/2 and
// -t[m - L/2] above (W_L^{L/2} = -1); one LDS read and no arithmetic per
// twiddle.  Used where L/2 points of LDS are affordable.
template <int L>
struct TwHalf {
  const float2 *t;
  __device__ __forceinline__ float2 operator()(unsigned m) const {
    const float2 w = t[m & (L / 2 - 1)];
    return (m & (L / 2)) ? make_float2(-w.x, -w.y) : w;
  }
};
template <int L>
__device__ __forceinline__ TwHalf<L> load_half_twiddles(float2 *twl, const float2 *__restrict__ tw, unsigned tid,
                                                        unsigned nthreads) {
  for (unsigned i = tid; i < (unsigned)(L / 2); i += nthreads) twl[i] = tw[i];
  return TwHalf<L>{twl};
}

// copy the two tables from the global table tw (L entries) into LDS twl;
// the caller synchronises before first use
template <int L>
__device__ __forceinline__ TwLds load_twiddles(float2 *twl, const float2 *__restrict__ tw, unsigned tid,
                                               unsigned nthreads) {
  constexpr int NHI = (L + kTwLo - 1) / kTwLo;
  for (unsigned i = tid; i < (unsigned)(kTwLo + NHI); i += nthreads)
    twl[i] = (i < (unsigned)kTwLo) ? tw[i < (unsigned)L ? i : 0] : tw[(i - kTwLo) * kTwLo];
  return TwLds{twl, twl + kTwLo};
}

// v[r] *= W^{base r}, r = 1 .. R-1.  With r = r1 + 4 r2 the twiddle factors
// as W^{base r1} W^{4 base r2}; the two factors are applied one after the
// other (the same multiply count as forming their product first), so only
// 2 x 3 table twiddles are live at a time.
template <int R, int L>
__device__ __forceinline__ void apply_twiddles(float2 *v, const TwHalf<L> &tw, unsigned base) {
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw(base * r));
}

template <int R>
__device__ __forceinline__ void apply_twiddles(float2 *v, const TwLds &tw, unsigned base) {
  if constexpr (R <= 4 || R % 4 != 0) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw(base * r));
  } else {
    float2 a[4], c[R / 4];
#pragma unroll
    for (int r1 = 1; r1 < 4; ++r1) a[r1] = tw(base * r1);
#pragma unroll
    for (int r2 = 1; r2 < R / 4; ++r2) c[r2] = tw(4 * base * r2);
#pragma unroll
    for (int r2 = 0; r2 < R / 4; ++r2)
#pragma unroll
      for (int r1 = 0; r1 < 4; ++r1) {
        const int r = r1 + 4 * r2;
        if (r1 != 0) v[r] = cmul(v[r], a[r1]);
        if (r2 != 0) v[r] = cmul(v[r], c[r2]);
      }
  }
}

// LDS index with one pad slot every 16 points (breaks the power-of-two
// strides of the first passes across banks)
__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 4); }
template <int L>
constexpr int lds_points() { return L + L / 16; }
// lds_idx(i + d) - lds_idx(i) for a compile-time d when it does not depend
// on i: d a multiple of 16 (d + d/16), or i mod 16 + d staying below 16 for
// every i the caller passes (d).  Padded addresses of a butterfly's points
// are then one base and immediate offsets.
constexpr int lds_step16(int d) { return d + d / 16; }

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
  template <int p, class TW>
  __device__ __forceinline__ static void pass(float2 (&v)[E], float2 *lds, int t, const TW &tw) {
    constexpr int R = Plan::list[p];
    constexpr int NS = ns_before(p);
    constexpr int NB = E / R;
    constexpr int TWS = L / (NS * R);  // table stride of this pass
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = t + i * NT;
      if constexpr (NS > 1) {
        const unsigned jm = (unsigned)(j % NS);
        apply_twiddles<R>(&v[i * R], tw, jm * TWS);
      }
      Dft<R>::template run<1>(&v[i * R]);
    }
    if constexpr (p + 1 < P) {
      constexpr int R2 = Plan::list[p + 1];
      constexpr int NB2 = E / R2;
      __syncthreads();  // previous readers of LDS are done
      // the outputs of a butterfly sit NS apart from base: when NS is a
      // multiple of 16, or the R outputs stay inside one aligned run of
      // NS R <= 16 points (base mod NS R = j mod NS), their padded addresses
      // are lds_idx(base) plus a compile-time offset
      constexpr bool kLin = NS % 16 == 0 || (NS * R <= 16 && 16 % (NS * R) == 0);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + i * NT;
        const int base = (j / NS) * NS * R + (j % NS);
        if constexpr (kLin) {
          float2 *pb = lds + lds_idx(base);
#pragma unroll
          for (int r = 0; r < R; ++r) pb[NS % 16 == 0 ? lds_step16(r * NS) : r * NS] = v[i * R + r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) lds[lds_idx(base + r * NS)] = v[i * R + r];
        }
      }
      __syncthreads();
      // inputs t + i NT + r L/R2: NT and L/R2 are multiples of 16, so every
      // padded address is lds_idx(t) plus a compile-time offset
      static_assert(NT % 16 == 0 && (L / R2) % 16 == 0, "read offsets must be multiples of 16");
      const float2 *pt = lds + lds_idx(t);
#pragma unroll
      for (int i = 0; i < NB2; ++i)
#pragma unroll
        for (int r = 0; r < R2; ++r) v[i * R2 + r] = pt[lds_step16(i * NT + r * (L / R2))];
    }
  }

  template <class TW, int... ps>
  __device__ __forceinline__ static void run_passes(float2 (&v)[E], float2 *lds, int t, const TW &tw,
                                                    std::integer_sequence<int, ps...>) {
    (pass<ps>(v, lds, t, tw), ...);
  }

  // forward FFT in place: v in "in_slot" layout -> v in "out_slot" layout
  template <class TW>
  __device__ __forceinline__ static void forward(float2 (&v)[E], float2 *lds, int t, const TW &tw) {
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

// ---------------------------------------------------------------------------
// One FFT per wavefront.  A single wave of 64 lanes holds all F points
// (E = F/64 per lane, point lane + 64 e in register e), so passes need no
// workgroup barrier: LDS operations of one wave execute in issue order, and a
// compiler-level wave barrier keeps them in program order.  Each exchange
// goes through a private LDS window of F/2 points in two halves (write the
// outputs that fall in a half, read the next pass's inputs from it, then the
// other half), halving the LDS a wave needs.
// ---------------------------------------------------------------------------
template <int F>
struct WaveShape;
template <> struct WaveShape<1024> { using Plan = Radices<16, 16, 4>; };
template <> struct WaveShape<2048> { using Plan = Radices<16, 16, 8>; };
template <> struct WaveShape<4096> { using Plan = Radices<16, 16, 16>; };

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int F>
struct WaveFft {
  static constexpr int NT = 64;
  static constexpr int E = F / NT;
  using Plan = typename WaveShape<F>::Plan;
  static constexpr int P = Plan::count;
  static constexpr int R_first = Plan::list[0];
  static constexpr int R_last = Plan::list[P - 1];
  // windows of F/2 points for F >= 2048 (32+ points per lane); smaller FFTs
  // exchange through a full window in one step
  static constexpr int PARTS = F >= 2048 ? 2 : 1;
  static constexpr int HALF = F / PARTS;
  static_assert(Plan::product() == F, "radix plan must multiply to F");

  __device__ __forceinline__ static constexpr int in_slot(int e) { return slot_of<E, R_first>(e); }
  __device__ __forceinline__ static constexpr int out_slot(int e) { return slot_of<E, R_last>(e); }
  static constexpr int ns_before(int p) {
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= Plan::list[i];
    return ns;
  }
  // LDS points of the private window
  static constexpr int window() { return F / (F >= 2048 ? 2 : 1) + F / (F >= 2048 ? 2 : 1) / 16; }

  template <int p, class TW>
  __device__ __forceinline__ static void pass(float2 (&v)[E], float2 *win, int lane, const TW &tw) {
    constexpr int R = Plan::list[p];
    constexpr int NS = ns_before(p);
    constexpr int NB = E / R;
    constexpr int TWS = F / (NS * R);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = lane + i * NT;
      if constexpr (NS > 1) {
        const unsigned jm = (unsigned)(j % NS);
        apply_twiddles<R>(&v[i * R], tw, jm * TWS);
      }
      Dft<R>::template run<1>(&v[i * R]);
      __builtin_amdgcn_sched_barrier(0);  // one butterfly's temporaries live at a time
    }
    if constexpr (p + 1 < P) {
      // inputs of the next pass go to nv: slots of v may still hold outputs
      // of the other half that have not been written yet
      float2 nv[E];
      exchange<p, 0>(v, nv, win, lane);
      if constexpr (PARTS == 2) exchange<p, 1>(v, nv, win, lane);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = nv[e];
    }
  }

  // Which half of the window output r of butterfly slot i lands in.  The
  // Stockham position (j/NS) NS R + j%NS + r NS is non-decreasing in j, so
  // checking lanes 0 and 63 decides it for the whole wave at compile time.
  template <int p, int i, int r>
  static constexpr bool out_upper() {
    if constexpr (PARTS == 1) return false;
    constexpr int R = Plan::list[p];
    constexpr int NS = ns_before(p);
    constexpr int j0 = i * NT, j1 = 63 + i * NT;
    constexpr int pos0 = (j0 / NS) * NS * R + j0 % NS + r * NS;
    constexpr int pos1 = (j1 / NS) * NS * R + j1 % NS + r * NS;
    static_assert((pos0 >= HALF) == (pos1 >= HALF), "an output slot straddles both halves");
    return pos0 >= HALF;
  }

  template <int p, int h, int i, int... rs>
  __device__ __forceinline__ static void write_slot(const float2 (&v)[E], float2 *win, int lane,
                                                    std::integer_sequence<int, rs...>) {
    constexpr int R = Plan::list[p];
    constexpr int NS = ns_before(p);
    const int j = lane + i * NT;
    const int base = (j / NS) * NS * R + (j % NS) - h * HALF;
    // as in Fft::pass: one padded base and compile-time offsets when the
    // outputs' spacing allows it (HALF is a multiple of 16)
    constexpr bool kLin = NS % 16 == 0 || (NS * R <= 16 && 16 % (NS * R) == 0);
    if constexpr (kLin) {
      float2 *pb = win + lds_idx(base);
      ((out_upper<p, i, rs>() == (h == 1) ? (void)(pb[NS % 16 == 0 ? lds_step16(rs * NS) : rs * NS] = v[i * R + rs])
                                          : (void)0),
       ...);
    } else {
      ((out_upper<p, i, rs>() == (h == 1) ? (void)(win[lds_idx(base + rs * NS)] = v[i * R + rs]) : (void)0), ...);
    }
  }
  template <int p, int h, int... is>
  __device__ __forceinline__ static void write_half(const float2 (&v)[E], float2 *win, int lane,
                                                    std::integer_sequence<int, is...>) {
    constexpr int R = Plan::list[p];
    (write_slot<p, h, is>(v, win, lane, std::make_integer_sequence<int, R>{}), ...);
  }

  // exchange of half h: write the outputs of pass p that fall in half h, then
  // read the inputs of pass p+1 held there (j + r2 F/R2 is in the upper half
  // exactly when r2 >= R2/2).  Reads of half 0 are issued before the writes
  // of half 1 and LDS executes a wave's operations in order, so the window is
  // reused safely.
  template <int p, int h>
  __device__ __forceinline__ static void exchange(const float2 (&v)[E], float2 (&nv)[E], float2 *win, int lane) {
    constexpr int R = Plan::list[p];
    constexpr int R2 = Plan::list[p + 1];
    constexpr int NB = E / R, NB2 = E / R2;
    wave_sync();
    write_half<p, h>(v, win, lane, std::make_integer_sequence<int, NB>{});
    wave_sync();
    // lane + i NT + r F/R2 - h HALF: every offset from lane is a multiple
    // of 16, so the padded addresses are lds_idx(lane) plus constants
    const float2 *pl = win + lds_idx(lane);
#pragma unroll
    for (int i = 0; i < NB2; ++i) {
#pragma unroll
      for (int r = h * (R2 / PARTS); r < (h + 1) * (R2 / PARTS); ++r)
        nv[i * R2 + r] = pl[lds_step16(i * NT + r * (F / R2) - h * HALF)];
    }
  }

  template <class TW, int... ps>
  __device__ __forceinline__ static void run_passes(float2 (&v)[E], float2 *win, int lane, const TW &tw,
                                                    std::integer_sequence<int, ps...>) {
    (pass<ps>(v, win, lane, tw), ...);
  }
  template <class TW>
  __device__ __forceinline__ static void forward(float2 (&v)[E], float2 *win, int lane, const TW &tw) {
    run_passes(v, win, lane, tw, std::make_integer_sequence<int, P>{});
  }
};

// Workgroup g of G (G a multiple of 8) -> work item q, numbered so that each
// XCD (dispatch is round-robin over 8) takes one contiguous run of q:
// neighbouring items share cache lines and table rows in that XCD's L2.
__device__ __forceinline__ int64_t xcd_item(int64_t g, int64_t G) { return (g & 7) * (G >> 3) + (g >> 3); }

// W_L^m for m < L from the two-level table tb: lo[i] = W_L^i (i < 2048),
// hi[i] = W_L^{2048 i}
__device__ __forceinline__ float2 big_twiddle(const float2 *__restrict__ tb, unsigned m) {
  return cmul(tb[m & 2047u], tb[2048u + (m >> 11)]);
}

}  // namespace tz
