// Split-precision chirp-Z transform: the radix-16 passes of both FFTs run on
// the matrix cores as a batched dense DFT-matrix product, the rest of the
// Bluestein pipeline is the FP32 path's.
//
// A radix-16 pass computes y_j = F16 x_j for every butterfly j.  In real form
//   [Re y; Im y] = [[Fr, -Fi], [Fi, Fr]] [Re x; Im x]   (32 x 32 times 32 x 1),
// so 32 butterflies make one 32x32x32 real product: two
// v_mfma_f32_32x32x16_{f16,bf16} per operand pair (K = 16 + 16).  Operands are
// split into a high and a low part in the 16-bit type, and the product is
// accumulated in FP32 as  Ah Bh + Ah Bl + Al Bh  (the Al Bl term is below the
// FP32 rounding of the sum).  For FP16 each butterfly's inputs are scaled by a
// power of two so that their largest component sits near 2^13: FP16's range
// holds the high part and its low part stays normal; the scale is exact and
// is undone on the FP32 result.  BF16 shares FP32's exponent range and needs
// no scaling.
//
// Lane layout of the 32x32x16 operations (checked on the device):
//   A (32 x 16): lane l holds row l%32, k = 8(l/32) + q, q < 8;
//   B (16 x 32): lane l holds column l%32, k = 8(l/32) + q;
//   C (32 x 32): lane l holds column l%32, rows (r%4) + 8(r/4) + 4(l/32), r < 16.
// The DFT matrix's rows are interleaved (row 2o: Re y_o, row 2o + 1: Im y_o),
// so accumulator registers 2c and 2c + 1 of a lane are the two parts of one
// output.  Wave w owns butterflies j = 64 w + 32 g + l%32 (g = 0, 1); lane
// half h = l/32 holds inputs 8h .. 8h+7 of its butterfly and, after the
// product, outputs 4(c/2) + 2h + c%2, c < 8.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fft_core.h"
#include "internal.h"
#include "thzspec.h"

namespace tz {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

template <int PREC>
struct Split;
template <>
struct Split<TZ_SPLIT_FP16> {
  using V = half8;
  using S = _Float16;
  __device__ static float16v mfma(V a, V b, float16v c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};
template <>
struct Split<TZ_SPLIT_BF16> {
  using V = bf8;
  using S = __bf16;
  __device__ static float16v mfma(V a, V b, float16v c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};

// cos(pi m / 8), m < 16, rounded to FP32: the entries of the 16-point DFT matrix
__constant__ float kCosPi8[16] = {
    1.0f, 0.92387953251128675613f, 0.70710678118654752440f, 0.38268343236508977173f,
    0.0f, -0.38268343236508977173f, -0.70710678118654752440f, -0.92387953251128675613f,
    -1.0f, -0.92387953251128675613f, -0.70710678118654752440f, -0.38268343236508977173f,
    0.0f, 0.38268343236508977173f, 0.70710678118654752440f, 0.92387953251128675613f};

// index of output c (c < 8) held by lane half h: 2h plus out_k0(c)
__device__ __forceinline__ constexpr int out_k0(int c) { return 4 * (c / 2) + c % 2; }

// NTERM = 2: operands split x = x_hi + x_lo, product A_hi B_hi + A_hi B_lo +
// A_lo B_hi (about 16 significant bits per BF16 operand, 22 per FP16 one).
// NTERM = 3 (BF16): x = x_hi + x_mid + x_lo and the six products of order
// <= 2 (hi.hi; hi.mid, mid.hi; hi.lo, mid.mid, lo.hi), about 24 bits: twice
// the matrix-core work, for chains of transforms whose two-term error adds up
// past 1e-5.
template <int L, int PREC, int NTERM = 2>
struct MfmaFft {
  static_assert(NTERM == 2 || NTERM == 3, "two- or three-term split");
  using SP = Split<PREC>;
  using V = typename SP::V;
  using S = typename SP::S;
  static constexpr int NT = L / 16;          // threads: one radix-16 butterfly each
  static constexpr int E = 16;               // points per thread
  // radix-16 passes on the matrix cores: three over 4096-point
  // sub-transforms from L = 4096 up, two over 256-point ones below
  static constexpr int NP = L >= 4096 ? 3 : 2;
  static constexpr int SUB = NP == 3 ? 4096 : 256;
  static constexpr int RT = L / SUB;         // trailing VALU radix (1, 2, 4 or 8)
  static constexpr int Q = L / 16;           // stride between the inputs of a butterfly
  static_assert(L == 1024 || L == 2048 || L == 4096 || L == 8192 || L == 16384,
                "radix-16 passes on the matrix cores plus a trailing radix of 1, 2, 4 or 8");

  // DFT-matrix operands: for lane l, rows i = l%32, columns k = 8h + q; a1
  // multiplies Re x, a2 multiplies Im x.  They are the same for every wave,
  // so they live in LDS (NOPS vectors x 64 lanes, lane-contiguous, one
  // conflict-free 16-byte read each) and are read right before each product
  // instead of holding 16-24 registers through the whole transform.
  static constexpr int NOPS = NTERM == 3 ? 6 : 4;  // a1h, a1l, a2h, a2l (+ a1m, a2m)
  static constexpr int kOpsBytes = NOPS * 64 * 16;
  const V *ops;

  // fill the operand table (the first wave of the workgroup); the caller
  // synchronises the workgroup before the first transform
  __device__ void init(void *lds_ops, int tid) {
    ops = (const V *)lds_ops;
    if (tid >= 64) return;
    const int lane = tid;
    V a1h, a1m, a1l, a2h, a2m, a2l;
    const int i = lane % 32, h = lane / 32;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 8 * h + q;
      const int m = ((i / 2) * k) % 16;        // row i: part i % 2 of output i / 2
      // e^{-j 2 pi m/16} = cos(pi m/8) - j sin(pi m/8), sin(pi m/8) = cos(pi (m-4)/8)
      const float fr = kCosPi8[m], fi = -kCosPi8[(m + 12) % 16];
      const float v1 = (i % 2 == 0) ? fr : fi;  // coefficient of Re x[k]
      const float v2 = (i % 2 == 0) ? -fi : fr; // coefficient of Im x[k]
      const S h1 = (S)v1, h2 = (S)v2;
      a1h[q] = h1;
      a2h[q] = h2;
      if constexpr (NTERM == 3) {
        const float r1 = v1 - (float)h1, r2 = v2 - (float)h2;
        const S m1 = (S)r1, m2 = (S)r2;
        a1m[q] = m1;
        a2m[q] = m2;
        a1l[q] = (S)(r1 - (float)m1);
        a2l[q] = (S)(r2 - (float)m2);
      } else {
        a1l[q] = (S)(v1 - (float)h1);
        a2l[q] = (S)(v2 - (float)h2);
      }
    }
    V *o = (V *)lds_ops;
    o[0 * 64 + lane] = a1h;
    o[1 * 64 + lane] = a1l;
    o[2 * 64 + lane] = a2h;
    o[3 * 64 + lane] = a2l;
    if constexpr (NTERM == 3) {
      o[4 * 64 + lane] = a1m;
      o[5 * 64 + lane] = a2m;
    }
  }

  // operand vector w of this lane; the index passes through an opaque zero
  // so that the read stays next to its product rather than being hoisted
  // and kept in registers
  __device__ __forceinline__ V op(int w, int lane) const { return ops[w * 64 + lane + (int)opaque_zero()]; }

  // the two-term operands of this lane, read once per pass and held in 16
  // registers through its products (the three-term ones stay in LDS and are
  // read next to each product)
  struct Areg {
    V a1h, a1l, a2h, a2l;
  };
  __device__ __forceinline__ Areg load_ops(int lane) const {
    if constexpr (NTERM == 2)
      return Areg{ops[lane], ops[64 + lane], ops[128 + lane], ops[192 + lane]};
    else
      return Areg{};
  }

  // y = F16 x for this lane's butterfly: x[q] are inputs 8h+q, results are
  // outputs 2h + out_k0(c), c < 8
  __device__ __forceinline__ void butterfly(float2 (&x)[8], float2 (&y)[8], const Areg &A) const {
    // FP16 needs the inputs brought near 2^13 (its range, and a normal low
    // part); BF16 has the FP32 exponent range and is split as it is
    constexpr bool kScale = PREC == TZ_SPLIT_FP16;
    float up = 1.f, down = 1.f;
    if constexpr (kScale) {
      float mx = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) mx = fmaxf(mx, fmaxf(fabsf(x[q].x), fabsf(x[q].y)));
      mx = fmaxf(mx, __shfl_xor(mx, 32));  // partner lane holds the other 8 inputs
      int ex = 0;
      (void)frexpf(mx, &ex);
      const int sh = (mx > 0.f) ? 13 - ex : 0;  // largest component near 2^13
      up = ldexpf(1.f, sh);
      down = ldexpf(1.f, -sh);
    }
    float16v c = {};
    const int lane = (int)(__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)));
    if constexpr (NTERM == 2) {
      V brh, brl, bih, bil;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float xr = kScale ? x[q].x * up : x[q].x, xi = kScale ? x[q].y * up : x[q].y;
        const S hr = (S)xr, hi = (S)xi;
        brh[q] = hr;
        brl[q] = (S)(xr - (float)hr);
        bih[q] = hi;
        bil[q] = (S)(xi - (float)hi);
      }
      c = SP::mfma(A.a1h, brh, c);
      c = SP::mfma(A.a1h, brl, c);
      c = SP::mfma(A.a1l, brh, c);
      c = SP::mfma(A.a2h, bih, c);
      c = SP::mfma(A.a2h, bil, c);
      c = SP::mfma(A.a2l, bih, c);
    } else {
      // the real parts' three operand vectors and their six products first,
      // then the imaginary parts': 12 operand registers live instead of 24
      auto split3 = [&](int comp, V &bh, V &bm, V &bl) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float xv = comp == 0 ? (kScale ? x[q].x * up : x[q].x) : (kScale ? x[q].y * up : x[q].y);
          const S hv = (S)xv;
          const float rv = xv - (float)hv;
          const S mv = (S)rv;
          bh[q] = hv;
          bm[q] = mv;
          bl[q] = (S)(rv - (float)mv);
        }
      };
      {
        V brh, brm, brl;
        split3(0, brh, brm, brl);
        const V a1h = op(0, lane), a1l = op(1, lane), a1m = op(4, lane);
        c = SP::mfma(a1h, brh, c);
        c = SP::mfma(a1h, brm, c);
        c = SP::mfma(a1m, brh, c);
        c = SP::mfma(a1h, brl, c);
        c = SP::mfma(a1m, brm, c);
        c = SP::mfma(a1l, brh, c);
      }
      {
        V bih, bim, bil;
        split3(1, bih, bim, bil);
        const V a2h = op(2, lane), a2l = op(3, lane), a2m = op(5, lane);
        c = SP::mfma(a2h, bih, c);
        c = SP::mfma(a2h, bim, c);
        c = SP::mfma(a2m, bih, c);
        c = SP::mfma(a2h, bil, c);
        c = SP::mfma(a2m, bim, c);
        c = SP::mfma(a2l, bih, c);
      }
    }
#pragma unroll
    for (int cc = 0; cc < 8; ++cc)  // output 2h + out_k0(cc)
      y[cc] = kScale ? make_float2(c[2 * cc] * down, c[2 * cc + 1] * down) : make_float2(c[2 * cc], c[2 * cc + 1]);
  }

  // one radix-16 pass p on the matrix cores: twiddle, product, exchange.
  // xin[g][q] = input 8h+q of butterfly j(g); on return xin holds the inputs
  // of pass p+1 in the same layout (p < NP - 1), or of the trailing pass in
  // the VALU layout v (the last one).
  //
  // LDS addresses are one per-lane base and compile-time offsets: the padded
  // index lds_idx(i + d) is lds_idx(i) + lds_step16(d) whenever d is a
  // multiple of 16, or i is a multiple of 16 and d < 16.  Butterfly j's
  // outputs go to (j / NS) 16 NS + j % NS + k NS; j and j + 32 (g = 0, 1)
  // differ by 512 in that index for NS <= 16, by 32 for NS = 256 (j % 256
  // stays below 224 for g = 0).
  template <int p>
  __device__ __forceinline__ void pass(float2 (&xin)[2][8], float2 (&v)[E], float2 *lds, int wave, int lane,
                                       const TwLds &tw) const {
    constexpr int NS = p == 0 ? 1 : (p == 1 ? 16 : 256);
    constexpr int TWS = L / (NS * 16);
    constexpr int S = lds_step16(NS);                      // between outputs k and k + 1
    constexpr int GW = lds_step16(NS == 256 ? 32 : 512);   // between butterflies j and j + 32
    constexpr int SQ = lds_step16(Q);                      // between inputs q and q + 1
    const int h = lane / 32;
    const int j0 = 64 * wave + lane % 32;
    const Areg A = load_ops(lane);
    float2 y[2][8];
    if constexpr (NS > 1) {
      // twiddles W_L^{jm (8h + q) TWS}, q < 8: two table values and powers
      // of the step, applied as they are formed (two complex values live);
      // for NS = 16 both butterflies of the lane share them
      auto twist = [&](int g, int g_end) {
        const unsigned jm = (unsigned)((j0 + 32 * g) % NS);
        const float2 d = tw(jm * TWS);
        float2 w = tw(jm * (unsigned)(8 * h) * TWS);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int gg = g; gg < g_end; ++gg) xin[gg][q] = cmul(xin[gg][q], w);
          if (q < 7) w = cmul(w, d);
        }
      };
      if constexpr (NS == 256) {
        twist(0, 1);
        twist(1, 2);
      } else {
        twist(0, 2);
      }
#pragma unroll
      for (int g = 0; g < 2; ++g) butterfly(xin[g], y[g], A);
    } else {
#pragma unroll
      for (int g = 0; g < 2; ++g) butterfly(xin[g], y[g], A);
    }
    __syncthreads();  // previous readers of LDS are done
    {
      float2 *pw = lds + lds_idx((j0 / NS) * NS * 16 + j0 % NS) + 2 * h * S;
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int c = 0; c < 8; ++c) pw[g * GW + out_k0(c) * S] = y[g][c];
    }
    __syncthreads();
    if constexpr (p < NP - 1) {
      const float2 *pr = lds + lds_idx(j0) + 8 * h * SQ;
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int q = 0; q < 8; ++q) xin[g][q] = pr[g * lds_step16(32) + q * SQ];
    } else {
      // layout of the trailing pass (radix RT) or, with RT = 1, the final
      // natural-order layout t + NT e
      constexpr int R = RT > 1 ? RT : 16;
      constexpr int NB = E / R;
      const float2 *pr = lds + lds_idx(64 * wave + lane);  // the transform's thread index
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) v[i * R + r] = pr[lds_step16(i * NT + r * (L / R))];
    }
  }

  // the matrix-core passes of one transform, xin in, v (trailing layout) out
  __device__ __forceinline__ void passes(float2 (&xin)[2][8], float2 (&v)[E], float2 *lds, int wave, int lane,
                                         const TwLds &tw) const {
    pass<0>(xin, v, lds, wave, lane, tw);
    pass<1>(xin, v, lds, wave, lane, tw);
    if constexpr (NP == 3) pass<2>(xin, v, lds, wave, lane, tw);
  }

  // trailing VALU pass of radix RT over the SUB-point sub-transforms; tl is
  // the thread's index in the transform
  __device__ __forceinline__ void trailing(float2 (&v)[E], const TwLds &tw, int tl) const {
    if constexpr (RT > 1) {
      constexpr int NB = E / RT;
      // a fresh thread index: the twiddle addresses of this pass are formed
      // here, not shared with (and held live from) the other transform's
      const int t = (int)(tl + opaque_zero());
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int j = t + i * NT;
        apply_twiddles<RT>(&v[i * RT], tw, (unsigned)(j % SUB));
        Dft<RT>::template run<1>(&v[i * RT]);
      }
    }
  }

  // register slot of element t + NT e after the transform
  __device__ __forceinline__ static constexpr int out_slot(int e) {
    return RT > 1 ? slot_of<E, RT>(e) : slot_of<E, 16>(e);
  }
};

// Bluestein CZT with split-precision radix-16 passes (single bin block,
// single segment, real input).  Same tables and algebra as k_czt.
template <int L, int PREC, int KIND>
__global__ void __launch_bounds__(L / 16, 4)
    k_czt_mfma(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ c_pre,
               const float2 *__restrict__ c_post, const float2 *__restrict__ V, const float2 *__restrict__ tw,
               float2 *__restrict__ X, int64_t os, int64_t M) {
  using MF = MfmaFft<L, PREC>;
  constexpr int NT = MF::NT, E = MF::E, Q = MF::Q;
  constexpr int XB = KIND == 1 ? 8 : 4;
  __shared__ float2 lds[lds_points<L>()];
  __shared__ float2 twl[tw_lds_points<L>()];
  __shared__ __attribute__((aligned(16))) char opl[MF::kOpsBytes];
  const int t = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64, h = lane / 32;
  const int64_t b = blockIdx.x;
  const TwLds twd = load_twiddles<L>(twl, tw, t, NT);
  MF mf;
  mf.init(opl, t);
  __syncthreads();
  const Rsrc rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
  const Rsrc rp = make_rsrc(c_pre, (uint64_t)N * 8);
  const Rsrc rV = make_rsrc(V, (uint64_t)L * 8);
  const Rsrc rq = make_rsrc(c_post, (uint64_t)M * 8);
  const Rsrc rX = make_rsrc(X + b * os, (uint64_t)M * 8);

  float2 xin[2][8];
  float2 v[E];
  // FFT 1: premultiplied input straight into the matrix-core layout
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int j = 64 * wave + 32 * g + lane % 32;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const unsigned n = (unsigned)(j + (8 * h + q) * Q);
      float xv;
      if constexpr (KIND == 1)
        xv = (float)ld_f64(rx, 8 * n);
      else
        xv = ld_f32(rx, 4 * n);
      xin[g][q] = cscale(ld_c64(rp, 8 * n), xv);
    }
  }
  mf.passes(xin, v, lds, wave, lane, twd);
  mf.trailing(v, twd, t);
  // spectral product with the conjugate chirp, then the inverse FFT as the
  // conjugate of a forward FFT of the conjugate
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k = (unsigned)(t + NT * e);
    v[MF::out_slot(e)] = cconj(cmul(v[MF::out_slot(e)], ld_c64(rV, 8 * k)));
  }
  __syncthreads();
  {
    float2 *pw = lds + lds_idx(t);
#pragma unroll
    for (int e = 0; e < E; ++e) pw[lds_step16(NT * e)] = v[MF::out_slot(e)];
  }
  __syncthreads();
  // fresh copies of the thread indices: the second transform recomputes its
  // LDS addresses instead of keeping those of the first one live
  const int t2 = (int)(t + opaque_zero()), wave2 = __builtin_amdgcn_readfirstlane(t2 / 64), lane2 = t2 % 64,
            h2 = lane2 / 32;
  {
    const float2 *pr = lds + lds_idx(64 * wave2 + lane2 % 32) + 8 * h2 * lds_step16(Q);
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int q = 0; q < 8; ++q) xin[g][q] = pr[g * lds_step16(32) + q * lds_step16(Q)];
  }
  mf.passes(xin, v, lds, wave2, lane2, twd);
  mf.trailing(v, twd, t2);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k = (unsigned)(t2 + NT * e);
    st_c64(cmul(cconj(v[MF::out_slot(e)]), ld_c64(rq, 8 * k)), rX, 8 * k);
  }
}

// The half-length form of k_czt_mfma (L = 8192, N and M at most L/2; the
// same algebra as k_czt_half): thread group h (256 threads) runs a
// 4096-point split-precision Bluestein pair on the trace twisted by W_L^{h n}
// and the bins 2k + h, in its own half of LDS; the two inverses are
// recombined with the second postmultiply table.  Each 4096-point transform
// is three matrix-core passes with no trailing VALU pass.
template <int PREC, int KIND>
__global__ void __launch_bounds__(512, 4)
    k_czt_mfma_half(const void *__restrict__ x, int64_t xs, int64_t N, const float2 *__restrict__ c_pre,
                    const float2 *__restrict__ c_pre1, const float2 *__restrict__ c_post,
                    const float2 *__restrict__ c_post1, const float2 *__restrict__ V, const float2 *__restrict__ tw,
                    float2 *__restrict__ X, int64_t os, int64_t M) {
  constexpr int L = 8192, LH = L / 2;
  using MF = MfmaFft<LH, PREC>;
  constexpr int NT = MF::NT, E = MF::E, Q = MF::Q;
  static_assert(2 * NT == 512 && MF::RT == 1, "two 4096-point transforms with no trailing pass");
  constexpr int XB = KIND == 1 ? 8 : 4;
  __shared__ float2 lds[2 * lds_points<LH>()];
  __shared__ float2 twl[tw_lds_points<LH>()];
  __shared__ __attribute__((aligned(16))) char opl[MF::kOpsBytes];
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const TwLds twd = load_twiddles<LH>(twl, tw, t, 2 * NT);
  MF mf;
  mf.init(opl, t);
  __syncthreads();
  const int hh = __builtin_amdgcn_readfirstlane(t / NT);  // the half of the bins (2k + hh)
  const int u = t - hh * NT, wave = __builtin_amdgcn_readfirstlane(u / 64), lane = u % 64, h = lane / 32;
  float2 *lh = lds + hh * lds_points<LH>();
  const Rsrc rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
  const Rsrc rp = make_rsrc(hh ? c_pre1 : c_pre, (uint64_t)N * 8);
  const Rsrc rV = make_rsrc(V, (uint64_t)L * 8);

  float2 xin[2][8];
  float2 v[E];
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int j = 64 * wave + 32 * g + lane % 32;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const unsigned n = (unsigned)(j + (8 * h + q) * Q);  // past N: 0
      float xv;
      if constexpr (KIND == 1)
        xv = (float)ld_f64(rx, 8 * n);
      else
        xv = ld_f32(rx, 4 * n);
      xin[g][q] = cscale(ld_c64(rp, 8 * n), xv);
    }
  }
  mf.passes(xin, v, lh, wave, lane, twd);
  // bins 2k + hh: times V, conjugated for the inverse
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k = (unsigned)(u + NT * e);
    v[MF::out_slot(e)] = cconj(cmul(v[MF::out_slot(e)], ld_c64(rV, 8 * (2 * k + hh))));
  }
  __syncthreads();
  {
    float2 *pw = lh + lds_idx(u);
#pragma unroll
    for (int e = 0; e < E; ++e) pw[lds_step16(NT * e)] = v[MF::out_slot(e)];
  }
  __syncthreads();
  const int u2 = (int)(u + opaque_zero()), wave2 = __builtin_amdgcn_readfirstlane(u2 / 64), lane2 = u2 % 64,
            h2 = lane2 / 32;
  {
    const float2 *pr = lh + lds_idx(64 * wave2 + lane2 % 32) + 8 * h2 * lds_step16(Q);
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int q = 0; q < 8; ++q) xin[g][q] = pr[g * lds_step16(32) + q * lds_step16(Q)];
  }
  mf.passes(xin, v, lh, wave2, lane2, twd);
  // a_hh[n] at out_slot(e), n = u + NT e: group 0 finishes n < LH/2, group 1
  // the rest, each taking the other's a of those n through LDS (two copies
  // of the code, so that every register index is a compile-time constant)
  const Rsrc rq0 = make_rsrc(c_post, (uint64_t)M * 8);
  const Rsrc rq1 = make_rsrc(c_post1, (uint64_t)M * 8);
  const Rsrc rX = make_rsrc(X + b * os, (uint64_t)M * 8);
  auto combine = [&](auto half) {
    constexpr int H = decltype(half)::value;
    constexpr int GIVE = H ? 0 : E / 2, KEEP = H ? E / 2 : 0;
    __syncthreads();  // the last pass's LDS reads are done
#pragma unroll
    for (int e = 0; e < E / 2; ++e) lds[u2 + NT * (GIVE + e)] = v[MF::out_slot(GIVE + e)];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
      const unsigned n = (unsigned)(u2 + NT * (KEEP + e));
      const float2 mine = v[MF::out_slot(KEEP + e)], other = lds[n];
      const float2 a0 = H ? other : mine, a1 = H ? mine : other;
      st_c64(cadd(cmul(cconj(a0), ld_c64(rq0, 8 * n)), cmul(cconj(a1), ld_c64(rq1, 8 * n))), rX, 8 * n);
    }
  };
  if (hh)
    combine(std::integral_constant<int, 1>{});
  else
    combine(std::integral_constant<int, 0>{});
}

// Row pass of the four-step path (the spectral product of eq. (15) on the
// rows of the L1 x L2 layout) with split-precision radix-16 passes: per row
// k1 of trace b,
//   Hc[k1][n2] = W_L^{k1 n2} FFT_L2( conj( V[k1 + L1 k2] FFT_L2( W_L^{k1 n2} Z[k1][.] ) ) ),
// in place; the same algebra as the FP32 row kernel, with its two L2-point
// FFTs as in k_czt_mfma.
template <int L1, int L2, int PREC>
__global__ void __launch_bounds__(L2 / 16, 4)
    k_long_rows_mfma(float2 *__restrict__ Z, const float2 *__restrict__ Vt, const float2 *__restrict__ tw_row,
                     const float2 *__restrict__ tbig, int64_t nb) {
  // BF16 takes the three-term split here: the two-term one measured 1.0e-5
  // on 256 x 2^20 long scans (L = 320 x 4096), at the 1e-5 bar
  using MF = MfmaFft<L2, PREC, PREC == TZ_SPLIT_BF16 ? 3 : 2>;
  constexpr int NT = MF::NT, E = MF::E, Q = MF::Q;
  constexpr int64_t L = (int64_t)L1 * L2;
  __shared__ float2 lds[lds_points<L2>()];
  __shared__ float2 twl[tw_lds_points<L2>()];
  __shared__ __attribute__((aligned(16))) char opl[MF::kOpsBytes];
  const int t = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64, h = lane / 32;
  // rows of equal k1 (one V row) for the traces of the chunk run back to back
  const int64_t q = xcd_item(blockIdx.x, gridDim.x);
  const unsigned k1 = (unsigned)(q / nb);
  const int64_t b = q % nb;
  const TwLds twd = load_twiddles<L2>(twl, tw_row, t, NT);
  MF mf;
  mf.init(opl, t);
  __syncthreads();
  const Rsrc rz = make_rsrc(Z + b * L + (int64_t)k1 * L2, (uint64_t)L2 * 8);
  const Rsrc rv = make_rsrc(Vt + (int64_t)k1 * L2, (uint64_t)L2 * 8);
  float2 xin[2][8];
  float2 v[E];
  // the row, times W_L^{k1 n2}, straight into the matrix-core layout
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int j = 64 * wave + 32 * g + lane % 32;
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      const unsigned n2 = (unsigned)(j + (8 * h + qq) * Q);
      xin[g][qq] = cmul(ld_c64(rz, 8 * n2), big_twiddle(tbig, k1 * n2));
    }
  }
  mf.passes(xin, v, lds, wave, lane, twd);
  mf.trailing(v, twd, t);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned k2 = (unsigned)(t + NT * e);
    v[MF::out_slot(e)] = cconj(cmul(v[MF::out_slot(e)], ld_c64(rv, 8 * k2)));
  }
  __syncthreads();
  {
    float2 *pw = lds + lds_idx(t);
#pragma unroll
    for (int e = 0; e < E; ++e) pw[lds_step16(NT * e)] = v[MF::out_slot(e)];
  }
  __syncthreads();
  // fresh copies of the thread indices for the second transform
  const int t2 = (int)(t + opaque_zero()), wave2 = __builtin_amdgcn_readfirstlane(t2 / 64), lane2 = t2 % 64,
            h2 = lane2 / 32;
  {
    const float2 *pr = lds + lds_idx(64 * wave2 + lane2 % 32) + 8 * h2 * lds_step16(Q);
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) xin[g][qq] = pr[g * lds_step16(32) + qq * lds_step16(Q)];
  }
  mf.passes(xin, v, lds, wave2, lane2, twd);
  mf.trailing(v, twd, t2);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned n2 = (unsigned)(t2 + NT * e);
    st_c64(cmul(v[MF::out_slot(e)], big_twiddle(tbig, k1 * n2)), rz, 8 * n2);
  }
}

bool long_rows_mfma_supported(int L1, int L2) {
  return (L1 == 320 || L1 == 512 || L1 == 1024) &&
         (L2 == 1024 || L2 == 2048 || L2 == 4096 || L2 == 8192 || L2 == 16384);
}

template <int L1, int L2>
static void long_rows_mfma_dispatch(const LongLaunch &a, int64_t nb, hipStream_t s) {
  const dim3 grid((unsigned)(nb * L1)), block(L2 / 16);
  if (a.precision == TZ_SPLIT_FP16)
    hipLaunchKernelGGL((k_long_rows_mfma<L1, L2, TZ_SPLIT_FP16>), grid, block, 0, s, a.work, a.Vt, a.tw_row, a.tbig,
                       nb);
  else
    hipLaunchKernelGGL((k_long_rows_mfma<L1, L2, TZ_SPLIT_BF16>), grid, block, 0, s, a.work, a.Vt, a.tw_row, a.tbig,
                       nb);
}

template <int L1>
static hipError_t long_rows_mfma_l2(const LongLaunch &a, int64_t nb, hipStream_t s) {
  switch (a.L2) {
    case 1024: long_rows_mfma_dispatch<L1, 1024>(a, nb, s); break;
    case 2048: long_rows_mfma_dispatch<L1, 2048>(a, nb, s); break;
    case 4096: long_rows_mfma_dispatch<L1, 4096>(a, nb, s); break;
    case 8192: long_rows_mfma_dispatch<L1, 8192>(a, nb, s); break;
    case 16384: long_rows_mfma_dispatch<L1, 16384>(a, nb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_long_rows_mfma(const LongLaunch &a, int L1, int64_t nb, hipStream_t s) {
  if (!long_rows_mfma_supported(L1, a.L2) ||
      (a.precision != TZ_SPLIT_FP16 && a.precision != TZ_SPLIT_BF16))
    return hipErrorInvalidValue;
  switch (L1) {
    case 320: return long_rows_mfma_l2<320>(a, nb, s);
    case 512: return long_rows_mfma_l2<512>(a, nb, s);
    default: return long_rows_mfma_l2<1024>(a, nb, s);
  }
}

bool czt_mfma_supported(int L, int nseg, int nblk, int in_kind) {
  return (L == 4096 || L == 8192 || L == 16384) && nseg == 1 && nblk == 1 && in_kind != 2;
}

template <int L, int PREC>
static void mfma_dispatch(const CztLaunch &a, hipStream_t s) {
  const dim3 grid((unsigned)a.B), block(L / 16);
  if constexpr (L == 8192) {
    if (a.c_pre1) {  // N and M within L/2 (the plan checked)
      if (a.in_kind == 1)
        hipLaunchKernelGGL((k_czt_mfma_half<PREC, 1>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_pre1,
                           a.c_post, a.c_post1, a.V, a.tw_half, a.X, a.os, a.M);
      else
        hipLaunchKernelGGL((k_czt_mfma_half<PREC, 0>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_pre1,
                           a.c_post, a.c_post1, a.V, a.tw_half, a.X, a.os, a.M);
      return;
    }
  }
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_czt_mfma<L, PREC, 1>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_post, a.V, a.tw,
                       a.X, a.os, a.M);
  else
    hipLaunchKernelGGL((k_czt_mfma<L, PREC, 0>), grid, block, 0, s, a.x, a.xs, a.N, a.c_pre, a.c_post, a.V, a.tw,
                       a.X, a.os, a.M);
}

hipError_t launch_czt_mfma(const CztLaunch &a, hipStream_t s) {
  if (!czt_mfma_supported(a.L, a.nseg, a.nblk, a.in_kind)) return hipErrorInvalidValue;
  const bool f16 = a.precision == TZ_SPLIT_FP16;
  switch (a.L) {
    case 4096: f16 ? mfma_dispatch<4096, TZ_SPLIT_FP16>(a, s) : mfma_dispatch<4096, TZ_SPLIT_BF16>(a, s); break;
    case 8192: f16 ? mfma_dispatch<8192, TZ_SPLIT_FP16>(a, s) : mfma_dispatch<8192, TZ_SPLIT_BF16>(a, s); break;
    default: f16 ? mfma_dispatch<16384, TZ_SPLIT_FP16>(a, s) : mfma_dispatch<16384, TZ_SPLIT_BF16>(a, s); break;
  }
  return hipGetLastError();
}

}  // namespace tz
