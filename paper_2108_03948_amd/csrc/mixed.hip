// Mixed-radix FFTs for any 7-smooth length L = 2^a 3^b 5^c 7^d: the
// zero-padded FFT of eqs. (2)-(5) when N_fft has no power-of-two
// factorisation the dedicated kernels take, and the inverse DFT (the IFFT
// Section 4 times against the FFT) at such lengths, without the two longer
// FFTs of the Bluestein form.
//
// Stockham autosort passes of radix 2, 3, 4, 5, 7 or 8 in the order of the
// plan.  Pass p (radix R, NS = product of the earlier radices) runs the L/R
// butterflies j: inputs j + r L/R (r < R), twiddled by W_{NS R}^{(j mod NS) r},
// a DFT_R in registers, outputs to (j / NS) NS R + j mod NS + r NS.  The first
// pass reads the row straight from global memory (coalesced: consecutive j,
// consecutive addresses); the passes exchange through LDS, each thread
// holding all of its butterflies' inputs in registers between two barriers,
// so the exchange is in place.  Each pass's twiddles sit in a table of their
// own, entry (r - 1) NS + (j mod NS): consecutive butterflies read
// consecutive entries.  Where the last pass's outputs go depends on the
// kernel: straight to the spectrum (inverse DFT), to LDS for the split of two
// real rows transformed as one complex row, or to a tile of LDS written out
// in runs of whole cache lines (the sub-transform kernels).
//
// Whole rows are dealt to groups of NT threads, ROWS groups per workgroup,
// with the row length bounded by LMAX: short rows run one wavefront each
// (wave barriers only), long rows a whole workgroup and up to all 160 KB of
// LDS.  Zero-padded rows whose N_fft = P F has a short factor F >= N run as
// P sub-transforms of F points, one wavefront each (k_fftpad_sub,
// k_fftpad_pairs).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

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

// Where the rows come from and where the spectra go.  RowIo mode 2 reads
// complex rows and writes their inverse DFT, scaled.  PairRowIo (real rows,
// f32 / f64) transforms two rows a, b zero-padded to L as one complex row
// z = a + j b and leaves Z in the group's LDS slice; the caller separates
//   A[k] = (Z[k] + conj(Z[L-k])) / 2,  B[k] = (Z[k] - conj(Z[L-k])) / 2j.
template <int MODE>
struct RowIo {
  static constexpr bool kStaged = false;
  Rsrc rx, rX;
  float scale;
  __device__ __forceinline__ float2 load(unsigned idx, unsigned) const {
    return cconj(ld_c64(rx, 8 * idx));  // inverse: conjugate, forward FFT, conjugate
  }
  __device__ __forceinline__ void store(unsigned pos, float2 v) const {
    st_c64(cscale(cconj(v), scale), rX, 8 * pos);
  }
};
template <int KIND>
struct PairRowIo {
  static constexpr bool kStaged = false;
  Rsrc ra, rb;  // samples past N (and a missing second row) read as 0
  float2 *slice;
  __device__ __forceinline__ float2 load(unsigned idx, unsigned) const {
    return make_float2(ld_real<KIND>(ra, idx), ld_real<KIND>(rb, idx));
  }
  __device__ __forceinline__ void store(unsigned pos, float2 v) const { slice[pos] = v; }
};

// HermPairIo (mode 3): two Hermitian half spectra a, b (bins 0 .. L/2 of
// real rows; the imaginary parts of bin 0 and, for even L, bin L/2 are
// taken as 0) inverted as one complex row: z = IDFT(A + j B) gives
// a = Re z, b = Im z.  Bin k > L/2 is conj(bin L - k).  The inverse is the
// conjugate of the forward FFT of the conjugate, scaled by 1/L; the last
// pass writes both real rows straight to global memory.
struct HermPairIo {
  static constexpr bool kStaged = false;
  Rsrc ra, rb;  // half spectra (a missing second row reads as 0)
  Rsrc oa, ob;  // real output rows (a missing second row drops its stores)
  unsigned L;
  float scale;
  __device__ __forceinline__ float2 bin(Rsrc r, unsigned k) const {
    const bool up = 2 * k > L;
    const unsigned m = up ? L - k : k;
    float2 v = ld_c64(r, 8 * m);
    if (up) v = cconj(v);
    if (m == 0 || 2 * m == L) v.y = 0.f;
    return v;
  }
  __device__ __forceinline__ float2 load(unsigned idx, unsigned) const {
    const float2 a = bin(ra, idx), b = bin(rb, idx);
    return make_float2(a.x - b.y, -(a.y + b.x));  // conj(A + j B)
  }
  __device__ __forceinline__ void store(unsigned pos, float2 v) const {
    // z = conj(v) / L: a = Re z, b = Im z
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b32(oa, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(U, v.x * scale), oa, (int)(4 * pos), 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(U, -v.y * scale), ob, (int)(4 * pos), 0, 0);
  }
};

// SubIo: sub-transform r (an F-point FFT) of a real row zero-padded to
// N_fft = P F, eq. (2) split by residue class of the bin:
//   X[q P + r] = sum_{n<N} (x[n] W_{N_fft}^{r n}) W_F^{q n},  q < F.
// The twiddle of input n = t + u (t the lane, u the same for the whole wave)
// is W^{r t} W^{r u}: one per-lane factor loaded once and one factor read
// from the same address by every lane.  Outputs go to column g of an F x RG
// tile in LDS that the workgroup then writes out in runs of RG bins; the
// column index is XOR-swizzled by the row so that 32 consecutive rows hit 32
// distinct bank pairs and a row stays a contiguous run of RG slots.
template <int KIND, int RG>
struct SubIo {
  static constexpr bool kStaged = true;
  static constexpr int kShift = RG == 16 ? 1 : 2;  // rows per bank-pair cycle: 32 / RG
  Rsrc rx;                // the row's N samples; reads past N give 0
  const float2 *root;     // W_{N_fft}^m, m < N_fft
  float2 wl;              // W_{N_fft}^{r t}
  unsigned r, g;          // sub-transform and its column in the tile
  float2 *tile;
  __device__ __forceinline__ float2 load(unsigned idx, unsigned u) const {
    return cscale(cmul(wl, root[r * u]), ld_real<KIND>(rx, idx));
  }
  __device__ __forceinline__ void store(unsigned pos, float2 v) const {
    tile[pos * RG + (g ^ ((pos >> kShift) & (RG - 1)))] = v;
  }
};

// Outputs into the wave's own LDS slice (the conjugate-pair kernel below):
// ColIo is sub-transform r as in SubIo; PairIo is the F-point FFT of
// z[n] = x[2n] + j x[2n+1], whose combine gives the 2F-point DFT of x.
template <int KIND>
struct ColIo {
  static constexpr bool kStaged = false;
  Rsrc rx;
  const float2 *root;
  float2 wl;
  unsigned r;
  float2 *slice;
  __device__ __forceinline__ float2 load(unsigned idx, unsigned u) const {
    return cscale(cmul(wl, root[r * u]), ld_real<KIND>(rx, idx));
  }
  __device__ __forceinline__ void store(unsigned pos, float2 v) const { slice[pos] = v; }
};
template <int KIND>
struct PairIo {
  static constexpr bool kStaged = false;
  Rsrc rx;  // samples past N read as 0
  float2 *slice;
  __device__ __forceinline__ float2 load(unsigned idx, unsigned) const {
    return make_float2(ld_real<KIND>(rx, 2 * idx), ld_real<KIND>(rx, 2 * idx + 1));
  }
  __device__ __forceinline__ void store(unsigned pos, float2 v) const { slice[pos] = v; }
};

template <int NT, int LMAX, int R, class Io>
__device__ __forceinline__ void mix_pass(int p, const MixPlan &pl, float2 *buf, const Io &io, const float2 *twp,
                                         unsigned t) {
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
        v[i * R + r] = first ? io.load(idx, idx - t) : buf[idx];
      }
    }
  }
  if (!first) group_sync<NT>();  // every input of this pass is in registers before any output lands
  // a staged last pass writes a tile that spans every group's buffer
  if (Io::kStaged && last) __syncthreads();
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
        if (last)
          io.store(pos, v[i * R + r]);
        else
          buf[pos] = v[i * R + r];
      }
    }
  }
  if (!last) group_sync<NT>();  // outputs visible to the next pass
}

// the passes of a plan, its radices grouped (8s, one 4 or 2, 3s, 5s, 7s):
// one loop per radix keeps each pass body's registers to itself
template <int NT, int LMAX, class Io>
__device__ __forceinline__ void mix_run(const MixPlan &pl, float2 *buf, const Io &io, const float2 *twp,
                                        unsigned t) {
  int p = 0;
  for (; p < pl.npass && pl.R[p] == 8; ++p) mix_pass<NT, LMAX, 8>(p, pl, buf, io, twp, t);
  for (; p < pl.npass && pl.R[p] == 4; ++p) mix_pass<NT, LMAX, 4>(p, pl, buf, io, twp, t);
  for (; p < pl.npass && pl.R[p] == 2; ++p) mix_pass<NT, LMAX, 2>(p, pl, buf, io, twp, t);
  for (; p < pl.npass && pl.R[p] == 3; ++p) mix_pass<NT, LMAX, 3>(p, pl, buf, io, twp, t);
  for (; p < pl.npass && pl.R[p] == 5; ++p) mix_pass<NT, LMAX, 5>(p, pl, buf, io, twp, t);
  for (; p < pl.npass && pl.R[p] == 7; ++p) mix_pass<NT, LMAX, 7>(p, pl, buf, io, twp, t);
}

// MODE 0 / 1: real f32 / f64 rows of N samples zero-padded to L, bins k < nout
// written, two rows per group (PairRowIo); MODE 2: complex rows of L points,
// inverse DFT with scale 1/L, one row per group; MODE 3: Hermitian half
// spectra (L/2 + 1 bins, xs complex elements apart) to real rows of L floats
// (os floats apart), scale 1/L, two rows per group (HermPairIo).
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
  constexpr int RPG = MODE == 2 ? 1 : 2;  // rows per group
  const int64_t b = ((int64_t)blockIdx.x * ROWS + g) * RPG;
  // a group past the last row leaves: with NT = 64 it is a wave of its own
  // and has no workgroup barrier to join; larger NT run one group per
  // workgroup, which always exists
  if (b >= B) return;
  float2 *buf = lds + g * LMAX;
  if constexpr (MODE == 3) {
    const bool two = b + 1 < B;
    const unsigned L = (unsigned)pl.L;
    HermPairIo io;
    io.ra = make_rsrc((const float2 *)x + b * xs, (uint64_t)(L / 2 + 1) * 8);
    io.rb = make_rsrc((const float2 *)x + (two ? b + 1 : b) * xs, two ? (uint64_t)(L / 2 + 1) * 8 : 0);
    io.oa = make_rsrc((float *)X + b * os, (uint64_t)L * 4);
    io.ob = make_rsrc((float *)X + (two ? b + 1 : b) * os, two ? (uint64_t)L * 4 : 0);
    io.L = L;
    io.scale = scale;
    mix_run<NT, LMAX>(pl, buf, io, twp, t);
  } else if constexpr (MODE == 2) {
    RowIo<MODE> io;
    io.rx = make_rsrc((const char *)x + b * xs * 8, (uint64_t)pl.L * 8);
    io.rX = make_rsrc(X + b * os, (uint64_t)nout * 8);
    io.scale = scale;
    mix_run<NT, LMAX>(pl, buf, io, twp, t);
  } else {
    constexpr int XB = MODE == 1 ? 8 : 4;
    const bool two = b + 1 < B;
    PairRowIo<MODE> io;
    io.ra = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
    io.rb = make_rsrc((const char *)x + (two ? b + 1 : b) * xs * XB, two ? (uint64_t)N * XB : 0);
    io.slice = buf;
    mix_run<NT, LMAX>(pl, buf, io, twp, t);
    group_sync<NT>();
    const Rsrc ra = make_rsrc(X + b * os, (uint64_t)nout * 8);
    const Rsrc rb = make_rsrc(X + (two ? b + 1 : b) * os, two ? (uint64_t)nout * 8 : 0);  // no second row: dropped
    const unsigned L = (unsigned)pl.L;
    for (unsigned k = t; k < (unsigned)nout; k += NT) {
      const float2 z = buf[k], c = cconj(buf[k == 0 ? 0u : L - k]);
      const float2 e = cscale(cadd(z, c), 0.5f), d = cscale(csub(z, c), 0.5f);
      st_c64(e, ra, 8 * k);
      st_c64(make_float2(d.y, -d.x), rb, 8 * k);  // (z - c) / 2j
    }
  }
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

// Zero-padded FFT by sub-transforms (eq. (2) with N_fft = P F, F >= N):
// workgroup (row b, sub-transforms r0 .. r0 + RG - 1) runs one F-point FFT
// per wave (SubIo above) and writes the F x RG tile of bins q P + r, so every
// run of RG bins (128 bytes at RG = 16) is written whole by one workgroup.
// The passes work in each wave's own F-point slice of the tile's LDS.
template <int RG, int FMAX, int KIND>
__global__ void __launch_bounds__(64 * RG)
    k_fftpad_sub(const void *__restrict__ x, int64_t xs, int64_t N, int P, float2 *__restrict__ X, int64_t os,
                 int64_t nout, MixPlan pl, const float2 *__restrict__ twg, const float2 *__restrict__ root) {
  __shared__ float2 tile[RG * FMAX];
  const int F = pl.L;
  const unsigned t = threadIdx.x % 64;
  const unsigned g = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int nrb = P / RG;
  const int64_t b = blockIdx.x / nrb;
  const unsigned r0 = (unsigned)(blockIdx.x % nrb) * RG;
  constexpr int XB = KIND == 1 ? 8 : 4;
  SubIo<KIND, RG> io;
  io.rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
  io.root = root;
  io.r = r0 + g;
  io.g = g;
  io.wl = root[io.r * t];  // r t < 64 P <= N_fft (F >= 64)
  io.tile = tile;
  mix_run<64, FMAX>(pl, tile + g * F, io, twg, t);
  __syncthreads();
  // bins q P + r0 + w (q < F, w < RG) in runs of RG; bins past nout dropped
  const Rsrc rX = make_rsrc(X + b * os, (uint64_t)nout * 8);
  constexpr int kShift = SubIo<KIND, RG>::kShift;
  for (unsigned f = threadIdx.x; f < (unsigned)F * RG; f += 64 * RG) {
    const unsigned q = f / RG, w = f % RG;
    st_c64(tile[q * RG + (w ^ ((q >> kShift) & (RG - 1)))], rX, 8 * (q * (unsigned)P + r0 + w));
  }
}

// Zero-padded FFT of real rows by conjugate pairs of sub-transforms
// (N_fft = P F, P = 2H in {16, 32}, F >= N, F <= FMAX).  For real x the
// bins of sub-transform P - r mirror those of r:
//   Y_{P-r}[F-1-q] = conj(Y_r[q])   (X[N_fft - k] = conj(X[k])),
// so workgroup b (one row, H waves) transforms only columns 1 .. H-1 (wave
// w: column w) and gets columns 0 and H, the even and odd bins of the
// 2F-point DFT of x, from one complex F-point FFT of
// z[n] = x[2n] + j x[2n+1] on wave 0:
//   E = (Z[k] + conj(Z[F-k])) / 2,  O = (Z[k] - conj(Z[F-k])) / 2j,
//   X_2F[k] = E + W_2F^k O,  X_2F[k+F] = E - W_2F^k O   (k < F),
// with W_2F^k = W_{N_fft}^{k H}.  About half the arithmetic of P
// sub-transforms.  The bins go out through an F x 16 tile in LDS (the same
// swizzle as above), columns 0-15 then, for P = 32, columns 16-31.
template <int H, int FMAX, int KIND>
__global__ void __launch_bounds__(64 * H)
    k_fftpad_pairs(const void *__restrict__ x, int64_t xs, int64_t N, float2 *__restrict__ X, int64_t os,
                   int64_t nout, MixPlan pl, const float2 *__restrict__ twg, const float2 *__restrict__ root) {
  static_assert(H == 8 || H == 16, "P = 16 or 32 sub-transforms");
  constexpr int P = 2 * H, NQ = (FMAX + 63) / 64;
  __shared__ float2 tile[16 * FMAX];
  const int F = pl.L;
  const unsigned t = threadIdx.x % 64;
  const unsigned w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t b = blockIdx.x;
  constexpr int XB = KIND == 1 ? 8 : 4;
  const Rsrc rx = make_rsrc((const char *)x + b * xs * XB, (uint64_t)N * XB);
  float2 *slice = tile + w * F;  // H F <= 16 FMAX
  if (w == 0) {
    PairIo<KIND> io;
    io.rx = rx;
    io.slice = slice;
    mix_run<64, FMAX>(pl, slice, io, twg, t);
  } else {
    ColIo<KIND> io;
    io.rx = rx;
    io.root = root;
    io.r = w;
    io.wl = root[w * t];  // w t < 64 P <= N_fft
    io.slice = slice;
    mix_run<64, FMAX>(pl, slice, io, twg, t);
  }
  wave_sync();
  // lane values: wave 0 the bins X_2F[k] (lo) and X_2F[k + F] (hi) of
  // k = t + 64 i; the other waves Y_w[q] of q = t + 64 i (lo)
  float2 lo[NQ], hi[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const unsigned k = t + 64u * i;
    lo[i] = hi[i] = make_float2(0.f, 0.f);
    if ((int)k < F) {
      const float2 a = slice[k];
      if (w == 0) {
        const float2 c = cconj(slice[k == 0 ? 0u : (unsigned)F - k]);
        const float2 e = cscale(cadd(a, c), 0.5f);
        const float2 d = cscale(csub(a, c), 0.5f);
        const float2 o = cmul(make_float2(d.y, -d.x), root[k * (unsigned)H]);  // W_2F^k (a - c) / 2j
        lo[i] = cadd(e, o);
        hi[i] = csub(e, o);
      } else {
        lo[i] = a;
      }
    }
  }
  __syncthreads();  // every slice read: the tile takes the bins
  auto put = [&](unsigned q, unsigned c, float2 v) { tile[q * 16 + (c ^ ((q >> 1) & 15))] = v; };
  const Rsrc rX = make_rsrc(X + b * os, (uint64_t)nout * 8);
  auto write_out = [&](unsigned c0) {
    for (unsigned f = threadIdx.x; f < (unsigned)F * 16; f += 64 * H) {
      const unsigned q = f / 16, c = f % 16;
      st_c64(tile[q * 16 + (c ^ ((q >> 1) & 15))], rX, 8 * (q * (unsigned)P + c0 + c));
    }
  };
  // bin m of the 2F-point DFT is Y_0[m / 2] (m even) or Y_H[(m - 1) / 2]
  // (m odd); with P = 32 column H = 16 belongs to the second tile
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const unsigned k = t + 64u * i;
    if ((int)k >= F) continue;
    if (w == 0) {
      const unsigned m2 = k + (unsigned)F;
      if (!(k & 1)) put(k >> 1, 0, lo[i]);
      else if (P == 16) put(k >> 1, H, lo[i]);
      if (!(m2 & 1)) put(m2 >> 1, 0, hi[i]);
      else if (P == 16) put(m2 >> 1, H, hi[i]);
    } else {
      put(k, w, lo[i]);
      if (P == 16) put((unsigned)F - 1 - k, P - w, cconj(lo[i]));
    }
  }
  __syncthreads();
  write_out(0);
  if constexpr (P == 32) {
    __syncthreads();  // the first tile is out
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const unsigned k = t + 64u * i;
      if ((int)k >= F) continue;
      if (w == 0) {
        const unsigned m2 = k + (unsigned)F;
        if (k & 1) put(k >> 1, 0, lo[i]);
        if (m2 & 1) put(m2 >> 1, 0, hi[i]);
      } else {
        put((unsigned)F - 1 - k, 16 - w, cconj(lo[i]));
      }
    }
    __syncthreads();
    write_out(16);
  }
}

template <int H>
void pairs_launch(const SubLaunch &a, hipStream_t s) {
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_fftpad_pairs<H, 640, 1>), dim3((unsigned)a.B), dim3(64 * H), 0, s, a.x, a.xs, a.N, a.X,
                       a.os, a.nout, a.plan, a.tw, a.root);
  else
    hipLaunchKernelGGL((k_fftpad_pairs<H, 640, 0>), dim3((unsigned)a.B), dim3(64 * H), 0, s, a.x, a.xs, a.N, a.X,
                       a.os, a.nout, a.plan, a.tw, a.root);
}

template <int RG, int FMAX>
void sub_launch(const SubLaunch &a, hipStream_t s) {
  const unsigned grid = (unsigned)(a.B * (a.P / RG));
  if (a.in_kind == 1)
    hipLaunchKernelGGL((k_fftpad_sub<RG, FMAX, 1>), dim3(grid), dim3(64 * RG), 0, s, a.x, a.xs, a.N, a.P, a.X, a.os,
                       a.nout, a.plan, a.tw, a.root);
  else
    hipLaunchKernelGGL((k_fftpad_sub<RG, FMAX, 0>), dim3(grid), dim3(64 * RG), 0, s, a.x, a.xs, a.N, a.P, a.X, a.os,
                       a.nout, a.plan, a.tw, a.root);
}

template <int NT, int LMAX, int ROWS, bool TWL, int MODE>
void mix_launch_tier(const MixLaunch &a, hipStream_t s) {
  const int64_t groups = MODE == 2 ? a.B : (a.B + 1) / 2;  // real rows go two to a group
  const unsigned grid = (unsigned)((groups + ROWS - 1) / ROWS);
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

// tiles of 16 sub-transforms of up to 640 points (80 KB) or 8 of up to 1024
// (64 KB): two workgroups per CU either way
int sub_tile_rows(int64_t F, int64_t P) {
  if (F < 64 || F > 1024 || P < 8) return 0;
  if (F <= 640 && P % 16 == 0) return 16;
  return P % 8 == 0 ? 8 : 0;
}

int sub_plan(int64_t N, int64_t nfft, int *F, int *P, MixPlan *pl) {
  const int64_t f0 = std::max<int64_t>(N, 64);
  // conjugate pairs for real rows: P = 16 or 32 sub-transforms of the
  // shortest 7-smooth F >= N up to 640 points (half the arithmetic)
  for (int64_t f = f0; f <= 640 && f <= nfft; ++f)
    if (nfft % f == 0 && (nfft / f == 16 || nfft / f == 32) && mix_plan(f, pl)) {
      *F = (int)f;
      *P = (int)(nfft / f);
      return 2;
    }
  // otherwise the shortest F >= N dividing N_fft that fills 16-row tiles
  // (whole 128-byte runs of bins: least work per bin, log F, and the most
  // sub-transforms); 8-row tiles (64-byte runs) only for power-of-two N_fft,
  // where they beat P workgroups each writing every P-th bin; other 7-smooth
  // N_fft run faster as one whole-row FFT
  for (int64_t f = f0; f <= 640 && f <= nfft; ++f)
    if (nfft % f == 0 && (nfft / f) % 16 == 0 && mix_plan(f, pl)) {
      *F = (int)f;
      *P = (int)(nfft / f);
      return 1;
    }
  if (nfft & (nfft - 1)) return 0;
  for (int64_t f = f0; f <= 1024 && f <= nfft; ++f)
    if (nfft % f == 0 && sub_tile_rows(f, nfft / f) && mix_plan(f, pl)) {
      *F = (int)f;
      *P = (int)(nfft / f);
      return 1;
    }
  return 0;
}

hipError_t launch_fftpad_sub(const SubLaunch &a, hipStream_t s) {
  if (a.pairs) {
    if (a.plan.L > 640 || (a.P != 16 && a.P != 32)) return hipErrorInvalidValue;
    if (a.P == 16)
      pairs_launch<8>(a, s);
    else
      pairs_launch<16>(a, s);
    return hipGetLastError();
  }
  const int rg = sub_tile_rows(a.plan.L, a.P);
  if (rg == 16)
    sub_launch<16, 640>(a, s);
  else if (rg == 8)
    sub_launch<8, 1024>(a, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fft_mixed(const MixLaunch &a, hipStream_t s) {
  switch (a.mode) {
    case 0: mix_launch<0>(a, s); break;
    case 1: mix_launch<1>(a, s); break;
    case 2: mix_launch<2>(a, s); break;
    case 3: mix_launch<3>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tz
