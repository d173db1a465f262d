// Uneven batch: thousands of traces, each with its own length N, band
// [f1, f2), bin count M and method (CZT or Zoom FFT), transformed by one
// persistent kernel that pulls work from a device queue, recorded once in a
// hipGraph.
//
// Work decomposition.  Every job is split into work items, one per bin block
// of its Bluestein plan (rows a2-a6; zoom jobs first pass through the front
// end, rows a7-a9, and then are a CZT of complex u, row a10).  Items with the
// same FFT length L form units of G = 1024 / NT(L) items, so a 1024-thread
// workgroup runs G independent L-point FFTs side by side in one LDS budget of
// ~139 KB for every L.  Units are dealt out by an atomic counter in an order
// chosen by the autotuner; every wave leaves when the counter passes the last
// unit, so the grid always drains.
//
// Tables.  Per-job chirps, conjugate-chirp spectra V and zoom taps/phasors
// are built at creation by batched FP64 kernels into one arena.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "fft_core.h"
#include "internal.h"
#include "phase.h"
#include "thzspec.h"

namespace tz {

// one bin block of one job
struct BatchItem {
  int64_t x_off;     // first input sample: f32 in x_flat, or complex in the u scratch
  int64_t X_off;     // first output bin of this block in X_flat (complex)
  int64_t pre_off;   // arena offsets (float2 units)
  int64_t post_off;  // post table of segment 0; segment s at + s * post_stride
  int64_t V_off;
  int32_t N;         // input samples (LD for zoom jobs)
  int32_t Ns;        // samples per segment
  int32_t nseg;
  int32_t kmax;      // bins of this block
  int32_t post_stride;
  int32_t complex_in;
};

// up to G items of one FFT-length class with the same input kind and the
// same segmentation, so every branch inside a workgroup is uniform
struct BatchUnit {
  int32_t first, count, lclass, flavor;  // flavor: bit 0 complex input, bit 1 segmented
};

struct ZoomJob {
  int64_t x_off, u_off, g_off, ph_off;
  int32_t N, LD, D, T;
};

// one workgroup of the zoom front end: outputs [m0, m0 + opb) of one job
struct ZoomTile {
  int32_t job, m0;
};

// workgroup size of the class kernels: 512 threads (two waves per SIMD, so
// the CZT body keeps its ~160 registers without spilling), or the FFT's own
// thread count when that is larger
template <int L>
constexpr int batch_threads() { return Fft<L>::NT > 512 ? Fft<L>::NT : 512; }
template <int L>
constexpr int group_size() { return batch_threads<L>() / Fft<L>::NT; }

// ---------------------------------------------------------------------------
// one item on one subgroup of NT threads (same arithmetic as k_czt)
// ---------------------------------------------------------------------------
template <int L, bool SEG, bool CIN>
__device__ __forceinline__ void czt_item(const BatchItem &it, bool active, const float *__restrict__ x,
                                         float2 *__restrict__ X, const float2 *__restrict__ u,
                                         const float2 *__restrict__ arena, float2 *lds, const TwLds &twd,
                                         unsigned t) {
  using F = Fft<L>;
  constexpr int NT = F::NT, E = F::E;
  const int kmax = active ? it.kmax : 0;  // an idle subgroup computes but stores nothing
  const Rsrc rV = make_rsrc(arena + it.V_off, (uint64_t)L * 8);
  const Rsrc rX = make_rsrc(X + it.X_off, (uint64_t)kmax * 8);
  float2 v[E];
  const int nloop = SEG ? it.nseg : 1;
  for (int s = 0; s < nloop; ++s) {
    // every segment (and the single pass of an unsegmented item) derives its
    // thread offsets afresh: none is held in registers across the loop or
    // from the unit's start (no spills in any class, 103 registers at 8192)
    const unsigned t1 = t + opaque_zero();
    const int64_t n0 = (int64_t)s * it.Ns;
    const int64_t nmax = (it.N - n0 < it.Ns) ? (it.N - n0) : it.Ns;
    const Rsrc rp = make_rsrc(arena + it.pre_off, (uint64_t)nmax * 8);
    const Rsrc rx = CIN ? make_rsrc(u + it.x_off + n0, (uint64_t)nmax * 8)
                        : make_rsrc(x + it.x_off + n0, (uint64_t)nmax * 4);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned n = t1 + NT * e;
      const float2 c = ld_c64(rp, 8 * n);
      if constexpr (CIN)
        v[F::in_slot(e)] = cmul(ld_c64(rx, 8 * n), c);
      else
        v[F::in_slot(e)] = cscale(c, ld_f32(rx, 4 * n));
    }
    F::forward(v, lds, t1, twd);
    // from L = 8192 up the spectral product and the second transform recompute
    // their thread-derived offsets (fewer live registers: no spills at 128)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t1 + NT * e;
      v[F::out_slot(e)] = cconj(cmul(v[F::out_slot(e)], ld_c64(rV, 8 * (L >= 8192 ? k + opaque_zero() : k))));
    }
    F::out_to_in(v);
    const unsigned t2 = L >= 8192 ? t + opaque_zero() : t1;
    F::forward(v, lds, (int)t2, twd);
    const Rsrc rq = make_rsrc(arena + it.post_off + (int64_t)s * it.post_stride, (uint64_t)it.kmax * 8);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned k = t2 + NT * e;
      const float2 r = cmul(cconj(v[F::out_slot(e)]), ld_c64(rq, 8 * k));
      // segments accumulate in X: each thread adds to its own stores of the
      // previous segment (same addresses, program order); bins past the block
      // are dropped
      st_c64((SEG && s > 0) ? cadd(ld_c64(rX, 8 * k), r) : r, rX, 8 * k);
    }
  }
}

// Persistent kernel for the units of one FFT-length class and flavour (SEG:
// segmented input, CIN: complex input): every workgroup takes units from the
// bucket's counter until it passes the last one.  The kernel asks for four
// waves per SIMD (128 VGPRs).
template <int L, bool SEG, bool CIN>
__global__ void __launch_bounds__(batch_threads<L>(), 4)
    k_batch_class(const float *__restrict__ x, float2 *__restrict__ X, const float2 *__restrict__ u,
                  const float2 *__restrict__ arena, const BatchItem *__restrict__ items,
                  const BatchUnit *__restrict__ units, int n_units, unsigned *counter,
                  const float2 *__restrict__ tw) {
  constexpr int NT = Fft<L>::NT;
  __shared__ float2 lds[group_size<L>() * lds_points<L>()];
  __shared__ float2 twl[tw_lds_points<L>()];
  __shared__ int next;
  const unsigned tid = threadIdx.x;
  // a subgroup spans whole waves (NT >= 64): its index, and the work item it
  // selects, are wave-uniform and live in scalar registers
  const unsigned sg = __builtin_amdgcn_readfirstlane(tid / NT), t = tid % NT;
  const TwLds twd = load_twiddles<L>(twl, tw, tid, batch_threads<L>());
  for (;;) {
    if (tid == 0) next = (int)atomicAdd(counter, 1u);
    __syncthreads();  // also orders the twiddle table load before first use
    const int ui = next;
    __syncthreads();  // every thread has read `next` before it is overwritten
    if (ui >= n_units) break;  // uniform: the whole workgroup leaves together
    const BatchUnit un = units[ui];
    const bool active = (int)sg < un.count;
    const BatchItem it = items[un.first + (active ? (int)sg : 0)];
    float2 *sub = lds + sg * lds_points<L>();
    // the thread index through an opaque zero: addresses derived from it are
    // formed per unit instead of being hoisted out of the loop and held live
    czt_item<L, SEG, CIN>(it, active, x, X, u, arena, sub, twd, t + opaque_zero());
  }
}

__global__ void k_batch_reset(unsigned *counters, int n) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n) counters[threadIdx.x] = 0u;
}

// zoom front end for every zoom job, one workgroup per tile of opb outputs
// of one job (a job of L_D outputs spans ceil(L_D / opb) tiles, so short and
// long jobs alike spread over the whole chip):
// u[m] = e^{-j 2 pi nu_N m D} sum_t g[t] x[mD - t], FP64 taps, phasors and
// sums (the T-term sum in FP32 would lose accuracy as sqrt(T)).  The tile's
// samples pass through LDS (buffer loads: zeros outside [0, N)); the tap
// index is the same across the wave, so the taps come through scalar loads.  When D is a multiple of 4 the tile has two
// pad words after every D samples (sample i at word i + 2 floor(i/D)): output
// j's base j (D + 2) then spreads the lanes over the banks, and the offset of
// tap c, c + 2 floor(c/D), is the same in every lane, an immediate of the LDS
// read within each block of D taps.  Other D keep a linear tile (the per-tap
// offsets fold the same way).  Filters longer than half the tile, and traces
// of 2^29 samples or more, read x and the taps straight from global memory.
constexpr int kBZTile = 6144;  // samples per chunk

// outputs per tile: their samples, (opb - 1) D + T, fit the LDS chunk
// (opb >= 1); jobs on the global-memory path take tiles of 256 outputs
__host__ __device__ inline int zoom_tile_outputs(int D, int T, int N) {
  if (2 * T > kBZTile || N >= (1 << 29)) return 256;
  const int o = (kBZTile - T) / D + 1;
  return o < 256 ? o : 256;
}

__global__ void __launch_bounds__(256)
    k_batch_zoom_front(const float *__restrict__ x, float2 *__restrict__ u, const float2 *__restrict__ arena,
                       const ZoomJob *__restrict__ jobs, const ZoomTile *__restrict__ tiles) {
  __shared__ float xl[kBZTile + kBZTile / 2 + 1];
  const ZoomTile tl = tiles[blockIdx.x];
  const ZoomJob j = jobs[tl.job];
  const double2 *g = (const double2 *)(arena + j.g_off);
  const double2 *ph = (const double2 *)(arena + j.ph_off);
  const float *xb = x + j.x_off;
  const int D = j.D, T = j.T, N = j.N, LD = j.LD;
  const int opb = zoom_tile_outputs(D, T, N);
  const int m_end = tl.m0 + opb < LD ? tl.m0 + opb : LD;
  if (2 * T > kBZTile || N >= (1 << 29)) {
    for (int m = tl.m0 + (int)threadIdx.x; m < m_end; m += 256) {
      const int64_t base = (int64_t)m * D;
      double ar = 0.0, ai = 0.0;
      for (int tt = 0; tt < T; ++tt) {
        const int64_t n = base - tt;
        if (n >= 0 && n < N) {
          const double xv = (double)xb[n];
          ar = fma(g[tt].x, xv, ar);
          ai = fma(g[tt].y, xv, ai);
        }
      }
      const double2 p = ph[m];
      u[j.u_off + m] = make_float2((float)(p.x * ar - p.y * ai), (float)(p.x * ai + p.y * ar));
    }
    return;
  }
  const int P = D % 4 == 0 ? 2 : 0;
  const uint32_t dmagic = P ? (uint32_t)((((uint64_t)1 << 32) + D - 1) / D) : 0u;  // floor(i/D) = umulhi(i, dmagic)
  // reads past N return 0; n < 0 wraps to an offset above 2^31 (N * 4 < 2^31)
  const Rsrc rx = make_rsrc(xb, (uint64_t)N * 4);
  const int jt = (int)threadIdx.x;
  const float *base = xl + jt * (D + P);
  const double2 *gp = g + (T - 1);  // tap of tile sample c (c = T - 1 - t): gp[-c]
  {
    const int m0 = tl.m0;
    const int64_t n0 = (int64_t)m0 * D - (T - 1);
    const int span = (opb - 1) * D + T;
    // every load of the tile is issued before the first LDS write (one
    // memory round trip per tile instead of one per group of loads); loads
    // past the span are harmless (read in range or as 0) and not stored
    constexpr int kPer = kBZTile / 256;
    float xv[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) xv[k] = ld_f32(rx, (unsigned)((n0 + jt + 256 * k) * 4));
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = jt + 256 * k;
      if (i < span) xl[i + (P ? P * __umulhi((unsigned)i, dmagic) : 0u)] = xv[k];
    }
    __syncthreads();
    const int m = m0 + jt;
    if (jt < opb && m < LD) {
      double ar = 0.0, ai = 0.0;
      int c = 0, cq = 0;
      while (c < T) {
        const int e = P ? ((cq + 1) * D < T ? (cq + 1) * D : T) : T;
        const float *row = base + P * cq;
#pragma unroll 8
        for (; c < e; ++c) {
          const double2 gt = gp[-c];
          const double xv = (double)row[c];
          ar = fma(gt.x, xv, ar);
          ai = fma(gt.y, xv, ai);
        }
        ++cq;
      }
      const double2 p = ph[m];
      u[j.u_off + m] = make_float2((float)(p.x * ar - p.y * ai), (float)(p.x * ai + p.y * ar));
    }
  }
}

// ---------------------------------------------------------------------------
// batched plan-time tables (FP64 on the GPU, rounded once to float)
// ---------------------------------------------------------------------------
struct TableJob {
  PhaseParams p;
  int64_t Ns, Mb, L, pre_off, post_off, V_off;
  int32_t nseg, nblk;
};

// pre[blk][n] = A^{-n} W^{blk Mb n} W^{n^2/2},
// post[s][blk][k] = W^{k^2/2} A^{-s Ns} W^{(blk Mb + k) s Ns}
__global__ void k_batch_chirps(float2 *arena, const TableJob *__restrict__ jobs) {
  const TableJob j = jobs[blockIdx.x];
  const int64_t npre = j.Ns * j.nblk, npost = j.Mb * j.nblk * j.nseg;
  for (int64_t i = threadIdx.x; i < npre; i += blockDim.x) {
    const int64_t blk = i / j.Ns, n = i % j.Ns;
    double cyc = chirp_cycles(j.p, n, true);
    if (blk) {
      cyc += shift_cycles(j.p, blk * j.Mb, n);
      cyc -= floor(cyc);
    }
    arena[j.pre_off + i] = unit_cycles(cyc);
  }
  for (int64_t i = threadIdx.x; i < npost; i += blockDim.x) {
    const int64_t k = i % j.Mb, blk = (i / j.Mb) % j.nblk, seg = i / (j.Mb * j.nblk);
    double cyc = chirp_cycles(j.p, k, false);
    if (seg) {
      const int64_t n0 = seg * j.Ns;
      if (j.p.rational) {
        const uint64_t q = (uint64_t)j.p.q;
        uint64_t r = mulmod((uint64_t)j.p.pa, (uint64_t)n0 % q, q);
        r = (r + mulmod(mulmod((uint64_t)j.p.pw, (uint64_t)(blk * j.Mb + k) % q, q), (uint64_t)n0 % q, q)) % q;
        cyc += (double)r / (double)q;
      } else {
        cyc += frac_mul(j.p.a, (double)n0) + frac_mul(j.p.w, (double)(blk * j.Mb + k) * (double)n0);
      }
      cyc -= floor(cyc);
    }
    arena[j.post_off + i] = unit_cycles(cyc);
  }
}

// v[l] = W^{-l^2/2} for l < Mb, v[L-l] for 1 <= l < Ns (FP64), for a chunk of
// jobs of one FFT length L laid out [chunk][L]
__global__ void k_batch_conj(double2 *v, const TableJob *__restrict__ jobs, int64_t L, int64_t n_jobs) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= L * n_jobs) return;
  const TableJob j = jobs[gi / L];
  const int64_t i = gi % L;
  int64_t l = -1;
  if (i < j.Mb) l = i;
  else if (L - i < j.Ns) l = L - i;
  if (l < 0) {
    v[gi] = make_double2(0.0, 0.0);
    return;
  }
  double s, c;
  sincospi(2.0 * chirp_cycles(j.p, l, false), &s, &c);
  v[gi] = make_double2(c, s);
}

// one radix-R Stockham pass (R = 2 or 4) over a chunk of FP64 transforms of length L
template <int R>
__global__ void k_batch_fft64_pass(const double2 *in, double2 *out, int64_t L, int64_t ns, int64_t n_jobs) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= (L / R) * n_jobs) return;
  const int64_t job = gi / (L / R), j = gi % (L / R);
  const double2 *a = in + job * L;
  double2 *o = out + job * L;
  const int64_t jm = j % ns;
  double2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double2 z = a[j + r * (L / R)];
    if (r && jm) {
      double s, c;
      sincospi(-2.0 * (double)(jm * r) / (double)(ns * R), &s, &c);
      z = make_double2(z.x * c - z.y * s, z.x * s + z.y * c);
    }
    v[r] = z;
  }
  const int64_t base = (j / ns) * ns * R + jm;
  if constexpr (R == 2) {
    o[base] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
    o[base + ns] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
  } else {
    const double2 t0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
    const double2 t1 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
    const double2 t2 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
    const double2 t3 = make_double2(v[1].y - v[3].y, -(v[1].x - v[3].x));  // -j (v1 - v3)
    o[base] = make_double2(t0.x + t2.x, t0.y + t2.y);
    o[base + 2 * ns] = make_double2(t0.x - t2.x, t0.y - t2.y);
    o[base + ns] = make_double2(t1.x + t3.x, t1.y + t3.y);
    o[base + 3 * ns] = make_double2(t1.x - t3.x, t1.y - t3.y);
  }
}

// V = FFT(v) / L into the arena
__global__ void k_batch_store_V(const double2 *v, float2 *arena, const TableJob *__restrict__ jobs, int64_t L,
                                int64_t n_jobs) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= L * n_jobs) return;
  const TableJob j = jobs[gi / L];
  const double s = 1.0 / (double)L;
  arena[j.V_off + gi % L] = make_float2((float)(v[gi].x * s), (float)(v[gi].y * s));
}

struct ZoomTableJob {
  int64_t g_off, ph_off;
  int32_t T, LD, D, pad;
  double nu_c, nu_N;
};

// Hamming-windowed sinc taps (unit DC gain) modulated by e^{j 2 pi nu_N t},
// and output phasors e^{-j 2 pi nu_N m D}, both kept in FP64 (two arena
// slots per value)
__global__ void k_batch_zoom_tables(float2 *arena, const ZoomTableJob *__restrict__ jobs) {
  const ZoomTableJob j = jobs[blockIdx.x];
  double2 *g = (double2 *)(arena + j.g_off);
  double2 *ph = (double2 *)(arena + j.ph_off);
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int pass = 0; pass < 2; ++pass)
      for (int t = 0; t < j.T; ++t) {
        double h = 1.0;
        if (j.T > 1) {
          const double c = (double)t - 0.5 * (double)(j.T - 1);
          const double uu = 2.0 * j.nu_c * c;
          const double sinc = (uu == 0.0) ? 1.0 : sinpi(uu) / (M_PI * uu);
          const double w = 0.54 - 0.46 * cospi(2.0 * (double)t / (double)(j.T - 1));
          h = w * 2.0 * j.nu_c * sinc;
        }
        if (pass == 0) {
          sum += h;
        } else {
          h /= sum;
          double s, c;
          sincospi(2.0 * frac_mul(j.nu_N, (double)t), &s, &c);
          g[t] = make_double2(h * c, h * s);
        }
      }
  }
  for (int m = threadIdx.x; m < j.LD; m += blockDim.x) {
    double s, c;
    sincospi(-2.0 * frac_mul(j.nu_N, (double)((int64_t)m * j.D)), &s, &c);
    ph[m] = make_double2(c, s);
  }
}

}  // namespace tz

// ===========================================================================
using namespace tz;

namespace tz {
void free_batch(tz_batch *b);
}

struct tz_batch {
  int device = 0;
  int64_t n_jobs = 0;
  int64_t x_extent = 0, X_extent = 0;  // elements of x_flat / X_flat the jobs reach
  std::vector<BatchItem> items;
  std::vector<BatchUnit> units;  // grouped by class; order inside a class chosen by the autotuner
  int cls_count[15] = {};                   // units per FFT-length class
  int bkt_first[60] = {}, bkt_count[60] = {};  // bucket = class * 4 + flavor
  std::vector<ZoomJob> zjobs;
  std::vector<ZoomTile> ztiles;
  void *d_arena = nullptr, *d_items = nullptr, *d_units = nullptr, *d_zjobs = nullptr, *d_ztiles = nullptr;
  void *d_u = nullptr, *d_counter = nullptr;
  void *d_tw[15] = {};
  int grid = 0;
  // 0: class kernels as independent graph branches; 1: two chains (real and
  // complex input) longest class first; 2: the same chains, both after the
  // zoom front end; 3: one chain, longest class first, after the front end
  int topology = 0;
  int inner = 0;     // 0: longest unit first inside a class, 1: creation order
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *last_x = nullptr;
  void *last_X = nullptr;
  bool tuned = false;
  bool tuned_from_cache = false;  // schedule read from the tune cache, no candidates timed
  double tuned_ms[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  std::string sig;  // hash of the job table: the key of its schedule in the tune cache
  hipEvent_t done = nullptr;  // recorded after every launch (tz_batch_wait)
  bool launched = false;
  bool failed = false;  // a launch returned an error: later launches are refused
  // every device buffer and graph object is released here, so an error
  // return anywhere in tz_batch_create frees what was allocated before it
  ~tz_batch() { tz::free_batch(this); }
};

namespace {

tz_status bfail(tz_status st, const std::string &m) {
  set_last_error(m.c_str());
  return st;
}

int ilog2(int64_t v) {
  int l = 0;
  while ((1LL << l) < v) ++l;
  return l;
}

#define BHIP(call, what)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return bfail(e_ == hipErrorOutOfMemory ? TZ_ENOMEM : TZ_EDEVICE,                            \
                   std::string(what) + ": " + hipGetErrorString(e_));                             \
  } while (0)

// unit cost: pieces x L log2 L
double unit_cost(const tz_batch &b, const BatchUnit &u) {
  double c = 0;
  for (int i = 0; i < u.count; ++i) c = std::max(c, (double)b.items[u.first + i].nseg);
  return c * (double)(1LL << u.lclass) * (double)u.lclass;
}

// units of each class and flavour in the order `inner` asks for (every
// bucket stays contiguous, at the same place for either order)
std::vector<BatchUnit> order_units(const tz_batch &b, const std::vector<BatchUnit> &units, int inner) {
  std::vector<BatchUnit> u = units;
  if (inner == 0)
    std::stable_sort(u.begin(), u.end(), [&](const BatchUnit &a, const BatchUnit &c) {
      if (a.lclass != c.lclass) return a.lclass > c.lclass;
      if (a.flavor != c.flavor) return a.flavor < c.flavor;
      return unit_cost(b, a) > unit_cost(b, c);
    });
  else
    std::stable_sort(u.begin(), u.end(), [](const BatchUnit &a, const BatchUnit &c) {
      if (a.lclass != c.lclass) return a.lclass > c.lclass;
      return a.flavor < c.flavor;
    });
  return u;
}

template <int L>
tz_status add_class_node(tz_batch *b, int bucket, const float *xf, float2 *Xc, const hipGraphNode_t *deps,
                         int ndeps, hipGraphNode_t *node) {
  const float2 *u = (const float2 *)b->d_u;
  const float2 *arena = (const float2 *)b->d_arena;
  const BatchItem *it = (const BatchItem *)b->d_items;
  const BatchUnit *un = (const BatchUnit *)b->d_units + b->bkt_first[bucket];
  int nu = b->bkt_count[bucket];
  unsigned *ctr = (unsigned *)b->d_counter + bucket;
  const float2 *tw = (const float2 *)b->d_tw[bucket / 4];
  void *args[] = {(void *)&xf, (void *)&Xc, (void *)&u, (void *)&arena, (void *)&it, (void *)&un,
                  (void *)&nu, (void *)&ctr, (void *)&tw};
  hipKernelNodeParams p{};
  const int fl = bucket % 4;
  // segmented items only occur at the longest length
  if constexpr (L == kMaxL) {
    static void *const f[4] = {(void *)k_batch_class<L, false, false>, (void *)k_batch_class<L, false, true>,
                               (void *)k_batch_class<L, true, false>, (void *)k_batch_class<L, true, true>};
    p.func = f[fl];
  } else {
    if (fl & 2) return bfail(TZ_EUNSUPPORTED, "segmented work item below the longest FFT length");
    p.func = (fl & 1) ? (void *)k_batch_class<L, false, true> : (void *)k_batch_class<L, false, false>;
  }
  // persistent grid: every workgroup the CUs can hold at once
  int per_cu = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p.func, batch_threads<L>(), 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  p.gridDim = dim3((unsigned)std::min(b->grid * per_cu, nu));
  p.blockDim = dim3(batch_threads<L>());
  p.kernelParams = args;
  BHIP(hipGraphAddKernelNode(node, b->graph, deps, ndeps, &p), "graph class node");
  return TZ_OK;
}

// graph: reset counters -> zoom front end -> one persistent kernel per class
// and flavour
tz_status build_graph(tz_batch *b, const void *x, void *X) {
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  // an injected failure fires before any graph object exists, so a failed
  // launch leaves no half-built graph behind
  if (fault_injected("graph")) return bfail(TZ_EDEVICE, "graph build: injected failure (TZ_FAULT=graph)");
  BHIP(hipGraphCreate(&b->graph, 0), "graph create");
  hipGraphNode_t reset, front = nullptr;
  {
    unsigned *ctr = (unsigned *)b->d_counter;
    int n = 60;
    void *args[] = {(void *)&ctr, (void *)&n};
    hipKernelNodeParams p{};
    p.func = (void *)k_batch_reset;
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.kernelParams = args;
    BHIP(hipGraphAddKernelNode(&reset, b->graph, nullptr, 0, &p), "graph reset node");
  }
  const float *xf = (const float *)x;
  float2 *Xc = (float2 *)X;
  if (!b->zjobs.empty()) {
    // the front end reads x and writes u only: it needs no counter reset
    float2 *u = (float2 *)b->d_u;
    const float2 *arena = (const float2 *)b->d_arena;
    const ZoomJob *zj = (const ZoomJob *)b->d_zjobs;
    const ZoomTile *zt = (const ZoomTile *)b->d_ztiles;
    void *args[] = {(void *)&xf, (void *)&u, (void *)&arena, (void *)&zj, (void *)&zt};
    hipKernelNodeParams p{};
    p.func = (void *)k_batch_zoom_front;
    p.gridDim = dim3((unsigned)b->ztiles.size());
    p.blockDim = dim3(256);
    p.kernelParams = args;
    BHIP(hipGraphAddKernelNode(&front, b->graph, nullptr, 0, &p), "graph front node");
  }
  // Real-input classes (CZT jobs) wait only for the counter reset, so they
  // run beside the zoom front end; complex-input classes (the zooms' short
  // DFTs) also wait for the front end.  Topology 0 makes every class its own
  // branch; 1 chains the classes of each input kind longest first; 2 is 1
  // with the real-input chain also after the front end (which then has the
  // GPU to itself instead of starving beside a persistent class kernel); 3
  // runs every class in one chain after the front end.
  hipGraphNode_t chain[2] = {nullptr, nullptr};
  const int topo = b->topology;
  for (int c = 14; c >= 8; --c)
    for (int fl = 0; fl < 4; ++fl) {
      const int bucket = c * 4 + fl;
      if (!b->bkt_count[bucket]) continue;
      const int cin = fl & 1;
      const int ch = topo == 3 ? 0 : cin;  // the chain this class joins
      hipGraphNode_t deps[2];
      int nd = 0;
      if (topo >= 1 && chain[ch]) {
        deps[nd++] = chain[ch];
      } else {
        deps[nd++] = reset;
        if (front && (cin || topo >= 2)) deps[nd++] = front;
      }
      hipGraphNode_t node;
      tz_status st = TZ_OK;
      switch (c) {
        case 8: st = add_class_node<256>(b, bucket, xf, Xc, deps, nd, &node); break;
        case 9: st = add_class_node<512>(b, bucket, xf, Xc, deps, nd, &node); break;
        case 10: st = add_class_node<1024>(b, bucket, xf, Xc, deps, nd, &node); break;
        case 11: st = add_class_node<2048>(b, bucket, xf, Xc, deps, nd, &node); break;
        case 12: st = add_class_node<4096>(b, bucket, xf, Xc, deps, nd, &node); break;
        case 13: st = add_class_node<8192>(b, bucket, xf, Xc, deps, nd, &node); break;
        default: st = add_class_node<16384>(b, bucket, xf, Xc, deps, nd, &node); break;
      }
      if (st) return st;
      chain[ch] = node;
    }
  BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
  b->last_x = x;
  b->last_X = X;
  return TZ_OK;
}

tz_status upload_units(tz_batch *b, hipStream_t s) {
  BHIP(hipMemcpyAsync(b->d_units, b->units.data(), sizeof(BatchUnit) * b->units.size(), hipMemcpyHostToDevice,
                      s),
       "batch units upload");
  BHIP(hipStreamSynchronize(s), "batch units upload");
  return TZ_OK;
}

}  // namespace

// a device allocation freed when it leaves scope (plan-time scratch)
struct ScopedDev {
  void *p = nullptr;
  ScopedDev() = default;
  ScopedDev(const ScopedDev &) = delete;
  ScopedDev &operator=(const ScopedDev &) = delete;
  ~ScopedDev() {
    if (p) (void)hipFree(p);
  }
};

namespace tz {
void free_batch(tz_batch *b) {
  bool any = b->exec || b->graph || b->done || b->d_arena || b->d_items || b->d_units || b->d_zjobs ||
             b->d_ztiles || b->d_u || b->d_counter;
  for (void *p : b->d_tw) any = any || p;
  if (!any) return;
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->done) (void)hipEventDestroy(b->done);
  b->exec = nullptr;
  b->graph = nullptr;
  b->done = nullptr;
  void **ptrs[] = {&b->d_arena, &b->d_items, &b->d_units, &b->d_zjobs, &b->d_ztiles, &b->d_u, &b->d_counter};
  for (void **p : ptrs)
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  for (void *&p : b->d_tw)
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
}
}  // namespace tz

extern "C" {

tz_status tz_batch_create(const tz_job *jobs, int64_t n_jobs, const tz_opts *opts, tz_batch **out) {
  if (!out) return bfail(TZ_EINVAL, "batch output pointer is NULL");
  *out = nullptr;
  if (!jobs || n_jobs < 1) return bfail(TZ_EINVAL, "need a non-empty job array");
  hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
  std::unique_ptr<tz_batch> b(new tz_batch());
  (void)hipGetDevice(&b->device);
  b->n_jobs = n_jobs;

  std::vector<TableJob> tjobs;
  std::vector<ZoomTableJob> ztjobs;
  std::vector<std::vector<BatchItem>> by_class(15 * 4);  // [class][flavor]
  int64_t arena = 0, uscratch = 0;
  auto take = [&](int64_t n) {
    const int64_t o = arena;
    arena += (n + 63) / 64 * 64;
    return o;
  };
  for (int64_t i = 0; i < n_jobs; ++i) {
    const tz_job &j = jobs[i];
    char msg[200];
    if ((j.kind != TZ_JOB_CZT && j.kind != TZ_JOB_ZOOM) || j.N < 1 || j.M < 1 || j.fs_hz < 1 || j.f1_hz < 0 ||
        j.f2_hz <= j.f1_hz || j.in_offset < 0 || j.out_offset < 0 || j.N > INT32_MAX || j.M > INT32_MAX) {
      snprintf(msg, sizeof msg, "job %lld: invalid kind, N, M, band or offsets", (long long)i);
      return bfail(TZ_EINVAL, msg);
    }
    b->x_extent = std::max(b->x_extent, j.in_offset + j.N);
    b->X_extent = std::max(b->X_extent, j.out_offset + j.M);
    PhaseParams p;
    int64_t Nin = j.N;
    int complex_in = 0;
    int64_t x_off = j.in_offset;
    if (j.kind == TZ_JOB_ZOOM) {
      const int64_t D = j.D;
      const int T = j.fir_taps ? j.fir_taps : 63;
      const int64_t K = zoom_short_length((double)j.fs_hz, (double)j.f1_hz, (double)j.f2_hz, j.M, D);
      if (D < 1 || T < 1 || K < 1) {
        snprintf(msg, sizeof msg, "job %lld: zoom needs D >= 1, taps >= 1 and K >= 1", (long long)i);
        return bfail(TZ_EINVAL, msg);
      }
      const int64_t LD = (j.N + D - 1) / D;
      ZoomJob zj{};
      zj.x_off = j.in_offset;
      zj.u_off = uscratch;
      zj.N = (int32_t)j.N;
      zj.LD = (int32_t)LD;
      zj.D = (int32_t)D;
      zj.T = T;
      ZoomTableJob zt{};
      zt.T = T;
      zt.LD = (int32_t)LD;
      zt.D = (int32_t)D;
      zt.nu_c = 1.0 / (2.0 * (double)D);
      const double nuN = 0.5 * ((double)j.f1_hz + (double)j.f2_hz) / (double)j.fs_hz;
      zt.nu_N = nuN - floor(nuN);
      zt.g_off = zj.g_off = take(2 * (int64_t)T);  // double2 = two float2 slots
      zt.ph_off = zj.ph_off = take(2 * LD);
      const int opb = zoom_tile_outputs(zj.D, zj.T, zj.N);
      for (int64_t m0 = 0; m0 < LD; m0 += opb)
        b->ztiles.push_back(ZoomTile{(int32_t)b->zjobs.size(), (int32_t)m0});
      b->zjobs.push_back(zj);
      ztjobs.push_back(zt);
      p = zoom_phase(K, j.M);
      Nin = LD;
      complex_in = 1;
      x_off = uscratch;
      uscratch += (LD + 63) / 64 * 64;
    } else {
      p = band_phase(j.fs_hz, j.f1_hz, j.f2_hz, j.M);
    }
    int L, nseg, nblk;
    int64_t Ns, Mb;
    if (!czt_shape(Nin, j.M, &L, &Ns, &nseg, &Mb, &nblk, true)) {
      snprintf(msg, sizeof msg, "job %lld: N=%lld, M=%lld too long for the single-pass path", (long long)i,
               (long long)Nin, (long long)j.M);
      return bfail(TZ_EUNSUPPORTED, msg);
    }
    TableJob tj{};
    tj.p = p;
    tj.Ns = Ns;
    tj.Mb = Mb;
    tj.L = L;
    tj.nseg = nseg;
    tj.nblk = nblk;
    tj.pre_off = take(Ns * nblk);
    tj.post_off = take(Mb * nblk * nseg);
    tj.V_off = take(L);
    tjobs.push_back(tj);
    for (int blk = 0; blk < nblk; ++blk) {
      BatchItem it{};
      it.x_off = x_off;
      it.X_off = j.out_offset + (int64_t)blk * Mb;
      it.pre_off = tj.pre_off + (int64_t)blk * Ns;
      it.post_off = tj.post_off + (int64_t)blk * Mb;
      it.V_off = tj.V_off;
      it.N = (int32_t)Nin;
      it.Ns = (int32_t)Ns;
      it.nseg = nseg;
      it.kmax = (int32_t)std::min<int64_t>(Mb, j.M - (int64_t)blk * Mb);
      it.post_stride = (int32_t)(Mb * nblk);
      it.complex_in = complex_in;
      by_class[ilog2(L) * 4 + complex_in + (nseg > 1 ? 2 : 0)].push_back(it);
    }
  }
  {
    // FNV-1a over the job records: equal job tables share a tuned schedule
    uint64_t h = 1469598103934665603ull;
    const unsigned char *pj = (const unsigned char *)jobs;
    for (size_t i = 0; i < sizeof(tz_job) * (size_t)n_jobs; ++i) h = (h ^ pj[i]) * 1099511628211ull;
    char hx[40];
    snprintf(hx, sizeof hx, "%016llx-%lld", (unsigned long long)h, (long long)n_jobs);
    b->sig = hx;
  }
  // units of G same-class items (segmented items only occur at L = 16384, G = 1)
  static const int kG[15] = {0, 0, 0, 0, 0, 0, 0, 0, group_size<256>(), group_size<512>(), group_size<1024>(),
                             group_size<2048>(), group_size<4096>(), group_size<8192>(), group_size<16384>()};
  std::vector<BatchUnit> units;
  for (int c = 14; c >= 8; --c)
    for (int fl = 0; fl < 4; ++fl) {
      const int G = kG[c];
      auto &v = by_class[c * 4 + fl];
      for (size_t i = 0; i < v.size(); i += G) {
        BatchUnit u{};
        u.first = (int32_t)b->items.size();
        u.count = (int32_t)std::min<size_t>(G, v.size() - i);
        u.lclass = c;
        u.flavor = fl;
        for (int k = 0; k < u.count; ++k) b->items.push_back(v[i + k]);
        units.push_back(u);
      }
    }
  b->units = order_units(*b, units, 0);
  tz_log("batch: %lld jobs (%zu zoom, %zu front-end tiles), %zu work items in %zu units", (long long)n_jobs,
         b->zjobs.size(), b->ztiles.size(), b->items.size(), units.size());
  for (size_t i = 0; i < b->units.size(); ++i) {
    const int c = b->units[i].lclass, bk = c * 4 + b->units[i].flavor;
    if (!b->bkt_count[bk]) b->bkt_first[bk] = (int)i;
    ++b->bkt_count[bk];
    ++b->cls_count[c];
  }

  // device buffers
  BHIP(dev_malloc((void **)&b->d_arena, sizeof(float2) * std::max<int64_t>(arena, 64)), "batch arena");
  BHIP(dev_malloc((void **)&b->d_items, sizeof(BatchItem) * b->items.size()), "batch items");
  BHIP(dev_malloc((void **)&b->d_units, sizeof(BatchUnit) * b->units.size()), "batch units");
  BHIP(dev_malloc((void **)&b->d_u, sizeof(float2) * std::max<int64_t>(uscratch, 64)), "batch zoom scratch");
  BHIP(dev_malloc((void **)&b->d_counter, sizeof(unsigned) * 64), "batch counters");
  if (!b->zjobs.empty()) {
    BHIP(dev_malloc((void **)&b->d_zjobs, sizeof(ZoomJob) * b->zjobs.size()), "batch zoom jobs");
    BHIP(hipMemcpy(b->d_zjobs, b->zjobs.data(), sizeof(ZoomJob) * b->zjobs.size(), hipMemcpyHostToDevice),
         "batch upload");
    BHIP(dev_malloc((void **)&b->d_ztiles, sizeof(ZoomTile) * b->ztiles.size()), "batch zoom tiles");
    BHIP(hipMemcpy(b->d_ztiles, b->ztiles.data(), sizeof(ZoomTile) * b->ztiles.size(), hipMemcpyHostToDevice),
         "batch upload");
  }
  BHIP(hipMemcpy(b->d_items, b->items.data(), sizeof(BatchItem) * b->items.size(), hipMemcpyHostToDevice),
       "batch upload");
  BHIP(hipMemcpy(b->d_units, b->units.data(), sizeof(BatchUnit) * b->units.size(), hipMemcpyHostToDevice),
       "batch upload");
  for (int c = 8; c <= 14; ++c) {
    const int64_t L = 1LL << c;
    BHIP(dev_malloc((void **)&b->d_tw[c], sizeof(float2) * L), "batch twiddles");
    BHIP(build_twiddles((float2 *)b->d_tw[c], L, s), "batch twiddles");
  }

  // tables: chirps (one workgroup per job), V per FFT-length class in chunks
  {
    ScopedDev tj_buf;
    BHIP(dev_malloc((void **)&tj_buf.p, sizeof(TableJob) * tjobs.size()), "table jobs");
    TableJob *d_tj = (TableJob *)tj_buf.p;
    BHIP(hipMemcpy(d_tj, tjobs.data(), sizeof(TableJob) * tjobs.size(), hipMemcpyHostToDevice), "table jobs");
    hipLaunchKernelGGL(k_batch_chirps, dim3((unsigned)tjobs.size()), dim3(256), 0, s, (float2 *)b->d_arena, d_tj);
    BHIP(hipGetLastError(), "chirp tables");
    BHIP(hipStreamSynchronize(s), "chirp tables");
    const int64_t chunk_points = (int64_t)1 << 25;  // FP64 scratch: 2 x 512 MiB
    ScopedDev va_buf, vb_buf, chunk_buf;
    BHIP(dev_malloc((void **)&va_buf.p, sizeof(double2) * chunk_points), "V scratch");
    BHIP(dev_malloc((void **)&vb_buf.p, sizeof(double2) * chunk_points), "V scratch");
    BHIP(dev_malloc((void **)&chunk_buf.p, sizeof(TableJob) * tjobs.size()), "V jobs");
    double2 *va = (double2 *)va_buf.p, *vb = (double2 *)vb_buf.p;
    TableJob *d_chunk = (TableJob *)chunk_buf.p;
    for (int c = 8; c <= 14; ++c) {
      const int64_t L = 1LL << c;
      std::vector<TableJob> cls;
      for (auto &t : tjobs)
        if (t.L == L) cls.push_back(t);
      const int64_t per = chunk_points / L;
      for (size_t i0 = 0; i0 < cls.size(); i0 += per) {
        const int64_t n = std::min<int64_t>(per, (int64_t)(cls.size() - i0));
        BHIP(hipMemcpy(d_chunk, cls.data() + i0, sizeof(TableJob) * n, hipMemcpyHostToDevice), "V jobs");
        const unsigned blocks = (unsigned)((L * n + 255) / 256);
        hipLaunchKernelGGL(k_batch_conj, dim3(blocks), dim3(256), 0, s, va, d_chunk, L, n);
        double2 *a = va, *bb = vb;
        int64_t ns = 1, rest = L;
        while (rest > 1) {
          const int R = (rest % 4 == 0) ? 4 : 2;
          const unsigned pb = (unsigned)(((L / R) * n + 255) / 256);
          if (R == 4)
            hipLaunchKernelGGL(k_batch_fft64_pass<4>, dim3(pb), dim3(256), 0, s, a, bb, L, ns, n);
          else
            hipLaunchKernelGGL(k_batch_fft64_pass<2>, dim3(pb), dim3(256), 0, s, a, bb, L, ns, n);
          ns *= R;
          rest /= R;
          std::swap(a, bb);
        }
        hipLaunchKernelGGL(k_batch_store_V, dim3(blocks), dim3(256), 0, s, a, (float2 *)b->d_arena, d_chunk, L, n);
        BHIP(hipGetLastError(), "V tables");
        BHIP(hipStreamSynchronize(s), "V tables");
      }
    }
    if (!ztjobs.empty()) {
      ScopedDev zt_buf;
      BHIP(dev_malloc((void **)&zt_buf.p, sizeof(ZoomTableJob) * ztjobs.size()), "zoom table jobs");
      ZoomTableJob *d_zt = (ZoomTableJob *)zt_buf.p;
      BHIP(hipMemcpy(d_zt, ztjobs.data(), sizeof(ZoomTableJob) * ztjobs.size(), hipMemcpyHostToDevice),
           "zoom table jobs");
      hipLaunchKernelGGL(k_batch_zoom_tables, dim3((unsigned)ztjobs.size()), dim3(256), 0, s,
                         (float2 *)b->d_arena, d_zt);
      BHIP(hipGetLastError(), "zoom tables");
      BHIP(hipStreamSynchronize(s), "zoom tables");
    }
  }

  // persistent grid per class: one workgroup per CU
  hipDeviceProp_t prop;
  BHIP(hipGetDeviceProperties(&prop, b->device), "device properties");
  b->grid = prop.multiProcessorCount;
  BHIP(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), "batch event");
  *out = b.release();
  return TZ_OK;
}

}  // extern "C"

namespace {

// the two events of the first launch's schedule timing, freed on every path
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair() = default;
  EventPair(const EventPair &) = delete;
  EventPair &operator=(const EventPair &) = delete;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

tz_status launch_batch(tz_batch *b, const void *x_flat, void *X_flat, hipStream_t s) {
  BatchTune cached;
  if (!b->tuned && tune_batch_lookup(b->sig, &cached)) {
    // a schedule this job table was tuned to before (this or an earlier process)
    b->topology = cached.topology;
    b->inner = cached.inner;
    b->units = order_units(*b, b->units, b->inner);
    tz_status st = upload_units(b, s);
    if (st) return st;
    st = build_graph(b, x_flat, X_flat);
    if (st) return st;
    b->tuned = true;
    b->tuned_from_cache = true;
    tz_log("batch autotune: schedule from the tune cache: topology %d, unit order %d", b->topology, b->inner);
  } else if (!b->tuned) {
    // first launch: time each candidate schedule on these buffers and keep
    // the fastest (every candidate computes the same outputs)
    const std::vector<BatchUnit> base = b->units;
    EventPair ev;
    BHIP(hipEventCreate(&ev.e0), "autotune events");
    BHIP(hipEventCreate(&ev.e1), "autotune events");
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    int best = 0;
    for (int cand = 0; cand < 8; ++cand) {
      b->topology = cand / 2;
      b->inner = cand % 2;
      b->units = order_units(*b, base, b->inner);
      tz_status st = upload_units(b, s);
      if (st) return st;
      st = build_graph(b, x_flat, X_flat);
      if (st) return st;
      BHIP(hipGraphLaunch(b->exec, s), "autotune launch");  // warm
      BHIP(hipEventRecord(e0, s), "autotune");
      BHIP(hipGraphLaunch(b->exec, s), "autotune launch");
      BHIP(hipEventRecord(e1, s), "autotune");
      BHIP(hipEventSynchronize(e1), "autotune");
      float ms = 0.f;
      BHIP(hipEventElapsedTime(&ms, e0, e1), "autotune");
      b->tuned_ms[cand] = ms;
      tz_log("batch autotune: topology %d, unit order %d: %.3f ms", b->topology, b->inner, ms);
      if (ms < b->tuned_ms[best]) best = cand;
    }
    b->topology = best / 2;
    b->inner = best % 2;
    b->units = order_units(*b, base, b->inner);
    tz_status st = upload_units(b, s);
    if (st) return st;
    st = build_graph(b, x_flat, X_flat);
    if (st) return st;
    b->tuned = true;
    BatchTune t;
    t.topology = b->topology;
    t.inner = b->inner;
    t.ms = b->tuned_ms[best];
    tune_batch_store(b->sig, t);
  } else if (x_flat != b->last_x || X_flat != b->last_X) {
    tz_status st = build_graph(b, x_flat, X_flat);
    if (st) return st;
  }
  BHIP(hipGraphLaunch(b->exec, s), "batch launch");
  BHIP(hipEventRecord(b->done, s), "batch launch");
  b->launched = true;
  return TZ_OK;
}

}  // namespace

extern "C" {

tz_status tz_batch_launch(tz_batch *b, const void *x_flat, void *X_flat, void *stream) {
  if (!b) return bfail(TZ_EINVAL, "batch is NULL");
  if (!x_flat || !X_flat) return bfail(TZ_EINVAL, "x_flat and X_flat must be device pointers");
  if (b->failed)
    return bfail(TZ_EDEVICE, "an earlier launch of this batch failed: destroy it and create a new one");
  const tz_status st = launch_batch(b, x_flat, X_flat, (hipStream_t)stream);
  if (st) b->failed = true;
  return st;
}

tz_status tz_batch_extents(const tz_batch *b, int64_t *x_elems, int64_t *X_elems) {
  if (!b || !x_elems || !X_elems) return bfail(TZ_EINVAL, "batch and both outputs must not be NULL");
  *x_elems = b->x_extent;
  *X_elems = b->X_extent;
  return TZ_OK;
}

tz_status tz_batch_wait(tz_batch *b, double timeout_ms) {
  if (!b) return bfail(TZ_EINVAL, "batch is NULL");
  if (!(timeout_ms >= 0.0)) return bfail(TZ_EINVAL, "timeout_ms must be >= 0");
  if (!b->launched) return TZ_OK;
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(b->done);
    if (e == hipSuccess) return TZ_OK;
    if (e != hipErrorNotReady) return bfail(TZ_EDEVICE, std::string("batch wait: ") + hipGetErrorString(e));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (ms >= timeout_ms) {
      char msg[160];
      snprintf(msg, sizeof msg, "the last launch of the batch had not finished after %.3f ms", ms);
      return bfail(TZ_ETIMEOUT, msg);
    }
    std::this_thread::sleep_for(std::chrono::microseconds(timeout_ms - ms > 1.0 ? 200 : 20));
  }
}

void tz_batch_destroy(tz_batch *b) { delete b; }

int64_t tz_batch_describe(const tz_batch *b, char *buf, int64_t len) {
  if (!b) return -1;
  std::string d = "jobs=" + std::to_string(b->n_jobs) + " items=" + std::to_string(b->items.size()) + " units:";
  for (int c = 8; c <= 14; ++c)
    if (b->cls_count[c]) d += " L" + std::to_string(1 << c) + "=" + std::to_string(b->cls_count[c]);
  static const char *names[8] = {"parallel/longest-first",   "parallel/creation-order",
                                 "chained/longest-first",    "chained/creation-order",
                                 "front-first/longest-first", "front-first/creation-order",
                                 "one-chain/longest-first",  "one-chain/creation-order"};
  if (b->tuned && b->tuned_from_cache) {
    d += std::string(" schedule=") + names[b->topology * 2 + b->inner] + " (tune cache)";
  } else if (b->tuned) {
    d += std::string(" schedule=") + names[b->topology * 2 + b->inner] + " candidates_ms:";
    for (int i = 0; i < 8; ++i) {
      char t[64];
      snprintf(t, sizeof t, " %s=%.3f", names[i], b->tuned_ms[i]);
      d += t;
    }
  } else {
    d += " schedule=untuned";
  }
  if (buf && len > 0) {
    const size_t n = std::min<size_t>((size_t)len - 1, d.size());
    memcpy(buf, d.data(), n);
    buf[n] = 0;
  }
  return (int64_t)d.size();
}

}  // extern "C"
