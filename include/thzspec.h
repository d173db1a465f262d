/*
 * thzspec — batched spectra of sampled THz-TDS traces on MI355X (gfx950):
 * zero-padded FFT, chirp-Z transform (Bluestein form) and Zoom FFT, as
 * defined in "Comparison of computing efficiency among FFT, CZT and Zoom FFT
 * in THz-TDS" (arXiv:2108.03948).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Traces are real samples x[n] = x(n T_s), n < N (Section 2.1, eq. (1)),
 *   one trace per row: trace b starts at element b * in_stride of x.
 *   Element type is float (TZ_F32, default) or double (TZ_F64).
 * - Spectra are written as interleaved complex float (re, im), one row per
 *   trace: row b starts at complex element b * out_stride of X.
 * - x and X are DEVICE pointers (HIP global memory, e.g. a torch tensor's
 *   data_ptr()).  The caller owns them; they must not overlap.  The library
 *   never copies traces or spectra to or from the host.
 * - Transforms are forward and unscaled (a plain sum over n, no 1/N), as in
 *   eqs. (2) and (11); the one exception is ifft(), the inverse DFT of
 *   complex spectra with its 1/N.
 * - Work is enqueued on opts->stream (a hipStream_t; NULL = the null stream)
 *   and returns before it finishes.  The first call with a new shape builds
 *   a plan (device tables, see below) and may allocate and synchronise that
 *   stream; later calls with the same shape reuse it and allocate nothing.
 * - Every call returns a tz_status.  On TZ_EINVAL / TZ_EUNSUPPORTED nothing
 *   is launched and X is untouched; tz_last_error() (thread-local) says why.
 *   TZ_EDEVICE reports a HIP error from an allocation or a launch.
 * - Plans (chirp tables, filter spectrum, twiddles, FIR taps) are owned by
 *   the library, cached per device, and freed by tz_release_plans() or at
 *   process exit.  All entry points are thread-safe.
 */
#ifndef THZSPEC_H
#define THZSPEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Complex parameter in double precision. */
typedef struct {
    double re, im;
} tz_c64;

typedef enum {
    TZ_OK = 0,
    TZ_EINVAL = 1,        /* an argument is out of range (nothing launched) */
    TZ_ENOMEM = 2,        /* a plan table could not be allocated            */
    TZ_EDEVICE = 3,       /* a HIP call failed                              */
    TZ_EUNSUPPORTED = 4,  /* valid arguments outside what the GPU path does */
    TZ_ETIMEOUT = 5       /* a bounded wait ended before the work was done  */
} tz_status;

/* input element type */
enum { TZ_F32 = 0, TZ_F64 = 1 };
/* arithmetic of the FFT stages.  TZ_SPLIT_FP16 / TZ_SPLIT_BF16 run the
 * radix-16 passes of czt() / czt_band_exact() on the matrix cores as dense
 * 16-point DFT-matrix products with operands split into high and low 16-bit
 * parts and FP32 accumulation: single-pass plans of FFT length 4096, 8192 or
 * 16384 with one bin block and real input, and four-step plans (N + M - 1 up
 * to 2^24) whose row FFTs have length 1024, 2048, 4096, 8192 or 16384 (there
 * BF16 splits each operand into three parts); the four-step column FFTs,
 * chirps and twiddles stay FP32.  zoom_fft() takes them for its short DFT
 * when that runs on the four-step path (its front end is FP64 either way).
 * Other shapes and the other transforms return TZ_EUNSUPPORTED.  TZ_FP64 evaluates czt() (one-shot or plan) by direct
 * summation of eq. (11) in FP64, X[k] = sum_n x[n] (A^{-1} W^k)^n, and
 * writes complex128 bins (X rows of M pairs of doubles, out_stride complex
 * elements apart): O(N M) work per trace, for any contour whose terms FP64
 * can hold (|ln| of every term's magnitude below 700), including the
 * spirals of eqs. (16)-(17) too steep for the FP32 tables; the other
 * transforms return TZ_EUNSUPPORTED for it. */
enum { TZ_FP32 = 0, TZ_SPLIT_FP16 = 1, TZ_SPLIT_BF16 = 2, TZ_FP64 = 3 };
/* flags */
enum {
    TZ_HALF = 1  /* fft_zeropad: write bins 0 .. N_fft/2 only (real input);
                    ifft: Hermitian half spectra in, real traces out */
};
/* job kinds for the uneven batch */
enum { TZ_JOB_CZT = 0, TZ_JOB_ZOOM = 1 };

typedef struct {
    int64_t batch;          /* B, number of traces (>= 1; 0 means 1)          */
    int64_t in_stride;      /* elements between trace starts (0 means N)      */
    int64_t out_stride;     /* complex elements between spectrum rows
                               (0 means the number of bins written)           */
    int32_t in_dtype;       /* TZ_F32 or TZ_F64                               */
    int32_t precision;      /* TZ_FP32, TZ_SPLIT_FP16, TZ_SPLIT_BF16, TZ_FP64 */
    int32_t flags;          /* TZ_HALF                                        */
    int32_t fir_taps;       /* zoom_fft low-pass length T (0 means 63)        */
    double fir_cutoff_hz;   /* zoom_fft cut-off f_c (0 means f_s / (2 D))     */
    void *stream;           /* hipStream_t, NULL = null stream                */
} tz_opts;

/* Fill *o with the defaults listed above. */
void tz_opts_init(tz_opts *o);

/*
 * Zero-padded FFT (Section 2.1, eqs. (2), (3) and (5)).
 *   X[k] = sum_{n<N} x[n] exp(-j 2 pi k n / N_fft),  N_fft = N + n_zeros,
 *   k = 0 .. N_fft - 1 (or 0 .. N_fft/2 with TZ_HALF).
 * n_zeros is the number of zeros appended to the trace (the "x" of eq. (5));
 * bin k sits at k f_s / N_fft (eq. (3)).
 * Errors: TZ_EINVAL if x or X is NULL, N < 1, n_zeros < 0, a stride is too
 * small, or N_fft exceeds 2^31 - 1.
 */
tz_status fft_zeropad(const void *x, int64_t N, int64_t n_zeros, void *X,
                      const tz_opts *opts);

/*
 * Chirp-Z transform (Section 2.3, eq. (11)), evaluated in Bluestein form
 * (eqs. (12)-(15)): chirp premultiply, convolution with the conjugate chirp
 * through FFT / pointwise product / inverse FFT, chirp postmultiply.
 *   X[k] = sum_{n<N} x[n] A^{-n} W^{k n},  k = 0 .. M-1.
 * A = A0 e^{j theta0} is the start point and W = W0 e^{-j phi0} the ratio
 * between contour points (eqs. (16)-(17)).  Off the unit circle (spirals,
 * A0 or W0 != 1) the chirp tables carry the magnitudes A0^{-n} W0^{n^2/2} and
 * W0^{-m^2/2}, computed in FP64 and rescaled by their exact maxima so that no
 * FFT operand exceeds |x|.  Because FP32 FFT rounding follows the largest
 * operands, the GPU path takes spirals whose two magnitude profiles together
 * span at most e^6 over the transform (relative L2 error then stays within
 * the FP32 bar), with N + M - 1 within one FFT pair (no bin blocks), in
 * TZ_FP32 only; steeper spirals return TZ_EUNSUPPORTED.
 * Errors: TZ_EINVAL for NULL pointers, N < 1, M < 1, zero or non-finite
 * A or W.
 */
tz_status czt(const void *x, int64_t N, int64_t M, tz_c64 W, tz_c64 A, void *X,
              const tz_opts *opts);

/*
 * CZT over the band [f1, f2) with M bins and rational phases: f_s, f1 and f2
 * in whole hertz.  Equivalent to czt() with A = e^{j 2 pi f1/f_s} and
 * W = e^{-j 2 pi (f2 - f1)/(M f_s)} (eqs. (22)-(23)); bin k sits at
 * f1 + k (f2 - f1)/M (eq. (24)).  The chirp phase of sample n is reduced as
 * an exact integer residue before any sine or cosine is taken.
 * Errors: TZ_EINVAL for NULL pointers, N < 1, M < 1, f_s < 1, f1 < 0,
 * f2 <= f1.
 */
tz_status czt_band_exact(const void *x, int64_t N, int64_t M, int64_t fs_hz,
                         int64_t f1_hz, int64_t f2_hz, void *X, const tz_opts *opts);

/*
 * Zoom FFT (Section 2.2, eqs. (6)-(10)).
 *   f_N = (f1 + f2)/2;  y[n] = x[n] e^{-j 2 pi f_N n / f_s};
 *   u[m] = sum_{t<T} h[t] y[mD - t],  m < ceil(N/D)   (y = 0 outside [0,N));
 *   K = round(M f_s / (D (f2 - f1)))  (half away from zero);
 *   X[k] = sum_m u[m] exp(-j 2 pi (k - floor(M/2)) m / K),  k < M.
 * h is a T-tap Hamming-windowed sinc with cut-off f_c, normalised to unit
 * DC gain (it stands in for the ideal low-pass of eq. (8)).  Bin k sits at
 * f_N + (k - floor(M/2)) f_s / (D K).
 * Errors: TZ_EINVAL for NULL pointers, N < 1, M < 1, D < 1, T < 1,
 * non-finite or non-positive f_s, f2 <= f1, f_c <= 0, K < 1.
 */
tz_status zoom_fft(const void *x, int64_t N, double fs, double f1, double f2,
                   int64_t M, int64_t D, void *X, const tz_opts *opts);

/*
 * Frequency response of sample/reference pairs (Section 1: the response of
 * the material under test is derived by comparing the sample trace with the
 * reference trace), on the CZT contour of czt() (eq. (11)):
 *   H[p][k] = X_s[k] / X_r[k],  X_r = CZT of row 2p, X_s = CZT of row 2p+1,
 *   k < M, p < B/2, with B = opts->batch traces (even; TZ_EINVAL otherwise).
 * Row p of H starts at complex element p * out_stride (0 means M).  Both CZTs
 * of a pair run in one workgroup and only H is written; the postmultiply of
 * eq. (13) cancels in the ratio.  A bin where X_r is exactly 0 gives IEEE
 * inf / nan.  Single-pass shapes only (N + M - 1 <= 16384, FP32 input f32 or
 * f64, TZ_FP32); other shapes return TZ_EUNSUPPORTED.  Errors otherwise as
 * czt().
 */
tz_status czt_transfer(const void *x, int64_t N, int64_t M, tz_c64 W, tz_c64 A, void *H,
                       const tz_opts *opts);

/*
 * Inverse DFT of complex spectra: the IFFT of the Bluestein convolution
 * (eq. (12)) as a transform of its own, which Section 4 times against the
 * FFT over the same resolutions:
 *   x[n] = (1/N) sum_{k<N} X[k] exp(+j 2 pi k n / N),  n = 0 .. N-1.
 * X: B = opts->batch rows of N complex64 (interleaved float re, im), row b
 * at complex element b * in_stride (0 means N); x: B rows of N complex64,
 * out_stride complex elements apart (0 means N).  Both are device memory
 * owned by the caller; X is only read.  Power-of-two N from 256 to 16384
 * run as one FFT per row (conjugate, forward FFT, conjugate, exact 1/N);
 * other 7-smooth N from 8 to 20480 as one mixed-radix FFT per row; any
 * other N with 2N - 1 <= 2^24 as the CZT of eq. (11) with A = 1,
 * W = e^{+j 2 pi / N} and exact integer chirp phases, the 1/N folded into
 * the plan's chirp spectrum.
 * With TZ_HALF in opts->flags, X holds the Hermitian half spectra of real
 * traces (the output of fft_zeropad with TZ_HALF): rows of N/2 + 1 complex64
 * bins 0 .. N/2 (in_stride 0 means N/2 + 1), bin k > N/2 being
 * conj(X[N - k]) and the imaginary parts of bin 0 and, for even N, bin N/2
 * taken as 0; x receives B real rows of N float32 samples (out_stride float
 * elements apart, 0 means N).  Two rows go through one complex mixed-radix
 * FFT (x_a = Re, x_b = Im of the inverse of X_a + j X_b); N must be 7-smooth
 * from 8 to 20480.
 * in_dtype must be TZ_F32 (the components of complex64).
 * Errors: TZ_EINVAL for NULL pointers, N < 1, strides below the row
 * lengths, in_dtype TZ_F64; TZ_EUNSUPPORTED for split precision,
 * 2N - 1 > 2^24, or TZ_HALF with N outside the 7-smooth range above.
 */
tz_status ifft(const void *X, int64_t N, void *x, const tz_opts *opts);

/* ---------------------------------------------------------------------- */
/* Multi-dimensional transforms (the 2-D and 3-D case Section 5 names as
 * the setting where CZT and Zoom FFT pay off).  x holds B = opts->batch
 * arrays x[N_0][N_1]...[N_{d-1}] (last index contiguous), consecutive arrays
 * opts->in_stride elements apart (0 means N_0 ... N_{d-1}); X receives
 * X[M_0]...[M_{d-1}] complex64 per array, opts->out_stride complex elements
 * apart (0 means M_0 ... M_{d-1}).  Input TZ_F32 or TZ_F64, arithmetic
 * TZ_FP32 only.  The transforms are separable: the one-dimensional
 * transform of each axis is applied along that axis in turn (the axis
 * parameters, one entry per dimension, describe axis 0 first).  Scratch:
 * two buffers of the largest intermediate, held per stream by the library
 * until tz_release_plans().                                               */
#define TZ_MAX_DIMS 3

/* One axis of czt_nd: N samples in, M bins out on the contour A W^-k. */
typedef struct {
    int64_t N, M;
    tz_c64 W, A;
} tz_czt_axis;

/*
 * d-dimensional CZT, 1 <= ndim <= TZ_MAX_DIMS:
 *   X[k_0..k_{d-1}] = sum_n x[n_0..n_{d-1}] prod_a A_a^{-n_a} W_a^{k_a n_a}
 * (eq. (11) along every axis).  Each axis accepts what czt() accepts
 * (spirals included).
 * Errors: TZ_EINVAL for NULL pointers, ndim out of range, N_a < 1, M_a < 1,
 * zero or non-finite A_a or W_a, strides below the array sizes;
 * TZ_EUNSUPPORTED for split precision and for an axis czt() refuses.
 */
tz_status czt_nd(const void *x, int ndim, const tz_czt_axis *axes, void *X,
                 const tz_opts *opts);

/* One axis of zoom_fft_nd: the arguments of zoom_fft() for that axis, and
 * its low-pass cut-off fc in hertz (0 means f_s / (2 D)). */
typedef struct {
    int64_t N, M, D;
    double fs, f1, f2, fc;
} tz_zoom_axis;

/*
 * d-dimensional Zoom FFT, 1 <= ndim <= TZ_MAX_DIMS: the Zoom FFT of
 * zoom_fft() (mix, T-tap low-pass, decimation by D_a, K_a-point short DFT on
 * M_a bins centred on the band) applied along every axis; opts->fir_taps
 * gives T for all axes and opts->fir_cutoff_hz must be 0 (cut-offs are per
 * axis).
 * Errors: TZ_EINVAL as zoom_fft() for any axis, NULL pointers, ndim out of
 * range, a non-zero fir_cutoff_hz; TZ_EUNSUPPORTED for split precision.
 */
tz_status zoom_fft_nd(const void *x, int ndim, const tz_zoom_axis *axes, void *X,
                      const tz_opts *opts);

/* ---------------------------------------------------------------------- */
/* Host-only helpers (pure functions, no device work).                     */

/* W and A for M bins over [f1, f2) at rate f_s, eqs. (22)-(23).
 * TZ_EINVAL if W or A is NULL, M < 1, f_s <= 0 or f2 <= f1. */
tz_status czt_band(double fs, double f1, double f2, int64_t M, tz_c64 *W, tz_c64 *A);

/* Zeros to append to an N_fft-point transform so that its bin spacing
 * shrinks by delta (eqs. (4)-(5)): the smallest integer count z with
 * f_s/N_fft - f_s/(N_fft + z) >= delta.  -1 if delta <= 0, N_fft < 1 or
 * delta >= f_s/N_fft (no finite count reaches it). */
int64_t fft_zero_count(double fs, int64_t N_fft, double delta);

/* CZT points giving the bin spacing of an N_fft-point FFT over [f1, f2)
 * (eq. (25)), rounded to the nearest integer; -1 on invalid input. */
int64_t czt_points_for_resolution(double fs, double f1, double f2, int64_t N_fft);

/* Short-DFT length K of the Zoom FFT (see zoom_fft); -1 on invalid input. */
int64_t zoom_short_length(double fs, double f1, double f2, int64_t M, int64_t D);

/* Device FFT length L the CZT path uses for N samples and M bins per block,
 * and the number of bin blocks (M is split into blocks when N + M - 1
 * exceeds the largest single-pass length).  TZ_EUNSUPPORTED if N is too long
 * for the single-pass path. */
tz_status czt_plan_shape(int64_t N, int64_t M, int64_t *L, int64_t *blocks);

/* ---------------------------------------------------------------------- */
/* Uneven batch: many traces of different length, band, M and method in   */
/* one launch (one persistent kernel, captured once in a hipGraph).        */

typedef struct {
    int32_t kind;        /* TZ_JOB_CZT or TZ_JOB_ZOOM                         */
    int32_t fir_taps;    /* zoom only (0 means 63)                            */
    int64_t N;           /* samples of this trace                             */
    int64_t M;           /* output bins                                       */
    int64_t D;           /* zoom decimation (ignored for CZT)                 */
    int64_t fs_hz;       /* sampling rate, whole hertz                        */
    int64_t f1_hz;       /* band start, whole hertz                           */
    int64_t f2_hz;       /* band end (exclusive), whole hertz                 */
    int64_t in_offset;   /* first sample of this trace in x_flat (elements)   */
    int64_t out_offset;  /* first bin of this spectrum in X_flat (complex)    */
} tz_job;

typedef struct tz_batch tz_batch;

/* Build device tables for every job, order the jobs longest-first and
 * record the launch in a hipGraph on opts->stream.  x_flat holds float
 * samples; X_flat complex float bins.  TZ_EINVAL for an invalid job (its
 * index is in tz_last_error()). */
tz_status tz_batch_create(const tz_job *jobs, int64_t n_jobs, const tz_opts *opts,
                          tz_batch **batch);
/* Run the batch on device buffers x_flat / X_flat (asynchronous on stream).
 * Once a launch has returned an error (TZ_EDEVICE: a HIP call or the graph
 * build failed), every later launch of the same batch returns TZ_EDEVICE
 * without touching the device: destroy the batch and create a new one. */
tz_status tz_batch_launch(tz_batch *batch, const void *x_flat, void *X_flat, void *stream);
/* Free the batch (synchronises the device first). */
void tz_batch_destroy(tz_batch *batch);
/* Elements of x_flat (floats) and X_flat (complex floats) the jobs reach:
 * max(in_offset + N) and max(out_offset + M) over the jobs.  tz_batch_launch
 * reads and writes exactly these ranges; buffers must hold at least that
 * many elements (the launch itself takes bare pointers and cannot check).
 * TZ_EINVAL for a NULL argument. */
tz_status tz_batch_extents(const tz_batch *batch, int64_t *x_elems, int64_t *X_elems);
/* Host-side bounded wait for the batch's last launch (a watchdog for the
 * persistent kernels): polls its completion for at most timeout_ms
 * milliseconds.  TZ_OK once it has finished (or if the batch was never
 * launched), TZ_ETIMEOUT if it is still running when the time is up (the
 * work itself continues and a later wait may succeed), TZ_EDEVICE if the
 * device reported an error, TZ_EINVAL for a NULL batch or a negative or NaN
 * timeout.  The kernels of a batch always terminate: every persistent
 * workgroup leaves when the shared work counter passes the last unit. */
tz_status tz_batch_wait(tz_batch *batch, double timeout_ms);
/* Write a one-line description of the batch into buf (NUL-terminated, at
 * most len bytes): jobs, work units per FFT length, and the schedule the
 * autotuner picked at the first launch with the time of every candidate.
 * Returns the length of the full description. */
int64_t tz_batch_describe(const tz_batch *batch, char *buf, int64_t len);

/* ---------------------------------------------------------------------- */
/* Explicit plans.  tz_plan_create() resolves everything one transform of  */
/* one shape needs (the chirp tables and filter spectrum of eqs. (13)-(15), */
/* FFT twiddles, FIR taps and mixing phasors of eqs. (6)-(10)) and builds   */
/* it on opts->stream, synchronising that stream.  tz_plan_execute() then   */
/* only enqueues kernels: it allocates no device memory and does not        */
/* synchronise, so it may be called inside HIP stream capture or a tight    */
/* serving loop.  Scratch memory (the four-step path's intermediates, the  */
/* Zoom FFT's decimated rows) is a caller-owned workspace of at least       */
/* tz_plan_workspace() bytes.                                               */

enum {
    TZ_PLAN_FFT_ZEROPAD = 0, TZ_PLAN_CZT = 1, TZ_PLAN_CZT_BAND_EXACT = 2, TZ_PLAN_ZOOM = 3,
    TZ_PLAN_IFFT = 4  /* ifft(): N complex64 in, N complex64 out */
};

typedef struct {
    int32_t kind;                 /* TZ_PLAN_*                                  */
    int64_t N;                    /* samples per trace (eq. (1)); ifft: points  */
    int64_t M;                    /* bins: czt, czt_band_exact, zoom            */
    int64_t n_zeros;              /* fft_zeropad: zeros appended (eq. (5))      */
    tz_c64 W, A;                  /* czt: contour A W^-k (eqs. (16)-(17))       */
    int64_t fs_hz, f1_hz, f2_hz;  /* czt_band_exact: integer-hertz band         */
    double fs, f1, f2;            /* zoom: band (Hz); fs also sets the bin      */
                                  /* frequencies of fft_zeropad and czt         */
    int64_t D;                    /* zoom decimation (eq. (9))                  */
} tz_plan_params;

typedef struct tz_plan tz_plan;

/* Build a plan for params with opts (batch, strides, in_dtype, precision,
 * flags, fir_taps, fir_cutoff_hz as in the one-shot calls; NULL = defaults).
 * The same argument checks and errors as fft_zeropad / czt /
 * czt_band_exact / zoom_fft / ifft; TZ_EINVAL for an unknown kind.  The plan owns
 * its tables (tz_release_plans() does not free them). */
tz_status tz_plan_create(const tz_plan_params *params, const tz_opts *opts, tz_plan **plan);
/* Bytes of workspace tz_plan_execute() needs (0 for most shapes). */
tz_status tz_plan_workspace(const tz_plan *plan, size_t *bytes);
/* Run the plan on device buffers x -> X (layouts as the one-shot call with
 * the plan's opts) with workspace (device memory of at least
 * tz_plan_workspace() bytes, or NULL when that is 0), asynchronously on
 * stream (NULL = the null stream).  Allocates nothing.  TZ_EINVAL for NULL
 * buffers, a missing workspace, or a current device other than the one the
 * plan was built on.  Executions that share a workspace must be ordered on
 * one stream; a plan itself is read-only and may run on several streams
 * with separate workspaces. */
tz_status tz_plan_execute(const tz_plan *plan, const void *x, void *X, void *workspace, void *stream);
/* Free the plan (synchronises the device first). */
void tz_plan_destroy(tz_plan *plan);

/* Bytes of the library's fixed device scratch array (one per GPU). */
#define TZ_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * tz_plan_execute() without a workspace argument, for callers that cannot
 * allocate device memory themselves (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the workspace is a fixed
 * array of TZ_STATIC_SCRATCH_BYTES inside this library, one copy per GPU,
 * held until the process ends.  Same outputs as tz_plan_execute(); the call
 * allocates nothing (the first call on a device looks up that device's copy
 * of the array).  The four-step path runs as many traces per chunk as fit
 * the array.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents: calls whose executions overlap on one GPU (different
 * streams, not ordered) race on it and give wrong results; order them on one
 * stream.  TZ_EINVAL, with nothing launched, for NULL buffers, a current
 * device other than the plan's, or a plan whose workspace cannot fit the
 * array (a Zoom FFT whose decimated rows, B ceil(N/D) complex64, exceed it,
 * or a four-step trace of more than TZ_STATIC_SCRATCH_BYTES / 8 points).
 */
tz_status tz_plan_execute_static(const tz_plan *plan, const void *x, void *X, void *stream);
/* Frequency in hertz of every output bin of params (host only, no device
 * work): fft_zeropad k fs / N_fft (eq. (3)), k < N_fft or N_fft/2 + 1 with
 * TZ_HALF in opts->flags; czt fs (nu_A + k nu_W) for A = e^{j 2 pi nu_A},
 * W = e^{-j 2 pi nu_W} (eqs. (16)-(17)); czt_band_exact f1 + k (f2 - f1)/M
 * (eq. (24)); zoom f_N + (k - floor(M/2)) fs / (D K) with f_N = (f1 + f2)/2
 * and K = zoom_short_length().  f_out holds one double per bin.  TZ_EINVAL
 * for TZ_PLAN_IFFT, whose outputs are time samples. */
tz_status tz_bin_freqs(const tz_plan_params *params, const tz_opts *opts, double *f_out);

/* ---------------------------------------------------------------------- */
/* Autotuner.  tz_autotune() times one Bluestein FFT pair (eq. (15)) of    */
/* every single-workgroup length 256 .. 16384 on the current device, on    */
/* opts->stream (synchronising it), and makes plans created afterwards     */
/* choose their FFT length and bin blocks from those times instead of the  */
/* built-in cost table (any FFT length >= N + M - 1 gives the same bins,   */
/* so only speed changes).  It allocates about 200 MB of device memory     */
/* while it runs and drops the one-shot calls' cached plans; explicit      */
/* plans keep their shape.  The uneven batch times its candidate schedules */
/* at its first launch (tz_batch_launch).  Both results persist in a JSON  */
/* file named by the environment variable TZ_TUNE_CACHE (default           */
/* $XDG_CACHE_HOME/thzspec/tune.json, else $HOME/.cache/thzspec/tune.json; */
/* "off" or an empty value disables reading and writing it), under the key */
/* "<device architecture name>/<tz_version()>": a later process on the     */
/* same architecture and library starts from them.  Entries under another  */
/* key are kept but not used; a file that does not parse is ignored (the  */
/* built-in defaults apply) and rewritten at the next save.  A file that   */
/* cannot be written leaves the results in memory for this process only.   */
/* Errors: TZ_EDEVICE / TZ_ENOMEM from the timing runs.                    */
tz_status tz_autotune(const tz_opts *opts);
/* One-line description of the tuning state: cache path and what loading   */
/* or saving it did, the device key, the FFT-pair times in use (measured   */
/* or built-in) and how many batch schedules are stored for this device.   */
/* Writes at most len bytes (NUL-terminated) and returns the full length;  */
/* needs no device (then device=none and the built-in costs).              */
int64_t tz_tune_describe(char *buf, int64_t len);

/* ---------------------------------------------------------------------- */
const char *tz_last_error(void);   /* thread-local message of the last failure */
const char *tz_version(void);
void tz_release_plans(void);       /* free every cached plan (synchronises)    */

#ifdef __cplusplus
}
#endif
#endif /* THZSPEC_H */
