/*
 * FP64 CPU oracle for the three spectral estimators compared in
 * "Comparison of computing efficiency among FFT, CZT and Zoom FFT in THz-TDS"
 * (arXiv:2108.03948).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  It shares no code,
 * header, table or helper with the HIP library: every quantity below is
 * computed from the paper's definitions by plain direct summation in double
 * precision, one output bin at a time, so that each function can be checked
 * against the paper by eye.  Nothing here is blocked, fused or reordered.
 *
 * Conventions
 *   - complex values are interleaved (re, im) doubles;
 *   - x is a batch of B traces, trace b starting at x + b*xs (xs = element
 *     stride between traces); real traces unless stated otherwise;
 *   - every transform is evaluated only at the bins listed in `bins`
 *     (nbins of them), output laid out [B][nbins];
 *   - loops over (trace, bin) run under OpenMP; the sum over samples for one
 *     bin runs sequentially in sample order.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* e^{-j 2 pi r / q} for an integer residue 0 <= r < q: the angle is formed
 * from the exact residue, so no phase precision is lost to large products. */
static double complex unit_phase(int64_t r, int64_t q)
{
    double a = 2.0 * M_PI * ((double)r / (double)q);
    return cos(a) - I * sin(a);
}

/* ------------------------------------------------------------------------ */
/* Zero-padded FFT (Section 2.1, eqs. (2), (3), (5)).
 * X[k] = sum_{n<N} x[n] e^{-j 2 pi k n / Nfft},   Nfft = N + n_zeros.
 * Eq. (2) prints the kernel as W^{-kn} with W = e^{-j2pi/N}; we take the
 * forward transform, which is what the CZT special case of Section 2.3
 * (A = 1, W = e^{-j2pi/N}) reproduces.  Appending n_zeros zeros (the "x" of
 * eqs. (4)-(5)) only lengthens the transform; the sum over the zeros is zero
 * and is not taken.  Phase residue (k*n) mod Nfft is exact in int64.        */
void orc_fft_zeropad(const double *x, int64_t xs, int64_t B, int64_t N,
                     int64_t n_zeros, const int64_t *bins, int64_t nbins,
                     double *out)
{
    const int64_t nfft = N + n_zeros;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t i = 0; i < nbins; ++i) {
            const int64_t k = bins[i];
            const double *xb = x + b * xs;
            double complex acc = 0.0;
            for (int64_t n = 0; n < N; ++n) {
                int64_t r = (int64_t)(((__int128)k * n) % nfft);
                acc += xb[n] * unit_phase(r, nfft);
            }
            out[2 * (b * nbins + i)] = creal(acc);
            out[2 * (b * nbins + i) + 1] = cimag(acc);
        }
}

/* ------------------------------------------------------------------------ */
/* Chirp-Z transform (Section 2.3, eq. (11)).
 * X[k] = sum_{n<N} x[n] A^{-n} W^{k n},   k = 0 .. M-1.
 * A and W are arbitrary non-zero complex numbers (eqs. (16)-(17): A0, W0 may
 * differ from 1).  The integer powers are evaluated as exp(p * log z) with the
 * principal logarithm; for an integer power every branch gives the same value.
 * x may be real (x_complex = 0) or complex interleaved (x_complex = 1).     */
void orc_czt(const double *x, int x_complex, int64_t xs, int64_t B, int64_t N,
             double Wr, double Wi, double Ar, double Ai, const int64_t *bins,
             int64_t nbins, double *out)
{
    const double complex lW = clog(Wr + I * Wi);
    const double complex lA = clog(Ar + I * Ai);
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t i = 0; i < nbins; ++i) {
            const int64_t k = bins[i];
            double complex acc = 0.0;
            for (int64_t n = 0; n < N; ++n) {
                double complex xn;
                if (x_complex)
                    xn = x[2 * (b * xs + n)] + I * x[2 * (b * xs + n) + 1];
                else
                    xn = x[b * xs + n];
                double complex e = -(double)n * lA + (double)(k * n) * lW;
                acc += xn * cexp(e);
            }
            out[2 * (b * nbins + i)] = creal(acc);
            out[2 * (b * nbins + i) + 1] = cimag(acc);
        }
}

/* ------------------------------------------------------------------------ */
/* Inverse DFT: the IFFT that closes the FFT convolution of eq. (12), which
 * Section 4 also times on its own against the FFT:
 *   x[n] = (1/N) sum_{k<N} X[k] e^{+j 2 pi k n / N},   n = 0 .. N-1.
 * X is complex interleaved, B rows of N (row b at complex element b*xs);
 * only the samples listed in `samples` are formed.  e^{+j 2 pi r/N} is
 * e^{-j 2 pi (N - r)/N}: the residue of -(k n) mod N is exact in int64.     */
void orc_ifft(const double *X, int64_t xs, int64_t B, int64_t N,
              const int64_t *samples, int64_t ns, double *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t i = 0; i < ns; ++i) {
            const int64_t n = samples[i];
            double complex acc = 0.0;
            for (int64_t k = 0; k < N; ++k) {
                const int64_t r = (int64_t)(((__int128)k * n) % N);
                const double complex Xk = X[2 * (b * xs + k)] + I * X[2 * (b * xs + k) + 1];
                acc += Xk * unit_phase((N - r) % N, N);
            }
            acc /= (double)N;
            out[2 * (b * ns + i)] = creal(acc);
            out[2 * (b * ns + i) + 1] = cimag(acc);
        }
}

/* CZT over a band given in integer hertz (eqs. (22)-(24)):
 * A = e^{j 2 pi f1/fs}, W = e^{-j 2 pi (f2-f1)/(M fs)}, so bin k sits at
 * f1 + k (f2 - f1)/M and   X[k] = sum_n x[n] e^{-j 2 pi (f1 + k(f2-f1)/M) n / fs}.
 * The phase numerator (M f1 + k (f2-f1)) n is reduced modulo M fs exactly in
 * 128-bit integers before the angle is formed.                              */
void orc_czt_band_exact(const double *x, int64_t xs, int64_t B, int64_t N,
                        int64_t M, int64_t fs_hz, int64_t f1_hz, int64_t f2_hz,
                        const int64_t *bins, int64_t nbins, double *out)
{
    const __int128 q = (__int128)M * fs_hz;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t i = 0; i < nbins; ++i) {
            const int64_t k = bins[i];
            const __int128 num = (__int128)M * f1_hz + (__int128)k * (f2_hz - f1_hz);
            double complex acc = 0.0;
            for (int64_t n = 0; n < N; ++n) {
                __int128 r = (num * n) % q;
                if (r < 0) r += q;
                double a = 2.0 * M_PI * ((double)r / (double)q);
                acc += x[b * xs + n] * (cos(a) - I * sin(a));
            }
            out[2 * (b * nbins + i)] = creal(acc);
            out[2 * (b * nbins + i) + 1] = cimag(acc);
        }
}

/* ------------------------------------------------------------------------ */
/* Zoom FFT (Section 2.2), one step per function, in the paper's order.      */

/* Low-pass taps standing in for the ideal filter of eq. (8): a Hamming
 * windowed sinc with cut-off nu_c = f_c / f_s (cycles per sample),
 *   h[t] = w[t] * 2 nu_c * sinc(2 nu_c (t - (T-1)/2)),
 *   w[t] = 0.54 - 0.46 cos(2 pi t / (T-1)),  sinc(u) = sin(pi u)/(pi u),
 * then scaled so that sum h = 1 (pass-band gain C = 1).  T = 1 gives h = [1]. */
void orc_zoom_taps(int64_t T, double nu_c, double *h)
{
    if (T == 1) {
        h[0] = 1.0;
        return;
    }
    double s = 0.0;
    for (int64_t t = 0; t < T; ++t) {
        double c = (double)t - 0.5 * (double)(T - 1);
        double u = 2.0 * nu_c * c;
        double sinc = (u == 0.0) ? 1.0 : sin(M_PI * u) / (M_PI * u);
        double w = 0.54 - 0.46 * cos(2.0 * M_PI * (double)t / (double)(T - 1));
        h[t] = w * 2.0 * nu_c * sinc;
        s += h[t];
    }
    for (int64_t t = 0; t < T; ++t) h[t] /= s;
}

/* Steps 1-3 of the zoom (eqs. (6), (7), (10)):
 *   f_N = (f1 + f2)/2                                  (centre of the band)
 *   y[n] = x[n] e^{-j 2 pi f_N n / f_s}                (shift f_N to DC)
 *   u[m] = sum_{t<T} h[t] y[mD - t],  y = 0 outside [0, N),  m < ceil(N/D).
 * Eq. (7) is printed without the sample index and 2 pi; the shift that moves
 * f_N to DC is the one taken.  Eq. (10) prints the tap sum up to N-1; the sum
 * runs over the T filter taps.  u is written to u_out as [B][ceil(N/D)]
 * complex.  x is real, or interleaved complex when x_complex != 0 (xs then
 * counts complex samples): the later axes of a multi-dimensional zoom.      */
void orc_zoom_frontend(const double *x, int x_complex, int64_t xs, int64_t B, int64_t N,
                       double fs, double f1, double f2, int64_t D,
                       const double *h, int64_t T, double *u_out)
{
    const double fN = 0.5 * (f1 + f2);
    const int64_t LD = (N + D - 1) / D;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < B; ++b) {
        const double *xb = x + b * xs * (x_complex ? 2 : 1);
        double complex *y = (double complex *)malloc(sizeof(double complex) * (size_t)N);
        for (int64_t n = 0; n < N; ++n) {
            const double complex xn = x_complex ? xb[2 * n] + I * xb[2 * n + 1] : xb[n];
            /* angle 2 pi f_N n / f_s, with the integer part of f_N n / f_s
             * removed first (fmod is exact) */
            double cyc = fmod(fN * (double)n / fs, 1.0);
            double a = 2.0 * M_PI * cyc;
            y[n] = xn * (cos(a) - I * sin(a));
        }
        for (int64_t m = 0; m < LD; ++m) {
            double complex acc = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                int64_t n = m * D - t;
                if (n >= 0 && n < N) acc += h[t] * y[n];
            }
            u_out[2 * (b * LD + m)] = creal(acc);
            u_out[2 * (b * LD + m) + 1] = cimag(acc);
        }
        free(y);
    }
}

/* Step 4 of the zoom: the short DFT of the decimated sequence (P. 2.2, the
 * "much shorter FFT", and its cost model).  With K points over the decimated
 * rate f_s/D, the M output bins are centred on f_N:
 *   X[k] = sum_{m<LD} u[m] e^{-j 2 pi (k - floor(M/2)) m / K},  k < M,
 * i.e. bin k sits at f_N + (k - floor(M/2)) f_s / (D K).  The residue
 * ((k - floor(M/2)) m) mod K is exact.                                      */
void orc_zoom_short_dft(const double *u, int64_t B, int64_t LD, int64_t K,
                        int64_t M, const int64_t *bins, int64_t nbins,
                        double *out)
{
    const int64_t half = M / 2;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b)
        for (int64_t i = 0; i < nbins; ++i) {
            const int64_t k = bins[i];
            double complex acc = 0.0;
            for (int64_t m = 0; m < LD; ++m) {
                int64_t r = ((k - half) * m) % K;
                if (r < 0) r += K;
                double complex um = u[2 * (b * LD + m)] + I * u[2 * (b * LD + m) + 1];
                acc += um * unit_phase(r, K);
            }
            out[2 * (b * nbins + i)] = creal(acc);
            out[2 * (b * nbins + i) + 1] = cimag(acc);
        }
}

/* Short-DFT length: the zoom keeps the CZT's bin spacing (f2 - f1)/M
 * (eq. (24)) at the decimated rate f_s/D, so K = round(M f_s / (D (f2-f1))),
 * rounded half away from zero.                                              */
int64_t orc_zoom_K(double fs, double f1, double f2, int64_t M, int64_t D)
{
    return (int64_t)llround((double)M * fs / ((double)D * (f2 - f1)));
}
