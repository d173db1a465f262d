/*
 * Sanitizer driver for the FP64 oracle (oracle/oracle.c), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
 * Every buffer is allocated at exactly the size the oracle's contract states
 * (B rows of xs elements, B x nbins outputs), so a read or write past any of
 * them is reported; edge cases cover N = 1, M = 1, one bin, strided rows,
 * complex input, T = 1 and D > N.  Exit status 0 when every result is finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_fft_zeropad(const double *x, int64_t xs, int64_t B, int64_t N, int64_t n_zeros, const int64_t *bins,
                     int64_t nbins, double *out);
void orc_czt(const double *x, int x_complex, int64_t xs, int64_t B, int64_t N, double Wr, double Wi, double Ar,
             double Ai, const int64_t *bins, int64_t nbins, double *out);
void orc_ifft(const double *X, int64_t xs, int64_t B, int64_t N, const int64_t *samples, int64_t ns, double *out);
void orc_czt_band_exact(const double *x, int64_t xs, int64_t B, int64_t N, int64_t M, int64_t fs_hz,
                        int64_t f1_hz, int64_t f2_hz, const int64_t *bins, int64_t nbins, double *out);
void orc_zoom_taps(int64_t T, double nu_c, double *h);
void orc_zoom_frontend(const double *x, int x_complex, int64_t xs, int64_t B, int64_t N, double fs, double f1,
                       double f2, int64_t D, const double *h, int64_t T, double *u_out);
void orc_zoom_short_dft(const double *u, int64_t B, int64_t LD, int64_t K, int64_t M, const int64_t *bins,
                        int64_t nbins, double *out);
int64_t orc_zoom_K(double fs, double f1, double f2, int64_t M, int64_t D);

static int bad = 0;

static double *rnd(int64_t n, unsigned *seed) {
    double *p = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        *seed = *seed * 1103515245u + 12345u;
        p[i] = ((double)(*seed >> 8) / 16777216.0) - 0.5;
    }
    return p;
}

static int64_t *all_bins(int64_t n) {
    int64_t *b = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) b[i] = i;
    return b;
}

static void check_finite(const char *what, const double *v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "%s: non-finite value at %lld\n", what, (long long)i);
            bad = 1;
            return;
        }
}

int main(void) {
    unsigned seed = 12345u;
    const int64_t shapes[][3] = {{1, 1, 1}, {1, 7, 2}, {5, 3, 1}, {64, 100, 3}, {333, 17, 2}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int64_t N = shapes[s][0], M = shapes[s][1], B = shapes[s][2], xs = N + 3;
        double *x = rnd(B * xs, &seed);
        double *xc = rnd(B * 2 * xs, &seed);
        int64_t *bins = all_bins(M);
        double *out = malloc(sizeof(double) * (size_t)(2 * B * M));

        orc_fft_zeropad(x, xs, B, N, M > N ? M - N : 0, bins, M, out);  /* bins 0 .. M-1 of N_fft >= M */
        check_finite("fft_zeropad", out, 2 * B * M);
        orc_czt(x, 0, xs, B, N, cos(0.01), -sin(0.01), cos(0.2), sin(0.2), bins, M, out);
        check_finite("czt real", out, 2 * B * M);
        orc_czt(xc, 1, xs, B, N, 1.0001 * cos(0.01), -sin(0.01), 0.999, 0.01, bins, M, out);
        check_finite("czt complex spiral", out, 2 * B * M);
        orc_czt_band_exact(x, xs, B, N, M, 20000000000000LL, 200000000000LL, 2500000000000LL, bins, M, out);
        check_finite("czt_band_exact", out, 2 * B * M);

        int64_t *samp = all_bins(N);
        double *y = malloc(sizeof(double) * (size_t)(2 * B * N));
        orc_ifft(xc, xs, B, N, samp, N, y);
        check_finite("ifft", y, 2 * B * N);

        for (int64_t T = 1; T <= 9; T += 8)
            for (int64_t D = 1; D <= N + 2; D += (N / 2 + 1)) {
                double *h = malloc(sizeof(double) * (size_t)T);
                orc_zoom_taps(T, 0.5 / (double)D, h);
                check_finite("taps", h, T);
                const int64_t LD = (N + D - 1) / D;
                double *u = malloc(sizeof(double) * (size_t)(2 * B * LD));
                orc_zoom_frontend(x, 0, xs, B, N, 20e12, 0.2e12, 2.5e12, D, h, T, u);
                check_finite("zoom front real", u, 2 * B * LD);
                orc_zoom_frontend(xc, 1, xs, B, N, 20e12, 0.2e12, 2.5e12, D, h, T, u);
                check_finite("zoom front complex", u, 2 * B * LD);
                const int64_t K = orc_zoom_K(20e12, 0.2e12, 2.5e12, M, D);
                orc_zoom_short_dft(u, B, LD, K > 0 ? K : 1, M, bins, M, out);
                check_finite("zoom short dft", out, 2 * B * M);
                free(u);
                free(h);
            }
        free(samp);
        free(y);
        free(out);
        free(bins);
        free(xc);
        free(x);
    }
    if (!bad) printf("oracle driver: ok\n");
    return bad;
}
