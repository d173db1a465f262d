"""Pins for the FP64 oracle against things other than itself.

Every transform in ``oracle/`` is checked against at least one of: a closed
form, an identity the paper states, a library routine computing the same
special case (numpy.fft, scipy.signal.czt, scipy.signal.firwin / lfilter),
mpmath brute force at tiny sizes, or a value the paper prints
(``tests/golden/paper_values.json``).  The cases are chosen so that a sign
flip, a dropped term, an off-by-one index or a transposed operand in the
oracle fails at least one of them.
"""
import json
import os

import mpmath
import numpy as np
import pytest
import scipy.signal as ss

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# --------------------------------------------------------------------------
# zero-padded FFT (Section 2.1, eqs. (2)-(5))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,nz", [(1, 0), (7, 0), (64, 0), (100, 28), (250, 750), (1024, 3072)])
def test_fft_zeropad_matches_numpy(orc, N, nz):
    x = np.random.default_rng(N).standard_normal((3, N))
    X = orc.fft_zeropad(x, nz)
    assert X.shape == (3, N + nz)
    assert rel(X, np.fft.fft(x, N + nz, axis=1)) < 1e-13


def test_fft_zeropad_impulse_closed_form(orc):
    N, nz, n0 = 37, 91, 5
    x = np.zeros(N)
    x[n0] = 1.0
    X = orc.fft_zeropad(x, nz)[0]
    k = np.arange(N + nz)
    assert np.abs(X - np.exp(-2j * np.pi * k * n0 / (N + nz))).max() < 1e-13
    # forward sign: an impulse at n0 = 5 has a negative phase slope
    assert X[1].imag < 0


def test_fft_zeropad_on_bin_cosine(orc):
    N, k0 = 96, 11
    n = np.arange(N)
    X = orc.fft_zeropad(np.cos(2 * np.pi * k0 * n / N), 0)[0]
    expect = np.zeros(N, complex)
    expect[k0] = expect[N - k0] = N / 2
    assert np.abs(X - expect).max() < 1e-12


def test_fft_zeropad_parseval_hermitian(orc):
    x = synth.single_trace(N=300)
    X = orc.fft_zeropad(x, 212)[0]
    nfft = 512
    assert abs(np.sum(np.abs(X) ** 2) - nfft * np.sum(x ** 2)) / (nfft * np.sum(x ** 2)) < 1e-13
    k = np.arange(1, nfft)
    assert np.abs(X[nfft - k] - np.conj(X[k])).max() < 1e-12


def test_fft_zeropad_bins_subset(orc):
    x = np.random.default_rng(3).standard_normal((2, 40))
    full = orc.fft_zeropad(x, 60)
    bins = np.array([99, 0, 17, 50])
    assert np.array_equal(orc.fft_zeropad(x, 60, bins), full[:, bins])


def test_fft_zeropad_mpmath(orc):
    mpmath.mp.dps = 40
    x = np.random.default_rng(9).standard_normal(9)
    nfft = 16
    X = orc.fft_zeropad(x, nfft - 9)[0]
    for k in range(nfft):
        s = mpmath.fsum(mpmath.mpf(float(x[n])) * mpmath.expj(-2 * mpmath.pi * k * n / nfft)
                        for n in range(9))
        assert abs(complex(s) - X[k]) < 1e-14


# --------------------------------------------------------------------------
# inverse DFT (the IFFT of eq. (12), timed against the FFT in Section 4)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 2, 7, 64, 500, 1031])
def test_ifft_matches_numpy(orc, N):
    rng = np.random.default_rng(400 + N)
    X = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    assert rel(orc.ifft(X), np.fft.ifft(X, axis=1)) < 1e-13


def test_ifft_closed_forms(orc):
    """A single line X[k] = delta[k - k0] gives x[n] = e^{+j 2 pi k0 n / N} / N
    (sign of the exponent and the 1/N); a flat spectrum gives an impulse at
    n = 0."""
    N, k0 = 97, 13
    X = np.zeros(N, dtype=complex)
    X[k0] = 1.0
    n = np.arange(N)
    assert np.max(np.abs(orc.ifft(X)[0] - np.exp(2j * np.pi * k0 * n / N) / N)) < 1e-15
    x = orc.ifft(np.ones(N, dtype=complex))[0]
    assert abs(x[0] - 1.0) < 1e-14 and np.max(np.abs(x[1:])) < 1e-14


def test_ifft_inverts_the_zero_padded_fft_and_keeps_energy(orc):
    """ifft(fft(x)) = x for the zero-padded FFT of eqs. (2)-(5) taken with
    no padding, and Parseval: sum |x|^2 = (1/N) sum |X|^2."""
    rng = np.random.default_rng(402)
    x = rng.standard_normal((2, 300))
    X = orc.fft_zeropad(x, 0)
    assert rel(orc.ifft(X), x.astype(complex)) < 1e-13
    xs = orc.ifft(X, samples=[0, 17, 299])
    assert rel(xs, x[:, [0, 17, 299]].astype(complex)) < 1e-13
    Y = rng.standard_normal((2, 211)) + 1j * rng.standard_normal((2, 211))
    y = orc.ifft(Y)
    assert abs(np.sum(np.abs(y) ** 2) - np.sum(np.abs(Y) ** 2) / 211) < 1e-12 * np.sum(np.abs(y) ** 2)


# --------------------------------------------------------------------------
# CZT (Section 2.3, eqs. (11)-(25))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 5, 64, 200])
def test_czt_dft_special_case(orc, N):
    # A = 1, W = e^{-j 2 pi / N}, M = N reproduces the DFT (text after eq. (11))
    x = np.random.default_rng(N + 1).standard_normal((2, N))
    X = orc.czt(x, N, np.exp(-2j * np.pi / N), 1.0)
    assert rel(X, np.fft.fft(x, axis=1)) < 1e-12


@pytest.mark.parametrize("W0,A0", [(1.0, 1.0), (1.0005, 0.999), (0.9993, 1.002)])
def test_czt_matches_scipy(orc, W0, A0):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 120))
    W = W0 * np.exp(-2j * np.pi * 0.0137)
    A = A0 * np.exp(2j * np.pi * 0.061)
    assert rel(orc.czt(x, 77, W, A), ss.czt(x, 77, W, A)) < 1e-12
    xc = x + 1j * rng.standard_normal((3, 120))
    assert rel(orc.czt(xc, 77, W, A), ss.czt(xc, 77, W, A)) < 1e-12


def test_czt_impulse_closed_form(orc):
    N, M, n0 = 50, 33, 7
    W = 1.001 * np.exp(-2j * np.pi * 0.02)
    A = 0.98 * np.exp(2j * np.pi * 0.3)
    x = np.zeros(N)
    x[n0] = 1.0
    k = np.arange(M)
    expect = A ** (-n0) * W ** (k * n0)
    assert rel(orc.czt(x, M, W, A)[0], expect) < 1e-13


def test_czt_tone_dirichlet(orc):
    # complex tone e^{j 2 pi nu0 n} on the band [nuA, nuA + M nuW):
    # X[k] = sum_n e^{j 2 pi (nu0 - nu_k) n} = e^{j pi (N-1) d} sin(pi N d)/sin(pi d)
    N, M = 128, 90
    nuA, nuW, nu0 = 0.05, 0.0011, 0.0987
    n = np.arange(N)
    x = np.exp(2j * np.pi * nu0 * n)
    X = orc.czt(x, M, np.exp(-2j * np.pi * nuW), np.exp(2j * np.pi * nuA))[0]
    d = nu0 - (nuA + np.arange(M) * nuW)
    expect = np.exp(1j * np.pi * (N - 1) * d) * np.sin(np.pi * N * d) / np.sin(np.pi * d)
    assert np.abs(X - expect).max() < 1e-10


def test_czt_on_fft_grid_equals_zero_padded_fft(orc):
    # every method samples the same DTFT: a CZT on the zero-padded FFT grid
    # returns exactly those FFT bins (Section 3.2: no resolution is gained)
    x = np.random.default_rng(11).standard_normal((2, 250))
    nfft, j0, M = 2000, 137, 300
    X = orc.czt(x, M, np.exp(-2j * np.pi / nfft), np.exp(2j * np.pi * j0 / nfft))
    F = orc.fft_zeropad(x, nfft - 250)
    # W and A enter as rounded doubles: arg(W) carries ~1e-16 rad, times
    # k n <= 7.5e4 gives ~1e-11 rad of phase at the far corner
    assert rel(X, F[:, j0:j0 + M]) < 1e-11


def test_czt_band_exact_matches_float_band(orc):
    x = np.random.default_rng(4).standard_normal((2, 300))
    fs, f1, f2, M = 20_000_000_000_000, 200_000_000_000, 2_500_000_000_000, 257
    X = orc.czt_band_exact(x, M, fs, f1, f2)
    W = np.exp(-2j * np.pi * (f2 - f1) / (M * fs))
    A = np.exp(2j * np.pi * f1 / fs)
    # float W, A: ~1e-16 rad of arg error times k n <= 7.7e4 (see above)
    assert rel(X, ss.czt(x, M, W, A)) < 1e-11
    assert rel(X, orc.czt(x, M, W, A)) < 1e-11


def test_czt_mpmath_spiral(orc):
    mpmath.mp.dps = 40
    rng = np.random.default_rng(2)
    x = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    W = 1.01 * np.exp(-0.7j)
    A = 0.95 * np.exp(0.4j)
    X = orc.czt(x, 5, W, A)[0]
    Wm, Am = mpmath.mpc(W), mpmath.mpc(A)
    for k in range(5):
        s = mpmath.fsum(mpmath.mpc(x[n]) * Am ** (-n) * Wm ** (k * n) for n in range(6))
        assert abs(complex(s) - X[k]) < 1e-13 * max(1.0, abs(complex(s)))


def test_paper_two_tone_grid(orc):
    # Section 3.1: 128 samples at 8 kHz, CZT over 100-1000 Hz -> 7.03 Hz.
    g = json.load(open(GOLDEN))["two_tone_czt_plotting_resolution"]
    fs, f1, f2, N = g["fs_hz"], g["f1_hz"], g["f2_hz"], g["samples"]
    M = N
    df = (f2 - f1) / M  # eq. (24)
    assert round(df, g["printed_digits"]) == g["printed_hz"]
    assert round((f2 - f1) / (M - 1), 2) != g["printed_hz"]  # the M-1 reading is excluded
    # a complex tone placed on bin j0 of that grid peaks exactly there with value N
    j0 = 53
    n = np.arange(N)
    x = np.exp(2j * np.pi * (f1 + j0 * df) * n / fs)
    X = orc.czt(x, M, np.exp(-2j * np.pi * (f2 - f1) / (M * fs)), np.exp(2j * np.pi * f1 / fs))[0]
    assert int(np.argmax(np.abs(X))) == j0
    assert abs(X[j0] - N) < 1e-10
    # and the same band through the exact rational form
    Xe = orc.czt_band_exact(np.cos(2 * np.pi * (f1 + j0 * df) * n / fs), M, fs, f1, f2)[0]
    assert int(np.argmax(np.abs(Xe))) == j0


def test_paper_thz_resolutions():
    g = json.load(open(GOLDEN))
    for key in ("thz_fft_resolution_N500", "thz_fft_resolution_N250"):
        e = g[key]
        assert abs(1.0 / (e["Ts_s"] * e["N"]) - e["printed_hz"]) < 1e-3  # eq. (3)
    # CZT: the printed 2.98 / 5.96 GHz are (f2 - f1)/M with M = N (eq. (24));
    # halving N doubles the spacing exactly, i.e. M tracks N
    a, b = g["thz_czt_resolution_N500"], g["thz_czt_resolution_N250"]
    assert abs(b["printed_hz"] / a["printed_hz"] - a["N"] / b["N"]) < 1e-12


# --------------------------------------------------------------------------
# Zoom FFT (Section 2.2, eqs. (6)-(10))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("T,D", [(63, 8), (255, 64), (31, 3), (2, 2)])
def test_zoom_taps_match_firwin(orc, T, D):
    fs = 20e12
    h = orc.zoom_taps(T, 1.0 / (2 * D))
    ref = ss.firwin(T, fs / (2 * D), window="hamming", fs=fs, scale=True)
    assert np.abs(h - ref).max() < 1e-14
    assert abs(h.sum() - 1) < 1e-14 and np.abs(h - h[::-1]).max() < 1e-15


def test_zoom_taps_one_tap(orc):
    assert np.array_equal(orc.zoom_taps(1, 0.1), np.array([1.0]))


def test_zoom_frontend_matches_lfilter(orc):
    fs, f1, f2, D = 20e12, 0.1e12, 3.0e12, 8
    x = synth.single_trace(N=1000)
    h = orc.zoom_taps(63, 1 / (2 * D))
    u = orc.zoom_frontend(x, fs, f1, f2, D, h)[0]
    # mixing pinned separately below; here the mixed input is formed with
    # an exact integer phase so lfilter sees the same y
    n = np.arange(1000)
    fN = 0.5 * (f1 + f2)
    y = x[0] * np.exp(-2j * np.pi * np.mod(fN * n / fs, 1.0))
    ref = ss.lfilter(h, [1.0], y)[::D]
    assert u.shape == ((1000 + D - 1) // D,)
    assert np.abs(u - ref).max() < 1e-14


def test_zoom_mix_sign_and_frequency(orc):
    # x = sin(2 pi f_N n / fs) mixed by e^{-j 2 pi f_N n/fs} and low-passed
    # leaves -j/2 at DC (a mix by e^{+j...} would leave +j/2; a wrong f_N
    # leaves a rotating phasor)
    fs, f1, f2, D, N = 20e12, 1.0e12, 1.6e12, 8, 4000
    fN = 0.5 * (f1 + f2)
    n = np.arange(N)
    h = orc.zoom_taps(63, 1 / (2 * D))
    u = orc.zoom_frontend(np.sin(2 * np.pi * fN * n / fs), fs, f1, f2, D, h)[0]
    steady = u[10:-10]
    assert np.abs(steady - (-0.5j)).max() < 2e-3
    uc = orc.zoom_frontend(np.cos(2 * np.pi * fN * n / fs), fs, f1, f2, D, h)[0]
    assert np.abs(uc[10:-10] - 0.5).max() < 2e-3


@pytest.mark.parametrize("LD,K,M", [(128, 883, 1024), (64, 200, 150), (300, 256, 200)])
def test_zoom_short_dft_matches_numpy(orc, LD, K, M):
    rng = np.random.default_rng(LD)
    u = rng.standard_normal((2, LD)) + 1j * rng.standard_normal((2, LD))
    X = orc.zoom_short_dft(u, K, M)
    # K-point DFT of u (time-aliased if K < LD) gathered at (k - M//2) mod K
    wrapped = np.zeros((2, K), complex)
    for m in range(LD):
        wrapped[:, m % K] += u[:, m]
    F = np.fft.fft(wrapped, axis=1)
    idx = (np.arange(M) - M // 2) % K
    assert rel(X, F[:, idx]) < 1e-12


def test_zoom_D1_T1_is_dtft_on_zoom_grid(orc):
    fs, f1, f2, M = 20e12, 0.4e12, 1.3e12, 180
    x = synth.single_trace(N=256)
    X = orc.zoom_fft(x, fs, f1, f2, M, D=1, taps=1)
    K = orc.zoom_K(fs, f1, f2, M, 1)
    fN = 0.5 * (f1 + f2)
    A = np.exp(2j * np.pi * (fN / fs - (M // 2) / K))
    W = np.exp(-2j * np.pi / K)
    assert rel(X, ss.czt(x, M, W, A)) < 1e-10


def test_zoom_tone_lands_in_predicted_bin(orc):
    fs, f1, f2, M, D = 20e12, 0.1e12, 3.0e12, 1024, 8
    N = 1024
    K = orc.zoom_K(fs, f1, f2, M, D)
    assert K == 883  # round(1024 * 20 / (8 * 2.9)) = round(882.76)
    fN = 0.5 * (f1 + f2)
    for j in (-40, 0, 7, 150):
        f0 = fN + j * fs / (D * K)
        n = np.arange(N)
        X = orc.zoom_fft(np.cos(2 * np.pi * f0 * n / fs), fs, f1, f2, M, D, taps=63)[0]
        assert int(np.argmax(np.abs(X))) % K == (M // 2 + j) % K


def test_zoom_K_rounding(orc):
    assert orc.zoom_K(20e12, 0.2e12, 2.5e12, 4096, 6) == 5936
    assert orc.zoom_K(100e12, 0.05e12, 0.10e12, 1 << 18, 64) == 8_192_000
    assert orc.zoom_K(8.0, 0.0, 2.0, 5, 2) == 10  # 10.0 exactly
    assert orc.zoom_K(10.0, 0.0, 4.0, 1, 1) == 3  # 2.5 rounds half away from zero


# ---------------------------------------------------------------------------
# frequency response of sample/reference pairs (Section 1)
# ---------------------------------------------------------------------------
def test_transfer_integer_delay_closed_form(orc):
    """A sample that is the reference delayed by d samples and scaled by g
    (reference zero over its last d samples) has X_s(nu) = g e^{-j 2 pi nu d}
    X_r(nu) exactly, so H[k] = g e^{-j 2 pi (a + k w) d} on the contour
    A = e^{j 2 pi a}, W = e^{-j 2 pi w}."""
    rng = np.random.default_rng(21)
    N, d, g, M = 900, 37, 0.63, 400
    xr = np.zeros(N)
    xr[: N - d] = rng.standard_normal(N - d)
    xs = np.zeros(N)
    xs[d:] = g * xr[: N - d]
    a, w = 0.0123, 0.37 / 1000
    A, W = np.exp(2j * np.pi * a), np.exp(-2j * np.pi * w)
    H = orc.transfer(np.stack([xr, xs]), M, W, A)[0]
    k = np.arange(M)
    ref = g * np.exp(-2j * np.pi * (a + k * w) * d)
    assert np.max(np.abs(H - ref)) < 1e-9


def test_transfer_identity_and_pair_order(orc):
    rng = np.random.default_rng(22)
    x = rng.standard_normal((2, 300))
    W, A = np.exp(-2j * np.pi * 0.0011), np.exp(2j * np.pi * 0.07)
    one = orc.transfer(np.stack([x[0], x[0]]), 120, W, A)
    assert np.max(np.abs(one - 1.0)) < 1e-12
    H = orc.transfer(x, 120, W, A)
    Hinv = orc.transfer(x[::-1].copy(), 120, W, A)
    assert np.max(np.abs(H * Hinv - 1.0)) < 1e-10
    with pytest.raises(ValueError):
        orc.transfer(x[:1], 120, W, A)


# ---------------------------------------------------------------------------
# multi-dimensional transforms (the 2-D / 3-D case of Section 5)
# ---------------------------------------------------------------------------
def _unit(rng):
    return np.exp(2j * np.pi * rng.uniform(0, 1))


@pytest.mark.parametrize("shape", [(2, 6, 10), (1, 4, 6, 10), (3, 7, 1)])
def test_czt_nd_dft_special_case(orc, shape):
    # A = 1, W = e^{-j 2 pi / N_a}, M_a = N_a on every axis is the d-D DFT;
    # unequal axis lengths make a swapped or transposed axis fail
    x = np.random.default_rng(len(shape)).standard_normal(shape)
    axes = [(n, np.exp(-2j * np.pi / n), 1.0) for n in shape[1:]]
    X = orc.czt_nd(x, axes)
    assert X.shape == shape
    assert rel(X, np.fft.fftn(x, axes=tuple(range(1, len(shape))))) < 1e-13


def _brute_nd(x, axes):
    """Direct d-fold sum of x[n] prod_a A_a^-n_a W_a^(k_a n_a), Python loops."""
    B = x.shape[0]
    Ns = x.shape[1:]
    Ms = tuple(ax[0] for ax in axes)
    out = np.zeros((B,) + Ms, complex)
    for b in range(B):
        for k in np.ndindex(*Ms):
            acc = 0j
            for n in np.ndindex(*Ns):
                term = complex(x[(b,) + n])
                for a, (M, W, A) in enumerate(axes):
                    term *= complex(A) ** (-n[a]) * complex(W) ** (k[a] * n[a])
                acc += term
            out[(b,) + k] = acc
    return out


def test_czt_nd_brute_force(orc):
    rng = np.random.default_rng(31)
    x2 = rng.standard_normal((2, 3, 5))
    ax2 = [(4, _unit(rng), _unit(rng)), (2, 1.02 * _unit(rng), 0.97 * _unit(rng))]
    assert rel(orc.czt_nd(x2, ax2), _brute_nd(x2, ax2)) < 1e-13
    x3 = rng.standard_normal((1, 2, 3, 4)) + 1j * rng.standard_normal((1, 2, 3, 4))
    ax3 = [(3, _unit(rng), _unit(rng)), (2, _unit(rng), _unit(rng)), (5, _unit(rng), _unit(rng))]
    assert rel(orc.czt_nd(x3, ax3), _brute_nd(x3, ax3)) < 1e-13


def test_czt_nd_impulse_closed_form(orc):
    rng = np.random.default_rng(32)
    N0, N1, n0, n1 = 9, 14, 4, 11
    x = np.zeros((1, N0, N1))
    x[0, n0, n1] = 1.0
    (W0, A0), (W1, A1) = (_unit(rng), _unit(rng)), (_unit(rng), _unit(rng))
    M0, M1 = 7, 12
    X = orc.czt_nd(x, [(M0, W0, A0), (M1, W1, A1)])[0]
    k0, k1 = np.meshgrid(np.arange(M0), np.arange(M1), indexing="ij")
    ref = A0 ** (-n0) * W0 ** (k0 * n0) * A1 ** (-n1) * W1 ** (k1 * n1)
    assert np.abs(X - ref).max() < 1e-12


def test_czt_nd_separable_product(orc):
    rng = np.random.default_rng(33)
    a, b = rng.standard_normal(40), rng.standard_normal(27)
    ax = [(30, _unit(rng), _unit(rng)), (35, _unit(rng), _unit(rng))]
    X = orc.czt_nd(np.outer(a, b)[None], ax)[0]
    ref = np.outer(orc.czt(a, *ax[0])[0], orc.czt(b, *ax[1])[0])
    assert rel(X, ref) < 1e-13


def test_zoom_frontend_complex_is_linear(orc):
    # the complex-input front end (later axes of a d-D zoom) equals the real
    # one on the real and imaginary parts: u(xr + j xi) = u(xr) + j u(xi)
    rng = np.random.default_rng(34)
    xr, xi = rng.standard_normal((2, 500)), rng.standard_normal((2, 500))
    fs, f1, f2, D = 20e12, 0.3e12, 1.1e12, 5
    h = orc.zoom_taps(31, 1 / (2 * D))
    u = orc.zoom_frontend(xr + 1j * xi, fs, f1, f2, D, h)
    ref = orc.zoom_frontend(xr, fs, f1, f2, D, h) + 1j * orc.zoom_frontend(xi, fs, f1, f2, D, h)
    assert rel(u, ref) < 1e-14


def test_zoom_nd_D1_T1_is_czt_on_zoom_grids(orc):
    # with D = 1 and one tap every axis reduces to the DTFT on its zoom grid:
    # scipy's CZT along each axis in turn
    rng = np.random.default_rng(35)
    x = rng.standard_normal((2, 40, 24))
    axes = [(20e12, 0.4e12, 1.3e12, 30, 1), (10e12, 1.0e12, 2.5e12, 20, 1)]
    X = orc.zoom_fft_nd(x, axes, taps=1)
    ref = x.astype(complex)
    for a, (fs, f1, f2, M, D) in enumerate(axes):
        K = orc.zoom_K(fs, f1, f2, M, D)
        fN = 0.5 * (f1 + f2)
        A = np.exp(2j * np.pi * (fN / fs - (M // 2) / K))
        ref = ss.czt(ref, M, np.exp(-2j * np.pi / K), A, axis=a + 1)
    assert X.shape == (2, 30, 20)
    assert rel(X, ref) < 1e-10


def test_zoom_nd_tone_lands_in_predicted_bins(orc):
    # a separable 2-D tone on the zoom grid of each axis peaks at
    # (M_0 // 2 + j_0, M_1 // 2 + j_1)
    ax = [(20e12, 0.2e12, 1.8e12, 128, 4), (16e12, 0.5e12, 1.5e12, 96, 6)]
    N0, N1 = 512, 600
    lines = []
    for (fs, f1, f2, M, D), j, N in zip(ax, (13, -9), (N0, N1)):
        K = orc.zoom_K(fs, f1, f2, M, D)
        f0 = 0.5 * (f1 + f2) + j * fs / (D * K)
        lines.append(np.cos(2 * np.pi * f0 * np.arange(N) / fs))
    X = orc.zoom_fft_nd(np.outer(*lines)[None], [a + (None,) for a in ax], taps=63)[0]
    k0, k1 = np.unravel_index(int(np.argmax(np.abs(X))), X.shape)
    assert (k0, k1) == (128 // 2 + 13, 96 // 2 - 9)


def test_nd_bins_subset_is_the_full_grid_subset(orc):
    # evaluating a grid of bins per axis (used for sampled checks of large
    # arrays) picks exactly those entries of the full transform
    rng = np.random.default_rng(36)
    x = rng.standard_normal((2, 30, 40))
    ax = [(25, _unit(rng), _unit(rng)), (33, _unit(rng), _unit(rng))]
    b0, b1 = np.array([0, 7, 24]), np.array([32, 1, 5, 5])
    full = orc.czt_nd(x, ax)
    assert np.array_equal(orc.czt_nd(x, ax, bins=[b0, b1]), full[:, b0][:, :, b1])
    zax = [(20e12, 0.4e12, 1.3e12, 30, 2, None), (10e12, 1.0e12, 2.5e12, 20, 1, None)]
    zfull = orc.zoom_fft_nd(x, zax, taps=15)
    assert np.array_equal(orc.zoom_fft_nd(x, zax, taps=15, bins=[b0, b1[:2] % 20]),
                          zfull[:, b0][:, :, b1[:2] % 20])
