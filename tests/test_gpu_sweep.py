"""GPU parity over every shape of the resolution sweep (Section 4, Figs. 11
and 12): N = 500 samples at f_s = 10 THz, df from 20 GHz down to 0.5 GHz in
0.5 GHz steps.  At each df the zero-padded FFT (full and half spectrum), the
CZT and the Zoom FFT over 0 - 2.5 THz, the inverse DFT of complex spectra and
the half-spectrum inverse back to the trace run on a small batch and are
checked against the FP64 oracle on sampled outputs.  The sweep itself only
times these calls; this test covers the plans it exercises (sub-transforms,
conjugate pairs, whole-row mixed radix, power-of-two, Bluestein).
Tolerance: relative L2 1e-6 per trace (FP32 path).
"""
import sys

import numpy as np
import pytest

import bench_sweep as sweep

pytestmark = pytest.mark.gpu
TOL = 1e-6
B = 6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tz():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_03948_amd as tz
    tz.lib()
    return tz


def close(got, ref, what):
    assert np.isfinite(got).all(), what
    e = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
    assert e.max() <= TOL, f"{what}: rel L2 {e.max():.3e}"
    return e.max()


@pytest.mark.parametrize("df", sweep.sweep_points())
def test_sweep_shape(tz, orc, df):
    import torch
    s = sweep.shapes(tz, df)
    N, nfft, M, D = sweep.N, s["n_fft"], s["M"], s["D"]
    rng = np.random.default_rng(int(df) % 100003)
    x = rng.standard_normal((B, N)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    bins = np.unique(np.r_[0, 1, nfft // 2, nfft - 1, rng.integers(0, nfft, 60)])
    hb = bins[bins <= nfft // 2]
    F = tz.fft_zeropad(xd, nfft - N).cpu().numpy()
    ef = close(F[:, bins], orc.fft_zeropad(x.astype(np.float64), nfft - N, bins), "fft_zeropad")
    Fh = tz.fft_zeropad(xd, nfft - N, half=True)
    close(Fh.cpu().numpy()[:, hb], orc.fft_zeropad(x.astype(np.float64), nfft - N, hb), "fft_zeropad half")
    W, A = tz.czt_band(sweep.FS, sweep.F1, sweep.F2, M)
    cb = np.unique(np.r_[0, M - 1, rng.integers(0, M, 40)])
    C = tz.czt(xd, M, W, A).cpu().numpy()
    close(C[:, cb], orc.czt(x.astype(np.float64), M, W, A, cb), "czt")
    Z = tz.zoom_fft(xd, sweep.FS, sweep.F1, sweep.F2, M, D, taps=sweep.TAPS).cpu().numpy()
    close(Z[:, cb], orc.zoom_fft(x.astype(np.float64), sweep.FS, sweep.F1, sweep.F2, M, D, taps=sweep.TAPS,
                                 bins=cb), "zoom_fft")
    # the inverse of complex spectra, and of the half spectrum back to the trace
    Xs = (rng.standard_normal((2, nfft)) + 1j * rng.standard_normal((2, nfft))).astype(np.complex64)
    samples = np.unique(np.r_[0, nfft - 1, rng.integers(0, nfft, 40)])
    I = tz.ifft(torch.from_numpy(Xs).cuda()).cpu().numpy()
    close(I[:, samples], orc.ifft(Xs.astype(np.complex128), samples=samples), "ifft")
    eh = float("nan")
    if nfft <= 20480 and sweep.smooth7(nfft):
        back = tz.ifft(Fh, half=True, N=nfft).cpu().numpy()
        ref = np.concatenate([x, np.zeros((B, nfft - N), np.float32)], axis=1)
        eh = close(back, ref, "half-spectrum inverse round trip")
    say(f"case: sweep df={df / 1e9:.1f} GHz N_fft={nfft} M={M} D={D}: fft {ef:.2e}, half inverse {eh:.2e}")
