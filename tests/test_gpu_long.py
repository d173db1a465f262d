"""GPU parity of the four-step long path: Bluestein CZT with N + M - 1 above
16384 where bin blocks x input segments would transform more points than one
long FFT pair (L = L1 L2 up to 2^24, a power of two or 5 * 2^a).

Checked against the FP64 oracle on sampled bins (first, last, middle and
seeded random ones) to relative L2 <= 1e-6, for float and integer-hertz
phases, f32 / f64 / complex (zoom) inputs, M below the row length, several
trace chunks, and the long-scan workload: 256 traces x 2^20 samples at
Ts = 0.01 ps, CZT M = 2^18 over 0.05 - 0.10 THz and Zoom FFT D = 64 with a
255-tap FIR.
"""
import sys
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
TOL = 1e-6


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


def sample_bins(M, rng, n=96):
    extra = rng.choice(M, min(n, M), replace=False)
    return np.unique(np.concatenate([[0, M - 1, M // 2], extra])).astype(np.int64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N,M,dtype", [(40000, 30000, np.float32), (1000000, 1000, np.float32),
                                       (70001, 60000, np.float64), (131071, 2, np.float32)])
def test_long_czt_float_phases(tz, orc, N, M, dtype):
    import torch
    L, blocks = tz.czt_plan_shape(N, M)
    say(f"case: long czt N={N} M={M} {np.dtype(dtype).name} plan L={L} blocks={blocks}")
    assert blocks == 1 and L >= N + M - 1 and L > 16384
    rng = np.random.default_rng(N + M)
    x = rng.standard_normal((3, N)).astype(dtype)
    W = np.exp(-2j * np.pi * 0.37 / (N + M))
    A = np.exp(2j * np.pi * 0.0123)
    X = tz.czt(torch.from_numpy(x).cuda(), M, W, A).cpu().numpy()
    bins = sample_bins(M, rng)
    ref = orc.czt(x.astype(np.float64), M, W, A, bins)
    for b in range(3):
        e = rel(X[b, bins], ref[b])
        say(f"  trace {b}: rel L2 {e:.3e}")
        assert e <= TOL


def test_long_czt_at_the_longest_fft(tz, orc):
    """N + M - 1 = 2^24, the longest Bluestein FFT the library runs (four-step
    rows of 16384 under 1024 columns); one point more is refused on the host
    (test_czt_plan_shape)."""
    import torch
    M = 64
    N = (1 << 24) - M + 1
    assert tz.czt_plan_shape(N, M) == (1 << 24, 1)
    rng = np.random.default_rng(24)
    x = rng.standard_normal((1, N)).astype(np.float32)
    W = np.exp(-2j * np.pi * 0.29 / (1 << 24))
    A = np.exp(2j * np.pi * 0.0417)
    say(f"case: long czt at the longest FFT: N={N} M={M} L=2^24")
    X = tz.czt(torch.from_numpy(x).cuda(), M, W, A).cpu().numpy()
    bins = sample_bins(M, rng, 13)
    ref = orc.czt(x.astype(np.float64), M, W, A, bins)
    e = rel(X[0, bins], ref[0])
    say(f"  rel L2 {e:.3e} over {bins.size} bins")
    assert np.isfinite(X).all() and e <= TOL


def test_long_czt_batch_of_eight_narrow_columns(tz, orc):
    """M below the row length L2 with a grid of whole column groups (8 traces)."""
    import torch
    N, M = 1000000, 1000
    assert tz.czt_plan_shape(N, M) == (1 << 20, 1)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((8, N)).astype(np.float32)
    say(f"case: long czt_band_exact N={N} M={M} B=8")
    fs, f1, f2 = 20_000_000_000_000, 300_000_000_000, 310_000_000_000
    X = tz.czt_band_exact(torch.from_numpy(x).cuda(), M, fs, f1, f2).cpu().numpy()
    for b in (0, 5, 7):
        bins = sample_bins(M, rng, 40)
        ref = orc.czt_band_exact(x[b:b + 1].astype(np.float64), M, fs, f1, f2, bins)[0]
        e = rel(X[b, bins], ref)
        say(f"  trace {b}: rel L2 {e:.3e}")
        assert e <= TOL


def test_long_fft_zeropad_without_fast_factor(tz, orc):
    """N_fft with no power-of-two factor >= N goes through the long Bluestein plan."""
    import torch
    N, nz = 30000, 120015                      # N_fft = 150015 = 3^2 5 3 ... (odd)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, N)).astype(np.float32)
    say(f"case: long fft_zeropad N={N} N_fft={N + nz}")
    X = tz.fft_zeropad(torch.from_numpy(x).cuda(), nz).cpu().numpy()
    bins = sample_bins(N + nz, rng)
    ref = orc.fft_zeropad(x.astype(np.float64), nz, bins)
    for b in range(2):
        assert rel(X[b, bins], ref[b]) <= TOL


FS, F1, F2 = 100_000_000_000_000, 50_000_000_000, 100_000_000_000
N_LONG, M_LONG, B_LONG = 1 << 20, 1 << 18, 256


@pytest.fixture(scope="module")
def long_scans():
    import torch
    t0 = time.time()
    x = synth.echoes(B_LONG, N=N_LONG, fs=float(FS))
    say(f"long scans generated in {time.time() - t0:.1f} s")
    return x, torch.from_numpy(x).cuda()


def timed(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = fn()
    e1.record()
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1) / reps


def test_long_scans_czt(tz, orc, long_scans):
    x, xd = long_scans
    say(f"case: long scans czt B={B_LONG} N={N_LONG} M={M_LONG} plan {tz.czt_plan_shape(N_LONG, M_LONG)}")
    X, ms = timed(lambda: tz.czt_band_exact(xd, M_LONG, FS, F1, F2))
    say(f"  {ms:.3f} ms per batch, {B_LONG * M_LONG / ms * 1e3:.3e} bins/s")
    Xh = X.cpu().numpy()
    assert np.isfinite(Xh).all()
    rng = np.random.default_rng(11)
    worst = 0.0
    for b in (0, 77, 255):
        bins = sample_bins(M_LONG, rng, 64)
        ref = orc.czt_band_exact(x[b:b + 1].astype(np.float64), M_LONG, FS, F1, F2, bins)[0]
        e = rel(Xh[b, bins], ref)
        worst = max(worst, e)
        assert e <= TOL, (b, e)
    say(f"  worst sampled rel L2 {worst:.3e}")


def test_long_scans_zoom(tz, orc, long_scans):
    x, xd = long_scans
    D, T = 64, 255
    say(f"case: long scans zoom B={B_LONG} N={N_LONG} M={M_LONG} D={D} T={T} "
        f"K={tz.zoom_short_length(FS, F1, F2, M_LONG, D)}")
    X, ms = timed(lambda: tz.zoom_fft(xd, FS, F1, F2, M_LONG, D, taps=T))
    say(f"  {ms:.3f} ms per batch, {B_LONG * M_LONG / ms * 1e3:.3e} bins/s")
    Xh = X.cpu().numpy()
    assert np.isfinite(Xh).all()
    rng = np.random.default_rng(12)
    worst = 0.0
    for b in (0, 128, 255):
        bins = sample_bins(M_LONG, rng, 64)
        ref = orc.zoom_fft(x[b:b + 1].astype(np.float64), FS, F1, F2, M_LONG, D, taps=T, bins=bins)[0]
        e = rel(Xh[b, bins], ref)
        worst = max(worst, e)
        assert e <= TOL, (b, e)
    say(f"  worst sampled rel L2 {worst:.3e}")


# ---------------------------------------------------------------------------
# split precision on the four-step path: the row FFTs' radix-16 passes on the
# matrix cores (hi + lo operands, FP32 accumulation); the column FFTs, chirps
# and twiddles stay FP32
# ---------------------------------------------------------------------------
TOL_SPLIT = 1e-5


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("N,M", [(1000000, 200000), (1500000, 100000), (2400000, 100000), (200000, 100000),
                                 (400000, 200000)])
def test_long_czt_split_precision(tz, orc, prec, N, M):
    """Rows of 4096 (L = 320 x 4096 and 512 x 4096), of 8192 (320 x 8192),
    and of 1024 and 2048 (320 x 1024, 320 x 2048: two matrix-core passes over
    256-point sub-transforms and a trailing radix 4 or 8)."""
    import torch
    L, blocks = tz.czt_plan_shape(N, M)
    say(f"case: long czt {prec} N={N} M={M} plan L={L} blocks={blocks}")
    rng = np.random.default_rng(N + M + 7)
    x = rng.standard_normal((2, N)).astype(np.float32)
    W = np.exp(-2j * np.pi * 0.37 / (N + M))
    A = np.exp(2j * np.pi * 0.0123)
    X = tz.czt(torch.from_numpy(x).cuda(), M, W, A, precision=prec).cpu().numpy()
    assert np.isfinite(X).all()
    bins = sample_bins(M, rng, 64)
    ref = orc.czt(x.astype(np.float64), M, W, A, bins)
    for b in range(2):
        e = rel(X[b, bins], ref[b])
        say(f"  trace {b}: rel L2 {e:.3e}")
        assert e <= TOL_SPLIT


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
def test_long_scans_zoom_split(tz, orc, long_scans, prec):
    """The long-scan Zoom FFT with its short DFT (four-step, rows of 1024) at
    split precision; the front end stays FP64."""
    x, xd = long_scans
    D, T = 64, 255
    say(f"case: long scans zoom {prec} B={B_LONG} N={N_LONG} M={M_LONG} D={D} T={T}")
    X, ms = timed(lambda: tz.zoom_fft(xd, FS, F1, F2, M_LONG, D, taps=T, precision=prec))
    _, ms32 = timed(lambda: tz.zoom_fft(xd, FS, F1, F2, M_LONG, D, taps=T))
    say(f"  {prec} {ms:.3f} ms per batch, FP32 {ms32:.3f} ms ({ms32 / ms:.2f}x)")
    Xh = X.cpu().numpy()
    assert np.isfinite(Xh).all()
    rng = np.random.default_rng(14)
    worst = 0.0
    for b in (0, 128, 255):
        bins = sample_bins(M_LONG, rng, 64)
        ref = orc.zoom_fft(x[b:b + 1].astype(np.float64), FS, F1, F2, M_LONG, D, taps=T, bins=bins)[0]
        e = rel(Xh[b, bins], ref)
        worst = max(worst, e)
        assert e <= TOL_SPLIT, (b, e)
    say(f"  worst sampled rel L2 {worst:.3e}")


def test_zoom_split_refuses_single_pass_short_dft(tz):
    """A short DFT that runs single-pass on complex u has no split kernel."""
    import torch
    x = torch.zeros((2, 4096), device="cuda")
    with pytest.raises(tz.ThzError) as e:
        tz.zoom_fft(x, 20e12, 0.2e12, 2.5e12, 4096, 6, precision="split_fp16")
    assert e.value.status == tz.TZ_EUNSUPPORTED


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
def test_long_scans_czt_split(tz, orc, long_scans, prec):
    """The long-scan CZT (256 x 2^20 -> 2^18 bins, L = 320 x 4096) at split
    precision: error against the FP64 oracle and time against the FP32 path."""
    x, xd = long_scans
    say(f"case: long scans czt {prec} B={B_LONG} N={N_LONG} M={M_LONG}")
    X, ms = timed(lambda: tz.czt_band_exact(xd, M_LONG, FS, F1, F2, precision=prec))
    _, ms32 = timed(lambda: tz.czt_band_exact(xd, M_LONG, FS, F1, F2))
    say(f"  {prec} {ms:.3f} ms per batch, FP32 {ms32:.3f} ms ({ms32 / ms:.2f}x)")
    Xh = X.cpu().numpy()
    assert np.isfinite(Xh).all()
    rng = np.random.default_rng(13)
    worst = 0.0
    for b in (0, 77, 255):
        bins = sample_bins(M_LONG, rng, 64)
        ref = orc.czt_band_exact(x[b:b + 1].astype(np.float64), M_LONG, FS, F1, F2, bins)[0]
        e = rel(Xh[b, bins], ref)
        worst = max(worst, e)
        assert e <= TOL_SPLIT, (b, e)
    say(f"  worst sampled rel L2 {worst:.3e}")
