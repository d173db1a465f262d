"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Bar (stated by the task for the FP32 path): relative L2 error per trace
<= 1e-6 against direct FP64 summation on the same (float32-rounded) inputs.
Sizes span several FFT tiles with ragged tails, the bin-block / input-segment
path, all three input kinds, strides, and the degenerate cases (N = 1,
M = 1, N + M - 1 exactly at a power of two).
"""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-6


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


@pytest.fixture(scope="module")
def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(x, dev, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def rel_rows(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.linalg.norm(a - b, axis=-1)
    den = np.maximum(np.linalg.norm(b, axis=-1), 1e-300)
    return num / den


def assert_close(gpu, ref, tol=TOL_FP32, what=""):
    r = rel_rows(gpu, ref)
    say(f"  {what}: max rel L2 {r.max():.3e} (median {np.median(r):.3e}) over {r.size} traces")
    assert np.all(np.isfinite(gpu))
    assert r.max() <= tol, f"{what}: rel L2 {r.max():.3e} > {tol}"


# ---------------------------------------------------------------------------
# single-trace workload: N = 1024 FP64, fs = 20 THz, band 0.1 - 3 THz
# ---------------------------------------------------------------------------
def test_single_trace_all_three(tz, dev, orc):
    x = synth.single_trace(N=1024)
    xd = to_dev(x, dev)
    fs, f1, f2, M = 20e12, 0.1e12, 3.0e12, 1024
    say("case: single trace fp64 N=1024: czt M=1024, fft_zeropad 16384, zoom D=8 T=63")
    W, A = tz.czt_band(fs, f1, f2, M)
    assert_close(tz.czt(xd, M, W, A).cpu().numpy(), orc.czt(x, M, W, A), what="czt")
    assert_close(tz.fft_zeropad(xd, 16384 - 1024).cpu().numpy(), orc.fft_zeropad(x, 16384 - 1024),
                 what="fft_zeropad")
    assert_close(tz.zoom_fft(xd, fs, f1, f2, M, 8, taps=63).cpu().numpy(),
                 orc.zoom_fft(x, fs, f1, f2, M, 8, taps=63), what="zoom (K=883 prime, M > K)")
    Xe = tz.czt_band_exact(xd, M, 20_000_000_000_000, 100_000_000_000, 3_000_000_000_000).cpu().numpy()
    assert_close(Xe, orc.czt_band_exact(x, M, 20_000_000_000_000, 100_000_000_000, 3_000_000_000_000),
                 what="czt_band_exact")


# ---------------------------------------------------------------------------
# batched pairs, the shapes of the 8192 x 4096 workload on a few traces
# ---------------------------------------------------------------------------
def test_pairs_czt_and_fft(tz, dev, orc):
    x = synth.pairs(3, N=4096)          # 6 traces, float32
    x64 = x.astype(np.float64)
    xd = to_dev(x, dev)
    fs, f1, f2, M = 20e12, 0.2e12, 2.5e12, 4096
    say("case: pairs B=6 N=4096 czt M=4096 (L=8192), fft_zeropad 65536 (16 x 4096)")
    W, A = tz.czt_band(fs, f1, f2, M)
    assert_close(tz.czt(xd, M, W, A).cpu().numpy(), orc.czt(x64, M, W, A), what="czt")
    F = tz.fft_zeropad(xd[:3], 65536 - 4096).cpu().numpy()
    assert_close(F, orc.fft_zeropad(x64[:3], 65536 - 4096), what="fft_zeropad split")
    Z = tz.zoom_fft(xd, fs, f1, f2, M, 6, taps=63).cpu().numpy()
    assert_close(Z, orc.zoom_fft(x64, fs, f1, f2, M, 6, taps=63), what="zoom D=6 K=5936")


@pytest.mark.parametrize("N,M", [(1, 1), (1, 300), (300, 1), (7, 5), (1000, 1049), (1000, 1050),
                                 (777, 1234), (4096, 4097), (2500, 13000), (8193, 8192)])
def test_czt_shapes_ragged(tz, dev, orc, N, M):
    rng = np.random.default_rng(N * 7 + M)
    x = rng.standard_normal((5, N)).astype(np.float32)
    W = np.exp(-2j * np.pi * 0.000731)
    A = np.exp(2j * np.pi * 0.0123)
    say(f"case: czt N={N} M={M} shape={tz.czt_plan_shape(N, M)}")
    X = tz.czt(to_dev(x, dev), M, W, A).cpu().numpy()
    assert_close(X, orc.czt(x.astype(np.float64), M, W, A), what=f"czt N={N} M={M}")


@pytest.mark.parametrize("N,M", [(12000, 6000), (16384, 8192), (3000, 15000), (16000, 2000), (16100, 8000)])
def test_czt_segments_and_blocks(tz, dev, orc, N, M):
    x = synth.pairs(1, N=N).astype(np.float32)
    fs, f1, f2 = 20e12, 0.05e12, 2.0e12
    W, A = tz.czt_band(fs, f1, f2, M)
    say(f"case: czt segmented/blocked N={N} M={M} shape={tz.czt_plan_shape(N, M)}")
    X = tz.czt(to_dev(x, dev), M, W, A).cpu().numpy()
    assert_close(X, orc.czt(x.astype(np.float64), M, W, A), what=f"czt seg N={N} M={M}")


@pytest.mark.parametrize("N,M", [(683, 4096), (1000, 8000), (200, 16000), (100, 100000), (3000, 15000)])
def test_czt_bin_blocks_on_shorter_ffts(tz, dev, orc, N, M):
    """Shapes whose FP32 plan splits the bins into blocks on a shorter FFT
    (the Bluestein length is free as long as it holds N + Mb - 1 points)."""
    rng = np.random.default_rng(N + 3 * M)
    x = rng.standard_normal((3, N)).astype(np.float32)
    W = np.exp(-2j * np.pi * 0.37 / M)
    A = np.exp(2j * np.pi * 0.0123)
    L, blocks = tz.czt_plan_shape(N, M)
    say(f"case: czt N={N} M={M} plan L={L} blocks={blocks}")
    assert blocks > 1 and L < 16384
    X = tz.czt(to_dev(x, dev), M, W, A).cpu().numpy()
    assert_close(X, orc.czt(x.astype(np.float64), M, W, A), what=f"czt blocks N={N} M={M}")


@pytest.mark.parametrize("N,M,dtype", [(4096, 4096, "float32"), (2500, 4000, "float32"), (4000, 300, "float32"),
                                       (4096, 4096, "float64"), (3500, 3000, "float32"), (4096, 100, "float32")])
def test_czt_half_length_form(tz, dev, orc, N, M, dtype):
    """Plans of L = 8192 whose trace and bins each fit in L/2 run as two
    4096-point Bluestein pairs (odd bins from the trace twisted by W_L^n, the
    inverse recombined with W_L^-n)."""
    rng = np.random.default_rng(N + 5 * M)
    x = rng.standard_normal((4, N)).astype(dtype)
    W = np.exp(-2j * np.pi * 0.61 / M)
    A = np.exp(2j * np.pi * 0.0417)
    L, blocks = tz.czt_plan_shape(N, M)
    say(f"case: czt half-length form N={N} M={M} {dtype} plan L={L} blocks={blocks}")
    assert (L, blocks) == (8192, 1)
    X = tz.czt(to_dev(x, dev), M, W, A).cpu().numpy()
    assert_close(X, orc.czt(x.astype(np.float64), M, W, A), what=f"czt half N={N} M={M}")


@pytest.mark.parametrize("dtype,precision", [("float32", "fp32"), ("float64", "fp32"), ("float32", "split_bf16"),
                                             ("float32", "split_fp16")])
def test_czt_half_length_form_strided_rows(tz, dev, orc, dtype, precision):
    """The half-length kernels (FP32 and matrix-core) on row views: traces
    4000 samples long at a row stride of 4500, bins written into rows 4100
    wide; the 100 columns past the bins keep their contents."""
    import torch
    N, M, B = 4000, 4000, 5
    rng = np.random.default_rng(91)
    big = rng.standard_normal((B, 4500)).astype(dtype)
    W = np.exp(-2j * np.pi * 0.53 / M)
    A = np.exp(2j * np.pi * 0.021)
    say(f"case: czt half-length form, strided rows, {dtype} {precision} plan {tz.czt_plan_shape(N, M)}")
    assert tz.czt_plan_shape(N, M) == (8192, 1)
    xd = to_dev(big, dev)[:, :N]
    full = torch.empty((B, 4100), dtype=torch.complex64, device=dev)
    torch.view_as_real(full).fill_(float("nan"))  # both parts NaN
    out = full[:, :M]
    assert tz.czt(xd, M, W, A, out=out, precision=precision) is out
    got = full.cpu().numpy()
    assert np.isnan(got[:, M:].real).all() and np.isnan(got[:, M:].imag).all()
    tol = 1e-5 if precision == "split_bf16" else TOL_FP32
    assert_close(got[:, :M], orc.czt(big[:, :N].astype(np.float64), M, W, A), tol=tol,
                 what=f"czt half strided {dtype} {precision}")


def test_zoom_short_dft_half_length_form(tz, dev, orc):
    """Complex input: the zoom's short DFT on u (3334 samples, 4000 bins)
    takes the half-length form of an 8192-point plan."""
    N, D, M = 20000, 6, 4000
    x = synth.pairs(1, N=N)[:1].astype(np.float32)
    fs, f1, f2 = 20e12, 0.2e12, 2.5e12
    say(f"case: zoom N={N} D={D} M={M}: short DFT of {-(-N // D)} samples, plan {tz.czt_plan_shape(-(-N // D), M)}")
    Z = tz.zoom_fft(to_dev(x, dev), fs, f1, f2, M, D, taps=63).cpu().numpy()
    assert_close(Z, orc.zoom_fft(x.astype(np.float64), fs, f1, f2, M, D, taps=63), what="zoom half-length short DFT")


def test_fft_zeropad_half_spectrum_with_bin_blocks_stays_in_rows(tz, dev, orc):
    """N_fft = 30001 has no power-of-two factor >= N: its bins come from a
    blocked Bluestein plan, of which TZ_HALF needs the first 15001 only.
    Blocks past them write nothing: the padding between output rows keeps
    its sentinel."""
    import torch
    N, nz = 1000, 29001
    nout = (N + nz) // 2 + 1
    rng = np.random.default_rng(77)
    x = rng.standard_normal((3, N)).astype(np.float32)
    full = torch.full((3, nout + 4096), complex(7.0, -7.0), dtype=torch.complex64, device=dev)
    out = full[:, :nout]
    say(f"case: fft_zeropad half N={N} Nfft={N + nz} plan {tz.czt_plan_shape(N, N + nz)}, padded rows")
    tz.fft_zeropad(to_dev(x, dev), nz, half=True, out=out)
    f = full.cpu().numpy()
    assert np.all(f[:, nout:] == np.complex64(complex(7.0, -7.0)))
    assert_close(f[:, :nout], orc.fft_zeropad(x.astype(np.float64), nz, np.arange(nout)),
                 what="fft half, blocked plan")


@pytest.mark.parametrize("N,nz,half", [(1, 0, False), (100, 156, False), (1000, 1048, False),
                                       (1024, 15360, False), (300, 212, True), (1000, 537, False),
                                       (4096, 61440, True), (5000, 11384, False), (2048, 30720, False),
                                       (4000, 28768, True), (7999, 57537, False), (511, 15873, False),
                                       (3, 16381, False), (4096, 61440, False)])
def test_fft_zeropad_shapes(tz, dev, orc, N, nz, half):
    rng = np.random.default_rng(N + nz)
    x = rng.standard_normal((3, N)).astype(np.float32)
    say(f"case: fft_zeropad N={N} n_zeros={nz} half={half}")
    F = tz.fft_zeropad(to_dev(x, dev), nz, half=half).cpu().numpy()
    nf = N + nz
    bins = np.arange(nf // 2 + 1 if half else nf)
    assert_close(F, orc.fft_zeropad(x.astype(np.float64), nz, bins), what=f"fft N={N} Nfft={nf}")


# 7-smooth N_fft that no power-of-two factorisation covers: the mixed-radix
# FFT (radices 2, 3, 4, 5, 7, 8) of the zero-padded row, both row kernels
# (up to 2560 points and past it), odd lengths, f64 input and the half
# spectrum
@pytest.mark.parametrize("N,nfft,half,dtype", [
    (500, 500, False, "float32"), (500, 1000, False, "float32"), (500, 588, True, "float32"),
    (300, 625, False, "float64"), (500, 1176, False, "float32"), (500, 2500, True, "float32"),
    (2000, 2646, False, "float32"), (500, 6615, False, "float32"), (4000, 10000, False, "float32"),
    (500, 16807, False, "float32"), (500, 19683, True, "float32"), (500, 20000, False, "float64"),
    (20000, 20000, False, "float32")])
def test_fft_zeropad_mixed_radix(tz, dev, orc, N, nfft, half, dtype):
    rng = np.random.default_rng(N + nfft)
    x = rng.standard_normal((3, N)).astype(dtype)
    nz = nfft - N
    nout = nfft // 2 + 1 if half else nfft
    say(f"case: fft_zeropad mixed radix N={N} N_fft={nfft} half={half} {dtype}")
    full = torch_full(dev, (3, nout + 5))
    tz.fft_zeropad(to_dev(x, dev), nz, half=half, out=full[:, :nout])
    f = full.cpu().numpy()
    assert np.all(f[:, nout:] == np.complex64(complex(7.0, -7.0))), "wrote past the row"
    bins = np.arange(nout) if nout <= 4096 else \
        np.unique(np.r_[0, 1, nout - 1, nout // 2, rng.integers(0, nout, 200)])
    assert_close(f[:, bins], orc.fft_zeropad(x.astype(np.float64), nz, bins), what=f"fft mixed N={N} Nfft={nfft}")


# N_fft = P F with a 7-smooth F >= N: sub-transforms of F points.  P = 16
# or 32 with F <= 640: conjugate pairs (columns 1 .. P/2 - 1 transformed,
# their mirrors conjugated, columns 0 and P/2 from one 2F-point real FFT);
# other multiples of 16: tiles of 16 independent sub-transforms; power-of-
# two N_fft: tiles of 8 up to F = 1024; other shapes keep the whole-row or
# Bluestein plans.  Odd and even F, the largest F of each kernel, N = 1,
# f64 input, the half spectrum, the sweep's N_fft = 20000 at N = 500
@pytest.mark.parametrize("N,nfft,half,dtype", [
    (500, 20000, False, "float32"),   # pairs: F = 625, P = 32
    (500, 10000, True, "float32"),    # pairs: F = 625, P = 16
    (300, 4800, False, "float64"),    # pairs: F = 300 (even), P = 16
    (100, 8192, False, "float32"),    # pairs: F = 256, P = 32
    (1, 1024, False, "float32"),      # pairs: F = 64, P = 16
    (640, 10240, True, "float32"),    # pairs: F = 640, P = 16: the largest F
    (500, 30000, False, "float32"),   # 16-row tiles: F = 625, P = 48
    (1000, 8192, True, "float32"),    # 8-row tiles: F = 1024, P = 8: the largest F
    (64, 512, False, "float32"),      # 8-row tiles: F = 64, P = 8
    (700, 131072, False, "float64"),  # 8-row tiles: F = 1024, P = 128
    (400, 4000, False, "float32"),    # no tile, not a power of two: whole-row FFT
    (999, 63 * 1000, False, "float32")])  # no tile fits (Bluestein plan)
def test_fft_zeropad_sub_transforms(tz, dev, orc, N, nfft, half, dtype):
    rng = np.random.default_rng(3 * N + nfft)
    x = rng.standard_normal((3, N)).astype(dtype)
    nz = nfft - N
    nout = nfft // 2 + 1 if half else nfft
    say(f"case: fft_zeropad sub-transforms N={N} N_fft={nfft} half={half} {dtype}")
    full = torch_full(dev, (3, nout + 5))
    tz.fft_zeropad(to_dev(x, dev), nz, half=half, out=full[:, :nout])
    f = full.cpu().numpy()
    assert np.isfinite(f).all()
    assert np.all(f[:, nout:] == np.complex64(complex(7.0, -7.0))), "wrote past the row"
    bins = np.arange(nout) if nout <= 8192 else \
        np.unique(np.r_[0, 1, nout - 1, nout // 2, rng.integers(0, nout, 300)])
    assert_close(f[:, bins], orc.fft_zeropad(x.astype(np.float64), nz, bins),
                 what=f"fft sub-transforms N={N} Nfft={nfft}")


def torch_full(dev, shape):
    import torch
    return torch.full(shape, complex(7.0, -7.0), dtype=torch.complex64, device=dev)


@pytest.mark.parametrize("N,M,D,T,band", [
    (1024, 1024, 8, 63, (0.1e12, 3.0e12)),
    (4096, 4096, 6, 63, (0.2e12, 2.5e12)),
    (3000, 500, 16, 255, (0.4e12, 0.9e12)),
    (999, 301, 3, 31, (1.0e12, 4.0e12)),
    (512, 256, 1, 1, (0.3e12, 1.2e12)),
    # long filters split over four waves, pad every D samples with D = 64 and
    # with D = 40 (a multiple of 8 that is no power of two), D % 8 == 4
    (20000, 700, 64, 511, (0.05e12, 0.15e12)),
    (6001, 300, 40, 300, (0.2e12, 0.4e12)),
    (4093, 1000, 12, 127, (0.3e12, 1.0e12)),
    (2999, 400, 5, 200, (0.5e12, 2.0e12)),
    # filters too long for two outputs per lane: one per lane, and a tile
    # narrower than its lanes
    (30000, 200, 128, 1000, (0.05e12, 0.1e12)),
    (30000, 200, 128, 2000, (0.05e12, 0.1e12)),
    # degenerate: decimation longer than the trace (one output, M = 1) and a
    # filter far longer than the trace
    (10, 1, 16, 127, (0.3e12, 1.2e12)),
    (3, 7, 1, 200, (0.3e12, 1.2e12)),
])
def test_zoom_shapes(tz, dev, orc, N, M, D, T, band):
    x = synth.pairs(2, N=N)
    f1, f2 = band
    fs = 20e12
    say(f"case: zoom N={N} M={M} D={D} T={T} K={tz.zoom_short_length(fs, f1, f2, M, D)}")
    Z = tz.zoom_fft(to_dev(x, dev), fs, f1, f2, M, D, taps=T).cpu().numpy()
    assert_close(Z, orc.zoom_fft(x.astype(np.float64), fs, f1, f2, M, D, taps=T), what="zoom")


@pytest.mark.parametrize("N,D,T", [(1001, 6, 63), (1003, 64, 255), (4097, 3, 130), (5, 2, 63), (1025, 8, 127)])
def test_zoom_padded_rows(tz, dev, orc, N, D, T):
    """Rows on 16-byte boundaries (stride a multiple of 4 samples) with N % 4 != 0:
    the front end's wide loads, including the one that holds sample N."""
    rng = np.random.default_rng(N + D)
    stride = (N + 3) // 4 * 4 + 4
    big = rng.standard_normal((3, stride)).astype(np.float32)
    xd = to_dev(big, dev)[:, :N]
    fs, f1, f2, M = 20e12, 0.3e12, 1.1e12, 300
    say(f"case: zoom padded rows N={N} stride={stride} D={D} T={T}")
    Z = tz.zoom_fft(xd, fs, f1, f2, M, D, taps=T).cpu().numpy()
    assert_close(Z, orc.zoom_fft(big[:, :N].astype(np.float64), fs, f1, f2, M, D, taps=T), what="zoom padded")


def test_strides_and_fp64_input(tz, dev, orc):
    import torch
    rng = np.random.default_rng(3)
    big = rng.standard_normal((4, 1500))
    xd = to_dev(big, dev)[:, :1200]             # in_stride 1500 > N = 1200, float64
    M = 700
    W = np.exp(-2j * np.pi * 0.00041)
    A = np.exp(2j * np.pi * 0.2)
    out = torch.zeros((4, 900), dtype=torch.complex64, device=dev)[:, :M]   # out_stride 900
    say("case: strided fp64 input, strided output")
    tz.czt(xd, M, W, A, out=out)
    assert_close(out.cpu().numpy(), orc.czt(big[:, :1200], M, W, A), what="strided czt")


def test_deterministic(tz, dev):
    x = to_dev(synth.pairs(4, N=4096), dev)
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 4096)
    say("case: determinism czt + fft_zeropad, two runs bitwise")
    a = tz.czt(x, 4096, W, A).cpu().numpy()
    b = tz.czt(x, 4096, W, A).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    f = tz.fft_zeropad(x, 61440).cpu().numpy()
    g = tz.fft_zeropad(x, 61440).cpu().numpy()
    assert np.array_equal(f.view(np.uint32), g.view(np.uint32))


def test_empty_batch_and_empty_traces(tz, dev):
    """A batch of no traces gives an empty result of the right shape on every
    transform (no library call); traces of no samples are refused."""
    import torch
    say("case: empty batches (0 x 300 traces) and traces of 0 samples")
    x0 = torch.empty((0, 300), dtype=torch.float32, device=dev)
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 50)
    assert tz.fft_zeropad(x0, 212).shape == (0, 512)
    assert tz.fft_zeropad(x0, 212, half=True).shape == (0, 257)
    assert tz.czt(x0, 50, W, A).shape == (0, 50)
    assert tz.czt(x0.double(), 50, W, A, precision="fp64").dtype == torch.complex128
    assert tz.czt_band_exact(x0, 50, 20 * 10**12, 2 * 10**11, 25 * 10**11).shape == (0, 50)
    assert tz.zoom_fft(x0, 20e12, 0.2e12, 2.5e12, 50, 3).shape == (0, 50)
    assert tz.czt_transfer(x0, 50, W, A).shape == (0, 50)
    X0 = torch.empty((0, 512), dtype=torch.complex64, device=dev)
    assert tz.ifft(X0).shape == (0, 512)
    assert tz.ifft(X0[:, :257], half=True).shape == (0, 512)
    out = torch.empty((0, 50), dtype=torch.complex64, device=dev)
    assert tz.czt(x0, 50, W, A, out=out) is out
    torch.cuda.synchronize()
    for empty in (torch.empty((3, 0), dtype=torch.float32, device=dev),
                  torch.empty((0,), dtype=torch.float32, device=dev)):
        with pytest.raises(ValueError):
            tz.czt(empty, 50, W, A)
        with pytest.raises(ValueError):
            tz.fft_zeropad(empty, 100)


def test_full_size_batch_sampled(tz, dev, orc):
    """The 8192 x 4096 batch exactly as the benchmark launches it; seeded
    traces and bins are recomputed one by one by the oracle."""
    import torch
    n_pairs = 4096
    say("case: full batch 8192 x 4096 (czt M=4096, fft_zeropad 65536, zoom D=6), sampled check")
    x = synth.pairs(n_pairs, N=4096)
    xd = to_dev(x, dev)
    fs, f1, f2, M = 20e12, 0.2e12, 2.5e12, 4096
    W, A = tz.czt_band(fs, f1, f2, M)
    X = tz.czt(xd, M, W, A)
    F = tz.fft_zeropad(xd, 65536 - 4096)
    Z = tz.zoom_fft(xd, fs, f1, f2, M, 6, taps=63)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    rows = np.sort(rng.choice(2 * n_pairs, 6, replace=False))
    rows[-1] = 2 * n_pairs - 1          # the last trace of the batch
    x64 = x[rows].astype(np.float64)
    bins = np.sort(rng.choice(M, 256, replace=False))
    assert_close(X[rows][:, bins].cpu().numpy(), orc.czt(x64, M, W, A, bins), what="czt sampled")
    fb = np.sort(rng.choice(65536, 256, replace=False))
    fb[-1] = 65535
    assert_close(F[rows][:, fb].cpu().numpy(), orc.fft_zeropad(x64, 65536 - 4096, fb),
                 what="fft sampled")
    zref = orc.zoom_fft(x64, fs, f1, f2, M, 6, taps=63)
    assert_close(Z[rows].cpu().numpy(), zref, what="zoom rows")
    # every output finite, and a property at full size: Hermitian symmetry of
    # the real-input spectrum, X[N-k] = conj X[k]
    assert bool(torch.isfinite(torch.view_as_real(X)).all())
    Fr = F[:64]
    k = torch.arange(1, 65536, device=dev)
    sym = (Fr[:, 65536 - k] - Fr[:, k].conj()).abs().max() / Fr.abs().max()
    say(f"  fft Hermitian defect {float(sym):.2e}")
    assert float(sym) < 1e-6


# ---------------------------------------------------------------------------
# split precision: radix-16 passes on the matrix cores (hi + lo operands)
# ---------------------------------------------------------------------------
TOL_SPLIT = 1e-5


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("N,M", [(2000, 2000), (4096, 4096), (8192, 8000), (3000, 1)])
def test_czt_split_precision(tz, dev, orc, prec, N, M):
    x = synth.pairs(2, N=N)
    fs, f1, f2 = 20e12, 0.2e12, 2.5e12
    W, A = tz.czt_band(fs, f1, f2, M)
    L, _ = tz.czt_plan_shape(N, M)
    say(f"case: czt {prec} N={N} M={M} L={L}")
    X = tz.czt(to_dev(x, dev), M, W, A, precision=prec).cpu().numpy()
    ref = orc.czt(x.astype(np.float64), M, W, A)
    r = rel_rows(X, ref)
    say(f"  {prec}: max rel L2 {r.max():.3e}")
    assert np.all(np.isfinite(X))
    # hi + lo keeps ~22 (fp16) or ~16 (bf16) significant bits per operand;
    # accumulation is FP32 in both cases
    assert r.max() <= TOL_SPLIT


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
def test_full_size_split_precision_sampled(tz, dev, orc, prec):
    """The split-precision CZT on the 8192 x 4096 batch exactly as the
    benchmark launches it (M = 4096, the half-length matrix-core kernel):
    sampled traces (the first and the last among them) on all bins and
    sampled bins of more traces against the oracle; every output finite."""
    import torch
    n_pairs, M = 4096, 4096
    say(f"case: full batch 8192 x 4096 czt M=4096 {prec}, sampled check")
    x = synth.pairs(n_pairs, N=4096)
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, M)
    X = tz.czt(to_dev(x, dev), M, W, A, precision=prec)
    assert bool(torch.isfinite(torch.view_as_real(X)).all())
    rng = np.random.default_rng(78)
    rows = np.r_[0, np.sort(rng.choice(np.arange(1, 2 * n_pairs - 1), 3, replace=False)), 2 * n_pairs - 1]
    assert_close(X[rows].cpu().numpy(), orc.czt(x[rows].astype(np.float64), M, W, A), tol=TOL_SPLIT,
                 what=f"{prec} rows")
    more = np.sort(rng.choice(2 * n_pairs, 24, replace=False))
    bins = np.sort(rng.choice(M, 128, replace=False))
    assert_close(X[more][:, bins].cpu().numpy(), orc.czt(x[more].astype(np.float64), M, W, A, bins),
                 tol=TOL_SPLIT, what=f"{prec} sampled bins")


def test_split_precision_rejects_other_shapes(tz, dev):
    x = to_dev(np.ones((1, 100), np.float32), dev)
    with pytest.raises(tz.ThzError) as e:
        tz.czt(x, 100, np.exp(-0.01j), 1.0, precision="split_fp16")   # L = 256
    assert e.value.status == tz.TZ_EUNSUPPORTED


# ---------------------------------------------------------------------------
# spiral contours (|A| or |W| != 1, eqs. (16)-(17))
# ---------------------------------------------------------------------------
# spreads of the two magnitude profiles (f, h): 2.5, 1.5, 3.4, 1.25, 5, 1.6
@pytest.mark.parametrize("N,M,A0,W0", [(1000, 800, 1.0005, 0.999998), (300, 300, 0.998, 1.00001),
                                       (4096, 4096, 1.0, 1.0000002), (2000, 2000, 0.9995, 0.9999995),
                                       (1000, 1000, 1.0, 1.000005), (40000, 30000, 1.0, 1.0 + 1e-9)])
def test_czt_spiral(tz, dev, orc, N, M, A0, W0):
    rng = np.random.default_rng(N + M)
    x = rng.standard_normal((3, N)).astype(np.float32)
    W = W0 * np.exp(-2j * np.pi * 0.37 / max(N, M))
    A = A0 * np.exp(2j * np.pi * 0.0123)
    say(f"case: spiral czt N={N} M={M} A0={A0} W0={W0} plan {tz.czt_plan_shape(N, M)}")
    X = tz.czt(to_dev(x, dev), M, W, A).cpu().numpy()
    if N * M <= 2_000_000:
        assert_close(X, orc.czt(x.astype(np.float64), M, W, A), what="spiral czt")
    else:
        bins = np.unique(np.concatenate([[0, M - 1], np.random.default_rng(1).choice(M, 80, replace=False)]))
        ref = orc.czt(x.astype(np.float64), M, W, A, bins)
        assert_close(X[:, bins], ref, what="spiral czt sampled")


# TZ_FP64: direct summation in FP64 for contours the FP32 tables cannot carry
# (bins spanning up to e^200, beyond FP32's range) and for the unit circle;
# complex128 bins, every one within 1e-9 of the oracle
@pytest.mark.parametrize("N,M,A0,W0,dtype", [(500, 400, 1.0, 1.001, "float32"),
                                              (2000, 1500, 0.99, 1.000003, "float64"),
                                              (300, 300, 1.02, 0.9999, "float32"),
                                              (1000, 700, 1.0, 1.0, "float32"),
                                              (1, 5, 1.0, 1.0, "float32")])
def test_czt_fp64_direct(tz, dev, orc, N, M, A0, W0, dtype):
    rng = np.random.default_rng(7 * N + M)
    x = rng.standard_normal((3, N)).astype(dtype)
    W = W0 * np.exp(-2j * np.pi * 0.37 / max(N, M))
    A = A0 * np.exp(2j * np.pi * 0.0123)
    xd = to_dev(x, dev)
    say(f"case: FP64 czt N={N} M={M} A0={A0} W0={W0} {dtype}")
    if (A0, W0) != (1.0, 1.0) and N > 1:
        with pytest.raises(tz.ThzError) as e:   # beyond the FP32 tables
            tz.czt(xd, M, W, A)
        assert e.value.status == tz.TZ_EUNSUPPORTED
    X = tz.czt(xd, M, W, A, precision="fp64").cpu().numpy()
    assert X.dtype == np.complex128
    ref = orc.czt(x.astype(np.float64), M, W, A)
    assert np.isfinite(X).all()
    err = np.abs(X - ref) / np.abs(ref)
    say(f"  max per-bin relative error {err.max():.3e}; |X| spans {np.abs(ref).min():.1e} .. {np.abs(ref).max():.1e}")
    assert err.max() <= 1e-9


def test_czt_fp64_plan_and_limits(tz, dev):
    x = to_dev(np.random.default_rng(5).standard_normal((2, 700)).astype(np.float32), dev)
    W, A = 1.0005 * np.exp(-0.003j), 0.999 * np.exp(0.1j)
    one = tz.czt(x, 600, W, A, precision="fp64").cpu().numpy()
    plan = tz.Plan("czt", N=700, batch=2, M=600, W=W, A=A, precision="fp64")
    assert plan.workspace_bytes == 0
    import torch
    out = torch.empty((2, 600), dtype=torch.complex128, device=dev)
    plan.execute(x, out)
    assert np.array_equal(out.cpu().numpy(), one)
    plan.close()
    with pytest.raises(tz.ThzError) as e:          # terms reach e^9950: outside FP64
        tz.czt(to_dev(np.ones((1, 1000), np.float32), dev), 1000, 1.01, 1.0, precision="fp64")
    assert e.value.status == tz.TZ_EUNSUPPORTED
    with pytest.raises(tz.ThzError) as e:          # FP64 is czt() only
        tz.czt_band_exact(x, 500, 20 * 10**12, 2 * 10**11, 25 * 10**11, precision="fp64")
    assert e.value.status == tz.TZ_EUNSUPPORTED
    with pytest.raises(tz.ThzError) as e:
        tz.zoom_fft(x, 20e12, 0.2e12, 2.5e12, 500, 6, precision="fp64")
    assert e.value.status == tz.TZ_EUNSUPPORTED


def test_czt_spiral_too_steep(tz, dev):
    x = to_dev(np.ones((1, 3000), np.float32), dev)
    with pytest.raises(tz.ThzError) as e:
        tz.czt(x, 3000, 1.001 * np.exp(-0.001j), 1.0)       # spread ~ e^9000
    assert e.value.status == tz.TZ_EUNSUPPORTED
