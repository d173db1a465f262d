"""GPU parity of the multi-dimensional transforms (czt_nd, zoom_fft_nd)
through the C-ABI against the FP64 oracle.

Shape and contour cases (random contours on every axis) take seeded white
noise; the zoom cases and the full-size cases take THz raster scans
(synth.raster): B-scans [B, pixels, samples] for 2-D and image cubes
[B, ny, nx, samples] for 3-D, with bands that hold the scans' energy.  Bar:
relative L2 error per array <= 1e-6 (the FP32 bar of the one-dimensional
transforms).  Shapes are ragged against the 64 x 64 transpose tiles, include
degenerate axes (N = 1, M = 1), strided and FP64 input, a spiral axis, and,
at full size, several chunks of arrays checked on sampled bin grids.
"""
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


def to_dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def assert_arrays_close(gpu, ref, tol=TOL_FP32, what=""):
    B = ref.shape[0]
    g = np.asarray(gpu).reshape(B, -1)
    r = np.asarray(ref).reshape(B, -1)
    assert np.all(np.linalg.norm(r, axis=1) > 0), f"{what}: a reference array is zero"
    err = np.linalg.norm(g - r, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)
    say(f"  {what}: max rel L2 {err.max():.3e} over {B} arrays")
    assert np.all(np.isfinite(g))
    assert err.max() <= tol, f"{what}: rel L2 {err.max():.3e} > {tol}"


def scans(B, pixels, N, seed, dtype=np.float32):
    """Raster scans with the pulse inside the window of every trace length."""
    return synth.raster(B, pixels, N, t0=0.4 * N / 20e12, seed=seed, dtype=dtype)


def white(B, pixels, N, seed, dtype=np.float32):
    """Seeded white noise [B, *pixels, N]: every contour, wherever it lies,
    sees a typical share of the input energy (shape and contour cases)."""
    return np.random.default_rng(seed).standard_normal((B,) + tuple(pixels) + (N,)).astype(dtype)


def unit(rng):
    return np.exp(2j * np.pi * rng.uniform(0, 1))


def random_axes(rng, Ms):
    return [(M, unit(rng), unit(rng)) for M in Ms]


# ---------------------------------------------------------------------------
# czt_nd
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B,pixels,N,Ms", [
    (3, (40,), 56, (24, 72)),        # both passes inside one transpose tile
    (2, (130,), 70, (129, 65)),      # ragged tiles on both sides
    (2, (1,), 33, (1, 20)),          # one-pixel axis, one bin
    (2, (300,), 17, (5, 400)),       # M far above N on one axis
    (1, (64,), 1, (64, 3)),          # one-sample traces
])
def test_czt_nd_2d(tz, dev, orc, B, pixels, N, Ms):
    rng = np.random.default_rng(sum(Ms) + N)
    x = white(B, pixels, N, seed=2000 + N)
    axes = random_axes(rng, Ms)
    say(f"case: czt_nd 2-D B={B} {pixels[0]}x{N} -> {Ms}")
    X = tz.czt_nd(to_dev(x, dev), axes).cpu().numpy()
    assert X.shape == (B,) + Ms
    assert_arrays_close(X, orc.czt_nd(x, axes), what=f"czt_nd {pixels[0]}x{N}->{Ms}")


@pytest.mark.parametrize("B,pixels,N,Ms", [
    (2, (12, 20), 36, (10, 16, 30)),
    (1, (64, 48), 100, (70, 40, 64)),
    (2, (3, 1), 5, (2, 1, 7)),
])
def test_czt_nd_3d(tz, dev, orc, B, pixels, N, Ms):
    rng = np.random.default_rng(sum(Ms) + 3 * N)
    x = white(B, pixels, N, seed=2100 + N)
    axes = random_axes(rng, Ms)
    say(f"case: czt_nd 3-D B={B} {pixels}x{N} -> {Ms}")
    X = tz.czt_nd(to_dev(x, dev), axes).cpu().numpy()
    assert X.shape == (B,) + Ms
    assert_arrays_close(X, orc.czt_nd(x, axes), what=f"czt_nd {pixels}x{N}->{Ms}")


def test_czt_nd_1d_is_czt(tz, dev):
    # one axis: the same plan and kernel as czt(), written straight to X
    x = to_dev(synth.pairs(8, N=1000), dev)
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 700)
    say("case: czt_nd 1-D vs czt, 16 x 1000 -> 700")
    a = tz.czt_nd(x, [(700, W, A)]).cpu().numpy()
    b = tz.czt(x, 700, W, A).cpu().numpy()
    assert np.array_equal(a, b)


def test_czt_nd_strides_fp64_and_spiral_axis(tz, dev, orc):
    import torch
    rng = np.random.default_rng(41)
    x = white(6, (50,), 90, seed=2200, dtype=np.float64)
    Ms = (45, 80)
    axes = [(45, 0.999 * unit(rng), 1.001 * unit(rng)), (80, unit(rng), unit(rng))]
    xd = to_dev(x, dev)[::2]                     # arrays 2 * 50 * 90 elements apart
    full = torch.empty((3, 45 * 80 + 13), dtype=torch.complex64, device=dev)
    out = full[:, : 45 * 80].view(3, 45, 80)     # output arrays padded apart
    say("case: czt_nd 2-D f64, strided arrays in and out, spiral axis 0")
    tz.czt_nd(xd, axes, out=out)
    assert_arrays_close(out.cpu().numpy(), orc.czt_nd(x[::2], axes), what="strided f64 spiral")


def test_czt_nd_full_size_chunks_sampled(tz, dev, orc):
    """B-scans at the size the benchmark times (64 x 512 pixels x 2048
    samples; spatial band [-1/4, 1/4) cycles per pixel on 512 bins, 0.2 -
    2.5 THz on 1024): several chunks of arrays; a 16 x 16 bin grid of three
    arrays, first, middle and last, is checked against the oracle."""
    B, P, N, M0, M1 = 64, 512, 2048, 512, 1024
    x = synth.raster(B, (P,), N, seed=3000)
    W0, A0 = np.exp(-2j * np.pi * 0.5 / M0), np.exp(2j * np.pi * -0.25)
    W1, A1 = tz.czt_band(20e12, 0.2e12, 2.5e12, M1)
    axes = [(M0, W0, A0), (M1, W1, A1)]
    say(f"case: czt_nd 2-D full size {B} x {P} x {N} -> {M0} x {M1}")
    X = tz.czt_nd(to_dev(x, dev), axes).cpu().numpy()
    rng = np.random.default_rng(42)
    b0 = np.sort(rng.choice(M0, 16, replace=False))
    b1 = np.sort(rng.choice(M1, 16, replace=False))
    rows = [0, B // 2 + 3, B - 1]
    ref = orc.czt_nd(x[rows], axes, bins=[b0, b1])
    assert_arrays_close(X[rows][:, b0][:, :, b1], ref, what="full size, sampled bins")


def test_czt_nd_cube_sampled(tz, dev, orc):
    """One image cube, 256 x 256 pixels x 1024 samples, to 256 x 256 x 512
    bins; an 8 x 8 x 8 bin grid against the oracle."""
    x = synth.raster(1, (256, 256), 1024, seed=3100)
    Wp, Ap = np.exp(-2j * np.pi * 0.5 / 256), np.exp(2j * np.pi * -0.25)
    Wt, At = tz.czt_band(20e12, 0.2e12, 2.5e12, 512)
    axes = [(256, Wp, Ap), (256, Wp, Ap), (512, Wt, At)]
    say("case: czt_nd 3-D cube 256 x 256 x 1024 -> 256 x 256 x 512")
    X = tz.czt_nd(to_dev(x, dev), axes).cpu().numpy()
    rng = np.random.default_rng(43)
    bins = [np.sort(rng.choice(M, 8, replace=False)) for M in (256, 256, 512)]
    ref = orc.czt_nd(x, axes, bins=bins)
    assert_arrays_close(X[:, bins[0]][:, :, bins[1]][:, :, :, bins[2]], ref, what="cube, sampled bins")


def test_czt_nd_arrays_larger_than_a_chunk(tz, dev, orc):
    """Arrays whose intermediates exceed the cache-sized chunk run one per
    chunk (here 2 arrays of 3000 x 3000 -> 3000 x 2500), written into padded
    output rows whose padding must stay untouched."""
    import torch
    B, N0, N1, M0, M1 = 2, 3000, 3000, 3000, 2500
    rng = np.random.default_rng(46)
    x = white(B, (N0,), N1, seed=2500)
    axes = random_axes(rng, (M0, M1))
    full = torch.full((B, M0 * M1 + 512), complex(5.0, 5.0), dtype=torch.complex64, device=dev)
    out = full[:, : M0 * M1].view(B, M0, M1)
    say(f"case: czt_nd 2-D {B} x {N0} x {N1} -> {M0} x {M1}, one array per chunk, padded output")
    tz.czt_nd(to_dev(x, dev), axes, out=out)
    f = full.cpu().numpy()
    assert np.all(f[:, M0 * M1:] == np.complex64(complex(5.0, 5.0)))
    b0 = np.sort(rng.choice(M0, 12, replace=False))
    b1 = np.sort(rng.choice(M1, 12, replace=False))
    X = f[:, : M0 * M1].reshape(B, M0, M1)
    assert_arrays_close(X[:, b0][:, :, b1], orc.czt_nd(x, axes, bins=[b0, b1]), what="large arrays, sampled")


# ---------------------------------------------------------------------------
# zoom_fft_nd
# ---------------------------------------------------------------------------
# fs (per pixel) and band [f1, f2) in cycles per pixel: centred on the
# spatial spectrum of the scans (gratings of 2 - 12 cycles per field and
# smooth delay maps), as the time-axis band 0.2 - 2.5 THz holds the pulse.
# FP32 rounding follows the energy a transform takes in, so a band that keeps
# a small part of it has a larger error relative to its own output.
SPATIAL = (1.0, -0.125, 0.125)


@pytest.mark.parametrize("B,pixels,N,zax,taps", [
    (2, (200,), 1000, [SPATIAL + (64, 2), (20e12, 0.2e12, 2.5e12, 256, 4)], 63),
    (3, (70,), 300, [SPATIAL + (40, 1), (20e12, 0.5e12, 1.5e12, 100, 8)], 31),
    (1, (33,), 64, [SPATIAL + (1, 3), (20e12, 0.5e12, 1.5e12, 17, 2)], 15),
])
def test_zoom_fft_nd_2d(tz, dev, orc, B, pixels, N, zax, taps):
    x = scans(B, pixels, N, seed=2300 + N)
    say(f"case: zoom_fft_nd 2-D B={B} {pixels[0]}x{N} axes {zax} taps {taps}")
    X = tz.zoom_fft_nd(to_dev(x, dev), zax, taps=taps).cpu().numpy()
    assert X.shape == (B, zax[0][3], zax[1][3])
    assert_arrays_close(X, orc.zoom_fft_nd(x, zax, taps=taps), what=f"zoom_fft_nd {pixels[0]}x{N}")


def test_zoom_fft_nd_3d_cutoffs(tz, dev, orc):
    x = scans(2, (40, 36), 400, seed=2400)
    zax = [SPATIAL + (24, 2, 0.2), SPATIAL + (20, 2), (20e12, 0.2e12, 2.5e12, 128, 3, 3e12)]
    say("case: zoom_fft_nd 3-D 40 x 36 x 400, explicit cut-offs on two axes")
    X = tz.zoom_fft_nd(to_dev(x, dev), zax, taps=63).cpu().numpy()
    ref = orc.zoom_fft_nd(x, [a if len(a) == 6 else a + (None,) for a in zax], taps=63)
    assert_arrays_close(X, ref, what="zoom_fft_nd 3-D")


def test_zoom_fft_nd_full_size_sampled(tz, dev, orc):
    """B-scans 64 x 512 x 2048: spatial zoom D = 3 on 512 bins, 0.2 - 2.5 THz
    zoom D = 6 on 1024 bins, 63 taps; a 16 x 16 bin grid of two arrays."""
    B, P, N = 64, 512, 2048
    x = synth.raster(B, (P,), N, seed=3000)
    zax = [SPATIAL + (512, 3), (20e12, 0.2e12, 2.5e12, 1024, 6)]
    say(f"case: zoom_fft_nd 2-D full size {B} x {P} x {N}")
    X = tz.zoom_fft_nd(to_dev(x, dev), zax, taps=63).cpu().numpy()
    rng = np.random.default_rng(44)
    b0 = np.sort(rng.choice(512, 16, replace=False))
    b1 = np.sort(rng.choice(1024, 16, replace=False))
    rows = [1, B - 2]
    ref = orc.zoom_fft_nd(x[rows], zax, taps=63, bins=[b0, b1])
    assert_arrays_close(X[rows][:, b0][:, :, b1], ref, what="zoom full size, sampled bins")
