"""GPU parity of the inverse DFT (ifft) against the FP64 oracle.

The inverse transform closes the FFT convolution of eq. (12) and is timed on
its own against the FFT in Section 4.  Power-of-two N from 256 to 16384 run
as one FFT per row (conjugate, forward FFT, conjugate, scale); other
7-smooth N from 8 to 20480 as one mixed-radix FFT per row (radices 2, 3, 4,
5, 7, 8; odd lengths included); every other N runs as a CZT with A = 1,
W = e^{+j 2 pi / N} and the 1/N folded into the chirp spectrum.  The cases
cover both ends of the direct range, sizes just outside it, both mixed-radix
row kernels, and every Bluestein shape: single pass (2N - 1 <= 16384), bin
blocks / input segments just past it, and the four-step path (2N - 1 up to a
few times 2^17).  Rows are strided on both sides; large N are checked on
sampled outputs.  A round trip through the zero-padded FFT must return the
trace.  With TZ_HALF the input is the Hermitian half spectrum of real traces
and the output the real traces, checked against the oracle's inverse of the
full Hermitian spectrum.  Tolerance: relative L2 1e-6 per row (FP32 path).
"""
import sys

import numpy as np
import pytest

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


def spectra(B, N, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((B, N)) + 1j * rng.standard_normal((B, N))).astype(np.complex64)


@pytest.mark.parametrize("N", [1, 2, 7, 128, 256, 500, 625, 1009, 1024, 1176, 2646, 3001, 4096, 6615, 8192, 8193,
                               12345, 16384, 16807, 19683, 20000, 65536, 100003])
def test_ifft_matches_oracle(tz, orc, N):
    import torch
    B = 3
    X = spectra(B, N, 500 + N % 1000)
    dev = torch.device("cuda:0")
    # strided rows on both sides: input rows N + 3 apart, output rows N + 5 apart
    Xbig = torch.zeros((B, N + 3), dtype=torch.complex64, device=dev)
    Xbig[:, :N] = torch.from_numpy(X).to(dev)
    obig = torch.full((B, N + 5), complex(9.0, 9.0), dtype=torch.complex64, device=dev)
    direct = 256 <= N <= 16384 and N & (N - 1) == 0
    m = N
    for f in (2, 3, 5, 7):
        while m % f == 0:
            m //= f
    mixed = not direct and m == 1 and 8 <= N <= 20480
    say(f"case: ifft N={N} B={B} " + ("direct FFT" if direct else "mixed radix" if mixed else
                                      f"Bluestein (L, blocks) = {tz.czt_plan_shape(N, N)}"))
    tz.ifft(Xbig[:, :N], out=obig[:, :N])
    torch.cuda.synchronize()
    got = obig.cpu().numpy()
    assert np.all(got[:, N:] == np.complex64(complex(9.0, 9.0))), "wrote past the row"
    samples = np.arange(N) if N <= 4096 else np.unique(np.r_[0, 1, N - 1, np.random.default_rng(N).integers(0, N, 61)])
    ref = orc.ifft(X.astype(np.complex128), samples=samples)
    g = got[:, samples]
    r = np.linalg.norm(g - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    say(f"  max rel L2 {r.max():.3e} over {samples.size} samples per row")
    assert np.isfinite(g).all() and r.max() <= TOL


def test_ifft_full_batch_sampled(tz, orc):
    """8192 spectra of 4096 bins, the size the benchmark times: the first, the
    last and sampled rows in full, and sampled samples of more rows, against
    the oracle; every output finite."""
    import torch
    B, N = 8192, 4096
    X = spectra(B, N, 4242)
    say(f"case: ifft full batch {B} x {N}, sampled check")
    out = tz.ifft(torch.from_numpy(X).cuda())
    assert bool(torch.isfinite(torch.view_as_real(out)).all())
    rng = np.random.default_rng(80)
    rows = np.r_[0, np.sort(rng.choice(np.arange(1, B - 1), 3, replace=False)), B - 1]
    got = out[rows].cpu().numpy()
    ref = orc.ifft(X[rows].astype(np.complex128))
    e = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    more = np.sort(rng.choice(B, 32, replace=False))
    samples = np.unique(np.r_[0, N - 1, rng.integers(0, N, 62)])
    got2 = out[more][:, samples].cpu().numpy()
    ref2 = orc.ifft(X[more].astype(np.complex128), samples=samples)
    e2 = np.linalg.norm(got2 - ref2, axis=1) / np.linalg.norm(ref2, axis=1)
    say(f"  full rows: max rel L2 {e.max():.3e}; sampled samples of 32 rows: {e2.max():.3e}")
    assert e.max() <= TOL and e2.max() <= TOL


@pytest.mark.parametrize("N", [1000, 4096, 30000])
def test_ifft_inverts_fft_zeropad(tz, N):
    """ifft(fft_zeropad(x, 0)) returns the real traces (imaginary part ~ 0)."""
    import torch
    x = np.random.default_rng(N).standard_normal((4, N)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    back = tz.ifft(tz.fft_zeropad(xd, 0)).cpu().numpy()
    r = np.linalg.norm(back - x, axis=1) / np.linalg.norm(x, axis=1)
    say(f"case: ifft(fft_zeropad(x)) N={N}: max rel L2 {r.max():.3e}")
    assert r.max() <= TOL


def hermitian_full(H, N):
    """The full spectrum of N bins whose half H (bins 0 .. N/2) is given:
    bin k > N/2 is conj(H[N - k]); bin 0 and, for even N, bin N/2 keep only
    their real parts."""
    Hc = H.astype(np.complex128).copy()
    Hc[:, 0] = Hc[:, 0].real
    if N % 2 == 0:
        Hc[:, N // 2] = Hc[:, N // 2].real
    full = np.empty((H.shape[0], N), dtype=np.complex128)
    full[:, :N // 2 + 1] = Hc
    k = np.arange(N // 2 + 1, N)
    full[:, k] = np.conj(Hc[:, N - k])
    return full


# Hermitian half spectra to real traces (ifft with TZ_HALF): two rows per
# mixed-radix FFT, so odd batches leave the last FFT with one row; odd and
# even N, the four row-kernel sizes, N = 20480 (the longest), strided rows,
# general half spectra (not from a real trace: bins 0 and N/2 carry
# imaginary parts the inverse must ignore)
@pytest.mark.parametrize("N,B", [(8, 3), (500, 3), (625, 4), (1176, 5), (2646, 2), (6615, 3), (10000, 1),
                                 (16807, 3), (20000, 2), (20480, 3)])
def test_ifft_half_spectrum_matches_oracle(tz, orc, N, B):
    import torch
    nb = N // 2 + 1
    H = spectra(B, nb, 900 + N % 1000)
    dev = torch.device("cuda:0")
    Hbig = torch.zeros((B, nb + 3), dtype=torch.complex64, device=dev)
    Hbig[:, :nb] = torch.from_numpy(H).to(dev)
    obig = torch.full((B, N + 5), 9.0, dtype=torch.float32, device=dev)
    say(f"case: ifft half spectrum N={N} B={B}")
    tz.ifft(Hbig[:, :nb], out=obig[:, :N], half=True, N=N)
    torch.cuda.synchronize()
    got = obig.cpu().numpy()
    assert np.all(got[:, N:] == np.float32(9.0)), "wrote past the row"
    samples = np.arange(N) if N <= 4096 else np.unique(np.r_[0, 1, N - 1, np.random.default_rng(N).integers(0, N, 61)])
    ref = orc.ifft(hermitian_full(H, N), samples=samples)
    assert np.max(np.abs(ref.imag)) <= 1e-12 * max(1.0, np.max(np.abs(ref.real)))  # a real trace
    g = got[:, samples]
    r = np.linalg.norm(g - ref.real, axis=1) / np.linalg.norm(ref.real, axis=1)
    say(f"  max rel L2 {r.max():.3e} over {samples.size} samples per row")
    assert np.isfinite(g).all() and r.max() <= TOL


def test_ifft_half_spectrum_inverts_fft_zeropad(tz):
    """ifft(fft_zeropad(x, z, half=True), half=True) returns the trace padded
    with z zeros (N_fft = 10000, an odd batch)."""
    import torch
    N, z = 4000, 6000
    x = np.random.default_rng(4).standard_normal((5, N)).astype(np.float32)
    back = tz.ifft(tz.fft_zeropad(torch.from_numpy(x).cuda(), z, half=True), half=True, N=N + z).cpu().numpy()
    ref = np.concatenate([x, np.zeros((5, z), np.float32)], axis=1)
    r = np.linalg.norm(back - ref, axis=1) / np.linalg.norm(x, axis=1)
    say(f"case: ifft_half(fft_zeropad_half(x)) N={N} N_fft={N + z}: max rel L2 {r.max():.3e}")
    assert r.max() <= TOL


def test_ifft_half_spectrum_refuses_other_lengths(tz):
    import torch
    H = torch.zeros((1, 6), dtype=torch.complex64, device="cuda")
    with pytest.raises(tz.ThzError, match="7-smooth"):
        tz.ifft(H, half=True, N=11)
    with pytest.raises(tz.ThzError, match="7-smooth"):
        tz.ifft(torch.zeros((1, 20481 // 2 + 1), dtype=torch.complex64, device="cuda"), half=True, N=20481)
