"""Seeded synthetic THz-TDS traces (inputs only; no spectral-estimation code).

The paper's measured traces (Section 3.2: T_s = 100 fs, N = 500) are not
available, so every workload uses synthetic stand-ins built from closed forms
in the time domain, in float64 with numpy's PCG64 generator:

* reference pulse: derivative of a Gaussian, peak-normalised,
  p(t) = -(dt/sigma) exp(-dt^2 / (2 sigma^2)) e^{1/2},  dt = t - t0;
* sample trace: the reference delayed by tau, scaled by g and passed through
  1-3 Lorentzian absorption lines.  A line of depth a, centre f_i and FWHM
  gamma has the transmission
      H_i(f) = 1 - a [ (gamma/2)/(gamma/2 + j(f - f_i)) + (gamma/2)/(gamma/2 + j(f + f_i)) ],
  whose impulse response is delta(t) plus causal damped exponentials.  The
  product of the lines is expanded in partial fractions over its poles and
  the pulse is convolved with each exponential in closed form (Faddeeva
  function), so no transform is used to build the inputs;
* white Gaussian noise at 60 dB SNR, sigma_n = rms(trace) * 10^(-60/20).

The random numbers are drawn in a fixed order from ``np.random.default_rng``
seeded per workload, so the oracle and the GPU path see identical inputs.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import wofz

PS = 1e-12
THZ = 1e12
GHZ = 1e9

SIGMA = 0.3 * PS
_KNORM = math.exp(0.5)  # makes max |p(t)| = 1


# --------------------------------------------------------------------------
# workload descriptions (sizes, bands, seeds)
# --------------------------------------------------------------------------
WORKLOADS = {
    0: dict(name="single-trace-fp64", B=1, N=1024, fs=20 * THZ, t0=15 * PS, seed=1000,
            dtype="f64", fft_nzeros=16384 - 1024,
            czt=dict(M=1024, f1=0.1 * THZ, f2=3.0 * THZ),
            zoom=dict(M=1024, f1=0.1 * THZ, f2=3.0 * THZ, D=8, taps=63)),
    1: dict(name="batched-fp32-pairs", B=8192, N=4096, fs=20 * THZ, t0=15 * PS, seed=1001,
            dtype="f32", fft_nzeros=65536 - 4096,
            czt=dict(M=4096, f1=0.2 * THZ, f2=2.5 * THZ),
            zoom=dict(M=4096, f1=0.2 * THZ, f2=2.5 * THZ, D=6, taps=63)),
    3: dict(name="uneven-batch", B=20000, fs=20 * THZ, t0=15 * PS, seed=1003, dtype="f32",
            Nmin=512, Nmax=16384, Mmin=256, Mmax=8192, taps=63),
    4: dict(name="long-scans", B=256, N=1 << 20, fs=100 * THZ, seed=1004, dtype="f32",
            czt=dict(M=1 << 18, f1=0.05 * THZ, f2=0.10 * THZ),
            zoom=dict(M=1 << 18, f1=0.05 * THZ, f2=0.10 * THZ, D=64, taps=255)),
}


# --------------------------------------------------------------------------
# closed-form pieces
# --------------------------------------------------------------------------
def pulse(dt: np.ndarray, sigma: float = SIGMA) -> np.ndarray:
    """Peak-normalised derivative-of-Gaussian THz pulse at time offset dt."""
    u = dt / sigma
    return -u * np.exp(-0.5 * u * u) * _KNORM


def _pulse_through_exp(dt: np.ndarray, beta: np.ndarray, sigma: float = SIGMA) -> np.ndarray:
    """(p * e^{-beta t} u(t))(dt) for complex beta with Re(beta) > 0.

    With G(t) = exp(-t^2/(2 sigma^2)) and p = sigma K G', the convolution is
    sigma K (G - beta E), E = G * e^{-beta t}u(t) = sigma sqrt(pi/2)
    exp(-beta dt + beta^2 sigma^2/2) erfc((beta sigma^2 - dt)/(sigma sqrt 2)).
    erfc is written through the Faddeeva function w on the branch where
    |w| <= 1, so nothing overflows.  dt and beta broadcast together."""
    s = sigma
    z = (beta * s * s - dt) / (s * math.sqrt(2.0))
    g = np.exp(-0.5 * (dt / s) ** 2)
    pos = z.real >= 0
    e = np.empty(np.broadcast(dt, beta).shape, dtype=np.complex128)
    zp = np.where(pos, z, 0.0)
    zn = np.where(pos, 0.0, z)
    e_pos = g * wofz(1j * zp)
    tail = np.exp(np.where(pos, 0.0, -beta * dt + 0.5 * beta * beta * s * s))
    e_neg = 2.0 * tail - g * wofz(-1j * zn)
    e = np.where(pos, e_pos, e_neg) * (s * math.sqrt(math.pi / 2.0))
    return s * _KNORM * (g - beta * e)


def line_poles(f0: np.ndarray, fwhm: np.ndarray, depth: np.ndarray):
    """Poles (in s = j 2 pi f) and residues of prod_i H_i(f) for one trace.

    Each line gives poles s = -pi gamma +- j 2 pi f_i with the factor
    1 - a pi gamma [1/(s - p+) + 1/(s - p-)].  Returns (poles, residues) so
    that prod_i H_i = 1 + sum_p c_p / (s - p)."""
    poles, owners = [], []
    for i in range(len(f0)):
        for sgn in (+1, -1):
            poles.append(-math.pi * fwhm[i] + sgn * 2j * math.pi * f0[i])
            owners.append(i)
    poles = np.array(poles)

    def factor(i, s):
        a, g = depth[i], fwhm[i]
        pp = -math.pi * g + 2j * math.pi * f0[i]
        pm = -math.pi * g - 2j * math.pi * f0[i]
        return 1.0 - a * math.pi * g * (1.0 / (s - pp) + 1.0 / (s - pm))

    res = []
    for p, i in zip(poles, owners):
        c = -depth[i] * math.pi * fwhm[i]
        for l in range(len(f0)):
            if l != i:
                c *= factor(l, p)
        res.append(c)
    return poles, np.array(res)


def sample_trace(t: np.ndarray, tc: float, gain: float, f0, fwhm, depth) -> np.ndarray:
    """Reference pulse centred at tc, scaled by gain, through the lines."""
    dt = t - tc
    out = pulse(dt)
    poles, res = line_poles(np.asarray(f0), np.asarray(fwhm), np.asarray(depth))
    for p, c in zip(poles, res):
        out = out + (c * _pulse_through_exp(dt, -p)).real
    return gain * out


def add_noise(x: np.ndarray, rng, snr_db: float = 60.0) -> np.ndarray:
    rms = np.sqrt(np.mean(x * x, axis=-1, keepdims=True))
    return x + rng.standard_normal(x.shape) * rms * 10.0 ** (-snr_db / 20.0)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def single_trace(N=1024, fs=20 * THZ, t0=15 * PS, seed=1000, snr_db=60.0) -> np.ndarray:
    """One reference trace [1, N] float64 (the single-trace workload)."""
    rng = np.random.default_rng(seed)
    t = np.arange(N) / fs
    x = pulse(t - t0)[None, :]
    return add_noise(x, rng, snr_db)


def pairs(n_pairs: int, N: int = 4096, fs: float = 20 * THZ, t0: float = 15 * PS,
          seed: int = 1001, snr_db: float = 60.0, dtype=np.float32):
    """Sample/reference pairs [2*n_pairs, N]: row 2i is reference i, row 2i+1
    its sample.  Reference: pulse at t0 + U(-0.1, 0.1) ps.  Sample: the same
    pulse delayed U[2, 8] ps, scaled U[0.3, 0.9], through U{1..3} Lorentzian
    lines with f_i ~ U[0.3, 2.5] THz, FWHM ~ U[20, 80] GHz, depth ~ U[0.2, 0.8]."""
    rng = np.random.default_rng(seed)
    t = np.arange(N) / fs
    jitter = rng.uniform(-0.1 * PS, 0.1 * PS, n_pairs)
    delay = rng.uniform(2 * PS, 8 * PS, n_pairs)
    gain = rng.uniform(0.3, 0.9, n_pairs)
    nlines = rng.integers(1, 4, n_pairs)
    f0 = rng.uniform(0.3 * THZ, 2.5 * THZ, (n_pairs, 3))
    fw = rng.uniform(20 * GHZ, 80 * GHZ, (n_pairs, 3))
    dp = rng.uniform(0.2, 0.8, (n_pairs, 3))
    out = np.empty((2 * n_pairs, N), dtype=np.float64)
    for i in range(n_pairs):
        tc = t0 + jitter[i]
        out[2 * i] = pulse(t - tc)
        k = nlines[i]
        out[2 * i + 1] = sample_trace(t, tc + delay[i], gain[i], f0[i, :k], fw[i, :k], dp[i, :k])
    out = add_noise(out, rng, snr_db)
    return out.astype(dtype, copy=False)


def pairs_meta(n_pairs: int, seed: int = 1001):
    """The per-pair parameters drawn by ``pairs`` (same order), for tests."""
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-0.1 * PS, 0.1 * PS, n_pairs)
    delay = rng.uniform(2 * PS, 8 * PS, n_pairs)
    gain = rng.uniform(0.3, 0.9, n_pairs)
    nlines = rng.integers(1, 4, n_pairs)
    f0 = rng.uniform(0.3 * THZ, 2.5 * THZ, (n_pairs, 3))
    return dict(jitter=jitter, delay=delay, gain=gain, nlines=nlines, f0=f0)


def echoes(B: int = 256, N: int = 1 << 20, fs: float = 100 * THZ, seed: int = 1004,
           snr_db: float = 60.0, dtype=np.float32, rows=None) -> np.ndarray:
    """Long scans: U{3..8} pulses per trace at U[0.05, 0.95] x window with
    amplitudes U[0.05, 1] plus noise.  `rows` selects a subset of the B traces
    (the draws for all B traces are made, so a subset is identical to the
    matching rows of the full batch)."""
    rng = np.random.default_rng(seed)
    window = N / fs
    npulse = rng.integers(3, 9, B)
    pos = rng.uniform(0.05, 0.95, (B, 8)) * window
    amp = rng.uniform(0.05, 1.0, (B, 8))
    noise_seeds = rng.integers(0, 2**63 - 1, B)
    rows = range(B) if rows is None else rows
    rows = list(rows)
    out = np.zeros((len(rows), N), dtype=np.float64)
    half = int(math.ceil(12 * SIGMA * fs))
    for j, b in enumerate(rows):
        for p in range(npulse[b]):
            c = int(round(pos[b, p] * fs))
            lo, hi = max(0, c - half), min(N, c + half + 1)
            n = np.arange(lo, hi)
            out[j, lo:hi] += amp[b, p] * pulse(n / fs - pos[b, p])
        r = np.random.default_rng(noise_seeds[b])
        out[j] = add_noise(out[j][None, :], r, snr_db)[0]
    return out.astype(dtype, copy=False)


def raster(B: int, pixels, N: int, fs: float = 20 * THZ, t0: float = 15 * PS, seed: int = 1005,
           snr_db: float = 60.0, dtype=np.float32) -> np.ndarray:
    """THz images for the multi-dimensional transforms: B reflection raster
    scans over `pixels` = (nx,) or (ny, nx) positions, [B, *pixels, N].  Each
    pixel's trace is the reference pulse delayed by a surface-height map and
    scaled by a reflectance map.  Per scan, with pixel coordinates p in
    [0, 1) per axis: delay t0 + sum of 4 Gaussian bumps (centres U[0, 1],
    widths U[0.05, 0.3], heights U[-1, 1] ps); reflectance
    0.6 + 0.4 cos(2 pi (k . p + phi)) with k ~ U[2, 12] per axis (a grating)
    and phi ~ U[0, 1); noise at snr_db per trace."""
    rng = np.random.default_rng(seed)
    pixels = tuple(int(v) for v in pixels)
    d = len(pixels)
    cen = rng.uniform(0.0, 1.0, (B, 4, d))
    wid = rng.uniform(0.05, 0.3, (B, 4))
    hgt = rng.uniform(-1.0, 1.0, (B, 4)) * PS
    kv = rng.uniform(2.0, 12.0, (B, d))
    phi = rng.uniform(0.0, 1.0, B)
    noise_seeds = rng.integers(0, 2**63 - 1, B)
    grids = np.meshgrid(*[np.arange(n) / n for n in pixels], indexing="ij")
    P = np.stack([g.ravel() for g in grids], axis=-1)  # [npix, d]
    t = np.arange(N) / fs
    out = np.empty((B, P.shape[0], N), dtype=dtype)
    for b in range(B):
        r2 = ((P[:, None, :] - cen[b][None, :, :]) ** 2).sum(-1)  # [npix, 4]
        tau = t0 + (hgt[b] * np.exp(-r2 / (2 * wid[b] ** 2))).sum(-1)
        refl = 0.6 + 0.4 * np.cos(2 * np.pi * (P @ kv[b] + phi[b]))
        nr = np.random.default_rng(noise_seeds[b])
        for lo in range(0, P.shape[0], 256):
            hi = min(P.shape[0], lo + 256)
            rows = refl[lo:hi, None] * pulse(t[None, :] - tau[lo:hi, None])
            out[b, lo:hi] = add_noise(rows, nr, snr_db)
    return out.reshape((B,) + pixels + (N,))


def uneven(B: int = 20000, fs: float = 20 * THZ, t0: float = 15 * PS, seed: int = 1003,
           Nmin: int = 512, Nmax: int = 16384, Mmin: int = 256, Mmax: int = 8192,
           taps: int = 63, snr_db: float = 60.0, dtype=np.float32):
    """Uneven batch: per-trace length, band, bin count and method.

    N ~ U{Nmin..Nmax}; f1 ~ U[0.05, 1] THz and f2 - f1 ~ U[0.1, 2] THz, both
    rounded to whole MHz; M ~ U{Mmin..Mmax}; method CZT or Zoom with
    probability 1/2; zoom decimation D = max(1, floor(fs / (1.25 (f2 - f1)))).
    Each trace is a reference pulse or a sample (probability 1/2) as in
    ``pairs``.  Returns (x_flat, offs, jobs) with jobs a list of dicts."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(Nmin, Nmax + 1, B)
    f1 = np.round(rng.uniform(0.05 * THZ, 1.0 * THZ, B) / 1e6) * 1e6
    bw = np.round(rng.uniform(0.1 * THZ, 2.0 * THZ, B) / 1e6) * 1e6
    Ms = rng.integers(Mmin, Mmax + 1, B)
    kind = rng.integers(0, 2, B)  # 0 = czt, 1 = zoom
    is_sample = rng.integers(0, 2, B)
    jitter = rng.uniform(-0.1 * PS, 0.1 * PS, B)
    delay = rng.uniform(2 * PS, 8 * PS, B)
    gain = rng.uniform(0.3, 0.9, B)
    nlines = rng.integers(1, 4, B)
    lf0 = rng.uniform(0.3 * THZ, 2.5 * THZ, (B, 3))
    lfw = rng.uniform(20 * GHZ, 80 * GHZ, (B, 3))
    ldp = rng.uniform(0.2, 0.8, (B, 3))
    offs = np.zeros(B + 1, dtype=np.int64)
    offs[1:] = np.cumsum(Ns)
    x = np.empty(int(offs[-1]), dtype=np.float64)
    jobs = []
    for b in range(B):
        N = int(Ns[b])
        t = np.arange(N) / fs
        tc = t0 + jitter[b]
        if is_sample[b]:
            k = nlines[b]
            tr = sample_trace(t, tc + delay[b], gain[b], lf0[b, :k], lfw[b, :k], ldp[b, :k])
        else:
            tr = pulse(t - tc)
        x[offs[b]:offs[b + 1]] = tr
        f2 = f1[b] + bw[b]
        D = max(1, int(math.floor(fs / (1.25 * bw[b])))) if kind[b] else 1
        jobs.append(dict(kind="zoom" if kind[b] else "czt", N=N, M=int(Ms[b]),
                         f1=float(f1[b]), f2=float(f2), D=D, taps=taps, fs=fs))
    # noise per trace, drawn in trace order
    for b in range(B):
        seg = x[offs[b]:offs[b + 1]]
        x[offs[b]:offs[b + 1]] = add_noise(seg[None, :], rng, snr_db)[0]
    return x.astype(dtype, copy=False), offs, jobs
