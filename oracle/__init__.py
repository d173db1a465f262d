"""FP64 CPU oracle for zero-padded FFT, chirp-Z transform and Zoom FFT.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the HIP library (``paper_2108_03948_amd``) and never imports it.

Each function is a thin ctypes wrapper over ``oracle.c`` (plain direct
summation in double precision, built with gcc + OpenMP); the docstrings cite
the paper passage each one follows.  Parity of the oracle itself is pinned by
``tests/test_oracle_pins.py`` against closed forms, library routines
(numpy.fft, scipy.signal.czt, scipy.signal.lfilter), mpmath brute force and the
values the paper prints (``tests/golden/``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP, FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            lib.orc_fft_zeropad.argtypes = [_pd, _i64, _i64, _i64, _i64, _pi, _i64, _pd]
            lib.orc_czt.argtypes = [_pd, ctypes.c_int, _i64, _i64, _i64, _dbl, _dbl, _dbl, _dbl, _pi, _i64, _pd]
            lib.orc_czt_band_exact.argtypes = [_pd, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _pi, _i64, _pd]
            lib.orc_zoom_taps.argtypes = [_i64, _dbl, _pd]
            lib.orc_zoom_frontend.argtypes = [_pd, ctypes.c_int, _i64, _i64, _i64, _dbl, _dbl, _dbl, _i64, _pd, _i64, _pd]
            lib.orc_zoom_short_dft.argtypes = [_pd, _i64, _i64, _i64, _i64, _pi, _i64, _pd]
            lib.orc_ifft.argtypes = [_pd, _i64, _i64, _i64, _pi, _i64, _pd]
            lib.orc_zoom_K.argtypes = [_dbl, _dbl, _dbl, _i64, _i64]
            lib.orc_zoom_K.restype = _i64
            for f in ("orc_fft_zeropad", "orc_czt", "orc_czt_band_exact", "orc_ifft", "orc_zoom_taps",
                      "orc_zoom_frontend", "orc_zoom_short_dft"):
                getattr(lib, f).restype = None
            _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_pd)


def _bins(bins, default_count):
    if bins is None:
        bins = np.arange(default_count, dtype=np.int64)
    return np.ascontiguousarray(np.asarray(bins, dtype=np.int64))


def _traces(x):
    x = np.asarray(x)
    if x.ndim == 1:
        x = x[None, :]
    return x


def _as_real(x):
    return np.ascontiguousarray(_traces(x), dtype=np.float64)


def _out(B, nb):
    return np.zeros((B, nb), dtype=np.complex128)


def fft_zeropad(x, n_zeros: int, bins=None) -> np.ndarray:
    """Zero-padded DFT, Section 2.1 eqs. (2), (3), (5):
    X[k] = sum_{n<N} x[n] exp(-j 2 pi k n / (N + n_zeros)).  Real x [B, N]."""
    lib = _load()
    x = _as_real(x)
    B, N = x.shape
    nfft = N + int(n_zeros)
    b = _bins(bins, nfft)
    out = _out(B, b.size)
    lib.orc_fft_zeropad(_p(x), N, B, N, int(n_zeros), b.ctypes.data_as(_pi), b.size,
                        out.view(np.float64).ctypes.data_as(_pd))
    return out


def czt(x, M: int, W: complex, A: complex, bins=None) -> np.ndarray:
    """Chirp-Z transform, Section 2.3 eq. (11): X[k] = sum_n x[n] A^-n W^(kn),
    k < M.  x real or complex, [B, N]."""
    lib = _load()
    x = _traces(x)
    is_c = np.iscomplexobj(x)
    xa = np.ascontiguousarray(x, dtype=np.complex128 if is_c else np.float64)
    B, N = xa.shape
    b = _bins(bins, M)
    out = _out(B, b.size)
    W = complex(W)
    A = complex(A)
    lib.orc_czt(xa.view(np.float64).ctypes.data_as(_pd) if is_c else _p(xa), int(is_c), N, B, N,
                W.real, W.imag, A.real, A.imag, b.ctypes.data_as(_pi), b.size,
                out.view(np.float64).ctypes.data_as(_pd))
    return out


def ifft(X, samples=None) -> np.ndarray:
    """Inverse DFT closing the convolution of eq. (12) (and timed on its own
    in Section 4): x[n] = (1/N) sum_{k<N} X[k] exp(+j 2 pi k n / N).
    X complex [B, N]; only the listed samples n are formed."""
    lib = _load()
    Xa = np.ascontiguousarray(_traces(X), dtype=np.complex128)
    B, N = Xa.shape
    s = _bins(samples, N)
    out = _out(B, s.size)
    lib.orc_ifft(Xa.view(np.float64).ctypes.data_as(_pd), N, B, N, s.ctypes.data_as(_pi), s.size,
                 out.view(np.float64).ctypes.data_as(_pd))
    return out


def transfer(x, M: int, W: complex, A: complex, bins=None) -> np.ndarray:
    """Frequency response of sample/reference pairs (Section 1: the material's
    response is the sample's spectrum relative to the reference's), on the CZT
    contour of eq. (11): rows 2p (reference) and 2p+1 (sample) of x give
    H[p][k] = X_{2p+1}[k] / X_{2p}[k], each X the direct FP64 sum of czt()."""
    X = czt(x, M, W, A, bins)
    if X.shape[0] % 2:
        raise ValueError("transfer needs reference/sample row pairs")
    return X[1::2] / X[0::2]


def czt_band_exact(x, M: int, fs_hz: int, f1_hz: int, f2_hz: int, bins=None) -> np.ndarray:
    """CZT over [f1, f2) with M bins, eqs. (22)-(24), integer-hertz band with
    exact rational phases.  Real x [B, N]."""
    lib = _load()
    x = _as_real(x)
    B, N = x.shape
    b = _bins(bins, M)
    out = _out(B, b.size)
    lib.orc_czt_band_exact(_p(x), N, B, N, int(M), int(fs_hz), int(f1_hz), int(f2_hz),
                           b.ctypes.data_as(_pi), b.size, out.view(np.float64).ctypes.data_as(_pd))
    return out


def zoom_taps(T: int, nu_c: float) -> np.ndarray:
    """Hamming-windowed sinc low-pass (stands in for eq. (8)), sum h = 1."""
    lib = _load()
    h = np.zeros(int(T), dtype=np.float64)
    lib.orc_zoom_taps(int(T), float(nu_c), _p(h))
    return h


def zoom_K(fs: float, f1: float, f2: float, M: int, D: int) -> int:
    """Short-DFT length K = round(M fs / (D (f2 - f1)))."""
    return int(_load().orc_zoom_K(float(fs), float(f1), float(f2), int(M), int(D)))


def zoom_frontend(x, fs: float, f1: float, f2: float, D: int, h) -> np.ndarray:
    """Zoom steps eqs. (6), (7), (10): mix f_N to DC, low-pass, keep every D-th
    output.  x real or complex [B, N]; returns u [B, ceil(N/D)] complex."""
    lib = _load()
    x = _traces(x)
    is_c = np.iscomplexobj(x)
    xa = np.ascontiguousarray(x, dtype=np.complex128 if is_c else np.float64)
    B, N = xa.shape
    h = np.ascontiguousarray(h, dtype=np.float64)
    LD = (N + D - 1) // D
    u = np.zeros((B, LD), dtype=np.complex128)
    lib.orc_zoom_frontend(xa.view(np.float64).ctypes.data_as(_pd) if is_c else _p(xa), int(is_c), N, B, N,
                          float(fs), float(f1), float(f2), int(D), _p(h), h.size,
                          u.view(np.float64).ctypes.data_as(_pd))
    return u


def zoom_short_dft(u, K: int, M: int, bins=None) -> np.ndarray:
    """Zoom step 4: X[k] = sum_m u[m] exp(-j 2 pi (k - M//2) m / K), k < M."""
    lib = _load()
    u = np.ascontiguousarray(_traces(u), dtype=np.complex128)
    B, LD = u.shape
    b = _bins(bins, M)
    out = _out(B, b.size)
    lib.orc_zoom_short_dft(u.view(np.float64).ctypes.data_as(_pd), B, LD, int(K), int(M),
                           b.ctypes.data_as(_pi), b.size, out.view(np.float64).ctypes.data_as(_pd))
    return out


def zoom_fft(x, fs: float, f1: float, f2: float, M: int, D: int, taps: int = 63,
             cutoff_hz: float | None = None, bins=None) -> np.ndarray:
    """Whole Zoom FFT (Section 2.2): taps, front end, short DFT."""
    nu_c = (fs / (2.0 * D) if cutoff_hz is None else cutoff_hz) / fs
    h = zoom_taps(taps, nu_c)
    u = zoom_frontend(x, fs, f1, f2, D, h)
    K = zoom_K(fs, f1, f2, M, D)
    return zoom_short_dft(u, K, M, bins)


def _along(x, axis: int, fn):
    """Apply fn (a map of [rows, n] to [rows, m]) to every line of x along axis."""
    y = np.moveaxis(np.asarray(x), axis, -1)
    lead = y.shape[:-1]
    z = fn(y.reshape(-1, y.shape[-1]))
    return np.moveaxis(z.reshape(lead + (z.shape[-1],)), -1, axis)


def czt_nd(x, axes, bins=None) -> np.ndarray:
    """Multi-dimensional CZT, the 2-D and 3-D transforms Section 5 names:
    X[k_0..k_{d-1}] = sum_n x[n_0..n_{d-1}] prod_a A_a^-n_a W_a^(k_a n_a).
    Each factor of the kernel depends on one index pair, so the d-fold sum is
    the one-dimensional CZT of eq. (11) taken along every axis in turn.
    x [B, N_0, ..., N_{d-1}] real or complex; axes = [(M_a, W_a, A_a), ...]
    for a = 0..d-1; returns [B, M_0, ..., M_{d-1}] complex.  bins = one
    index list per axis evaluates only that grid of bins."""
    x = np.asarray(x)
    d = len(axes)
    if x.ndim != d + 1:
        raise ValueError("x must be [B] + one dimension per axis")
    y = x
    for a, (M, W, A) in enumerate(axes):
        b = None if bins is None else bins[a]
        y = _along(y, a + 1, lambda r, M=M, W=W, A=A, b=b: czt(r, M, W, A, b))
    return y


def zoom_fft_nd(x, axes, taps: int = 63, bins=None) -> np.ndarray:
    """Multi-dimensional Zoom FFT (Section 2.2 along every axis, for the 2-D
    and 3-D transforms of Section 5): the mix, low-pass, decimation and short
    DFT of each axis act on that axis' index alone, so the transform is the
    one-dimensional Zoom FFT taken along every axis in turn (real input on
    the first, complex on the later ones).  axes = [(fs, f1, f2, M, D, fc),
    ...] with fc the cut-off in Hz (None = fs / (2 D)); x [B, N_0, ...];
    returns [B, M_0, ...] complex (bins: as czt_nd)."""
    x = np.asarray(x)
    d = len(axes)
    if x.ndim != d + 1:
        raise ValueError("x must be [B] + one dimension per axis")
    y = x
    for a, ax in enumerate(axes):
        fs, f1, f2, M, D = ax[:5]
        fc = ax[5] if len(ax) > 5 else None
        b = None if bins is None else bins[a]
        y = _along(y, a + 1, lambda r, fs=fs, f1=f1, f2=f2, M=M, D=D, fc=fc, b=b:
                   zoom_fft(r, fs, f1, f2, M, D, taps, fc, b))
    return y
