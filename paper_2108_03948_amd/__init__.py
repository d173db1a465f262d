"""Python binding of libthzspec (HIP, gfx950): zero-padded FFT, chirp-Z
transform and Zoom FFT of batched THz-TDS traces.

The binding only marshals arguments: every transform runs in the library's
HIP kernels.  torch is used for device memory and streams.  There is no CPU
fallback: if ``libthzspec.so`` is missing, or a tensor is not on the GPU,
the call raises.

Build the library with ``python -m paper_2108_03948_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "fft_zeropad", "czt", "czt_band_exact", "zoom_fft", "czt_transfer", "ifft", "czt_nd", "zoom_fft_nd",
    "czt_band", "fft_zero_count",
    "czt_points_for_resolution", "zoom_short_length", "czt_plan_shape", "lib", "ThzError",
    "Batch", "Plan", "bin_freqs", "release_plans", "version",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libthzspec.so")

TZ_OK, TZ_EINVAL, TZ_ENOMEM, TZ_EDEVICE, TZ_EUNSUPPORTED, TZ_ETIMEOUT = range(6)
TZ_F32, TZ_F64 = 0, 1
TZ_FP32, TZ_SPLIT_FP16, TZ_SPLIT_BF16, TZ_FP64 = 0, 1, 2, 3
TZ_HALF = 1
TZ_JOB_CZT, TZ_JOB_ZOOM = 0, 1
PRECISIONS = {"fp32": TZ_FP32, "split_fp16": TZ_SPLIT_FP16, "split_bf16": TZ_SPLIT_BF16, "fp64": TZ_FP64}
_STATUS = {1: "TZ_EINVAL", 2: "TZ_ENOMEM", 3: "TZ_EDEVICE", 4: "TZ_EUNSUPPORTED", 5: "TZ_ETIMEOUT"}


class ThzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class tz_c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class tz_opts(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_int64), ("in_stride", ctypes.c_int64), ("out_stride", ctypes.c_int64),
        ("in_dtype", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("fir_taps", ctypes.c_int32), ("fir_cutoff_hz", ctypes.c_double), ("stream", ctypes.c_void_p),
    ]


class tz_job(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("fir_taps", ctypes.c_int32), ("N", ctypes.c_int64),
        ("M", ctypes.c_int64), ("D", ctypes.c_int64), ("fs_hz", ctypes.c_int64),
        ("f1_hz", ctypes.c_int64), ("f2_hz", ctypes.c_int64), ("in_offset", ctypes.c_int64),
        ("out_offset", ctypes.c_int64),
    ]


class tz_czt_axis(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("M", ctypes.c_int64), ("W", tz_c64), ("A", tz_c64)]


class tz_zoom_axis(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int64), ("D", ctypes.c_int64), ("fs", ctypes.c_double),
        ("f1", ctypes.c_double), ("f2", ctypes.c_double), ("fc", ctypes.c_double),
    ]


class tz_plan_params(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("N", ctypes.c_int64), ("M", ctypes.c_int64), ("n_zeros", ctypes.c_int64),
        ("W", tz_c64), ("A", tz_c64), ("fs_hz", ctypes.c_int64), ("f1_hz", ctypes.c_int64),
        ("f2_hz", ctypes.c_int64), ("fs", ctypes.c_double), ("f1", ctypes.c_double), ("f2", ctypes.c_double),
        ("D", ctypes.c_int64),
    ]


TZ_PLAN_KINDS = {"fft_zeropad": 0, "czt": 1, "czt_band_exact": 2, "zoom": 3, "ifft": 4}
TZ_MAX_DIMS = 3

# every symbol declared in include/thzspec.h
EXPORTS = (
    "tz_opts_init", "fft_zeropad", "czt", "czt_band_exact", "czt_transfer", "ifft", "zoom_fft", "czt_nd",
    "zoom_fft_nd", "czt_band",
    "fft_zero_count",
    "czt_points_for_resolution", "zoom_short_length", "czt_plan_shape", "tz_batch_create",
    "tz_batch_launch", "tz_batch_destroy", "tz_batch_describe", "tz_batch_extents", "tz_batch_wait",
    "tz_last_error", "tz_version",
    "tz_release_plans", "tz_plan_create", "tz_plan_workspace", "tz_plan_execute", "tz_plan_execute_static",
    "tz_plan_destroy",
    "tz_bin_freqs", "tz_autotune", "tz_tune_describe",
)

_lock = threading.Lock()
_lib = None


def lib() -> ctypes.CDLL:
    """Load libthzspec.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2108_03948_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        po = ctypes.POINTER(tz_opts)
        L.tz_opts_init.argtypes = [po]
        L.tz_opts_init.restype = None
        L.fft_zeropad.argtypes = [vp, i64, i64, vp, po]
        L.czt.argtypes = [vp, i64, i64, tz_c64, tz_c64, vp, po]
        L.czt_transfer.argtypes = [vp, i64, i64, tz_c64, tz_c64, vp, po]
        L.ifft.argtypes = [vp, i64, vp, po]
        L.czt_band_exact.argtypes = [vp, i64, i64, i64, i64, i64, vp, po]
        L.zoom_fft.argtypes = [vp, i64, dbl, dbl, dbl, i64, i64, vp, po]
        L.czt_nd.argtypes = [vp, ctypes.c_int, ctypes.POINTER(tz_czt_axis), vp, po]
        L.zoom_fft_nd.argtypes = [vp, ctypes.c_int, ctypes.POINTER(tz_zoom_axis), vp, po]
        L.czt_band.argtypes = [dbl, dbl, dbl, i64, ctypes.POINTER(tz_c64), ctypes.POINTER(tz_c64)]
        L.fft_zero_count.argtypes = [dbl, i64, dbl]
        L.fft_zero_count.restype = i64
        L.czt_points_for_resolution.argtypes = [dbl, dbl, dbl, i64]
        L.czt_points_for_resolution.restype = i64
        L.zoom_short_length.argtypes = [dbl, dbl, dbl, i64, i64]
        L.zoom_short_length.restype = i64
        L.czt_plan_shape.argtypes = [i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.tz_batch_create.argtypes = [ctypes.POINTER(tz_job), i64, po, ctypes.POINTER(vp)]
        L.tz_batch_launch.argtypes = [vp, vp, vp, vp]
        L.tz_batch_destroy.argtypes = [vp]
        L.tz_batch_destroy.restype = None
        L.tz_batch_describe.argtypes = [vp, ctypes.c_char_p, i64]
        L.tz_batch_describe.restype = i64
        L.tz_batch_extents.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.tz_batch_wait.argtypes = [vp, dbl]
        L.tz_last_error.restype = ctypes.c_char_p
        L.tz_version.restype = ctypes.c_char_p
        L.tz_release_plans.restype = None
        pp = ctypes.POINTER(tz_plan_params)
        L.tz_plan_create.argtypes = [pp, po, ctypes.POINTER(vp)]
        L.tz_plan_workspace.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.tz_plan_execute.argtypes = [vp, vp, vp, vp, vp]
        L.tz_plan_execute_static.argtypes = [vp, vp, vp, vp]
        L.tz_plan_destroy.argtypes = [vp]
        L.tz_plan_destroy.restype = None
        L.tz_bin_freqs.argtypes = [pp, po, ctypes.POINTER(ctypes.c_double)]
        L.tz_autotune.argtypes = [po]
        L.tz_tune_describe.argtypes = [ctypes.c_char_p, i64]
        L.tz_tune_describe.restype = i64
        for f in ("fft_zeropad", "czt", "czt_band_exact", "czt_transfer", "ifft", "zoom_fft", "czt_band",
                  "czt_plan_shape",
                  "tz_batch_create", "tz_batch_launch", "tz_batch_extents", "tz_batch_wait", "tz_plan_create", "tz_plan_workspace", "tz_plan_execute",
                  "tz_plan_execute_static", "tz_bin_freqs", "tz_autotune"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
        return L


def _check(st: int):
    if st != TZ_OK:
        raise ThzError(st, lib().tz_last_error().decode())


def version() -> str:
    return lib().tz_version().decode()


def release_plans():
    lib().tz_release_plans()


def autotune(stream=None):
    """Time one Bluestein FFT pair of every single-workgroup length on the
    current device; later plans pick FFT lengths and bin blocks from these
    times, which persist in the tune cache (TZ_TUNE_CACHE)."""
    torch = _torch()
    o = tz_opts()
    lib().tz_opts_init(ctypes.byref(o))
    if stream is None:
        stream = torch.cuda.current_stream()
    o.stream = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(lib().tz_autotune(ctypes.byref(o)))


def tune_describe() -> str:
    """Cache path, load/save outcome, device key and the FFT-pair costs in use."""
    n = lib().tz_tune_describe(None, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    lib().tz_tune_describe(buf, len(buf))
    return buf.value.decode()


# ---------------------------------------------------------------------------
# tensor plumbing
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _traces(x):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("x must be a torch tensor on the GPU")
    if x.dim() == 1:
        x = x.unsqueeze(0)
    if x.dim() != 2:
        raise ValueError("x must be [N] or [B, N]")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    if x.stride(1) != 1:
        x = x.contiguous()
    return x


def _opts(x, out_stride=0, precision="fp32", flags=0, taps=0, cutoff=0.0, stream=None):
    torch = _torch()
    o = tz_opts()
    lib().tz_opts_init(ctypes.byref(o))
    o.batch = x.shape[0]
    o.in_stride = x.stride(0) if x.shape[0] > 1 else x.shape[1]
    o.out_stride = out_stride
    o.in_dtype = TZ_F64 if x.dtype == torch.float64 else TZ_F32
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.flags = flags
    o.fir_taps = taps
    o.fir_cutoff_hz = cutoff
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    o.stream = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    return o


def _empty(x) -> bool:
    """A batch of no rows (of at least one sample each) has an empty result:
    the transforms return it without a library call (the C entry points read
    batch = 0 as one trace)."""
    if x.shape[1] < 1:
        raise ValueError("traces must hold at least one sample")
    return x.shape[0] == 0


def _out(x, bins, out, dtype=None):
    torch = _torch()
    dtype = dtype or torch.complex64
    if out is None:
        return torch.empty((x.shape[0], bins), dtype=dtype, device=x.device)
    if out.dtype != dtype or not out.is_cuda or out.shape != (x.shape[0], bins) or out.stride(1) != 1:
        raise ValueError(f"out must be a {dtype} GPU tensor [B, bins] with unit inner stride")
    return out


# ---------------------------------------------------------------------------
# transforms
# ---------------------------------------------------------------------------
def fft_zeropad(x, n_zeros: int, *, half: bool = False, out=None, stream=None):
    """X[k] = sum_{n<N} x[n] exp(-j 2 pi k n / (N + n_zeros)) for each row of x."""
    x = _traces(x)
    nfft = x.shape[1] + int(n_zeros)
    bins = nfft // 2 + 1 if half else nfft
    out = _out(x, bins, out)
    o = _opts(x, out.stride(0), flags=TZ_HALF if half else 0, stream=stream)
    if _empty(x):
        return out
    with _torch().cuda.device(x.device):
        _check(lib().fft_zeropad(x.data_ptr(), x.shape[1], int(n_zeros), out.data_ptr(), ctypes.byref(o)))
    return out


def czt(x, M: int, W: complex, A: complex, *, out=None, precision="fp32", stream=None):
    """X[k] = sum_n x[n] A^-n W^(kn), k < M, for each row of x; complex64, or
    complex128 with precision="fp64" (direct FP64 summation, any contour)."""
    x = _traces(x)
    out = _out(x, int(M), out, _torch().complex128 if precision == "fp64" else None)
    o = _opts(x, out.stride(0), precision=precision, stream=stream)
    W, A = complex(W), complex(A)
    if _empty(x):
        return out
    with _torch().cuda.device(x.device):
        _check(lib().czt(x.data_ptr(), x.shape[1], int(M), tz_c64(W.real, W.imag), tz_c64(A.real, A.imag),
                         out.data_ptr(), ctypes.byref(o)))
    return out


def ifft(X, *, out=None, stream=None, half=False, N=None):
    """x[n] = (1/N) sum_k X[k] exp(+j 2 pi k n / N) for each row of the
    complex64 spectra X ([N] or [B, N]); returns [B, N] complex64.
    half=True: X holds the Hermitian half spectra of real traces ([B, N/2 + 1]
    bins, as fft_zeropad(..., half=True) writes them) and the result is the
    real traces [B, N] float32; N (default 2 (bins - 1)) picks odd lengths."""
    torch = _torch()
    if not isinstance(X, torch.Tensor) or not X.is_cuda:
        raise TypeError("X must be a torch tensor on the GPU")
    if X.dim() == 1:
        X = X.unsqueeze(0)
    if X.dim() != 2 or X.dtype != torch.complex64:
        raise TypeError("X must be a complex64 tensor [N] or [B, N]")
    if X.stride(1) != 1:
        X = X.contiguous()
    B, nb = X.shape
    if half:
        N = int(N) if N is not None else 2 * (nb - 1)
        if N // 2 + 1 != nb:
            raise ValueError(f"{nb} bins are not the half spectrum of N = {N}")
        if out is None:
            out = torch.empty((B, N), dtype=torch.float32, device=X.device)
        elif out.dtype != torch.float32 or not out.is_cuda or out.shape != (B, N) or out.stride(1) != 1:
            raise ValueError("out must be a float32 GPU tensor [B, N] with unit inner stride")
    else:
        N = nb
        out = _out(X, N, out)
    o = tz_opts()
    lib().tz_opts_init(ctypes.byref(o))
    o.batch = B
    o.in_stride = X.stride(0) if B > 1 else nb
    o.out_stride = out.stride(0)
    o.flags = TZ_HALF if half else 0
    if stream is None:
        stream = torch.cuda.current_stream(X.device)
    o.stream = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    if _empty(X):
        return out
    with torch.cuda.device(X.device):
        _check(lib().ifft(X.data_ptr(), N, out.data_ptr(), ctypes.byref(o)))
    return out


def czt_transfer(x, M: int, W: complex, A: complex, *, out=None, stream=None):
    """H[p][k] = CZT(x[2p+1])[k] / CZT(x[2p])[k]: frequency response of
    reference/sample row pairs, one [B/2, M] complex64 row per pair."""
    torch = _torch()
    x = _traces(x)
    if x.shape[0] % 2:
        raise ValueError("x must hold reference/sample row pairs (even number of rows)")
    M = int(M)
    if out is None:
        out = torch.empty((x.shape[0] // 2, M), dtype=torch.complex64, device=x.device)
    elif out.dtype != torch.complex64 or not out.is_cuda or out.shape != (x.shape[0] // 2, M) or out.stride(1) != 1:
        raise ValueError("out must be a complex64 GPU tensor [B/2, M] with unit inner stride")
    o = _opts(x, out.stride(0), stream=stream)
    W, A = complex(W), complex(A)
    if _empty(x):
        return out
    with torch.cuda.device(x.device):
        _check(lib().czt_transfer(x.data_ptr(), x.shape[1], M, tz_c64(W.real, W.imag), tz_c64(A.real, A.imag),
                                  out.data_ptr(), ctypes.byref(o)))
    return out


def czt_band_exact(x, M: int, fs_hz: int, f1_hz: int, f2_hz: int, *, out=None, precision="fp32", stream=None):
    """CZT over [f1, f2) with M bins, integer-hertz band (exact phase residues)."""
    x = _traces(x)
    out = _out(x, int(M), out)
    o = _opts(x, out.stride(0), precision=precision, stream=stream)
    if _empty(x):
        return out
    with _torch().cuda.device(x.device):
        _check(lib().czt_band_exact(x.data_ptr(), x.shape[1], int(M), int(fs_hz), int(f1_hz), int(f2_hz),
                                    out.data_ptr(), ctypes.byref(o)))
    return out


def zoom_fft(x, fs: float, f1: float, f2: float, M: int, D: int, *, taps: int = 63,
             cutoff_hz: float | None = None, out=None, precision="fp32", stream=None):
    """Zoom FFT: mix f_N = (f1+f2)/2 to DC, T-tap Hamming low-pass, decimate by
    D, K-point DFT on M bins centred on f_N."""
    x = _traces(x)
    out = _out(x, int(M), out)
    o = _opts(x, out.stride(0), precision=precision, taps=int(taps), cutoff=float(cutoff_hz or 0.0),
              stream=stream)
    if _empty(x):
        return out
    with _torch().cuda.device(x.device):
        _check(lib().zoom_fft(x.data_ptr(), x.shape[1], float(fs), float(f1), float(f2), int(M), int(D),
                              out.data_ptr(), ctypes.byref(o)))
    return out


def _arrays(x, ndim: int):
    """x as [B, N_0, ..., N_{d-1}] with each array packed (last index fastest)."""
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("x must be a torch tensor on the GPU")
    if not 1 <= ndim <= TZ_MAX_DIMS:
        raise ValueError(f"1 to {TZ_MAX_DIMS} axes")
    if x.dim() == ndim:
        x = x.unsqueeze(0)
    if x.dim() != ndim + 1:
        raise ValueError(f"x must be [N_0, ...] or [B, N_0, ...] with {ndim} array dimensions")
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    if not x[0].is_contiguous():
        x = x.contiguous()
    return x


def _nd_call(fn, x, Ms, axes_arr, out, taps, stream):
    torch = _torch()
    B = x.shape[0]
    shape = (B,) + tuple(Ms)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=x.device)
    elif out.dtype != torch.complex64 or not out.is_cuda or tuple(out.shape) != shape or not out[0].is_contiguous():
        raise ValueError(f"out must be a complex64 GPU tensor {list(shape)} with packed arrays")
    o = _opts(x, taps=taps, stream=stream)
    o.in_stride = x.stride(0) if B > 1 else x[0].numel()
    o.out_stride = out.stride(0) if B > 1 else out[0].numel()
    with torch.cuda.device(x.device):
        _check(fn(x.data_ptr(), len(Ms), axes_arr, out.data_ptr(), ctypes.byref(o)))
    return out


def czt_nd(x, axes, *, out=None, stream=None):
    """X[k_0..k_{d-1}] = sum_n x[n] prod_a A_a^-n_a W_a^(k_a n_a) for every
    array of x [B, N_0, ..., N_{d-1}] (or one array [N_0, ...]);
    axes = [(M_a, W_a, A_a), ...], axis 0 first.  Returns [B, M_0, ...]."""
    ndim = len(axes)
    x = _arrays(x, ndim)
    arr = (tz_czt_axis * ndim)()
    Ms = []
    for a, (M, W, A) in enumerate(axes):
        W, A = complex(W), complex(A)
        arr[a] = tz_czt_axis(x.shape[a + 1], int(M), tz_c64(W.real, W.imag), tz_c64(A.real, A.imag))
        Ms.append(int(M))
    return _nd_call(lib().czt_nd, x, Ms, arr, out, 0, stream)


def zoom_fft_nd(x, axes, *, taps: int = 63, out=None, stream=None):
    """Zoom FFT along every axis of x [B, N_0, ..., N_{d-1}];
    axes = [(fs, f1, f2, M, D[, fc]), ...], axis 0 first (fc = cut-off in Hz,
    default fs / (2 D)).  Returns [B, M_0, ...]."""
    ndim = len(axes)
    x = _arrays(x, ndim)
    arr = (tz_zoom_axis * ndim)()
    Ms = []
    for a, ax in enumerate(axes):
        fs, f1, f2, M, D = ax[:5]
        fc = ax[5] if len(ax) > 5 and ax[5] is not None else 0.0
        arr[a] = tz_zoom_axis(x.shape[a + 1], int(M), int(D), float(fs), float(f1), float(f2), float(fc))
        Ms.append(int(M))
    return _nd_call(lib().zoom_fft_nd, x, Ms, arr, out, int(taps), stream)


# ---------------------------------------------------------------------------
# host helpers
# ---------------------------------------------------------------------------
def czt_band(fs: float, f1: float, f2: float, M: int):
    W, A = tz_c64(), tz_c64()
    _check(lib().czt_band(float(fs), float(f1), float(f2), int(M), ctypes.byref(W), ctypes.byref(A)))
    return complex(W.re, W.im), complex(A.re, A.im)


def fft_zero_count(fs: float, N_fft: int, delta: float) -> int:
    return int(lib().fft_zero_count(float(fs), int(N_fft), float(delta)))


def czt_points_for_resolution(fs: float, f1: float, f2: float, N_fft: int) -> int:
    return int(lib().czt_points_for_resolution(float(fs), float(f1), float(f2), int(N_fft)))


def zoom_short_length(fs: float, f1: float, f2: float, M: int, D: int) -> int:
    return int(lib().zoom_short_length(float(fs), float(f1), float(f2), int(M), int(D)))


def czt_plan_shape(N: int, M: int):
    L, blocks = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().czt_plan_shape(int(N), int(M), ctypes.byref(L), ctypes.byref(blocks)))
    return L.value, blocks.value


# ---------------------------------------------------------------------------
# uneven batch
# ---------------------------------------------------------------------------
class Batch:
    """Many traces of different length / band / M / method in one launch.

    jobs: list of dicts with keys kind ("czt" | "zoom"), N, M, fs_hz, f1_hz,
    f2_hz, D (zoom), taps (zoom), in_offset, out_offset."""

    def __init__(self, jobs, stream=None):
        torch = _torch()
        arr = (tz_job * len(jobs))()
        for i, j in enumerate(jobs):
            a = arr[i]
            a.kind = TZ_JOB_ZOOM if j["kind"] == "zoom" else TZ_JOB_CZT
            a.fir_taps = int(j.get("taps", 0))
            a.N, a.M, a.D = int(j["N"]), int(j["M"]), int(j.get("D", 1))
            a.fs_hz, a.f1_hz, a.f2_hz = int(j["fs_hz"]), int(j["f1_hz"]), int(j["f2_hz"])
            a.in_offset, a.out_offset = int(j["in_offset"]), int(j["out_offset"])
        o = tz_opts()
        lib().tz_opts_init(ctypes.byref(o))
        if stream is None:
            stream = torch.cuda.current_stream()
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        h = ctypes.c_void_p()
        _check(lib().tz_batch_create(arr, len(jobs), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.n_jobs = len(jobs)
        xe, Xe = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tz_batch_extents(self._h, ctypes.byref(xe), ctypes.byref(Xe)))
        self.x_elems, self.X_elems = xe.value, Xe.value

    def launch(self, x_flat, X_flat, stream=None):
        """Run every job: x_flat float32 and X_flat complex64, contiguous GPU
        tensors of at least x_elems / X_elems elements."""
        torch = _torch()
        if x_flat.dtype != torch.float32 or X_flat.dtype != torch.complex64:
            raise TypeError("x_flat must be float32 and X_flat complex64")
        if not (x_flat.is_cuda and X_flat.is_cuda):
            raise TypeError("x_flat and X_flat must be GPU tensors")
        if not (x_flat.is_contiguous() and X_flat.is_contiguous()):
            raise ValueError("x_flat and X_flat must be contiguous")
        if x_flat.numel() < self.x_elems or X_flat.numel() < self.X_elems:
            raise ValueError(f"the jobs reach {self.x_elems} samples and {self.X_elems} bins; got buffers of "
                             f"{x_flat.numel()} and {X_flat.numel()}")
        if x_flat.device != X_flat.device:
            raise ValueError("x_flat and X_flat must be on the same GPU")
        if stream is None:
            stream = torch.cuda.current_stream(x_flat.device)
        _check(lib().tz_batch_launch(self._h, x_flat.data_ptr(), X_flat.data_ptr(),
                                     ctypes.c_void_p(stream.cuda_stream)))
        return X_flat

    def wait(self, timeout_ms: float) -> bool:
        """Wait at most timeout_ms for the last launch; False on TZ_ETIMEOUT."""
        st = lib().tz_batch_wait(self._h, float(timeout_ms))
        if st == TZ_ETIMEOUT:
            return False
        _check(st)
        return True

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        lib().tz_batch_describe(self._h, buf, len(buf))
        return buf.value.decode()

    def close(self):
        if self._h:
            lib().tz_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# explicit plans
# ---------------------------------------------------------------------------
def _plan_params(kind, N, M, n_zeros, W, A, fs, f1, f2, D, fs_hz, f1_hz, f2_hz):
    p = tz_plan_params()
    p.kind = TZ_PLAN_KINDS[kind]
    p.N, p.M, p.n_zeros, p.D = int(N), int(M), int(n_zeros), int(D)
    p.W, p.A = tz_c64(complex(W).real, complex(W).imag), tz_c64(complex(A).real, complex(A).imag)
    p.fs, p.f1, p.f2 = float(fs), float(f1), float(f2)
    p.fs_hz, p.f1_hz, p.f2_hz = int(fs_hz), int(f1_hz), int(f2_hz)
    return p


def _plan_opts(batch, in_stride, out_stride, dtype, precision, half, taps, cutoff_hz, stream):
    o = tz_opts()
    lib().tz_opts_init(ctypes.byref(o))
    o.batch = int(batch)
    o.in_stride, o.out_stride = int(in_stride), int(out_stride)
    o.in_dtype = TZ_F64 if str(dtype).endswith("float64") else TZ_F32
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.flags = TZ_HALF if half else 0
    o.fir_taps, o.fir_cutoff_hz = int(taps), float(cutoff_hz)
    if stream is not None:
        o.stream = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    return o


def bin_freqs(kind: str, *, N: int = 1, M: int = 1, n_zeros: int = 0, W: complex = 1.0, A: complex = 1.0,
              fs: float = 0.0, f1: float = 0.0, f2: float = 0.0, D: int = 1, fs_hz: int = 0, f1_hz: int = 0,
              f2_hz: int = 0, half: bool = False, taps: int = 0, cutoff_hz: float = 0.0):
    """Frequency in Hz of every output bin of a transform (host only)."""
    import numpy as np
    p = _plan_params(kind, N, M, n_zeros, W, A, fs, f1, f2, D, fs_hz, f1_hz, f2_hz)
    o = _plan_opts(1, 0, 0, "float32", "fp32", half, taps, cutoff_hz, None)
    n = (N + n_zeros if not half else (N + n_zeros) // 2 + 1) if kind == "fft_zeropad" else M
    f = np.empty(max(int(n), 1), dtype=np.float64)
    _check(lib().tz_bin_freqs(ctypes.byref(p), ctypes.byref(o), f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return f[:n]


class Plan:
    """A transform of one shape built once (tz_plan_create): execute() only
    enqueues kernels, with a caller-owned workspace of workspace_bytes.

    kind: "fft_zeropad" (N, n_zeros, half), "czt" (N, M, W, A),
    "czt_band_exact" (N, M, fs_hz, f1_hz, f2_hz) or "zoom" (N, M, fs, f1, f2,
    D, taps, cutoff_hz) or "ifft" (N: complex64 spectra in, N samples out;
    with half, N/2 + 1 Hermitian bins in and N float32 samples out);
    batch traces of dtype, rows in_stride / out_stride elements apart
    (0 = packed)."""

    def __init__(self, kind: str, *, N: int, batch: int = 1, M: int = 0, n_zeros: int = 0, W: complex = 1.0,
                 A: complex = 1.0, fs: float = 0.0, f1: float = 0.0, f2: float = 0.0, D: int = 1, fs_hz: int = 0,
                 f1_hz: int = 0, f2_hz: int = 0, dtype="float32", precision="fp32", half: bool = False,
                 taps: int = 0, cutoff_hz: float = 0.0, in_stride: int = 0, out_stride: int = 0, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.kind, self.N, self.batch = kind, int(N), int(batch)
        self.dtype = torch.float64 if str(dtype).endswith("float64") else torch.float32
        self.out_dtype = torch.complex128 if (kind == "czt" and precision == "fp64") else torch.complex64
        self.in_len = self.N
        if kind == "ifft":
            self.dtype = torch.complex64
            self.bins = int(N)
            if half:
                self.in_len = self.N // 2 + 1
                self.out_dtype = torch.float32
        elif kind == "fft_zeropad":
            self.bins = N + n_zeros if not half else (N + n_zeros) // 2 + 1
        else:
            self.bins = int(M)
        self.in_stride = int(in_stride) or self.in_len
        self.out_stride = int(out_stride) or self.bins
        p = _plan_params(kind, N, M, n_zeros, W, A, fs, f1, f2, D, fs_hz, f1_hz, f2_hz)
        o = _plan_opts(batch, in_stride, out_stride, "float32" if kind == "ifft" else dtype, precision, half, taps,
                       cutoff_hz, stream)
        h = ctypes.c_void_p()
        _check(lib().tz_plan_create(ctypes.byref(p), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        _check(lib().tz_plan_workspace(self._h, ctypes.byref(n)))
        self.workspace_bytes = n.value

    def _check_buffers(self, x, out):
        torch = _torch()
        if not (x.is_cuda and out.is_cuda) or x.dtype != self.dtype or out.dtype != self.out_dtype:
            raise TypeError("x and out must be GPU tensors of the plan's input and output dtypes")
        if x.shape[0] != self.batch or x.shape[-1] != self.in_len or out.shape != (self.batch, self.bins):
            raise ValueError("x must be [batch, N] (ifft half: N/2 + 1) and out [batch, bins] of the plan")
        if self.batch > 1 and (x.stride(0) != self.in_stride or out.stride(0) != self.out_stride):
            raise ValueError("row strides must be the plan's in_stride / out_stride")
        if x.stride(-1) != 1 or out.stride(-1) != 1:
            raise ValueError("rows must be contiguous")

    def execute(self, x, out, workspace=None, stream=None):
        """x: [batch, N] (rows in_stride apart), out: [batch, bins] complex64
        (rows out_stride apart), workspace: a GPU tensor of at least
        workspace_bytes bytes (None when that is 0).  Asynchronous."""
        torch = _torch()
        self._check_buffers(x, out)
        ws = 0
        if self.workspace_bytes:
            if workspace is None or not workspace.is_cuda or \
                    workspace.numel() * workspace.element_size() < self.workspace_bytes:
                raise ValueError(f"this plan needs a GPU workspace of {self.workspace_bytes} bytes")
            ws = workspace.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        _check(lib().tz_plan_execute(self._h, x.data_ptr(), out.data_ptr(), ws, ctypes.c_void_p(stream.cuda_stream)))
        return out

    def execute_static(self, x, out, stream=None):
        """execute() with the library's fixed device scratch array as the
        workspace (tz_plan_execute_static): no workspace argument and no
        allocation.  Calls on one GPU share that array, so they must be
        ordered on one stream.  Asynchronous."""
        self._check_buffers(x, out)
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        _check(lib().tz_plan_execute_static(self._h, x.data_ptr(), out.data_ptr(),
                                            ctypes.c_void_p(stream.cuda_stream)))
        return out

    def close(self):
        if self._h:
            lib().tz_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
