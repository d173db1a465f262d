"""CPU checks of the C-ABI library: it loads, exports every symbol declared in
include/thzspec.h, its host helpers follow the paper's formulas and values,
and invalid arguments are rejected before any device work."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thzspec.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "paper_values.json")


@pytest.fixture(scope="module")
def tz():
    import paper_2108_03948_amd as tz
    if not os.path.exists(tz.LIB_PATH):
        from paper_2108_03948_amd import build
        build.build()
    tz.lib()
    return tz


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(tz):
    declared = header_functions()
    assert "czt" in declared and "fft_zeropad" in declared and "zoom_fft" in declared
    L = ctypes.CDLL(tz.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), f"{name} declared in thzspec.h but not exported"
    assert sorted(tz.EXPORTS) == declared


def test_version(tz):
    assert "gfx950" in tz.version()


def test_czt_band_eq22_23(tz):
    fs, f1, f2, M = 20e12, 0.2e12, 2.5e12, 4096
    W, A = tz.czt_band(fs, f1, f2, M)
    assert abs(W - np.exp(-2j * np.pi * (f2 - f1) / (M * fs))) < 1e-15
    assert abs(A - np.exp(2j * np.pi * f1 / fs)) < 1e-15
    with pytest.raises(tz.ThzError):
        tz.czt_band(fs, f2, f1, M)


def test_fft_zero_count_inverts_eq4(tz):
    # eq. (5) gives the zeros x reaching a resolution change delta (eq. (4))
    g = json.load(open(GOLDEN))["timing_sweep_step"]
    fs, N = 10e12, 500                      # Section 3.2: T_s = 100 fs, N = 500
    df = fs / N
    assert df == pytest.approx(g["start_hz"])
    for steps in range(1, 30):
        delta = steps * g["step_hz"]        # Fig. 11: 0.5 GHz steps from 20 GHz
        z = tz.fft_zero_count(fs, N, delta)
        assert df - fs / (N + z) >= delta * (1 - 1e-12)
        assert z == 0 or df - fs / (N + z - 1) < delta
        x = fs * N / (fs - delta * N) - N   # eq. (5) with L = N_FFT
        assert z == math.ceil(x - 1e-9)
    assert tz.fft_zero_count(fs, N, df) == -1
    assert tz.fft_zero_count(fs, N, 0.0) == -1


def test_paper_resolutions_through_helpers(tz):
    g = json.load(open(GOLDEN))
    # eq. (25): CZT points over [f1, f2) matching an N_FFT-point FFT's spacing
    assert tz.czt_points_for_resolution(8000, 100, 1000, 128) == round(900 / 8000 * 128)
    e = g["thz_fft_resolution_N500"]
    fs = 1.0 / e["Ts_s"]
    assert fs / e["N"] == pytest.approx(e["printed_hz"])
    # a CZT with M = N over a band B has spacing B/N; 2.98 GHz at N = 500
    # means B = 1.49 THz, and the same band at N = 250 gives 5.96 GHz
    c500, c250 = g["thz_czt_resolution_N500"], g["thz_czt_resolution_N250"]
    band = c500["printed_hz"] * 500
    W, _ = tz.czt_band(fs, 0.0, band, 250)
    assert -np.angle(W) / (2 * np.pi) * fs == pytest.approx(c250["printed_hz"], rel=1e-12)


def test_zoom_short_length(tz):
    assert tz.zoom_short_length(20e12, 0.1e12, 3.0e12, 1024, 8) == 883
    assert tz.zoom_short_length(100e12, 0.05e12, 0.10e12, 1 << 18, 64) == 8_192_000
    assert tz.zoom_short_length(20e12, 0.2e12, 2.5e12, 4096, 6) == 5936
    assert tz.zoom_short_length(10.0, 0.0, 4.0, 1, 1) == 3  # 2.5 rounds away from zero
    assert tz.zoom_short_length(1.0, 2.0, 1.0, 1, 1) == -1


def test_czt_plan_shape(tz):
    assert tz.czt_plan_shape(4096, 4096) == (8192, 1)
    assert tz.czt_plan_shape(1024, 1024) == (2048, 1)
    assert tz.czt_plan_shape(1, 1) == (256, 1)
    assert tz.czt_plan_shape(8193, 8192) == (16384, 1)
    L, blocks = tz.czt_plan_shape(16384, 8192)
    assert L == 16384 and blocks > 1
    # long traces: one four-step FFT pair of length next_pow2(N + M - 1)
    # (power of two or 5 * 2^a, whichever is smaller)
    assert tz.czt_plan_shape(1 << 20, 1 << 18) == (5 << 18, 1)
    assert tz.czt_plan_shape(16384, 1 << 18) == (5 << 16, 1)
    assert tz.czt_plan_shape(40000, 30000) == (5 << 14, 1)
    assert tz.czt_plan_shape(70001, 60000) == (1 << 17, 1)
    with pytest.raises(tz.ThzError):
        tz.czt_plan_shape(1 << 24, 2)


def _raw(tz, fn, *args):
    st = fn(*args)
    return st, tz.lib().tz_last_error().decode()


def test_invalid_arguments_rejected_before_device_work(tz):
    L = tz.lib()
    o = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o))
    one = tz.tz_c64(1.0, 0.0)
    w = tz.tz_c64(math.cos(0.1), -math.sin(0.1))
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation
    cases = [
        (L.czt, (None, 10, 10, w, one, fake, ctypes.byref(o)), "NULL"),
        (L.czt, (fake, 0, 10, w, one, fake, ctypes.byref(o)), "N must be"),
        (L.czt, (fake, 10, 0, w, one, fake, ctypes.byref(o)), "M must be"),
        (L.czt, (fake, 10, 10, tz.tz_c64(0.0, 0.0), one, fake, ctypes.byref(o)), "non-zero"),
        (L.czt, (fake, 10, 10, tz.tz_c64(float("nan"), 0.0), one, fake, ctypes.byref(o)), "finite"),
        (L.fft_zeropad, (fake, 10, -1, fake, ctypes.byref(o)), "n_zeros"),
        (L.fft_zeropad, (fake, 10, 1 << 31, fake, ctypes.byref(o)), "2^31"),
        (L.zoom_fft, (fake, 100, 20e12, 2e12, 1e12, 64, 4, fake, ctypes.byref(o)), "f2 > f1"),
        (L.zoom_fft, (fake, 100, 20e12, 1e12, 2e12, 64, 0, fake, ctypes.byref(o)), "D must be"),
        (L.czt_band_exact, (fake, 10, 10, 0, 1, 2, fake, ctypes.byref(o)), "fs >= 1"),
        (L.czt_transfer, (fake, 10, 0, w, one, fake, ctypes.byref(o)), "M must be"),
        (L.ifft, (None, 10, fake, ctypes.byref(o)), "NULL"),
        (L.ifft, (fake, 0, fake, ctypes.byref(o)), "N must be"),
    ]
    for fn, args, msg in cases:
        st, err = _raw(tz, fn, *args)
        assert st == tz.TZ_EINVAL, (fn.__name__, st, err)
        assert msg in err, (fn.__name__, err)
    # the transfer function takes reference/sample pairs
    o1 = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o1))
    o1.batch = 3
    st, err = _raw(tz, L.czt_transfer, fake, 10, 10, w, one, fake, ctypes.byref(o1))
    assert st == tz.TZ_EINVAL and "pairs" in err
    # a spiral contour whose chirp magnitudes span too wide a range for FP32
    # is valid input but outside the GPU path (refused before any device work)
    o2 = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o2))
    st, err = _raw(tz, L.czt, fake, 5000, 5000, tz.tz_c64(1.01, 0.0), one, fake, ctypes.byref(o2))
    assert st == tz.TZ_EUNSUPPORTED and "too steep" in err
    st, err = _raw(tz, L.czt, fake, 100000, 100, tz.tz_c64(1.0 + 1e-9, 1e-6), one, fake, ctypes.byref(o2))
    assert st == tz.TZ_EUNSUPPORTED and "bin blocks" in err
    # strides smaller than a row
    o3 = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o3))
    o3.batch, o3.in_stride = 4, 5
    st, err = _raw(tz, L.czt, fake, 10, 10, w, one, fake, ctypes.byref(o3))
    assert st == tz.TZ_EINVAL and "in_stride" in err
    # the inverse DFT takes complex64 spectra and runs in FP32
    o4 = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o4))
    o4.in_dtype = tz.TZ_F64
    st, err = _raw(tz, L.ifft, fake, 10, fake, ctypes.byref(o4))
    assert st == tz.TZ_EINVAL and "complex64" in err
    o4.in_dtype, o4.precision = tz.TZ_F32, tz.TZ_SPLIT_FP16
    st, err = _raw(tz, L.ifft, fake, 10, fake, ctypes.byref(o4))
    assert st == tz.TZ_EUNSUPPORTED and "FP32" in err


def test_nd_invalid_arguments_rejected_before_device_work(tz):
    L = tz.lib()
    o = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o))
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation
    one = tz.tz_c64(1.0, 0.0)
    w = tz.tz_c64(math.cos(0.1), -math.sin(0.1))

    def czt_axes(*spec):
        arr = (tz.tz_czt_axis * max(1, len(spec)))()
        for i, (N, M, W) in enumerate(spec):
            arr[i] = tz.tz_czt_axis(N, M, W, one)
        return arr

    def zoom_axes(*spec):
        arr = (tz.tz_zoom_axis * len(spec))()
        for i, sp in enumerate(spec):
            arr[i] = tz.tz_zoom_axis(*sp)
        return arr

    good = czt_axes((16, 8, w), (12, 6, w))
    cases = [
        (L.czt_nd, (fake, 0, good, fake, ctypes.byref(o)), "ndim"),
        (L.czt_nd, (fake, 4, czt_axes(*[(4, 4, w)] * 4), fake, ctypes.byref(o)), "ndim"),
        (L.czt_nd, (fake, 2, None, fake, ctypes.byref(o)), "axes"),
        (L.czt_nd, (None, 2, good, fake, ctypes.byref(o)), "NULL"),
        (L.czt_nd, (fake, 2, czt_axes((16, 8, w), (12, 0, w)), fake, ctypes.byref(o)), "axis 1"),
        (L.czt_nd, (fake, 2, czt_axes((0, 8, w), (12, 6, w)), fake, ctypes.byref(o)), "axis 0"),
        (L.czt_nd, (fake, 2, czt_axes((16, 8, tz.tz_c64(0.0, 0.0)), (12, 6, w)), fake, ctypes.byref(o)),
         "non-zero"),
        (L.zoom_fft_nd, (fake, 2, zoom_axes((64, 16, 2, 20e12, 1e12, 2e12, 0.0), (64, 16, 0, 20e12, 1e12, 2e12, 0.0)),
                         fake, ctypes.byref(o)), "D must be"),
        (L.zoom_fft_nd, (fake, 1, zoom_axes((64, 16, 2, 20e12, 2e12, 1e12, 0.0)), fake, ctypes.byref(o)),
         "f2 > f1"),
        (L.zoom_fft_nd, (fake, 1, zoom_axes((64, 16, 2, 20e12, 1e12, 2e12, -1.0)), fake, ctypes.byref(o)),
         "cutoff"),
    ]
    for fn, args, msg in cases:
        st, err = _raw(tz, fn, *args)
        assert st == tz.TZ_EINVAL, (fn.__name__, st, err)
        assert msg in err, (fn.__name__, err)
    # the cut-off is per axis
    oc = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(oc))
    oc.fir_cutoff_hz = 1e12
    st, err = _raw(tz, L.zoom_fft_nd, fake, 1, zoom_axes((64, 16, 2, 20e12, 1e12, 2e12, 0.0)), fake,
                   ctypes.byref(oc))
    assert st == tz.TZ_EINVAL and "per axis" in err
    # arrays closer together than their size
    os_ = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(os_))
    os_.batch, os_.in_stride = 3, 16 * 12 - 1
    st, err = _raw(tz, L.czt_nd, fake, 2, good, fake, ctypes.byref(os_))
    assert st == tz.TZ_EINVAL and "in_stride" in err
    # split precision is refused
    op = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(op))
    op.precision = tz.TZ_SPLIT_BF16
    st, err = _raw(tz, L.czt_nd, fake, 2, good, fake, ctypes.byref(op))
    assert st == tz.TZ_EUNSUPPORTED and "FP32" in err


def test_binding_refuses_cpu_tensors(tz):
    import torch
    with pytest.raises(TypeError):
        tz.czt(torch.zeros(4, 16), 8, 1.0, 1.0)


def test_resolution_sweep_shapes(tz):
    """The sweep of the paper's timing comparison (Section 4): N = 500 samples at
    T_s = 100 fs give the 20 GHz FFT resolution of Section 3.2 with no zeros;
    each 0.5 GHz step sets N_fft from eq. (3), M from eq. (25) and K from the
    zoom grid."""
    import bench_sweep as bs
    pts = bs.sweep_points()
    assert len(pts) == 40 and pts[0] == 20e9 and pts[-1] == 0.5e9
    assert all(abs((a - b) - 0.5e9) < 1 for a, b in zip(pts, pts[1:]))
    s0, s1 = bs.shapes(tz, pts[0]), bs.shapes(tz, pts[-1])
    assert (s0["n_fft"], s0["n_zeros"], s0["M"]) == (500, 0, 125)
    assert (s1["n_fft"], s1["n_zeros"], s1["M"]) == (20000, 19500, 5000)
    assert s0["D"] == s1["D"] == 3
    assert s0["K"] == 167 and s1["K"] == 6667
    # eq. (4): the zero count of each point reaches its resolution from 20 GHz
    for df in pts[1:]:
        s = bs.shapes(tz, df)
        assert abs(bs.FS / s["n_fft"] - df) <= bs.FS / s["n_fft"] ** 2


def test_bin_freqs_closed_forms(tz):
    """Frequencies of the output bins (host helper, no device work)."""
    # eq. (24): czt_band_exact bins at f1 + k (f2 - f1)/M, f2 excluded
    f = tz.bin_freqs("czt_band_exact", M=4096, fs_hz=20 * 10**12, f1_hz=2 * 10**11, f2_hz=25 * 10**11)
    assert len(f) == 4096 and f[0] == 2e11 and f[-1] < 2.5e12
    assert np.allclose(np.diff(f), 2.3e12 / 4096, rtol=1e-12, atol=0)
    # the W, A of eqs. (22)-(23) trace the same grid on the plain CZT
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 4096)
    g = tz.bin_freqs("czt", M=4096, W=W, A=A, fs=20e12)
    assert np.max(np.abs(g - f)) < 1e-3 * (2.3e12 / 4096)
    # Section 3.1: 128 samples at 8 kHz over 100-1000 Hz are 7.03 Hz apart
    t = json.load(open(GOLDEN))["two_tone_czt_plotting_resolution"]
    h = tz.bin_freqs("czt_band_exact", M=t["samples"], fs_hz=t["fs_hz"], f1_hz=t["f1_hz"], f2_hz=t["f2_hz"])
    assert round(h[1] - h[0], t["printed_digits"]) == t["printed_hz"]
    # eq. (3): FFT bin k at k fs / N_fft; the half spectrum ends at fs / 2
    z = tz.bin_freqs("fft_zeropad", N=1000, n_zeros=1048, fs=20e12)
    assert len(z) == 2048 and z[0] == 0.0 and z[1] == 20e12 / 2048
    zh = tz.bin_freqs("fft_zeropad", N=1000, n_zeros=1048, fs=20e12, half=True)
    assert len(zh) == 1025 and zh[-1] == 10e12
    # zoom grid: bin floor(M/2) at f_N = (f1 + f2)/2, spacing fs / (D K)
    K = tz.zoom_short_length(20e12, 0.2e12, 2.5e12, 4096, 6)
    q = tz.bin_freqs("zoom", M=4096, fs=20e12, f1=0.2e12, f2=2.5e12, D=6)
    assert q[2048] == pytest.approx(1.35e12, rel=1e-15)
    assert np.allclose(np.diff(q), 20e12 / (6 * K), rtol=1e-12, atol=0)


def test_plan_invalid_arguments_rejected_before_device_work(tz):
    L = tz.lib()
    h = ctypes.c_void_p()

    def create(kind, **kw):
        p = tz._plan_params(kind, kw.get("N", 100), kw.get("M", 50), kw.get("n_zeros", 0), kw.get("W", 1.0),
                            kw.get("A", 1.0), kw.get("fs", 20e12), kw.get("f1", 1e12), kw.get("f2", 2e12),
                            kw.get("D", 4), kw.get("fs_hz", 20 * 10**12), kw.get("f1_hz", 10**12),
                            kw.get("f2_hz", 2 * 10**12))
        return _raw(tz, L.tz_plan_create, ctypes.byref(p), None, ctypes.byref(h))

    for (kind, kw, msg) in [("fft_zeropad", dict(N=0), "N must be"), ("fft_zeropad", dict(n_zeros=-1), "n_zeros"),
                            ("czt", dict(M=0), "M must be"), ("czt", dict(W=0.0), "non-zero"),
                            ("czt_band_exact", dict(f2_hz=10**12), "f2 > f1"),
                            ("zoom", dict(f2=0.5e12), "f2 > f1"), ("zoom", dict(D=0), "D must be")]:
        st, err = create(kind, **kw)
        assert st == tz.TZ_EINVAL and msg in err, (kind, kw, err)
        assert not h.value
    p = tz._plan_params("czt", 100, 50, 0, 1.0, 1.0, 0, 0, 0, 1, 0, 0, 0)
    p.kind = 9
    st, err = _raw(tz, L.tz_plan_create, ctypes.byref(p), None, ctypes.byref(h))
    assert st == tz.TZ_EINVAL and "unknown plan kind" in err
    n = ctypes.c_size_t()
    assert L.tz_plan_workspace(None, ctypes.byref(n)) == tz.TZ_EINVAL
    assert L.tz_plan_execute(None, 1, 1, None, None) == tz.TZ_EINVAL
    st, err = _raw(tz, L.tz_bin_freqs, None, None, None)
    assert st == tz.TZ_EINVAL
    # the inverse-DFT plan takes complex64 spectra; its outputs are time samples
    p = tz._plan_params("ifft", 100, 0, 0, 1.0, 1.0, 20e12, 0, 0, 1, 0, 0, 0)
    o = tz._plan_opts(1, 0, 0, "float64", "fp32", False, 0, 0.0, None)
    st, err = _raw(tz, L.tz_plan_create, ctypes.byref(p), ctypes.byref(o), ctypes.byref(h))
    assert st == tz.TZ_EINVAL and "complex64" in err and not h.value
    f = (ctypes.c_double * 100)()
    st, err = _raw(tz, L.tz_bin_freqs, ctypes.byref(p), None, f)
    assert st == tz.TZ_EINVAL and "time samples" in err


def test_batch_wait_and_extents_reject_null(tz):
    L = tz.lib()
    a, b = ctypes.c_int64(), ctypes.c_int64()
    assert L.tz_batch_extents(None, ctypes.byref(a), ctypes.byref(b)) == tz.TZ_EINVAL
    assert L.tz_batch_wait(None, 1.0) == tz.TZ_EINVAL
    assert "NULL" in L.tz_last_error().decode()
    assert tz.TZ_ETIMEOUT == 5


def _no_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("passes stand-in device pointers: CPU only")


def test_fault_injection_alloc_one_shot_and_batch(tz, monkeypatch):
    """TZ_FAULT=alloc fails the first device allocation of a plan as out of
    memory, before hipMalloc is called: the one-shot call and the batch return
    TZ_ENOMEM with the allocation named (without the injection the same calls
    on a machine with no GPU fail as TZ_EDEVICE instead)."""
    _no_gpu()
    L = tz.lib()
    o = tz.tz_opts()
    L.tz_opts_init(ctypes.byref(o))
    fake_x, fake_X = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    monkeypatch.delenv("TZ_FAULT", raising=False)
    L.tz_release_plans()
    st, err = _raw(tz, L.fft_zeropad, fake_x, 100, 28, fake_X, ctypes.byref(o))
    assert st == tz.TZ_EDEVICE, err
    monkeypatch.setenv("TZ_FAULT", "alloc")
    L.tz_release_plans()
    st, err = _raw(tz, L.fft_zeropad, fake_x, 100, 28, fake_X, ctypes.byref(o))
    assert st == tz.TZ_ENOMEM and "out of memory" in err, err
    job = tz.tz_job(kind=0, fir_taps=0, N=300, M=40, D=1, fs_hz=20 * 10**12, f1_hz=2 * 10**11,
                    f2_hz=25 * 10**11, in_offset=0, out_offset=0)
    h = ctypes.c_void_p()
    st, err = _raw(tz, L.tz_batch_create, ctypes.byref(job), 1, None, ctypes.byref(h))
    assert st == tz.TZ_ENOMEM and "batch arena" in err and not h.value, err


def test_log_names_plan_decisions():
    """TZ_LOG=1 writes the library's plan decisions to stderr (here the
    batch's work items, logged before its first allocation, which TZ_FAULT
    makes fail so that no device is needed)."""
    _no_gpu()
    import subprocess
    import sys
    code = ("import ctypes, paper_2108_03948_amd as tz\n"
            "L = tz.lib()\n"
            "job = tz.tz_job(kind=1, fir_taps=0, N=3000, M=500, D=6, fs_hz=20 * 10**12, f1_hz=2 * 10**11, "
            "f2_hz=25 * 10**11, in_offset=0, out_offset=0)\n"
            "h = ctypes.c_void_p()\n"
            "print(L.tz_batch_create(ctypes.byref(job), 1, None, ctypes.byref(h)))\n")
    env = dict(os.environ, TZ_LOG="1", TZ_FAULT="alloc")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.stdout.strip().splitlines()[-1] == str(2), r.stdout + r.stderr   # TZ_ENOMEM
    assert "thzspec: batch: 1 jobs (1 zoom, 2 front-end tiles), 1 work items in 1 units" in r.stderr, r.stderr
    env.pop("TZ_LOG")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert "thzspec:" not in r.stderr


def test_tune_cache_states_without_a_device(tz, tmp_path, monkeypatch):
    """tz_tune_describe needs no device: with the cache switched off, with a
    file that does not parse (ignored: the built-in costs stay), and with a
    well-formed file for some device, which is read (its entry is used only
    under the current device's key)."""
    import json
    monkeypatch.setenv("TZ_TUNE_CACHE", "off")
    d = tz.tune_describe()
    assert "cache=off" in d and "persistence off" in d and "fft_pair_ns=built-in" in d, d
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": 1, "entries": {')
    monkeypatch.setenv("TZ_TUNE_CACHE", str(bad))
    d = tz.tune_describe()
    assert f"cache={bad}" in d and "cache ignored" in d and "fft_pair_ns=built-in" in d, d
    monkeypatch.setenv("TZ_TUNE_CACHE", str(tmp_path / "bad2.json"))
    (tmp_path / "bad2.json").write_text('{"format": 2, "entries": {}}')  # another format: ignored as a whole
    assert "cache ignored" in tz.tune_describe()
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"format": 1, "entries": {"gfx000:test/thzspec 0.0": {
        "fft_pair_ns": {str(1 << c): float(c) for c in range(8, 15)}, "batches": {}}}}))
    monkeypatch.setenv("TZ_TUNE_CACHE", str(good))
    d = tz.tune_describe()
    assert "cache ignored" not in d and "fft_pair_ns=built-in" in d, d  # no entry for this device
    monkeypatch.setenv("TZ_TUNE_CACHE", str(tmp_path / "absent.json"))
    assert "no cache file" in tz.tune_describe()
