"""GPU checks of the explicit plans (tz_plan_create / tz_plan_execute).

A plan runs the same kernels on the same tables as the one-shot call of its
shape, so its spectra must equal the one-shot call's bit for bit, on every
path: single-pass CZT (float and integer-hertz phases, f32 and f64 input),
split precision, the four-step long path (workspace), the three forms of the
zero-padded FFT (real whole-spectrum, power-of-two factor, Bluestein with
the half spectrum) and the Zoom FFT (its decimated rows in the workspace,
short and long short-DFT).  One case is also checked against the FP64
oracle.  Plans keep their tables past tz_release_plans(), refuse a missing
workspace, and an execution captured in a HIP graph replays correctly with
new inputs, each replay checked against the eager call.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def traces(B, N, seed, dev, dtype=np.float32):
    import torch
    x = np.random.default_rng(seed).standard_normal((B, N)).astype(dtype)
    return x, torch.from_numpy(x).to(dev)


def run_plan(plan, x):
    import torch
    out = torch.empty((plan.batch, plan.bins), dtype=plan.out_dtype, device=x.device)
    ws = None
    if plan.workspace_bytes:
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=x.device)
    plan.execute(x, out, ws)
    torch.cuda.synchronize()
    return out


FS_HZ = 20_000_000_000_000
W0 = np.exp(-2j * np.pi * 0.37 / 140000)
A0 = np.exp(2j * np.pi * 0.0123)


def cases(tz):
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 4096)
    zoom_short = dict(fs=20e12, f1=0.2e12, f2=2.5e12, D=6)
    zoom_long = dict(fs=100e12, f1=0.05e12, f2=0.1e12, D=16)
    return [
        ("czt single pass", 4, 4096, np.float32, dict(kind="czt", M=4096, W=W, A=A),
         lambda x: tz.czt(x, 4096, W, A), False),
        ("czt f64 input, bin blocks", 3, 3000, np.float64, dict(kind="czt", M=15000, W=W, A=A),
         lambda x: tz.czt(x, 15000, W, A), False),
        ("czt split fp16", 2, 4096, np.float32, dict(kind="czt", M=4096, W=W, A=A, precision="split_fp16"),
         lambda x: tz.czt(x, 4096, W, A, precision="split_fp16"), False),
        ("czt four-step", 3, 100000, np.float32, dict(kind="czt", M=40000, W=W0, A=A0),
         lambda x: tz.czt(x, 40000, W0, A0), True),
        ("czt_band_exact", 3, 1000, np.float32,
         dict(kind="czt_band_exact", M=700, fs_hz=FS_HZ, f1_hz=300_000_000_000, f2_hz=1_100_000_000_000),
         lambda x: tz.czt_band_exact(x, 700, FS_HZ, 300_000_000_000, 1_100_000_000_000), False),
        ("fft_zeropad real, 65536 bins", 3, 4096, np.float32, dict(kind="fft_zeropad", n_zeros=61440),
         lambda x: tz.fft_zeropad(x, 61440), False),
        ("fft_zeropad power-of-two factor", 3, 300, np.float32, dict(kind="fft_zeropad", n_zeros=212),
         lambda x: tz.fft_zeropad(x, 212), False),
        ("fft_zeropad Bluestein, half spectrum", 2, 1000, np.float32,
         dict(kind="fft_zeropad", n_zeros=537, half=True), lambda x: tz.fft_zeropad(x, 537, half=True), False),
        ("zoom", 4, 4096, np.float32, dict(kind="zoom", M=4096, taps=63, **zoom_short),
         lambda x: tz.zoom_fft(x, 20e12, 0.2e12, 2.5e12, 4096, 6, taps=63), True),
        ("zoom f64 input", 3, 4096, np.float64, dict(kind="zoom", M=4096, taps=63, **zoom_short),
         lambda x: tz.zoom_fft(x, 20e12, 0.2e12, 2.5e12, 4096, 6, taps=63), True),
        ("zoom, long short-DFT, 255 taps", 2, 300000, np.float32, dict(kind="zoom", M=20000, taps=255, **zoom_long),
         lambda x: tz.zoom_fft(x, 100e12, 0.05e12, 0.1e12, 20000, 16, taps=255), True),
    ]


def test_plan_equals_one_shot_on_every_path(tz, dev):
    for i, (name, B, N, dtype, kw, one_shot, needs_ws) in enumerate(cases(tz)):
        kw = dict(kw)
        kind = kw.pop("kind")
        x, xd = traces(B, N, 100 + i, dev, dtype)
        plan = tz.Plan(kind, N=N, batch=B, dtype=np.dtype(dtype).name, **kw)
        say(f"case: plan {name}: B={B} N={N} bins={plan.bins} workspace {plan.workspace_bytes} B")
        assert (plan.workspace_bytes > 0) == needs_ws, name
        got = run_plan(plan, xd).cpu().numpy()
        ref = one_shot(xd).cpu().numpy()
        assert got.shape == ref.shape and np.isfinite(got).all()
        assert np.array_equal(got, ref), f"{name}: plan differs from the one-shot call"
        plan.close()


@pytest.mark.parametrize("N", [4096, 3000, 70000])
def test_ifft_plan_equals_one_shot(tz, dev, N):
    """The inverse-DFT plan (direct power-of-two FFT, Bluestein single pass
    with bin blocks, and the four-step path with its workspace) equals the
    one-shot ifft() bit for bit."""
    import torch
    rng = np.random.default_rng(N)
    X = torch.from_numpy((rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))).astype(np.complex64)).to(dev)
    plan = tz.Plan("ifft", N=N, batch=3)
    say(f"case: ifft plan N={N}: workspace {plan.workspace_bytes} B")
    got = run_plan(plan, X).cpu().numpy()
    ref = tz.ifft(X).cpu().numpy()
    assert np.array_equal(got, ref)
    plan.close()


@pytest.mark.parametrize("N", [10000, 945])
def test_ifft_half_plan_equals_one_shot(tz, dev, N):
    """The half-spectrum inverse plan (Hermitian bins in, real traces out)
    equals the one-shot ifft(..., half=True) bit for bit, through both
    execute() and execute_static()."""
    import torch
    rng = np.random.default_rng(N)
    nb = N // 2 + 1
    H = torch.from_numpy((rng.standard_normal((3, nb)) + 1j * rng.standard_normal((3, nb))).astype(np.complex64))
    H = H.to(dev)
    plan = tz.Plan("ifft", N=N, batch=3, half=True)
    assert plan.workspace_bytes == 0
    say(f"case: ifft half plan N={N}")
    got = run_plan(plan, H).cpu().numpy()
    ref = tz.ifft(H, half=True, N=N).cpu().numpy()
    assert got.dtype == np.float32 and np.array_equal(got, ref)
    out = torch.empty((3, N), dtype=torch.float32, device=dev)
    plan.execute_static(H, out)
    assert np.array_equal(out.cpu().numpy(), ref)
    plan.close()


def test_plan_against_oracle(tz, dev, orc):
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 1500)
    x, xd = traces(3, 2000, 7, dev)
    plan = tz.Plan("czt", N=2000, batch=3, M=1500, W=W, A=A)
    got = run_plan(plan, xd).cpu().numpy()
    ref = orc.czt(x.astype(np.float64), 1500, W, A)
    r = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    say(f"case: plan czt vs FP64 oracle: max rel L2 {r.max():.3e}")
    assert r.max() <= 1e-6


def test_plan_outlives_release_plans_and_strided_rows(tz, dev):
    import torch
    W, A = tz.czt_band(20e12, 0.3e12, 1.2e12, 900)
    x, _ = traces(3, 1000, 11, dev)
    big = torch.zeros((3, 1024), device=dev)
    big[:, :1000] = torch.from_numpy(x).to(dev)
    xv = big[:, :1000]
    plan = tz.Plan("czt", N=1000, batch=3, M=900, W=W, A=A, in_stride=1024, out_stride=960)
    tz.release_plans()  # the plan holds its own tables
    full = torch.full((3, 960), complex(7.0, 7.0), dtype=torch.complex64, device=dev)
    out = full[:, :900]
    plan.execute(xv, out)
    torch.cuda.synchronize()
    ref = tz.czt(xv.contiguous(), 900, W, A)
    say("case: plan after release_plans, strided rows")
    assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
    assert np.all(full[:, 900:].cpu().numpy() == np.complex64(complex(7.0, 7.0)))


def test_plan_refuses_missing_workspace(tz, dev):
    import torch
    plan = tz.Plan("zoom", N=4096, batch=2, M=4096, fs=20e12, f1=0.2e12, f2=2.5e12, D=6)
    assert plan.workspace_bytes > 0
    x = torch.zeros((2, 4096), device=dev)
    out = torch.empty((2, 4096), dtype=torch.complex64, device=dev)
    with pytest.raises(ValueError):
        plan.execute(x, out, None)
    st = tz.lib().tz_plan_execute(plan._h, x.data_ptr(), out.data_ptr(), None, None)
    assert st == tz.TZ_EINVAL and b"workspace" in tz.lib().tz_last_error()


@pytest.mark.parametrize("kind", ["czt", "zoom"])
def test_plan_in_hip_graph(tz, dev, kind):
    """An execution captured in a HIP graph: every replay, with new inputs
    copied in between, equals the eager one-shot call."""
    import torch
    B, N, M = 8, 4096, 4096
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, M)
    if kind == "czt":
        plan = tz.Plan("czt", N=N, batch=B, M=M, W=W, A=A)
        eager = lambda t: tz.czt(t, M, W, A)  # noqa: E731
    else:
        plan = tz.Plan("zoom", N=N, batch=B, M=M, fs=20e12, f1=0.2e12, f2=2.5e12, D=6)
        eager = lambda t: tz.zoom_fft(t, 20e12, 0.2e12, 2.5e12, M, 6)  # noqa: E731
    x = torch.zeros((B, N), device=dev)
    out = torch.zeros((B, M), dtype=torch.complex64, device=dev)
    ws = torch.empty(max(plan.workspace_bytes, 16), dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.execute(x, out, ws if plan.workspace_bytes else None, stream=s)  # first launch outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.execute(x, out, ws if plan.workspace_bytes else None, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        xn, xnd = traces(B, N, 50 + rep, dev)
        x.copy_(xnd)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = eager(xnd).cpu().numpy()
        say(f"case: {kind} plan graph replay {rep}")
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep} differs from the eager call"
    del g
    plan.close()
