"""tz_plan_execute_static (the allocation-free execution with the library's
fixed device scratch array) against tz_plan_execute with a caller-owned
workspace: the same kernels on the same inputs, so the outputs must agree bit
for bit.  Two calls in a row on one GPU, the second with a smaller input,
for a Zoom FFT (decimated rows in the scratch) and a four-step CZT (L-point
intermediates in the scratch, with fewer traces per chunk than the plan's
own execution), and the refusal of a plan whose rows exceed the array."""
import sys

import numpy as np
import pytest

import synth

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


def both(tz, plan, x):
    """Run plan on x through tz_plan_execute (torch workspace) and
    tz_plan_execute_static; return both outputs."""
    import torch
    dev = x.device
    ref = torch.full((plan.batch, plan.bins), complex("nan"), dtype=torch.complex64, device=dev)
    ws = None
    if plan.workspace_bytes:
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    plan.execute(x, ref, ws)
    out = torch.full_like(ref, complex("nan"))
    plan.execute_static(x, out)
    torch.cuda.synchronize()
    return ref, out


def same(ref, out, what):
    assert torch_isfinite(out), f"{what}: non-finite output"
    d = (ref != out).sum().item()
    say(f"  {what}: {ref.numel()} bins, {d} differ")
    assert d == 0


def torch_isfinite(t):
    import torch
    return bool(torch.isfinite(torch.view_as_real(t)).all().item())


def test_static_zoom_then_smaller(tz):
    import torch
    fs, f1, f2 = 20e12, 0.2e12, 2.5e12
    shapes = [(64, 4096, 4096, 6), (16, 2048, 1024, 4)]   # second call: smaller input
    for B, N, M, D in shapes:
        say(f"case: static zoom B={B} N={N} M={M} D={D}")
        x = torch.from_numpy(synth.pairs(B // 2, N=N).astype(np.float32)).cuda()
        plan = tz.Plan("zoom", N=N, batch=B, M=M, fs=fs, f1=f1, f2=f2, D=D, taps=63)
        assert plan.workspace_bytes > 0
        ref, out = both(tz, plan, x)
        same(ref, out, f"zoom B={B} N={N}")
        plan.close()


def test_static_four_step_then_smaller(tz):
    import torch
    # N + M - 1 > 2^17: the four-step path, 2 MiB of intermediates per trace.
    # 40 traces need 80 MiB, more than the 64 MiB array: the static call runs
    # two chunks (32 + 8 traces) where the plan's own execution runs one.
    cases = [(40, 1 << 17, 1 << 17), (3, 100000, 40000)]
    for B, N, M in cases:
        say(f"case: static four-step czt_band_exact B={B} N={N} M={M}")
        rng = np.random.default_rng(77 + B)
        x = torch.from_numpy(rng.standard_normal((B, N)).astype(np.float32)).cuda()
        plan = tz.Plan("czt_band_exact", N=N, batch=B, M=M, fs_hz=20_000_000_000_000,
                       f1_hz=200_000_000_000, f2_hz=2_500_000_000_000)
        assert plan.workspace_bytes > 0
        ref, out = both(tz, plan, x)
        same(ref, out, f"four-step B={B} N={N} M={M}")
        plan.close()


def test_static_single_pass_and_refusal(tz):
    import torch
    say("case: static czt single pass (no workspace)")
    x = torch.from_numpy(synth.pairs(4, N=4096).astype(np.float32)).cuda()
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 4096)
    plan = tz.Plan("czt", N=4096, batch=8, M=4096, W=W, A=A)
    ref, out = both(tz, plan, x)
    same(ref, out, "czt single pass")
    plan.close()
    # decimated rows of 8192 traces x 2048 outputs = 128 MiB > 64 MiB: refused
    say("case: static zoom refusal (rows exceed the array)")
    B, N = 8192, 4096
    plan = tz.Plan("zoom", N=N, batch=B, M=1024, fs=20e12, f1=0.2e12, f2=2.5e12, D=2, taps=63)
    xb = torch.zeros((B, N), dtype=torch.float32, device="cuda")
    ob = torch.zeros((B, 1024), dtype=torch.complex64, device="cuda")
    with pytest.raises(tz.ThzError) as e:
        plan.execute_static(xb, ob)
    assert e.value.status == tz.TZ_EINVAL and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert not ob.abs().any().item()     # nothing was launched
    plan.close()
