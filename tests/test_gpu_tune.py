"""The autotuner on the GPU (the benchmark spec batching (2): schedules picked by an
autotuner the project writes) and its persisted cache.

tz_autotune() times one Bluestein FFT pair per single-workgroup length and
writes the times under the device's key; plans made afterwards still match
the FP64 oracle (any FFT length >= N + M - 1 gives the same bins).  The
uneven batch stores the schedule its first launch picked; a new batch of the
same job table reads it back instead of timing the candidates, and computes
bitwise the same outputs.  A file that does not parse is ignored and then
rewritten.
"""
import json
import os
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


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("TZ_TUNE_CACHE", str(path))
    return path


def test_autotune_measures_and_persists(tz, orc, cache):
    import torch
    say("case: autotune, fresh cache file")
    assert "fft_pair_ns=built-in" in tz.tune_describe()
    tz.autotune()
    torch.cuda.synchronize()
    d = tz.tune_describe()
    say(f"  {d}")
    assert "fft_pair_ns=measured" in d
    data = json.loads(cache.read_text())
    assert data["format"] == 1
    (key, ent), = data["entries"].items()
    assert "gfx950" in key and key.endswith(tz.version())
    t = [ent["fft_pair_ns"][str(1 << c)] for c in range(8, 15)]
    say(f"  FFT pair ns per length 256 .. 16384: {[round(v, 1) for v in t]}")
    assert all(v > 0 for v in t) and t[-1] > t[0]  # longer pairs cost more
    # plans made with the measured costs still give the oracle's bins
    W, A = tz.czt_band(20e12, 0.2e12, 2.5e12, 3000)
    x = np.random.default_rng(3).standard_normal((2, 1500)).astype(np.float32)
    got = tz.czt(torch.from_numpy(x).cuda(), 3000, W, A).cpu().numpy()
    ref = orc.czt(x.astype(np.float64), 3000, W, A)
    r = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    say(f"  czt N=1500 M=3000 after autotune, plan {tz.czt_plan_shape(1500, 3000)}: rel L2 {r.max():.3e}")
    assert r.max() <= 1e-6


def test_corrupt_cache_is_ignored_then_rewritten(tz, cache):
    import torch
    cache.write_text("{ this is not json")
    d = tz.tune_describe()
    say(f"case: corrupt cache: {d}")
    assert "cache ignored" in d and "fft_pair_ns=built-in" in d
    tz.autotune()
    torch.cuda.synchronize()
    assert json.loads(cache.read_text())["format"] == 1


def test_batch_schedule_is_reused_from_the_cache(tz, cache):
    import torch
    dev = torch.device("cuda:0")
    x_flat, offs, meta = synth.uneven(B=24, seed=21, Nmin=300, Nmax=9000, Mmin=64, Mmax=4000)
    jobs, out = [], 0
    for i, j in enumerate(meta):
        jobs.append(dict(kind=j["kind"], N=j["N"], M=j["M"], D=j["D"], taps=j["taps"],
                         fs_hz=int(round(j["fs"])), f1_hz=int(round(j["f1"])), f2_hz=int(round(j["f2"])),
                         in_offset=int(offs[i]), out_offset=out))
        out += j["M"]
    xd = torch.from_numpy(x_flat).to(dev)
    say(f"case: batch of {len(jobs)} jobs, first process-wide launch times the candidates")
    X1 = torch.zeros(out, dtype=torch.complex64, device=dev)
    b = tz.Batch(jobs)
    b.launch(xd, X1)
    torch.cuda.synchronize()
    d1 = b.describe()
    say(f"  {d1}")
    assert "candidates_ms" in d1
    b.close()
    data = json.loads(cache.read_text())
    (ent,) = data["entries"].values()
    assert len(ent["batches"]) == 1
    X2 = torch.zeros(out, dtype=torch.complex64, device=dev)
    b = tz.Batch(jobs)
    b.launch(xd, X2)
    torch.cuda.synchronize()
    d2 = b.describe()
    say(f"  {d2}")
    assert "(tune cache)" in d2 and d1.split(" schedule=")[1].split(" ")[0] in d2
    assert np.array_equal(X1.cpu().numpy().view(np.uint32), X2.cpu().numpy().view(np.uint32))
    b.close()
