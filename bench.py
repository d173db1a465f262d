"""Benchmark: spectra of a batch of THz-TDS traces on one MI355X.

Workload (one "step" = one pass of the whole path over the batch):
  8192 synthetic traces (4096 sample/reference pairs) x 4096 FP32 samples at
  f_s = 20 THz, already resident in HBM;
    czt         M = 4096 bins over 0.2 - 2.5 THz        (Bluestein, L = 8192)
    fft_zeropad to N_fft = 65536 (61440 zeros)          (16 x 4096-point FFTs)
    zoom_fft    same band, M = 4096, D = 6, 63 taps     (K = 5936)
value = CZT outputs (8192 x 4096 bins) per second of the whole step.
The same run reports each transform's own rate, the roofline of the
dominant kernel (HIP events on the launch stream), and the FP64 oracle timed
on the host cores over a bounded sample.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--calib-copy]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CZT outputs/s over batched THz traces; %HBM peak; MFMA vs FP32 at 1e-5 err"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# profiled durations of the dominant kernel over the timed steps of a
# rocprofv3 run of this script (bench_profiles.py timed)
PROFILED_FILE = os.path.join(ROOT, "profiles", "bench_batched8192x4096_fft_zeropad_timed.json")
CSRC = os.path.join(ROOT, "paper_2108_03948_amd", "csrc")

N_PAIRS, N, FS = 4096, 4096, 20e12
F1, F2, M = 0.2e12, 2.5e12, 4096
NFFT = 65536
ZOOM_D, ZOOM_T = 6, 63


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of every library source (kernels, launch sizing, tables): byte
    counters taken with other sources are stale."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


# algorithmic work per launch (minimum bytes: read x once, write X once;
# flops: 5 L log2 L per complex FFT plus the pointwise complex products)
def fft_work(B):
    by = B * (N * 4 + NFFT * 8)
    P, F = NFFT // 4096, 4096
    fl = B * P * (5 * F * 12 + 6 * N)
    return by, fl


def czt_work(B, L=8192):
    by = B * (N * 4 + M * 8)
    fl = B * (2 * 5 * L * 13 + 6 * (N + L + M))
    return by, fl


def zoom_work(B):
    LD = -(-N // ZOOM_D)
    by = B * (N * 4 + M * 8)
    fl = B * (LD * ZOOM_T * 4 + 2 * 5 * 8192 * 13 + 6 * (LD + 8192 + M))
    return by, fl


def cpu_baseline(x_np, budget_s=12.0):
    """Time the FP64 oracle on a bounded sample of the same workload and
    scale it to CZT outputs per second of the whole step."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    x64 = x_np.astype(np.float64)
    W = np.exp(-2j * np.pi * (F2 - F1) / (M * FS))
    A = np.exp(2j * np.pi * F1 / FS)
    # calibrate on one trace, then size the sample to the budget
    t0 = time.perf_counter()
    oracle.czt(x64[:1], M, W, A)
    t_czt1 = time.perf_counter() - t0
    n = max(1, min(64, int(budget_s * 0.5 / max(t_czt1, 1e-6))))
    t0 = time.perf_counter()
    oracle.czt(x64[:n], M, W, A)
    t_czt = (time.perf_counter() - t0) / n
    fb = np.arange(0, NFFT, 16)          # every 16th bin of the zero-padded FFT
    nf = max(1, n // 4)
    t0 = time.perf_counter()
    oracle.fft_zeropad(x64[:nf], NFFT - N, fb)
    t_fft = (time.perf_counter() - t0) / nf * (NFFT / fb.size)
    t0 = time.perf_counter()
    oracle.zoom_fft(x64[:nf], FS, F1, F2, M, ZOOM_D, taps=ZOOM_T)
    t_zoom = (time.perf_counter() - t0) / nf
    per_trace = t_czt + t_fft + t_zoom
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {
        "value": M / per_trace,
        "unit": "CZT outputs/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"FP64 direct-summation oracle, {cores} OpenMP threads: czt on {n} traces x {M} bins, "
                   f"zoom on {nf} traces x {M} bins, fft_zeropad on {nf} traces x every 16th of {NFFT} "
                   f"bins (scaled x16); per-trace times summed and scaled to the 8192-trace step"),
        "seconds_per_trace": {"czt": t_czt, "fft_zeropad": t_fft, "zoom": t_zoom},
        "extrapolated_step_s": per_trace * 2 * N_PAIRS,
        "cpu_model": _cpu_model(),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _event_ms(stream, fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def fp64_czt(tz, xn, M, W, A, dev):
    """Reference bins for the error figures of this run: the library's FP64
    direct summation of eq. (11) on the GPU (complex128, relative rounding
    ~ n 2^-53; the tests pin it to the FP64 oracle at 1e-9), independent of
    the FP32 / split-precision Bluestein kernels it checks."""
    import numpy as np
    import torch
    x = torch.from_numpy(np.ascontiguousarray(xn, dtype=np.float64)).to(dev)
    return tz.czt(x, M, W, A, precision="fp64").cpu().numpy()


def bench_single(tz, synth, dev, stream):
    """One FP64 trace of 1024 samples at f_s = 20 THz: czt M = 1024 over
    0.1 - 3.0 THz, fft_zeropad to 16384, zoom D = 8 with 63 taps; microseconds
    per call (launch latency); the relative L2 error of every bin of the czt
    (against the FP64 direct summation) and of the zero-padded FFT (against
    torch's complex128 FFT); the zoom's parity is in the tests."""
    import numpy as np
    import torch
    x64 = synth.single_trace(N=1024).reshape(1, -1)
    x = torch.from_numpy(x64).to(dev)
    fs, f1, f2 = 20e12, 0.1e12, 3.0e12
    W, A = tz.czt_band(fs, f1, f2, 1024)
    Xc = torch.empty((1, 1024), dtype=torch.complex64, device=dev)
    Xf = torch.empty((1, 16384), dtype=torch.complex64, device=dev)
    Xz = torch.empty((1, 1024), dtype=torch.complex64, device=dev)
    calls = {"czt": lambda: tz.czt(x, 1024, W, A, out=Xc, stream=stream),
             "fft_zeropad": lambda: tz.fft_zeropad(x, 16384 - 1024, out=Xf, stream=stream),
             "zoom_fft": lambda: tz.zoom_fft(x, fs, f1, f2, 1024, 8, taps=63, out=Xz, stream=stream)}
    refs = {"czt": lambda: fp64_czt(tz, x64, 1024, W, A, dev),
            "fft_zeropad": lambda: torch.fft.fft(torch.from_numpy(x64).to(dev), n=16384).cpu().numpy()}
    outs = {"czt": Xc, "fft_zeropad": Xf, "zoom_fft": Xz}
    res = {}
    for name, fn in calls.items():
        us = _event_ms(stream, fn, 200) * 1e3
        res[name] = {"us_per_call": us}
        if name in refs:
            ref = refs[name]()
            got = outs[name].cpu().numpy()
            res[name]["rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    log("bench: single trace " + ", ".join(f"{k} {v['us_per_call']:.1f} us" for k, v in res.items()))
    return res


def bench_uneven(tz, synth, dev, stream, reps):
    """The uneven batch: 20000 traces, N ~ U{512..16384}, own band and M ~
    U{256..8192}, CZT / Zoom FFT 50/50, in one graph launch of the batch API.
    Algorithmic bytes: every sample read once (4 B) and every bin written once
    (8 B).  Error figure: 4 CZT jobs against the FP64 direct summation on
    48 bins each (the zoom jobs' parity is in the tests)."""
    import numpy as np
    import torch
    t0 = time.time()
    x_flat, offs, meta = synth.uneven(B=20000, seed=1003)
    jobs, out = [], 0
    for i, j in enumerate(meta):
        jobs.append(dict(kind=j["kind"], N=j["N"], M=j["M"], D=j["D"], taps=j["taps"],
                         fs_hz=int(round(j["fs"])), f1_hz=int(round(j["f1"])), f2_hz=int(round(j["f2"])),
                         in_offset=int(offs[i]), out_offset=out))
        out += j["M"]
    log(f"bench: uneven batch of {len(jobs)} jobs generated in {time.time() - t0:.1f} s")
    xd = torch.from_numpy(x_flat).to(dev)
    Xd = torch.zeros(out, dtype=torch.complex64, device=dev)
    b = tz.Batch(jobs)
    b.launch(xd, Xd, stream=stream)  # first launch: the schedule autotuner
    torch.cuda.synchronize()
    ms = _event_ms(stream, lambda: b.launch(xd, Xd, stream=stream), reps)
    nbytes = 4 * int(x_flat.size) + 8 * out
    # FFT work of the shapes the batch runs: every bin block (x input
    # segment) of a job is one Bluestein pair of length L, 2 x 5 L log2 L
    # flops (zoom jobs: the short DFT on ceil(N/D) decimated samples)
    flops = 0.0
    for j in jobs:
        n_in = j["N"] if j["kind"] == "czt" else -(-j["N"] // j["D"])
        L, pieces = tz.czt_plan_shape(n_in, j["M"])
        flops += pieces * 10.0 * L * np.log2(L)
    X = Xd.cpu().numpy()
    rng = np.random.default_rng(9)
    worst = 0.0
    for i0 in (0, 4999, 12345, 19990):
        i = next(k for k in range(i0, len(jobs)) if jobs[k]["kind"] == "czt")
        j = jobs[i]
        bins = np.unique(np.r_[0, j["M"] - 1, rng.integers(0, j["M"], 46)])
        W, A = tz.czt_band(j["fs_hz"], j["f1_hz"], j["f2_hz"], j["M"])
        ref = fp64_czt(tz, x_flat[offs[i]:offs[i + 1]][None], j["M"], W, A, dev)[0][bins]
        got = X[j["out_offset"] + bins]
        worst = max(worst, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    res = {"jobs": len(jobs), "samples": int(x_flat.size), "bins": out, "ms": ms, "bins_per_s": out / (ms * 1e-3),
           "alg_bytes": nbytes, "alg_GBps": nbytes / (ms * 1e-3) / 1e9,
           "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "fft_flops": flops,
           "TFLOPs": flops / (ms * 1e-3) / 1e12, "fp32_frac": flops / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
           "rel_l2_sampled": worst,
           "schedule": b.describe()}
    log(f"bench: uneven batch {ms:.3f} ms, {res['bins_per_s']:.3e} bins/s, {res['alg_GBps']:.0f} GB/s "
        f"algorithmic, rel L2 {worst:.2e}")
    b.close()
    return res


def bench_long(tz, synth, dev, stream, reps):
    """Long scans: 256 traces x 2^20 samples at T_s = 0.01 ps; czt M = 2^18
    over 0.05 - 0.10 THz with integer-hertz phases and the Zoom FFT with
    D = 64 and 255 taps, each in FP32 and the two split precisions.  Error
    figure of the czt: one trace, 48 bins, against the FP64 direct summation
    (the zoom's parity on these scans is in the tests)."""
    import numpy as np
    import torch
    B, NL, ML, fs, f1, f2 = 256, 1 << 20, 1 << 18, 100 * 10**12, 5 * 10**10, 10**11
    t0 = time.time()
    xn = synth.echoes(B, NL)
    log(f"bench: long scans generated in {time.time() - t0:.1f} s")
    x = torch.from_numpy(xn).to(dev)
    X = torch.empty((B, ML), dtype=torch.complex64, device=dev)
    bins = np.unique(np.r_[0, ML - 1, np.random.default_rng(13).integers(0, ML, 46)])
    Wl, Al = tz.czt_band(fs, f1, f2, ML)
    ref_c = fp64_czt(tz, xn[77:78], ML, Wl, Al, dev)[0][bins]
    res = {}
    for prec in ("fp32", "split_fp16", "split_bf16"):
        ms = _event_ms(stream, lambda: tz.czt_band_exact(x, ML, fs, f1, f2, out=X, precision=prec,
                                                          stream=stream), reps)
        got = X[77].cpu().numpy()[bins]
        res["czt_" + prec] = {"ms": ms, "bins_per_s": B * ML / (ms * 1e-3),
                              "rel_l2_sampled": float(np.linalg.norm(got - ref_c) / np.linalg.norm(ref_c))}
    for prec in ("fp32", "split_fp16", "split_bf16"):
        ms = _event_ms(stream, lambda: tz.zoom_fft(x, fs, f1, f2, ML, 64, taps=255, out=X, precision=prec,
                                                   stream=stream), reps)
        res["zoom_" + prec] = {"ms": ms, "bins_per_s": B * ML / (ms * 1e-3)}
    for t in ("czt", "zoom"):
        for k in (t + "_split_fp16", t + "_split_bf16"):
            res[k]["speedup_vs_fp32"] = res[t + "_fp32"]["ms"] / res[k]["ms"]
    log("bench: long scans " + ", ".join(f"{k} {v['ms']:.3f} ms" + (f" ({v['rel_l2_sampled']:.1e})" if
                                         "rel_l2_sampled" in v else "") for k, v in res.items()))
    del x, X
    return res


def bench_nd(tz, synth, dev, stream, reps):
    """Multi-dimensional CZT / Zoom FFT on THz images: 64 B-scans of 512
    pixels x 2048 samples (spatial band [-1/4, 1/4) cycles per pixel on 512
    bins, 0.2 - 2.5 THz on 1024 bins; the zoom: [-1/8, 1/8) with D = 3 and
    0.2 - 2.5 THz with D = 6, 63 taps) and one 256 x 256 pixel x 1024 sample
    cube (256 x 256 x 512 bins).  Each entry: ms per call, output bins/s, the
    algorithmic bytes (input read once, output written once) per second
    (parity of these launches is in the tests)."""
    import numpy as np
    import torch

    log("bench: generating THz images (64 x 512 x 2048 B-scans, 256 x 256 x 1024 cube)")
    scans = synth.raster(64, (512,), 2048, seed=3000)
    cube = synth.raster(1, (256, 256), 1024, seed=3100)
    Wp, Ap = np.exp(-2j * np.pi * 0.5 / 512), np.exp(2j * np.pi * -0.25)
    Wc, Ac = np.exp(-2j * np.pi * 0.5 / 256), np.exp(2j * np.pi * -0.25)
    Wt, At = tz.czt_band(FS, F1, F2, 1024)
    Wt2, At2 = tz.czt_band(FS, F1, F2, 512)
    cases = {
        "czt_2d": (scans, "czt", [(512, Wp, Ap), (1024, Wt, At)]),
        "czt_3d": (cube, "czt", [(256, Wc, Ac), (256, Wc, Ac), (512, Wt2, At2)]),
        "zoom_2d": (scans, "zoom", [(1.0, -0.125, 0.125, 512, 3), (FS, F1, F2, 1024, ZOOM_D)]),
    }
    res = {}
    rng = np.random.default_rng(45)
    for name, (xn, kind, axes) in cases.items():
        x = torch.from_numpy(xn).to(dev)
        Ms = [a[0] if kind == "czt" else a[3] for a in axes]
        X = torch.empty([x.shape[0]] + Ms, dtype=torch.complex64, device=dev)
        if kind == "czt":
            call = lambda: tz.czt_nd(x, axes, out=X, stream=stream)
        else:
            call = lambda: tz.zoom_fft_nd(x, axes, taps=ZOOM_T, out=X, stream=stream)
        for _ in range(2):
            call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        assert bool(torch.isfinite(torch.view_as_real(X)).all())
        nbytes = xn.nbytes + X.numel() * 8
        res[name] = {"shape_in": list(xn.shape), "shape_out": [x.shape[0]] + Ms, "ms": ms,
                     "bins_per_s": X.numel() / (ms * 1e-3), "alg_GBps": nbytes / (ms * 1e-3) / 1e9}
        log(f"bench: {name} {list(xn.shape)} -> {Ms}: {ms:.3f} ms, {X.numel() / (ms * 1e-3):.3e} bins/s")
        del x, X
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--step-only", action="store_true",
                    help="skip the single-trace, uneven-batch and long-scan workloads")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the per-trace path has no "
              "cross-GPU step: traces are independent, so N GPUs would each take B/N of the batch "
              "with no collective.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2108_03948_amd as tz
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # the autotuner's FFT-pair costs pick the Bluestein lengths of every plan
    # below (read from the tune cache when this device was tuned before)
    if "fft_pair_ns=measured" not in tz.tune_describe():
        tz.autotune()
    tune = tz.tune_describe()
    log(f"bench: autotune: {tune}")
    log("bench: generating 8192 x 4096 synthetic traces")
    x_np = synth.pairs(N_PAIRS, N=N, fs=FS)
    x = torch.from_numpy(x_np).to(dev)
    B = x.shape[0]
    W, A = tz.czt_band(FS, F1, F2, M)
    Xc = torch.empty((B, M), dtype=torch.complex64, device=dev)
    Xf = torch.empty((B, NFFT), dtype=torch.complex64, device=dev)
    Xz = torch.empty((B, M), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        tz.czt(x, M, W, A, out=Xc, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        tz.fft_zeropad(x, NFFT - N, out=Xf, stream=stream)
        if ev is not None:
            ev[2].record(stream)
        tz.zoom_fft(x, FS, F1, F2, M, ZOOM_D, taps=ZOOM_T, out=Xz, stream=stream)
        if ev is not None:
            ev[3].record(stream)

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("bench: calibration copy of 1 GiB done")

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step_events = sum(e[0].elapsed_time(e[3]) for e in evs) / args.steps
    ms_czt = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    ms_fft = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    ms_zoom = sum(e[2].elapsed_time(e[3]) for e in evs) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    log(f"bench: step {ms_per_step:.3f} ms (events {ms_step_events:.3f}); czt {ms_czt:.3f}, "
        f"fft_zeropad {ms_fft:.3f}, zoom {ms_zoom:.3f} ms")

    kernels = {}
    for name, ms, (by, fl), bins in (("czt", ms_czt, czt_work(B), B * M),
                                     ("fft_zeropad", ms_fft, fft_work(B), B * NFFT),
                                     ("zoom_fft", ms_zoom, zoom_work(B), B * M)):
        kernels[name] = {
            "ms": ms, "bins_per_s": bins / (ms * 1e-3),
            "alg_bytes": by, "alg_flops": fl,
            "GBps": by / (ms * 1e-3) / 1e9, "hbm_frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "TFLOPs": fl / (ms * 1e-3) / 1e12, "fp32_frac": fl / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
        }
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    dk = kernels[dom]
    hbm_bound = dk["alg_flops"] / dk["alg_bytes"] < FP32_VECTOR_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = None
    try:
        t = json.load(open(TRAFFIC_FILE))
        if t.get("source_hash") == kernel_source_hash() and dom in t.get("kernels", {}):
            traffic = t["kernels"][dom]["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None
    # the same kernel's average over the timed dispatches of the committed
    # rocprofv3 run, if the sources still hash to the profiled ones
    profiled = None
    try:
        t = json.load(open(PROFILED_FILE))
        if t.get("source_hash") == kernel_source_hash() and t.get("kernel") == dom:
            us = t["timed_average_us"]
            profiled = {"avg_us": us, "median_us": t["timed_median_us"], "dispatches": t["timed_dispatches"],
                        "achieved": dk["alg_bytes"] / (us * 1e-6) / 1e9,
                        "frac": dk["alg_bytes"] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                        "source": os.path.relpath(PROFILED_FILE, ROOT)}
    except (OSError, ValueError, KeyError):
        profiled = None
    if hbm_bound:
        roof = {"bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["hbm_frac"], "traffic": traffic, "kernel": dom,
                "event_avg_us": dk["ms"] * 1e3, "profiled": profiled}
    else:
        roof = {"bound": "alu", "achieved": dk["TFLOPs"], "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": dk["fp32_frac"], "traffic": traffic, "kernel": dom}

    # the error of this very run on two traces, against the FP64 direct summation
    rows = [0, B - 1]
    ref = fp64_czt(tz, x_np[rows], M, W, A, dev)

    def rel_err(Xd):
        got = Xd[rows].cpu().numpy()
        return float(np.max(np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)))

    err = rel_err(Xc)

    # the same CZT with the radix-16 passes on the matrix cores
    mfma = {"fp32_ms": ms_czt}
    Xs = torch.empty_like(Xc)
    for prec in ("split_fp16", "split_bf16"):
        for _ in range(2):
            tz.czt(x, M, W, A, out=Xs, precision=prec, stream=stream)
        reps = max(5, args.steps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            tz.czt(x, M, W, A, out=Xs, precision=prec, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        mfma[prec] = {"ms": ms, "speedup_vs_fp32": ms_czt / ms, "rel_l2_sampled": rel_err(Xs),
                      "bins_per_s": B * M / (ms * 1e-3)}
        log(f"bench: czt {prec} {ms:.3f} ms ({ms_czt / ms:.2f}x fp32), rel L2 {mfma[prec]['rel_l2_sampled']:.2e}")

    # frequency response of the 4096 reference/sample pairs, fused
    Ht = torch.empty((B // 2, M), dtype=torch.complex64, device=dev)
    for _ in range(2):
        tz.czt_transfer(x, M, W, A, out=Ht, stream=stream)
    reps = max(5, args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        tz.czt_transfer(x, M, W, A, out=Ht, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_tr = e0.elapsed_time(e1) / reps
    Xo = fp64_czt(tz, x_np[:2], M, W, A, dev)
    werr = float(np.linalg.norm(Xo[0] * (Ht[0].cpu().numpy() - Xo[1] / Xo[0])) / np.linalg.norm(Xo[1]))
    transfer = {"ms": ms_tr, "pairs": B // 2, "H_bins_per_s": (B // 2) * M / (ms_tr * 1e-3),
                "weighted_rel_l2_sampled": werr}
    log(f"bench: czt_transfer {ms_tr:.3f} ms for {B // 2} pairs, weighted rel L2 {werr:.2e}")

    # inverse DFT of the 8192 CZT spectra (4096 complex points each: the
    # direct one-FFT-per-row form), back to 4096 time samples per row
    Xi = torch.empty_like(Xc)
    for _ in range(2):
        tz.ifft(Xc, out=Xi, stream=stream)
    reps = max(5, args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        tz.ifft(Xc, out=Xi, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_if = e0.elapsed_time(e1) / reps
    # every sample of two rows: a pulse concentrates its energy in a few
    # samples, so a sparse sample of a row would weigh the rounding floor of
    # the near-zero ones
    ri = torch.fft.ifft(Xc[:2].to(torch.complex128), dim=1).cpu().numpy()  # torch's FFT in complex128
    ierr = float(np.linalg.norm(Xi[:2].cpu().numpy() - ri) / np.linalg.norm(ri))
    ifft_b = 2 * B * M * 8
    inverse = {"ms": ms_if, "rows": B, "points": M, "alg_GBps": ifft_b / (ms_if * 1e-3) / 1e9,
               "hbm_frac": ifft_b / (ms_if * 1e-3) / 1e9 / HBM_PEAK_GBS, "rel_l2_sampled": ierr}
    log(f"bench: ifft {ms_if:.3f} ms for {B} x {M}, {inverse['alg_GBps']:.0f} GB/s, rel L2 {ierr:.2e}")

    nd = bench_nd(tz, synth, dev, stream, max(3, args.steps // 4))
    single = uneven = longs = None
    if not args.step_only:
        single = bench_single(tz, synth, dev, stream)
        uneven = bench_uneven(tz, synth, dev, stream, max(5, args.steps // 2))
        longs = bench_long(tz, synth, dev, stream, 5)

    out = {
        "metric": METRIC,
        "value": B * M / (ms_per_step * 1e-3),
        "unit": "CZT outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "8192 THz-TDS traces (4096 sample/reference pairs) x 4096 FP32 samples, fs 20 THz; "
                        "per step: czt M=4096 over 0.2-2.5 THz + fft_zeropad to 65536 + zoom_fft "
                        "(same band, M=4096, D=6, 63 taps)",
            "traces": B, "samples": N, "czt_bins": M, "fft_bins": NFFT, "zoom_decimation": ZOOM_D,
            "zoom_taps": ZOOM_T,
        },
        "roofline": roof,
        "czt_only": {"value": B * M / (ms_czt * 1e-3), "ms": ms_czt},
        "kernels": kernels,
        "mfma_vs_fp32": mfma,
        "transfer": transfer,
        "ifft": inverse,
        "nd": nd,
        "single_trace_1024_fp64": single,
        "uneven_batch_20000": uneven,
        "long_scans_256x2p20": longs,
        "czt_rel_l2_sampled": err,
        "autotune": tune,
    }
    if not args.no_cpu:
        log("bench: timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(x_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
