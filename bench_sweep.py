"""Resolution sweep: the paper's timing comparison (Section 4, Fig. 11) on one
MI355X.

For a THz trace of N = 500 samples at T_s = 100 fs (the measured trace of
Section 3.2; a synthetic pulse here) the plotting resolution df runs from
20 GHz down to 0.5 GHz in 0.5 GHz steps.  At each df:

  fft_zeropad  N_fft = round(f_s/df) (eq. (3)), i.e. N_fft - N zeros (eq. (5))
  czt          band 0 - 2.5 THz, M = round((f2 - f1) N_fft / f_s) bins (eq. (25))
  zoom_fft     same band and M, f_N = 1.25 THz, D = floor(f_s / (1.25 (f2 - f1))),
               63-tap low-pass; short DFT length K = round(M f_s / (D (f2 - f1)))
  ifft         the N_fft-point inverse DFT of the fft_zeropad spectrum back to
               N_fft time samples (the FFT/IFFT comparison of Section 4, Fig. 12)
  fft / ifft   for 7-smooth N_fft (up to 20480): also the half spectrum, bins
  half         0 .. N_fft/2 (fft_zeropad with TZ_HALF), and its inverse back
               to the real trace (ifft with TZ_HALF), the pair a real THz
               trace goes through

Each method is timed (HIP events on the launch stream, plans built before the
timed region) for one trace, as the paper does, and for a batch of 8192
traces, and normalised to its own time at 20 GHz; the dashed curves of the
paper's figure (theoretical cost) are given as L log2 L of the FFTs each
method runs, normalised the same way.

  python bench_sweep.py [--reps 200] [--batch 8192] [--out FILE.md]

Prints one JSON line per df and, with --out, writes a markdown table.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FS = 10e12            # T_s = 100 fs
N = 500
F1, F2 = 0.0, 2.5e12
TAPS = 63


def sweep_points():
    """df in Hz from 20 GHz down to 0.5 GHz in 0.5 GHz steps."""
    return [(40 - i) * 0.5e9 for i in range(40)]


def shapes(tz, df):
    """Transform sizes the sweep uses at resolution df."""
    nfft = int(round(FS / df))
    M = tz.czt_points_for_resolution(FS, F1, F2, nfft)
    D = max(1, int(math.floor(FS / (1.25 * (F2 - F1)))))
    K = tz.zoom_short_length(FS, F1, F2, M, D)
    return {"df_hz": df, "n_fft": nfft, "n_zeros": nfft - N, "M": M, "D": D, "K": K}


def smooth7(n):
    for f in (2, 3, 5, 7):
        while n % f == 0:
            n //= f
    return n == 1


def direct_ifft(n):
    """ifft runs one FFT of length n (power of two 256..16384, or 7-smooth
    8..20480 on the mixed-radix kernel) rather than the Bluestein form."""
    return (256 <= n <= 16384 and n & (n - 1) == 0) or (8 <= n <= 20480 and smooth7(n))


def theory(tz, s):
    """FFT work of each method: sum of L log2 L over the FFTs it runs."""
    def c(L):
        return L * math.log2(L)
    L_czt, _ = tz.czt_plan_shape(N, s["M"])
    LD = -(-N // s["D"])
    L_zoom, _ = tz.czt_plan_shape(LD, s["M"])
    n = s["n_fft"]
    L_ifft = n if direct_ifft(n) else tz.czt_plan_shape(n, n)[0]
    return {"fft": c(n), "czt": 2 * c(L_czt), "zoom": 2 * c(L_zoom),
            "ifft": c(L_ifft) * (1 if direct_ifft(n) else 2)}


def pow2_neighbour(n):
    """The power of two nearest to n in log scale, at least N."""
    lo = 1 << int(math.floor(math.log2(n)))
    hi = lo * 2
    p = lo if math.log2(n) - math.log2(lo) <= math.log2(hi) - math.log2(n) else hi
    return max(p, 1 << int(math.ceil(math.log2(N))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=200, help="timed calls per point (single trace)")
    ap.add_argument("--batch", type=int, default=8192, help="traces in the batched measurement")
    ap.add_argument("--out", default=None, help="also write a markdown table here")
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2108_03948_amd as tz
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    x1 = torch.from_numpy(synth.single_trace(N=N, fs=FS, t0=15e-12).astype(np.float32)).to(dev).reshape(1, N)
    xb = torch.from_numpy(synth.pairs(args.batch // 2, N=N, fs=FS, t0=15e-12)).to(dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3  # us

    rows = []
    for df in sweep_points():
        s = shapes(tz, df)
        W, A = tz.czt_band(FS, F1, F2, s["M"])
        out = {}
        for tag, x, reps in (("single", x1, args.reps), ("batch", xb, max(3, args.reps // 20))):
            Xf = torch.empty((x.shape[0], s["n_fft"]), dtype=torch.complex64, device=dev)
            Xc = torch.empty((x.shape[0], s["M"]), dtype=torch.complex64, device=dev)
            Xz = torch.empty_like(Xc)
            Xi = torch.empty_like(Xf)
            tz.fft_zeropad(x, s["n_zeros"], out=Xf, stream=stream)
            out[tag] = {
                "fft": timed(lambda: tz.fft_zeropad(x, s["n_zeros"], out=Xf, stream=stream), reps),
                "czt": timed(lambda: tz.czt(x, s["M"], W, A, out=Xc, stream=stream), reps),
                "zoom": timed(lambda: tz.zoom_fft(x, FS, F1, F2, s["M"], s["D"], taps=TAPS, out=Xz,
                                                  stream=stream), reps),
                "ifft": timed(lambda: tz.ifft(Xf, out=Xi, stream=stream), reps),
            }
            if s["n_fft"] <= 20480 and smooth7(s["n_fft"]):
                nh = s["n_fft"] // 2 + 1
                Xh = torch.empty((x.shape[0], nh), dtype=torch.complex64, device=dev)
                xr = torch.empty((x.shape[0], s["n_fft"]), dtype=torch.float32, device=dev)
                tz.fft_zeropad(x, s["n_zeros"], half=True, out=Xh, stream=stream)
                out[tag]["fft_half"] = timed(lambda: tz.fft_zeropad(x, s["n_zeros"], half=True, out=Xh,
                                                                    stream=stream), reps)
                out[tag]["ifft_half"] = timed(lambda: tz.ifft(Xh, half=True, N=s["n_fft"], out=xr,
                                                              stream=stream), reps)
                del Xh, xr
            # the zero-padded FFT at the nearest power-of-two length, for the
            # cost of a 7-smooth N_fft against it
            n2 = pow2_neighbour(s["n_fft"])
            X2 = torch.empty((x.shape[0], n2), dtype=torch.complex64, device=dev)
            out[tag]["fft_pow2"] = timed(lambda: tz.fft_zeropad(x, n2 - N, out=X2, stream=stream), reps)
            del Xf, Xc, Xz, Xi, X2
        row = dict(s, us=out, theory=theory(tz, s), pow2=pow2_neighbour(s["n_fft"]),
                   smooth7=smooth7(s["n_fft"]))
        rows.append(row)
        print(json.dumps(row), flush=True)

    base = rows[0]
    methods = ("fft", "czt", "zoom", "ifft")
    for r in rows:
        r["rel"] = {tag: {m: r["us"][tag][m] / base["us"][tag][m] for m in methods}
                    for tag in ("single", "batch")}
        r["rel_theory"] = {m: r["theory"][m] / base["theory"][m] for m in methods}
    if args.out:
        cmd = "python bench_sweep.py " + " ".join(sys.argv[1:])
        lines = ["# Resolution sweep: time per call vs plotting resolution", "",
                 f"Command:\n\n    {cmd}\n",
                 f"N = {N} samples at f_s = {FS / 1e12:g} THz, band {F1 / 1e12:g}-{F2 / 1e12:g} THz, "
                 f"zoom {TAPS} taps; single trace ({args.reps} calls per point) and "
                 f"{args.batch} traces; times in microseconds, rel = time / time at 20 GHz.  "
                 "7s: N_fft is 7-smooth (mixed-radix FFT and IFFT); pow2: the nearest power-of-two "
                 "N_fft, fft 2^k B its batched zero-padded FFT time; fft/2^k and ifft/fft are ratios of "
                 "the batched times; fft h B / ifft h B: the half spectrum and its inverse to the real "
                 "trace (7-smooth N_fft), ih/fh their ratio.", "",
                 "| df (GHz) | N_fft | 7s | M | D | K | fft 1 | czt 1 | zoom 1 | ifft 1 | fft B | czt B | zoom B | "
                 "ifft B | pow2 | fft 2^k B | fft/2^k | ifft/fft | fft h B | ifft h B | ih/fh | "
                 "rel fft B | rel czt B | rel zoom B | "
                 "rel ifft B | theory fft | theory czt | theory zoom | theory ifft |",
                 "|" + "---|" * 29]
        for r in rows:
            u1, ub, rb, th = r["us"]["single"], r["us"]["batch"], r["rel"]["batch"], r["rel_theory"]
            lines.append(f"| {r['df_hz'] / 1e9:.1f} | {r['n_fft']} | {'y' if r['smooth7'] else ''} | {r['M']} | "
                         f"{r['D']} | {r['K']} | "
                         f"{u1['fft']:.1f} | {u1['czt']:.1f} | {u1['zoom']:.1f} | {u1['ifft']:.1f} | "
                         f"{ub['fft']:.1f} | {ub['czt']:.1f} | {ub['zoom']:.1f} | {ub['ifft']:.1f} | "
                         f"{r['pow2']} | {ub['fft_pow2']:.1f} | {ub['fft'] / ub['fft_pow2']:.2f} | "
                         f"{ub['ifft'] / ub['fft']:.2f} | "
                         + (f"{ub['fft_half']:.1f} | {ub['ifft_half']:.1f} | {ub['ifft_half'] / ub['fft_half']:.2f} | "
                            if "fft_half" in ub else " |  |  | ") +
                         f"{rb['fft']:.2f} | {rb['czt']:.2f} | {rb['zoom']:.2f} | {rb['ifft']:.2f} | "
                         f"{th['fft']:.2f} | {th['czt']:.2f} | {th['zoom']:.2f} | {th['ifft']:.2f} |")
        with open(args.out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
