"""Summarise rocprofv3 output of bench.py into short text files under profiles/.

  python bench_profiles.py stats <kernel_stats.csv> <out.md> "<command>"
  python bench_profiles.py traffic <fetch_counter.csv> <write_counter.csv> <out.json> "<cmd>"
  python bench_profiles.py kernel-traffic <fetch_counter.csv> <write_counter.csv> <kernel_trace.csv>
         <calibration.json> <out.md> "<cmd>" <name-substring> ...
  python bench_profiles.py utilization <counter.csv> <out.md> "<cmd>" <name-substring> ...
  python bench_profiles.py timed <kernel_trace.csv> <out.json> "<cmd>" <warmup> <steps>
  python bench_profiles.py instructions <counter.csv> <out.md> "<cmd>"

Byte counters are scaled by what the same counters read for the 1 GiB device
copy that ``bench.py --calib-copy`` runs first (dispatch with the largest grid
among the runtime's copy kernels).
"""
from __future__ import annotations

import csv
import json
import os
import sys

# bench dispatches: (kernel-name substring, grid size in work-items or None);
# the grid tells the timed 8192 x 4096 launches from the same kernels' use in
# the multi-dimensional transforms
KERNEL_KEYS = {"czt": ("k_czt_half<8192, 0>", 4194304), "fft_zeropad": ("k_fftpad_real<2048, 16, 0>", None),
               "zoom_front": ("k_zoom_front<0, 1, false>", 6291456),
               "zoom_short_dft": ("k_czt<2048, 2, false>", 3145728),
               "transpose_2d_scans": ("k_transpose_c64", 524288), "transpose_3d_cube": ("k_transpose_c64", 2097152),
               "ifft": ("k_ifft_pow2<4096>", None)}


def stats(path, out, cmd):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics\n", f"Command:\n\n    {cmd}\n",
             "| kernel | calls | average (us) | min (us) | max (us) | share (%) |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.2f} | "
                     f"{float(r['MinNs'])/1e3:.2f} | {float(r['MaxNs'])/1e3:.2f} | {float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path, counter):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def traffic(fetch_csv, write_csv, out, cmd, source_hash):
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")
    copy_f = max((x for x in f if "copyBuffer" in x[0]), key=lambda x: x[1])
    copy_w = max((x for x in w if "copyBuffer" in x[0]), key=lambda x: x[1])
    gib_kib = 1024.0 * 1024.0
    sf, sw = gib_kib / copy_f[2], gib_kib / copy_w[2]
    res = {"command": cmd, "source_hash": source_hash,
           "calibration": {"copy_bytes": 1 << 30, "fetch_kib": copy_f[2], "write_kib": copy_w[2],
                           "fetch_scale": sf, "write_scale": sw},
           "kernels": {}}
    for name, (key, grid) in KERNEL_KEYS.items():
        fv = [x[2] for x in f if key in x[0] and grid in (None, x[1])]
        wv = [x[2] for x in w if key in x[0] and grid in (None, x[1])]
        if fv and wv:
            fb = sum(fv) / len(fv) * 1024 * sf
            wb = sum(wv) / len(wv) * 1024 * sw
            res["kernels"][name] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                                    "hbm_bytes_per_launch": fb + wb}
    json.dump(res, open(out, "w"), indent=1)


def kernel_traffic(fetch_csv, write_csv, stats_csv, calib_json, out, cmd, keys):
    """Per-dispatch HBM bytes of the named kernels (counters scaled by the
    copy calibration recorded in calib_json) against their average durations."""
    cal = json.load(open(calib_json))["calibration"]
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")
    # average duration per (kernel, grid size) from the kernel trace
    acc = {}
    for r in csv.DictReader(open(stats_csv)):
        key = (r["Kernel_Name"].split("(")[0],
               int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
        a = acc.setdefault(key, [0.0, 0])
        a[0] += float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        a[1] += 1
    dur = {k: v[0] / v[1] for k, v in acc.items()}
    lines = ["# HBM traffic per dispatch", "", f"Command (counters, one run per counter):\n\n    {cmd}\n",
             f"Scaled by the 1 GiB copy calibration of `profiles/traffic.json` (FETCH x{cal['fetch_scale']:.3f}, "
             f"WRITE x{cal['write_scale']:.3f}); durations from the kernel-trace run of the same command, "
             "per kernel and grid size (work-items).", "",
             "| kernel | grid | dispatches | fetch (MB) | write (MB) | average (us) | GB/s |",
             "|---|---|---|---|---|---|---|"]
    groups = sorted({(x[0].split("(")[0], x[1]) for x in f if any(k in x[0] for k in keys)})
    for name, grid in groups:
        fv = [x[2] for x in f if x[0].split("(")[0] == name and x[1] == grid]
        wv = [x[2] for x in w if x[0].split("(")[0] == name and x[1] == grid]
        if not fv or not wv or (name, grid) not in dur:
            continue
        fb = sum(fv) / len(fv) * 1024 * cal["fetch_scale"]
        wb = sum(wv) / len(wv) * 1024 * cal["write_scale"]
        us = dur[(name, grid)] / 1e3
        lines.append(f"| `{name}` | {grid} | {len(fv)} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {us:.1f} | "
                     f"{(fb + wb) / (us * 1e-6) / 1e9:.0f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def utilization(counter_csv, out, cmd, keys):
    """VALUBusy and MfmaUtil (percent of the dispatch's GPU-active time the
    vector ALUs / matrix cores were busy) per kernel and grid size."""
    acc = {}
    for r in csv.DictReader(open(counter_csv)):
        name = r["Kernel_Name"].split("(")[0]
        if not any(k in r["Kernel_Name"] for k in keys):
            continue
        d = acc.setdefault((name, int(r["Grid_Size"])), {})
        d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["# Vector ALU and matrix-core utilization per dispatch", "",
             f"Command:\n\n    {cmd}\n",
             "VALUBusy = 100 SQ_ACTIVE_INST_VALU / (CUs x GRBM_GUI_ACTIVE); MfmaUtil = 100 "
             "SQ_VALU_MFMA_BUSY_CYCLES / (SIMDs x GRBM_GUI_ACTIVE), averaged over the dispatches of each "
             "kernel and grid size (work-items).", "",
             "| kernel | grid | dispatches | VALUBusy (%) | MfmaUtil (%) |", "|---|---|---|---|---|"]
    for (name, grid), d in sorted(acc.items()):
        vb, mu = d.get("VALUBusy", []), d.get("MfmaUtil", [])
        if not vb:
            continue
        lines.append(f"| `{name}` | {grid} | {len(vb)} | {sum(vb) / len(vb):.1f} | "
                     f"{(sum(mu) / len(mu)) if mu else float('nan'):.1f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def timed(trace_csv, out, cmd, warmup, steps, source_hash):
    """Durations of the dominant kernel's dispatches in the timed steps of a
    profiled bench.py run: the first `warmup` dispatches of the kernel (one
    per warm-up step) are dropped, the next `steps` kept, so the average is
    taken over the same launches the bench line's event timing covers."""
    key, grid = KERNEL_KEYS["fft_zeropad"]
    rows = [r for r in csv.DictReader(open(trace_csv)) if key in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    if len(d) < warmup + steps:
        raise SystemExit(f"{len(d)} dispatches of {key}, expected {warmup} warm-up + {steps} timed")
    t = sorted(d[warmup:warmup + steps])
    res = {"command": cmd, "source_hash": source_hash, "kernel": "fft_zeropad", "name": key,
           "warmup_dispatches_us": d[:warmup], "timed_dispatches": steps,
           "timed_average_us": sum(t) / len(t), "timed_median_us": t[len(t) // 2],
           "timed_min_us": t[0], "timed_max_us": t[-1]}
    json.dump(res, open(out, "w"), indent=1)


# the bench step's kernels: (name substring, grid size, points per dispatch, what a point is)
STEP_POINTS = [
    ("k_czt_half<8192, 0>", 4194304, 8192 * 8192,
     "czt: 8192 Bluestein pairs of L = 8192, as two 4096-point pairs each (per point of L: premultiply, "
     "two FFTs, x V, postmultiply)"),
    ("k_fftpad_real<2048, 16, 0>", None, 8192 * 16 * 2048,
     "fft_zeropad: 8192 traces x 16 FFTs of 2048 + the real-input combine to 65536 bins (per complex FFT point)"),
    ("k_czt<2048, 2, false>", 3145728, 8192 * 3 * 2048,
     "zoom short DFT: 8192 x 3 bin blocks, Bluestein pairs of L = 2048 (per point of L)"),
    ("k_zoom_front<0, 1, false>", 6291456, 8192 * 683,
     "zoom front end: 8192 x 683 outputs of 63 FP64 taps (per output)"),
]


def instructions(counter_csv, out, cmd):
    """SQ_INSTS_VALU / SALU / LDS of the step's kernels per point (a wave's
    instruction counts once for its 64 lanes)."""
    acc = {}
    for r in csv.DictReader(open(counter_csv)):
        for key, grid, pts, what in STEP_POINTS:
            if key in r["Kernel_Name"] and (grid is None or int(r["Grid_Size"]) == grid):
                d = acc.setdefault((key, int(r["Grid_Size"])), {"pts": pts, "what": what, "n": {}, "v": {}})
                c = r["Counter_Name"]
                d["v"][c] = d["v"].get(c, 0.0) + float(r["Counter_Value"])
                d["n"][c] = d["n"].get(c, 0) + 1
    lines = ["# Instructions per point of the bench step's kernels\n", f"Command:\n\n    {cmd}\n",
             "Counters are per dispatch, summed over the waves (one instruction of a wave counts once, for 64 "
             "lanes); per point = counter x 64 / points of the launch.\n",
             "| kernel | grid | waves | VALU / point | SALU / point | LDS / point | what a point is |",
             "|---|---|---|---|---|---|---|"]
    for (key, grid), d in acc.items():
        avg = {c: d["v"][c] / d["n"][c] for c in d["v"]}
        per = {c: avg.get(c, 0.0) * 64 / d["pts"] for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS")}
        lines.append(f"| `{key}` | {grid} | {avg.get('SQ_WAVES', 0):.0f} | {per['SQ_INSTS_VALU']:.1f} | "
                     f"{per['SQ_INSTS_SALU']:.1f} | {per['SQ_INSTS_LDS']:.1f} | {d['what']} |")
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "timed":
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import bench
        timed(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]), bench.kernel_source_hash())
    elif sys.argv[1] == "utilization":
        utilization(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:])
    elif sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "instructions":
        instructions(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "kernel-traffic":
        kernel_traffic(*sys.argv[2:8], sys.argv[8:])
    else:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import bench
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], bench.kernel_source_hash())
