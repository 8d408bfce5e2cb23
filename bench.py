#!/usr/bin/env python3
"""Throughput of the Spectral Ewald k-space evaluation on one MI355X.

One step = one full pass of the hot path on the device-resident inputs:
bin/sort, spread (eq. 4.5), forward FFT, scaling + k-space energy (eq. 4.6),
inverse FFT, gather of phi and F (eqs. 4.9, 4.12).  Default workload:
synthetic 3-site water at liquid density, L = 100 A (100,200 atoms),
xi = 0.3 A^-1, M = 96, P = 8.  At these parameters the FP32 form matches the
FP64 oracle to a relative rms force error of about 2e-6 (the implementation
error, held to 1e-5); the method's own error against a converged reference
is 1.5e-4 here, and P = 10 brings it to 1.0e-5 (the matched-accuracy row).
The headline value is FP32; the FP64 form at the same parameters is reported
beside it, and the 10^6-ion SE/SPME comparison after it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SE k-space E+F atom-evals/s at rms force err 1e-5, FP32 vs FP64; %HBM peak"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
CALIB_COPY_BYTES = 256 << 20     # bytes read (and written) by the calibration copy
REAL_SPACE_RC = 10.0             # A: the usual MD cutoff, for the real-space line
# FP32 operations of the real-space kernel: the distance test of a tested
# pair (3 differences, 3 scalings, |r|^2) and the terms of a pair in range
# (rsqrt, xi r, e^{-x^2}, t, eight-term polynomial, phi and force updates)
RS_FLOPS_TEST, RS_FLOPS_PAIR = 11, 38
PROFILES = os.path.join(ROOT, "profiles")

# source files each kernel is built from (a change voids stored counters and traces)
CSRC = os.path.join(ROOT, "paper_1712_04718_amd", "csrc")
KERNEL_SOURCES = {
    "gather": ("gather.hip", "window.hpp", "se_common.hpp"),
    "spread": ("spread.hip", "window.hpp", "se_common.hpp"),
    "fold": ("spread.hip", "se_common.hpp"),
    "bin_count": ("bin.hip", "se_common.hpp"),
    "bin_scan": ("bin.hip", "se_common.hpp"),
    "bin_scatter": ("bin.hip", "se_common.hpp"),
}
for _st in ("fft_x", "fft_y", "fft_z_scale", "ifft_y", "ifft_x", "fft_xy", "ifft_yx"):
    KERNEL_SOURCES[_st] = ("fft.hip", "se_common.hpp")

# kernel names of each stage in a rocprofv3 trace (FP32 instantiations)
STAGE_KERNEL_RE = {
    "bin_count": r"k_bin_count_(lds|run)<float", "bin_scan": r"k_bin_scan\b",
    "bin_scatter": r"k_bin_scatter(_scan)?<float>",
    "spread": r"k_spread(_lane)?<float,", "fold": r"k_fold(_tiles)?<float",
    "fft_x": r"k_fft_x_r2c<float,", "fft_y": r"k_fft_y<float, -?\d+, \d+, false>",
    "fft_z_scale": r"k_fft_z_scale<float,", "ifft_y": r"k_fft_y<float, -?\d+, \d+, true>",
    "ifft_x": r"k_fft_x_c2r<float,", "gather": r"k_gather(_lane)?<float,",
    "fft_xy": r"k_fft_xy_r2c<float,", "ifft_yx": r"k_fft_yx_c2r<float,",
}
CALIB_KERNEL_RE = r"neg_kernel"

# the 10^6-ion comparison (tuned to a relative rms force error of 1e-4,
# tests/golden/spme_tuned_grid.json): (window, support or order, M)
C5_CASES = (("gaussian", 8, 192), ("gaussian", 10, 192), ("bspline", 4, 432),
            ("bspline", 6, 192))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(stage):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[stage]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_work(stage, N, M, P, rs):
    """Algorithmic work of one launch of a stage: (kind, amount).  Bytes for
    the grid passes and binning, flops for spread and gather.  The fold's
    algorithmic bytes are the grid it writes (the spread step's output,
    4 M^3 in FP32): the tile blocks it reads are this implementation's
    overhead, which the counter traffic shows."""
    K = M // 2 + 1
    grid, spec = M ** 3 * rs, M * M * K * 2 * rs
    if stage == "bin_count":
        return "bytes", N * 4 * rs + N * 8                  # x, q in; keys out
    if stage == "bin_scan":
        return "bytes", 0                                  # a handful of counters
    if stage == "bin_scatter":  # x, q, keys in; sorted particles and indices out
        return "bytes", N * 4 * rs + N * 8 + N * (4 * rs + 8)
    if stage == "spread":
        return "flops", N * 2 * P ** 3                      # a multiply and an add per point
    if stage == "gather":
        return "flops", N * 4 * P ** 3                      # two multiply-adds per point
    if stage == "fold":
        return "bytes", grid
    if stage in ("fft_x", "fft_xy"):
        return "bytes", grid + spec
    if stage in ("ifft_x", "ifft_yx"):
        return "bytes", spec + grid
    return "bytes", 2 * spec                                # fft_y, fft_z_scale, ifft_y


def step_bytes(N, M, rs):
    """What one step must move through HBM (r = bytes per real): x, q in and
    phi, F out (8 r N), the sorted copy written and read (8 r N), the spread
    grid written (r M^3), three grid passes read and written (6 r M^3) and
    the grid read by the gather (r M^3): 8 r M^3 + 16 r N."""
    return 8 * rs * M ** 3 + 16 * rs * N


def stored(kind, stage, workload, P, window, tag="f32"):
    """A committed per-kernel figure (kind 'traffic': HBM bytes per launch
    from counters; kind 'trace': mean kernel duration from a rocprofv3
    kernel trace) for this kernel, workload and the kernel's current sources,
    else (None, None)."""
    name = {"traffic": f"traffic_{workload}_{window}_P{P}_{tag}.json",
            "trace": f"kernels_{workload}_{window}_P{P}_{tag}.json"}[kind]
    path = os.path.join(PROFILES, name)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, None
    st = rec.get("stages", {}).get(stage)
    if st is None or st.get("source_sha256_16") != source_hash(stage):
        return None, None
    key = "traffic_bytes_per_launch" if kind == "traffic" else "mean_us"
    return st.get(key), os.path.relpath(path, ROOT)


def lds_atomic_peak():
    """Measured LDS integer-atomic rate of the MI355X in the spread's access
    pattern (lane-atomics per second), from the committed probe summary."""
    try:
        with open(os.path.join(PROFILES, "lds_atomic_rate.json")) as f:
            rec = json.load(f)
        return rec["spread_pattern_float_lane_atomics_per_s"], "profiles/lds_atomic_rate.json"
    except (OSError, ValueError, KeyError):
        return None, None


def _bench_line(log_path):
    """The JSON line a bench.py run printed (None if absent)."""
    try:
        with open(log_path) as f:
            for line in f:
                if line.startswith("{") and '"metric"' in line:
                    return json.loads(line)
    except OSError:
        pass
    return None


def _csv_rows(d, suffix):
    import csv
    rows = []
    for path in glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True):
        with open(path) as f:
            rows.extend(csv.DictReader(f))
    return rows


def _workload_of(line):
    cfg = line["config"]
    return cfg["workload"].split(":")[0], cfg["P"], cfg.get("window", "gaussian"), cfg["M"], cfg["N"]


def summarize_counters(fetch_dir, write_dir, fetch_log, write_log):
    """Turn two rocprofv3 --pmc runs of bench.py (FETCH_SIZE, WRITE_SIZE, in
    KiB per dispatch) into HBM bytes per launch of each k-space kernel,
    scaled by what the same counters read for the calibration copy of
    CALIB_COPY_BYTES.  Writes profiles/traffic_<workload>_<window>_P<P>_f32.json
    (read back by stored()) and a markdown table beside it."""
    line = _bench_line(fetch_log) or _bench_line(write_log)
    if line is None:
        raise SystemExit("no bench.py JSON line in the counter runs' logs")
    workload, P, window, M, N = _workload_of(line)
    hashes = line.get("sources") or {}
    fetch = [(r["Kernel_Name"], float(r["Counter_Value"]))
             for r in _csv_rows(fetch_dir, "counter_collection.csv") if r["Counter_Name"] == "FETCH_SIZE"]
    write = [(r["Kernel_Name"], float(r["Counter_Value"]))
             for r in _csv_rows(write_dir, "counter_collection.csv") if r["Counter_Name"] == "WRITE_SIZE"]

    def mean_of(rows, pattern):
        v = [val for name, val in rows if re.search(pattern, name)]
        return (sum(v) / len(v), len(v)) if v else (None, 0)

    cf, _ = mean_of(fetch, CALIB_KERNEL_RE)
    cw, _ = mean_of(write, CALIB_KERNEL_RE)
    if not cf or not cw:
        raise SystemExit("calibration copy not found in the counter runs")
    kf, kw = CALIB_COPY_BYTES / (cf * 1024.0), CALIB_COPY_BYTES / (cw * 1024.0)
    rec = {"workload": workload, "P": P, "window": window, "dtype": "f32", "M": M, "N": N,
           "counters": "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE (KiB per dispatch)",
           "calibration": {"kernel": "torch.neg over float32 (elementwise copy)",
                           "bytes_read": CALIB_COPY_BYTES, "bytes_written": CALIB_COPY_BYTES,
                           "fetch_kib": cf, "write_kib": cw,
                           "fetch_factor": kf, "write_factor": kw},
           "step_algorithmic_bytes": step_bytes(N, M, 4),
           "stages": {}}
    cmd = line.get("command", "python3 bench.py")
    md = [f"# HBM traffic per launch: {workload}, {window} window, P={P}, M={M}, N={N}, FP32\n",
          "Counters from two `rocprofv3 --pmc` runs of bench.py (FETCH_SIZE, then WRITE_SIZE; "
          "KiB per dispatch), each scaled by what the counter reads for a calibration copy of "
          f"{CALIB_COPY_BYTES >> 20} MiB (torch.neg): fetch factor {kf:.4f}, write factor {kw:.4f}.\n",
          "```",
          f"cd /tmp && rocprofv3 --pmc FETCH_SIZE -f csv -d <out-dir> -o bench -- {cmd}",
          f"cd /tmp && rocprofv3 --pmc WRITE_SIZE -f csv -d <out-dir> -o bench -- {cmd}",
          "```\n",
          "| stage | dispatches | fetch MB | write MB | traffic MB | algorithmic | ratio |",
          "|---|---|---|---|---|---|---|"]
    total = 0.0
    for st, pat in STAGE_KERNEL_RE.items():
        f_kib, nf = mean_of(fetch, pat)
        w_kib, nw = mean_of(write, pat)
        if f_kib is None or w_kib is None:
            continue
        traffic = f_kib * 1024.0 * kf + w_kib * 1024.0 * kw
        total += traffic
        kind, amount = kernel_work(st, N, M, P, 4)
        rec["stages"][st] = {"dispatches": min(nf, nw), "fetch_kib": f_kib, "write_kib": w_kib,
                             "traffic_bytes_per_launch": traffic,
                             "algorithmic": {"kind": kind, "per_launch": amount},
                             "source_sha256_16": hashes.get(st, source_hash(st))}
        alg = f"{amount / 1e6:.2f} MB" if kind == "bytes" else f"{amount / 1e9:.3f} GFLOP"
        ratio = f"{traffic / amount:.2f}" if kind == "bytes" and amount else "-"
        md.append(f"| {st} | {min(nf, nw)} | {f_kib * 1024 * kf / 1e6:.2f} | "
                  f"{w_kib * 1024 * kw / 1e6:.2f} | {traffic / 1e6:.2f} | {alg} | {ratio} |")
    rec["step_traffic_bytes"] = total
    md.append("")
    md.append(f"One step's counter traffic {total / 1e6:.1f} MB against the algorithmic "
              f"8 r M^3 + 16 r N = {step_bytes(N, M, 4) / 1e6:.1f} MB (r = 4): ratio "
              f"{total / step_bytes(N, M, 4):.2f}.")
    base = os.path.join(PROFILES, f"traffic_{workload}_{window}_P{P}_f32")
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    with open(base + ".md", "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def _short_name(name):
    """A kernel's name without its namespace, return type and arguments."""
    name = name.replace("sek::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0]


SQ_PASSES = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
             "SQ_WAIT_INST_LDS SQ_INSTS_VALU SQ_INSTS_LDS",
             "SQ_WAVES SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE SQ_WAIT_ANY SQ_ACTIVE_INST_ANY "
             "SQ_INSTS_LDS_ATOMIC SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE")


def summarize_sq(dir1, dir2, bench_log):
    """Turn the two rocprofv3 --pmc passes of SQ_PASSES over this script into
    per-launch means for each k-space stage's FP32 kernels: instruction mix,
    the shares of the waves' resident cycles spent issuing VALU work or
    waiting (on LDS issue, on anything), and the share of the LDS pipe's
    active cycles lost to bank conflicts.  Writes
    profiles/counters_sq_<workload>_<window>_P<P>_f32.md."""
    line = _bench_line(bench_log)
    if line is None:
        raise SystemExit("no bench.py JSON line in the counter run's log")
    workload, P, window, M, N = _workload_of(line)
    rows = _csv_rows(dir1, "counter_collection.csv") + _csv_rows(dir2, "counter_collection.csv")

    def mean(pat, counter):
        v = [float(r["Counter_Value"]) for r in rows
             if r["Counter_Name"] == counter and re.search(pat, r["Kernel_Name"])]
        return sum(v) / len(v) if v else None

    def share(a, b):
        return f"{a / b:.2f}" if a is not None and b else "-"

    cmd = line.get("command", "python3 bench.py")
    md = [f"# SQ counters per launch: {workload} (N={N}, M={M}, {window} window, P={P}), FP32\n",
          "Two `rocprofv3 --pmc` passes over the FP32 bench; means per dispatch of each "
          "stage's kernels.\n", "```"]
    md += [f"cd /tmp && rocprofv3 --pmc {ps} -f csv -d <out-dir> -o bench -- {cmd}"
           for ps in SQ_PASSES]
    md += ["```\n",
           "Shares are ratios of counters in the same units: of the waves' resident cycles "
           "(SQ_WAVE_CYCLES) those issuing VALU work, waiting to issue an LDS instruction, or "
           "waiting on anything; of the LDS pipe's active cycles (SQ_LDS_IDX_ACTIVE) those lost "
           "to bank conflicts.\n",
           "| stage | waves | VALU insts / wave | LDS insts / wave | LDS atomic insts | "
           "VALU-active share | LDS-wait share | any-wait share | LDS bank-conflict share |",
           "|---|---|---|---|---|---|---|---|---|"]
    for st, pat in STAGE_KERNEL_RE.items():
        c = {k: mean(pat, k) for k in ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU",
                                        "SQ_WAIT_INST_LDS", "SQ_INSTS_VALU", "SQ_INSTS_LDS",
                                        "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE",
                                        "SQ_WAIT_ANY", "SQ_INSTS_LDS_ATOMIC")}
        if not c["SQ_WAVES"] or not c["SQ_WAVE_CYCLES"]:
            continue
        w, cyc = c["SQ_WAVES"], c["SQ_WAVE_CYCLES"]
        md.append(f"| {st} | {w:.0f} | {(c['SQ_INSTS_VALU'] or 0) / w:.0f} | "
                  f"{(c['SQ_INSTS_LDS'] or 0) / w:.0f} | {c['SQ_INSTS_LDS_ATOMIC'] or 0:.0f} | "
                  f"{share(c['SQ_ACTIVE_INST_VALU'], cyc)} | {share(c['SQ_WAIT_INST_LDS'], cyc)} | "
                  f"{share(c['SQ_WAIT_ANY'], cyc)} | "
                  f"{share(c['SQ_LDS_BANK_CONFLICT'], c['SQ_LDS_IDX_ACTIVE'])} |")
    base = os.path.join(PROFILES, f"counters_sq_{workload}_{window}_P{P}_f32")
    with open(base + ".md", "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_lds_probe(log_path):
    """Store the LDS-atomic probe's output (paper_1712_04718_amd/probes/
    lds_atomic_rate.hip) as profiles/lds_atomic_rate.{json,md}; the JSON is
    what lds_atomic_peak() reads."""
    with open(log_path) as f:
        text = f.read().splitlines()
    rec = next((json.loads(t) for t in text if t.startswith("{")), None)
    if rec is None:
        raise SystemExit("no JSON line in the probe's output")
    build = ("hipcc --offload-arch=gfx950 -O3 paper_1712_04718_amd/probes/lds_atomic_rate.hip "
             "-o lds_atomic_rate && ./lds_atomic_rate")
    rec["command"] = build
    with open(os.path.join(PROFILES, "lds_atomic_rate.json"), "w") as f:
        json.dump(rec, f, indent=1)
    md = ["# LDS integer-atomic rate in the spread's access pattern\n",
          "A 19^3 block of 32-bit integers per 512-thread work-group, each lane adding 64 "
          "values (8 x 8 rows at a random anchor) with `ds_add_u32`, as the Gaussian spread "
          "does; plain integers, float products rounded to integers (the spread's fixed-point "
          "step), and a conflict-free pattern for reference.\n",
          "```", build, "```\n", "```"] + [t for t in text if not t.startswith("{")] + ["```"]
    with open(os.path.join(PROFILES, "lds_atomic_rate.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_trace(trace_dir, bench_log):
    """Turn a rocprofv3 --kernel-trace --stats run of bench.py into mean
    kernel durations per stage (FP32 instantiations, every dispatch of the
    run).  Writes profiles/kernels_<workload>_<window>_P<P>_f32.json (read back
    by stored()) and a markdown table of every kernel beside it."""
    line = _bench_line(bench_log)
    if line is None:
        raise SystemExit("no bench.py JSON line in the traced run's log")
    workload, P, window, M, N = _workload_of(line)
    hashes = line.get("sources") or {}
    stats = _csv_rows(trace_dir, "kernel_stats.csv")
    if not stats:
        raise SystemExit("no kernel_stats.csv under " + trace_dir)
    # the headline configuration's instantiations (support P, grid M)
    pats = dict(STAGE_KERNEL_RE)
    pats["spread"] = rf"k_spread(_lane)?<float, (\d, )?{P}, \d+>"
    pats["gather"] = rf"k_gather(_lane)?<float, (\d, )?{P}, \d+>"
    pats["fold"] = rf"k_fold_tiles<float, \d, {P}, \d+>|k_fold<float>"
    for st in ("fft_x", "fft_y", "fft_z_scale", "ifft_y", "ifft_x", "fft_xy", "ifft_yx"):
        pats[st] = pats[st].replace(r"-?\d+", str(M)).replace("<float,", f"<float, {M},")
    pats["fft_y"] = rf"k_fft_y<float, {M}, \d+, false>"
    pats["ifft_y"] = rf"k_fft_y<float, {M}, \d+, true>"
    cmd = line.get("command", "python3 bench.py")
    rec = {"workload": workload, "P": P, "window": window, "dtype": "f32", "M": M, "N": N,
           "command": f"rocprofv3 --kernel-trace --stats -f csv -d <out-dir> -o bench -- {cmd}",
           "stages": {}}
    for st, pat in pats.items():
        rows = [r for r in stats if re.search(pat, r["Name"])]
        if not rows:
            continue
        calls = sum(int(r["Calls"]) for r in rows)
        total_ns = sum(float(r["TotalDurationNs"]) for r in rows)
        rec["stages"][st] = {"kernels": [_short_name(r["Name"]) for r in rows], "calls": calls,
                             "mean_us": total_ns / calls / 1e3,
                             "min_us": min(float(r["MinNs"]) for r in rows) / 1e3,
                             "source_sha256_16": hashes.get(st, source_hash(st))}
    md = [f"# Kernel durations: {workload} (N={N}, M={M}, {window} window, P={P})\n",
          "```", f"cd /tmp && {rec['command']}", "```\n",
          "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        name = _short_name(r["Name"])
        md.append(f"| `{name[:100]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                  f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                  f"{float(r['Percentage']):.1f} |")
    step = sum(v["mean_us"] for v in rec["stages"].values())
    md.append("")
    parts = ", ".join(f"{k} {v['mean_us']:.2f}" for k, v in rec["stages"].items())
    md.append(f"Sum of one FP32 k-space step's stage means: {step:.1f} us ({parts}). "
              "The bench line's `stages_us` come from the library's timing plan (each launch's "
              "own start and stop events) over its timed region.")
    base = os.path.join(PROFILES, f"kernels_{workload}_{window}_P{P}_f32")
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    with open(base + ".md", "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def method_error(workload, M, P, window):
    """Relative rms k-space force error of the method itself at (M, P)
    against a converged reference, from the stored oracle-only sweeps
    (tests/golden), or None when none covers this configuration."""
    golden = os.path.join(ROOT, "tests", "golden")
    path = os.path.join(golden, f"{workload}_method_error.json")
    if window == "gaussian" and os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("M") == M and str(P) in rec.get("rel_rms_force", {}):
            return {"rel_rms_force": rec["rel_rms_force"][str(P)], "reference": rec["reference"],
                    "source": os.path.relpath(path, ROOT)}
    path = os.path.join(golden, "spme_tuned_grid.json")
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("workload") != workload:
            return None
        if window == "gaussian":
            for p_, err in rec["se"]["trail"]:
                if p_ == P and rec["se"]["M"] == M:
                    return {"rel_rms_force": err, "reference": rec["reference"],
                            "source": os.path.relpath(path, ROOT)}
        else:
            sp = rec["spme"].get(f"p{P}")
            if sp:
                for m_, err in sp["trail"]:
                    if m_ == M:
                        return {"rel_rms_force": err, "reference": rec["reference"],
                                "source": os.path.relpath(path, ROOT)}
    return None


def percentile(sorted_vals, p):
    if not sorted_vals:
        return float("nan")
    k = (len(sorted_vals) - 1) * p
    lo, hi = math.floor(k), math.ceil(k)
    return sorted_vals[lo] + (sorted_vals[hi] - sorted_vals[lo]) * (k - lo)


# ----------------------------------------------------------------- GPU legs

class Case:
    """One configuration on the device: plan, inputs, outputs, step function."""

    def __init__(self, x, q, L, xi, M, P, window, dtype, dev, timing=False):
        import torch
        from paper_1712_04718_amd import SEPlan, _lib
        self.torch, self._lib = torch, _lib
        self.lib = _lib.load()
        self.N, self.M, self.P, self.L, self.xi, self.window = len(q), M, P, L, xi, window
        self.dtype = dtype
        self.plan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=self.N, device=dev,
                           timing=timing)
        self.xt = torch.tensor(x, dtype=dtype, device=dev)
        self.qt = torch.tensor(q, dtype=dtype, device=dev)
        self.E = torch.empty((), dtype=torch.float64, device=dev)
        self.phi = torch.empty(self.N, dtype=dtype, device=dev)
        self.F = torch.empty(self.N, 3, dtype=dtype, device=dev)
        self.ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (self.xt, self.qt, self.E, self.phi,
                                                             self.F)]

    def step(self):
        s = self.torch.cuda.current_stream().cuda_stream
        self._lib.check(self.lib.se_plan_set_stream(self.plan._plan, ctypes.c_void_p(s)))
        self._lib.check(self.lib.se_kspace(self.plan._plan, self.N, *self.ptrs))

    def time_steps(self, steps, warmup, per_step=False):
        """Mean ms per step of eager launches (and the sorted per-step times)."""
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        evs[0].record()
        for i in range(steps):
            self.step()
            if per_step:
                evs[i + 1].record()
        evs[-1].record()
        torch.cuda.synchronize()
        ms = evs[0].elapsed_time(evs[-1]) / steps
        each = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps)) if per_step else []
        return ms, each

    def time_graph(self, steps, warmup):
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            self.step()  # warm the capture stream
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.step()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def time_autograd(self, steps, warmup, graph=True):
        """(eager, graph) ms per SEEnergy forward + backward step: E = SEEnergy(x, q),
        then E.backward() (the adjoint gather on the stored grid)."""
        torch = self.torch
        from paper_1712_04718_amd import SEEnergy
        xg = self.xt.clone().requires_grad_(True)
        qg = self.qt.clone().requires_grad_(True)
        plan = self.plan

        def fwd_bwd():
            xg.grad = None
            qg.grad = None
            SEEnergy.apply(xg, qg, plan).backward()

        for _ in range(warmup):
            fwd_bwd()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fwd_bwd()
        e1.record()
        torch.cuda.synchronize()
        eager = e0.elapsed_time(e1) / steps
        if not graph:
            return eager, None
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                fwd_bwd()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        xg.grad = None
        qg.grad = None
        ga = torch.cuda.CUDAGraph()
        with torch.cuda.graph(ga):
            SEEnergy.apply(xg, qg, plan).backward()
        for _ in range(warmup):
            ga.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            ga.replay()
        e1.record()
        torch.cuda.synchronize()
        return eager, e0.elapsed_time(e1) / steps

    def stage_times(self, steps, warmup):
        """Mean kernel duration per stage (ms) over a timed region of `steps`
        steps, from a plan recording each launch's own start and stop."""
        from paper_1712_04718_amd import SEPlan
        torch = self.torch
        tplan = SEPlan(self.M, self.P, self.L, self.xi, window=self.window, dtype=self.dtype,
                       n_max=self.N, device=self.xt.device, timing=True)
        main = self.plan
        self.plan = tplan
        try:
            for _ in range(warmup):
                self.step()
            tplan.stage_times()  # discard the warm-up launches
            for _ in range(steps):
                self.step()
            torch.cuda.synchronize()
            return tplan.stage_times()
        finally:
            self.plan = main
            tplan.close()

    def impl_error(self, nsample=2000):
        """(relative rms force error, relative energy error) of this run
        against the FP64 oracle at the same parameters, on sampled particles."""
        import numpy as np
        from oracle import se_oracle as O
        torch = self.torch
        self.step()
        torch.cuda.synchronize()
        xo, qo = self.xt.double().cpu().numpy(), self.qt.double().cpu().numpy()
        L, xi, M, P = self.L, self.xi, self.M, self.P
        idx = np.random.default_rng(0).choice(self.N, size=min(self.N, nsample), replace=False)
        if self.window == "gaussian":
            eta = O.se_eta(L, xi, M, P)
            G = O.se_spread(xo, qo, L, M, P, xi, eta)
            Eo, Phi = O.scale_and_energy(G, O.se_influence(L, xi, M, eta), L)
            _, Fo = O.se_gather(xo[idx], qo[idx], L, M, P, xi, eta, Phi)
        else:
            G = O.spme_spread(xo, qo, L, M, P)
            Eo, Phi = O.scale_and_energy(G, O.spme_influence(L, xi, M, P), L)
            _, Fo = O.spme_gather(xo[idx], qo[idx], L, M, P, Phi)
        Fg = self.F.double().cpu().numpy()[idx]
        return O.rel_rms(Fg, Fo), abs(self.E.item() - Eo) / abs(Eo)

    def close(self):
        self.plan.close()


def roofline(stages_ms, N, M, P, window, workload):
    """The dominant kernel's algorithmic work per launch over its kernel
    duration (the timing plan's own start/stop events of every launch in the
    timed region), against the peak of what bounds it; the committed
    counters and kernel trace of the same kernel beside it when its sources
    still hash the same."""
    dom = max(stages_ms, key=stages_ms.get)
    kind, amount = kernel_work(dom, N, M, P, 4)
    dur_s = stages_ms[dom] * 1e-3
    if kind == "bytes":
        roof = {"bound": "hbm", "achieved": amount / dur_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": amount / dur_s / 1e12,
                "peak": VALU_PEAK_TFLOPS["f32"], "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    traffic, traffic_src = stored("traffic", dom, workload, P, window)
    roof["traffic"] = traffic
    roof["kernel"] = dom
    roof["kernel_us"] = stages_ms[dom] * 1e3
    roof["algorithmic"] = {"kind": kind, "per_launch": amount}
    roof["traffic_source"] = traffic_src
    trace_us, trace_src = stored("trace", dom, workload, P, window)
    if trace_us:
        roof["trace"] = {"kernel_us": trace_us, "frac": amount / (trace_us * 1e-6) /
                         (roof["peak"] * (1e9 if kind == "bytes" else 1e12)),
                         "source": trace_src}
    # the LDS integer atomics of the spread: N P^3 lane-atomics per launch
    # against the measured rate of the chip in this access pattern
    peak_atom, atom_src = lds_atomic_peak()
    if "spread" in stages_ms and peak_atom and window == "gaussian":
        rate = N * P ** 3 / (stages_ms["spread"] * 1e-3)
        roof["spread_lds_atomic"] = {"achieved": rate, "peak": peak_atom,
                                     "unit": "lane-atomics/s", "frac": rate / peak_atom,
                                     "source": atom_src}
    return roof


def run(args):
    import numpy as np
    import torch

    from workloads import make_system

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x, q, spec = make_system(args.workload)
    N, L, xi = len(q), spec.L, spec.xi
    M = args.M if args.M else spec.M
    P = args.P
    window = args.window
    log(f"workload {args.workload}: N={N} L={L} xi={xi} M={M} P={P} window={window}")

    # Calibration copy for the HBM byte counters: one elementwise pass that
    # reads and writes CALIB_COPY_BYTES (torch.neg into a second buffer).
    src = torch.ones(CALIB_COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst

    dtypes = [(torch.float32, "f32")] + ([] if args.no_fp64 else [(torch.float64, "f64")])
    out = {}
    for dtype, tag in dtypes:
        c = Case(x, q, L, xi, M, P, window, dtype, dev)
        ms_eager, per_step = c.time_steps(args.steps, args.warmup, per_step=True)
        ms_graph = c.time_graph(args.steps, args.warmup)
        ms_ag, ms_ag_graph = c.time_autograd(args.steps, args.warmup)
        stages = c.stage_times(args.steps, max(2, args.warmup // 4))
        err_F, err_E = c.impl_error()
        log(f"{tag}: eager {ms_eager * 1e3:.1f} us/step (median "
            f"{percentile(per_step, 0.5) * 1e3:.1f}), graph {ms_graph * 1e3:.1f} us/step, "
            f"rms force err vs oracle {err_F:.2e}")
        out[tag] = dict(ms_eager=ms_eager, ms_graph=ms_graph, per_step=per_step,
                        ms_autograd=ms_ag, ms_autograd_graph=ms_ag_graph, err_F=err_F,
                        err_E=err_E, stages_ms=stages)
        c.close()

    # matched accuracy: the support at which the method itself reaches a
    # relative rms force error of 1e-5 on this system (P = 10 on water_L100)
    matched = None
    if not args.no_matched and args.workload == "water_L100" and window == "gaussian":
        matched = {"P": 10, "M": M,
                   "method_error": method_error(args.workload, M, 10, window)}
        for dtype, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
            c = Case(x, q, L, xi, M, 10, window, dtype, dev)
            ms, _ = c.time_steps(args.steps, args.warmup)
            ms_ag, _ = c.time_autograd(max(10, args.steps // 4), max(3, args.warmup // 4),
                                       graph=False)
            err_F, _ = c.impl_error()
            matched[tag] = {"ms_per_step": ms, "value": N / (ms * 1e-3),
                            "autograd_ms_per_step": ms_ag,
                            "rms_force_err_vs_fp64_oracle": err_F}
            c.close()
        matched["fp32_over_fp64"] = matched["f64"]["ms_per_step"] / matched["f32"]["ms_per_step"]
        log(f"matched accuracy (P=10): f32 {matched['f32']['ms_per_step'] * 1e3:.1f} us, "
            f"f64 {matched['f64']['ms_per_step'] * 1e3:.1f} us")

    # the 10^6-ion SE vs SPME comparison, FP32, each tuned to 1e-4
    c5 = None
    if not args.no_c5:
        xi_, qi_, sp5 = make_system("ions_1M")
        c5 = {"workload": f"ions_1M: {len(qi_)} random +-1 ions, L={sp5.L} A, xi={sp5.xi}",
              "dtype": "f32", "target_rel_rms_force": 1e-4, "rows": []}
        for win, p, m in C5_CASES:
            c = Case(xi_, qi_, sp5.L, sp5.xi, m, p, win, torch.float32, dev)
            steps = max(10, args.steps // 4)
            ms, _ = c.time_steps(steps, max(3, args.warmup // 4))
            ms_ag, ms_ag_g = c.time_autograd(steps, max(3, args.warmup // 4))
            err_F, _ = c.impl_error()
            me = method_error("ions_1M", m, p, win)
            c5["rows"].append({"window": win, "P" if win == "gaussian" else "p": p, "M": m,
                               "ms_per_step": ms, "value": len(qi_) / (ms * 1e-3),
                               "autograd_ms_per_step": ms_ag,
                               "autograd_graph_ms_per_step": ms_ag_g,
                               "rms_force_err_vs_fp64_oracle": err_F,
                               "method_error": me["rel_rms_force"] if me else None})
            log(f"ions_1M {win} {p} M={m}: {ms * 1e3:.1f} us/step, fwd+bwd {ms_ag * 1e3:.1f} us, "
                f"impl err {err_F:.2e}")
            c.close()
        del xi_, qi_
        c5["method_error_source"] = "tests/golden/spme_tuned_grid.json"

    # Real-space sum beside the path (FP32, cutoff REAL_SPACE_RC): timed on its
    # own, reported next to the k-space line
    real_space = None
    if not args.no_real_space and 3 * REAL_SPACE_RC <= L:
        real_space = real_space_leg(args, x, q, L, xi, M, P, window, N, dev)

    cpu = None if args.no_cpu else cpu_baseline(args, x, q, L, xi, M, P, window, N)

    f32 = out["f32"]
    ms = f32["ms_eager"]
    value = N / (ms * 1e-3)
    stages = f32["stages_ms"]
    roof = roofline(stages, N, M, P, window, args.workload)
    hbm_frac = {}
    for st in stages:
        k, b = kernel_work(st, N, M, P, 4)
        if k == "bytes" and b:
            hbm_frac[st] = round(b / (stages[st] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    ps = f32["per_step"]
    desc = {"water": "3-site water", "ions": "random +-1 ions"}[spec.kind]
    wname = "SE Gaussian window" if window == "gaussian" else "SPME B-spline window"
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}, {N} atoms, L={L} A, "
                               f"xi={xi}, M={M}, {'P' if window == 'gaussian' else 'p'}={P}, "
                               f"{wname}",
                   "N": N, "L": L, "xi": xi, "M": M, "P": P, "window": window,
                   "mode": "eager launches on one stream"},
        "command": "python3 bench.py " + " ".join(sys.argv[1:]),
        "step_ms": {"median": percentile(ps, 0.5), "p10": percentile(ps, 0.1),
                    "p90": percentile(ps, 0.9)},
        "rms_force_err_vs_fp64_oracle": f32["err_F"],
        "method_error": method_error(args.workload, M, P, window),
        "energy_rel_err_vs_fp64_oracle": f32["err_E"],
        "graph": {"ms_per_step": f32["ms_graph"], "value": N / (f32["ms_graph"] * 1e-3)},
        "autograd": {"ms_per_step": f32["ms_autograd"],
                     "value": N / (f32["ms_autograd"] * 1e-3),
                     "graph_ms_per_step": f32["ms_autograd_graph"],
                     "graph_value": N / (f32["ms_autograd_graph"] * 1e-3),
                     "step": "SEEnergy forward + backward (dE/dx, dE/dq); graph: the same "
                             "captured once in a HIP graph and replayed"},
        "stages_us": {k: round(v * 1e3, 2) for k, v in stages.items()},
        "stages_sum_us": round(sum(stages.values()) * 1e3, 2),
        "grid_pass_hbm_frac": hbm_frac,
        "hbm_frac_step": step_bytes(N, M, 4) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_algorithmic_bytes": step_bytes(N, M, 4),
        "roofline": roof,
        "cpu_baseline": cpu,
        "matched_accuracy": matched,
        "c5": c5,
        "real_space": real_space,
        "sources": {st: source_hash(st) for st in KERNEL_SOURCES},
    }
    if "f64" in out:
        f64 = out["f64"]
        res["fp64"] = {"value": N / (f64["ms_eager"] * 1e-3), "ms_per_step": f64["ms_eager"],
                       "graph_ms_per_step": f64["ms_graph"],
                       "autograd_ms_per_step": f64["ms_autograd"],
                       "step_ms_median": percentile(f64["per_step"], 0.5),
                       "rms_force_err_vs_fp64_oracle": f64["err_F"],
                       "hbm_frac_step": step_bytes(N, M, 8) / (f64["ms_eager"] * 1e-3) / 1e9
                       / HBM_PEAK_GBS,
                       "stages_us": {k: round(v * 1e3, 2) for k, v in f64["stages_ms"].items()}}
        res["fp32_over_fp64"] = f64["ms_eager"] / ms
    print(json.dumps(res), flush=True)


def real_space_leg(args, x, q, L, xi, M, P, window, N, dev):
    import torch

    from paper_1712_04718_amd import RealSpacePlan, SEPlan, ewald_total
    from paper_1712_04718_amd import _lib as rs_lib, tolerance as rs_tol
    xt = torch.tensor(x, dtype=torch.float32, device=dev)
    qt = torch.tensor(q, dtype=torch.float32, device=dev)
    rplan = RealSpacePlan(L, xi, REAL_SPACE_RC, dtype=torch.float32, n_max=N, device=dev)
    reps = max(10, args.steps // 4)
    for _ in range(max(3, args.warmup // 4)):
        rplan.eval(xt, qt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rplan.eval(xt, qt)
    e1.record()
    torch.cuda.synchronize()
    ms_rs = e0.elapsed_time(e1) / reps
    # the total Ewald sum (k space with self terms + real space), the two
    # parts in sequence on one stream and overlapped on two streams
    kplan = SEPlan(M, P, L, xi, window=window, dtype=torch.float32, n_max=N, device=dev,
                   add_self=True)
    total_ms = {}
    for mode in (() if args.no_total else (False, True)):
        for _ in range(3):
            ewald_total(xt, qt, kplan, rplan, overlap=mode)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            ewald_total(xt, qt, kplan, rplan, overlap=mode)
        e1.record()
        torch.cuda.synchronize()
        total_ms["overlapped" if mode else "sequential"] = e0.elapsed_time(e1) / reps
    kplan.close()
    rplan.close()
    if total_ms:
        log(f"total Ewald sum: sequential {total_ms['sequential'] * 1e3:.1f} us, "
            f"overlapped {total_ms['overlapped'] * 1e3:.1f} us")
    # the cell list the library takes for this N: its cell count from the
    # runtime model's per-cell term; the fine list (more cells than the
    # coarse one) searches 5 cells wide, the coarse one 3
    unit = {n: 0.0 for n, _ in rs_lib.SeCostModel._fields_}
    unit["real_cell"] = 1.0
    nc = round(rs_tol.predict(unit, "f32", N, L, REAL_SPACE_RC, 48, 4)[0] ** (1.0 / 3.0))
    w = 5 if nc > int(L // REAL_SPACE_RC) else 3
    tested = N * float(w) ** 3 * (L / nc) ** 3 * N / L ** 3
    in_range = N * 4.0 / 3.0 * math.pi * REAL_SPACE_RC ** 3 * N / L ** 3
    flops = tested * RS_FLOPS_TEST + in_range * RS_FLOPS_PAIR
    log(f"real space rc={REAL_SPACE_RC}: {ms_rs * 1e3:.1f} us/eval")
    return {"rc": REAL_SPACE_RC, "ms_per_eval": ms_rs, "reps": reps,
            "value": N / (ms_rs * 1e-3), "unit": "atom-evals/s",
            "pairs_in_range_per_s": in_range / (ms_rs * 1e-3),
            "tested_pairs_per_s": tested / (ms_rs * 1e-3),
            "alu": {"achieved": flops / (ms_rs * 1e-3) / 1e12,
                    "peak": VALU_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                    "frac": flops / (ms_rs * 1e-3) / 1e12 / VALU_PEAK_TFLOPS["f32"]},
            "step": "se_rs_eval: cell-list binning + pair kernel + energy reduction",
            "total_ms": {k: round(v, 4) for k, v in total_ms.items()},
            "total_step": "ewald_total: k space (same M, P, self terms) + real space, "
                          "in sequence on one stream or overlapped on two"}


def cpu_baseline(args, x, q, L, xi, M, P, window, N):
    """The oracle as it stands, FP64, repeated full evaluations of the same
    workload for about args.cpu_seconds, then on one thread for about 3 s."""
    from oracle import se_oracle as O
    if window == "gaussian":
        evaluate = lambda xx, qq: O.se_kspace(xx, qq, L, xi, M, P)  # noqa: E731
    else:
        evaluate = lambda xx, qq: O.spme_kspace(xx, qq, L, xi, M, P)  # noqa: E731
    evaluate(x[:100], q[:100])  # load the library
    t0 = time.perf_counter()
    evaluate(x, q)
    t1 = time.perf_counter() - t0
    reps = max(1, min(200, int(math.ceil(args.cpu_seconds / max(t1, 1e-6))) - 1))
    t0 = time.perf_counter()
    for _ in range(reps):
        evaluate(x, q)
    dt = (time.perf_counter() - t0 + t1) / (reps + 1)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu = {"value": N / dt, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
           "sample": f"{reps + 1} full FP64 evaluations of the same {N}-atom workload "
                     f"({(reps + 1) * dt:.1f} s; spread and FFT on one thread, gather "
                     f"on {cores} OpenMP threads)"}
    log(f"oracle: {dt:.3f} s per evaluation")
    # the same oracle on one thread (the OpenMP runtime it links), for
    # comparison with per-core CPU figures; a bounded sample of ~3 s
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_get_max_threads.restype = ctypes.c_int
        nthr = gomp.omp_get_max_threads()
        gomp.omp_set_num_threads(1)
        try:
            t0 = time.perf_counter()
            evaluate(x, q)
            n1 = 1
            while time.perf_counter() - t0 < 3.0 and n1 < 50:
                evaluate(x, q)
                n1 += 1
            dt1 = (time.perf_counter() - t0) / n1
        finally:
            gomp.omp_set_num_threads(nthr)
        cpu["single_thread"] = {"value": N / dt1, "unit": "atom-evals/s", "cores": 1,
                                "sample": f"{n1} full FP64 evaluations on one thread "
                                          f"({n1 * dt1:.1f} s)"}
        log(f"oracle, one thread: {dt1:.3f} s per evaluation")
    except OSError:
        pass
    return cpu


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="water_L100")
    ap.add_argument("--P", type=int, default=8, help="Gaussian support P or B-spline order p")
    ap.add_argument("--M", type=int, default=0, help="grid size (default: the workload's)")
    ap.add_argument("--window", choices=("gaussian", "bspline"), default="gaussian")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-matched", action="store_true",
                    help="skip the matched-accuracy (P = 10) row")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the 10^6-ion SE/SPME comparison")
    ap.add_argument("--no-real-space", action="store_true")
    ap.add_argument("--no-total", action="store_true",
                    help="skip the total Ewald sum timing (its overlapped form runs k-space "
                         "kernels beside the pair kernel, which a kernel trace would mix in)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "FETCH_LOG",
                                                       "WRITE_LOG"),
                    help="summarize two rocprofv3 --pmc runs of this script into profiles/ "
                         "(host only)")
    ap.add_argument("--trace-from", nargs=2, metavar=("TRACE_DIR", "LOG"),
                    help="summarize a rocprofv3 --kernel-trace --stats run of this script "
                         "into profiles/ (host only)")
    ap.add_argument("--sq-from", nargs=3, metavar=("PASS1_DIR", "PASS2_DIR", "LOG"),
                    help="summarize the two SQ counter passes (SQ_PASSES) of this script into "
                         "profiles/ (host only)")
    ap.add_argument("--lds-probe-from", metavar="LOG",
                    help="store the LDS-atomic probe's output in profiles/ (host only)")
    args = ap.parse_args()
    if args.sq_from:
        summarize_sq(*args.sq_from)
        return
    if args.lds_probe_from:
        summarize_lds_probe(args.lds_probe_from)
        return
    if args.traffic_from:
        summarize_counters(*args.traffic_from)
        return
    if args.trace_from:
        summarize_trace(*args.trace_from)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
