#!/usr/bin/env python3
"""Throughput of the Spectral Ewald k-space evaluation on one MI355X.

One step = one full pass of the hot path on the device-resident inputs:
bin/sort, spread (eq. 4.5), forward FFT, scaling + k-space energy (eq. 4.6),
inverse FFT, gather of phi and F (eqs. 4.9, 4.12).  Default workload:
synthetic 3-site water at liquid density, L = 100 A (100,200 atoms),
xi = 0.3 A^-1, M = 96, P = 8 (relative rms force error of the method
~1e-5).  The headline value is FP32; the FP64 form at the same parameters is
reported beside it.

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

# source files each kernel is built from (a change voids stored counters)
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
    "bin_count": r"k_bin_count_(lds|run)<float", "bin_scan": r"k_bin_scan",
    "bin_scatter": r"k_bin_scatter(_scan)?<float>",
    "spread": r"k_spread<float,", "fold": r"k_fold(_tiles)?<float",
    "fft_x": r"k_fft_x_r2c<float,", "fft_y": r"k_fft_y<float, -?\d+, \d+, false>",
    "fft_z_scale": r"k_fft_z_scale<float,", "ifft_y": r"k_fft_y<float, -?\d+, \d+, true>",
    "ifft_x": r"k_fft_x_c2r<float,", "gather": r"k_gather<float,",
    "fft_xy": r"k_fft_xy_r2c<float,", "ifft_yx": r"k_fft_yx_c2r<float,",
}
CALIB_KERNEL_RE = r"neg_kernel"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(stage):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[stage]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def tile_edge(M, P, window, rs):
    """Tile edge the library picks: the largest of 16, 12, 8 leaving at least
    512 tiles (LDS limits do not bind for the supports used here)."""
    for T in (16, 12):
        if (-(-M // T)) ** 3 >= 512:
            return T
    return 8


def kernel_work(stage, N, M, P, rs, window):
    """Algorithmic work of one launch of a stage: (kind, amount).
    Bytes for the grid passes and binning, flops for spread and gather."""
    K = M // 2 + 1
    grid, spec = M ** 3 * rs, M * M * K * 2 * rs
    T = tile_edge(M, P, window, rs)
    ntiles = ((M + T - 1) // T) ** 3
    if stage == "bin_count":
        return "bytes", N * 4 * rs + N * 8                  # x, q in; keys out
    if stage == "bin_scan":
        return "bytes", ntiles * 12                        # counts in and reset; offsets out
    if stage == "bin_scatter":  # x, q, keys, counts in; sorted, meta, offsets out
        return "bytes", N * 4 * rs + N * 8 + N * (4 * rs + 8) + ntiles * 8
    if stage == "spread":
        return "flops", N * 2 * P ** 3                      # a multiply and an add per point
    if stage == "gather":
        return "flops", N * 4 * P ** 3                      # two multiply-adds per point
    if stage == "fold":
        ts = T + P - 1
        return "bytes", ((M + T - 1) // T) ** 3 * ts ** 3 * rs + grid
    if stage in ("fft_x", "fft_xy"):
        return "bytes", grid + spec
    if stage in ("ifft_x", "ifft_yx"):
        return "bytes", spec + grid
    return "bytes", 2 * spec                                # fft_y, fft_z_scale, ifft_y


def stored_traffic(stage, workload, P, window, tag):
    """HBM bytes per launch from a committed counter summary, or None when
    none matches this kernel, workload and the kernel's current sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{window}_P{P}_{tag}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, None
    st = rec.get("stages", {}).get(stage)
    if st is None or st.get("source_sha256_16") != source_hash(stage):
        return None, None
    return st.get("traffic_bytes_per_launch"), os.path.relpath(path, ROOT)


def _counter_rows(d, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 --pmc csv run."""
    import csv
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


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


def summarize_counters(fetch_dir, write_dir, fetch_log, write_log):
    """Turn two rocprofv3 --pmc runs of bench.py (FETCH_SIZE, WRITE_SIZE, in
    KiB per dispatch) into HBM bytes per launch of each k-space kernel,
    scaled by what the same counters read for the calibration copy of
    CALIB_COPY_BYTES.  Writes profiles/traffic_<workload>_<window>_P<P>_f32.json
    (read back by stored_traffic) and a markdown table beside it."""
    import re
    line = _bench_line(fetch_log) or _bench_line(write_log)
    if line is None:
        raise SystemExit("no bench.py JSON line in the counter runs' logs")
    cfg = line["config"]
    workload = cfg["workload"].split(":")[0]
    P, window, M, N = cfg["P"], cfg.get("window", "gaussian"), cfg["M"], cfg["N"]
    hashes = line.get("sources") or {}
    fetch, write = _counter_rows(fetch_dir, "FETCH_SIZE"), _counter_rows(write_dir, "WRITE_SIZE")

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
           "stages": {}}
    rs = 4
    md = [f"# HBM traffic per launch: {workload}, {window} window, P={P}, M={M}, N={N}, FP32\n",
          "Counters from two `rocprofv3 --pmc` runs of bench.py (FETCH_SIZE, then WRITE_SIZE; "
          "KiB per dispatch), each scaled by what the counter reads for a calibration copy of "
          f"{CALIB_COPY_BYTES >> 20} MiB (torch.neg): fetch factor {kf:.4f}, write factor {kw:.4f}.\n",
          "```",
          f"cd /tmp && rocprofv3 --pmc FETCH_SIZE -f csv -d <out-dir> -o bench -- "
          f"python3 <repo>/bench.py --steps 5 --warmup 2 --no-cpu --no-fp64 --no-real-space",
          f"cd /tmp && rocprofv3 --pmc WRITE_SIZE -f csv -d <out-dir> -o bench -- "
          f"python3 <repo>/bench.py --steps 5 --warmup 2 --no-cpu --no-fp64 --no-real-space",
          "```\n",
          "| stage | dispatches | fetch MB | write MB | traffic MB | algorithmic | ratio |",
          "|---|---|---|---|---|---|---|"]
    for st, pat in STAGE_KERNEL_RE.items():
        f_kib, nf = mean_of(fetch, pat)
        w_kib, nw = mean_of(write, pat)
        if f_kib is None or w_kib is None:
            continue
        traffic = f_kib * 1024.0 * kf + w_kib * 1024.0 * kw
        kind, amount = kernel_work(st, N, M, P, rs, window)
        rec["stages"][st] = {"dispatches": min(nf, nw), "fetch_kib": f_kib, "write_kib": w_kib,
                             "traffic_bytes_per_launch": traffic,
                             "algorithmic": {"kind": kind, "per_launch": amount},
                             "source_sha256_16": hashes.get(st, source_hash(st))}
        alg = f"{amount / 1e6:.2f} MB" if kind == "bytes" else f"{amount / 1e9:.3f} GFLOP"
        ratio = f"{traffic / amount:.2f}" if kind == "bytes" else "-"
        md.append(f"| {st} | {min(nf, nw)} | {f_kib * 1024 * kf / 1e6:.2f} | "
                  f"{w_kib * 1024 * kw / 1e6:.2f} | {traffic / 1e6:.2f} | {alg} | {ratio} |")
    base = os.path.join(ROOT, "profiles", f"traffic_{workload}_{window}_P{P}_f32")
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    with open(base + ".md", "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def method_error(workload, M, P, window):
    """Relative rms k-space force error of the method itself at (M, P)
    against a converged reference, from the stored oracle-only sweep
    (tests/golden), or None when none covers this configuration."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_method_error.json")
    if window != "gaussian" or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("M") != M or str(P) not in rec.get("rel_rms_force", {}):
        return None
    return {"rel_rms_force": rec["rel_rms_force"][str(P)], "reference": rec["reference"],
            "source": os.path.relpath(path, ROOT)}


def percentile(sorted_vals, p):
    if not sorted_vals:
        return float("nan")
    k = (len(sorted_vals) - 1) * p
    lo, hi = math.floor(k), math.ceil(k)
    return sorted_vals[lo] + (sorted_vals[hi] - sorted_vals[lo]) * (k - lo)


def run(args):
    import numpy as np
    import torch

    from paper_1712_04718_amd import SEPlan, _lib
    from workloads import make_system

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x, q, spec = make_system(args.workload)
    N, L, xi = len(q), spec.L, spec.xi
    M = args.M if args.M else spec.M
    P = args.P
    window = args.window
    log(f"workload {args.workload}: N={N} L={L} xi={xi} M={M} P={P} window={window}")
    lib = _lib.load()

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
        plan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=N, device=dev)
        xt = torch.tensor(x, dtype=dtype, device=dev)
        qt = torch.tensor(q, dtype=dtype, device=dev)
        E = torch.empty((), dtype=torch.float64, device=dev)
        phi = torch.empty(N, dtype=dtype, device=dev)
        F = torch.empty(N, 3, dtype=dtype, device=dev)
        ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (xt, qt, E, phi, F)]

        def step(p=plan):
            s = torch.cuda.current_stream().cuda_stream
            _lib.check(lib.se_plan_set_stream(p._plan, ctypes.c_void_p(s)))
            _lib.check(lib.se_kspace(p._plan, N, *ptrs))

        # eager launches on one stream (headline); an event after every step
        # gives the per-step distribution
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        evs[0].record()
        for i in range(args.steps):
            step()
            evs[i + 1].record()
        torch.cuda.synchronize()
        per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
        ms_eager = evs[0].elapsed_time(evs[-1]) / args.steps

        # the same step captured once in a HIP graph and replayed
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            step()  # warm the capture stream
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / args.steps
        log(f"{tag}: eager {ms_eager * 1e3:.1f} us/step (median "
            f"{percentile(per_step, 0.5) * 1e3:.1f}), graph {ms_graph * 1e3:.1f} us/step")

        # the autograd form: E = SEEnergy(x, q), then E.backward() (the
        # adjoint gather on the stored grid gives dE/dx and dE/dq)
        from paper_1712_04718_amd import SEEnergy
        xg = xt.clone().requires_grad_(True)
        qg = qt.clone().requires_grad_(True)

        def fwd_bwd():
            xg.grad = None
            qg.grad = None
            SEEnergy.apply(xg, qg, plan).backward()

        for _ in range(args.warmup):
            fwd_bwd()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            fwd_bwd()
        e1.record()
        torch.cuda.synchronize()
        ms_autograd = e0.elapsed_time(e1) / args.steps

        # the same forward + backward captured once in a HIP graph (the
        # adjoint reads dL/dE from device memory, so the whole step replays)
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
        for _ in range(args.warmup):
            ga.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            ga.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_autograd_graph = e0.elapsed_time(e1) / args.steps

        # per-kernel durations: a plan that records a HIP event pair around
        # every launch on its stream, over a timed region of K steps
        tplan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=N, device=dev,
                       timing=True)
        for _ in range(max(2, args.warmup // 4)):
            step(tplan)
        tplan.stage_times()  # discard the warm-up launches
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            step(tplan)
        e1.record()
        torch.cuda.synchronize()
        ms_timed_eager = e0.elapsed_time(e1) / args.steps
        stages = tplan.stage_times()

        # accuracy of this precision against the FP64 oracle (sampled particles)
        from oracle import se_oracle as O
        xo, qo = xt.double().cpu().numpy(), qt.double().cpu().numpy()
        idx = np.random.default_rng(0).choice(N, size=min(N, 2000), replace=False)
        if window == "gaussian":
            eta = O.se_eta(L, xi, M, P)
            G = O.se_spread(xo, qo, L, M, P, xi, eta)
            Eo, Phi = O.scale_and_energy(G, O.se_influence(L, xi, M, eta), L)
            phio, Fo = O.se_gather(xo[idx], qo[idx], L, M, P, xi, eta, Phi)
        else:
            G = O.spme_spread(xo, qo, L, M, P)
            Eo, Phi = O.scale_and_energy(G, O.spme_influence(L, xi, M, P), L)
            phio, Fo = O.spme_gather(xo[idx], qo[idx], L, M, P, Phi)
        Fg = F.double().cpu().numpy()[idx]
        err_F = O.rel_rms(Fg, Fo)
        err_E = abs(E.item() - Eo) / abs(Eo)
        out[tag] = dict(ms_eager=ms_eager, ms_graph=ms_graph, per_step=per_step,
                        ms_autograd=ms_autograd, ms_autograd_graph=ms_autograd_graph,
                        ms_timed_eager=ms_timed_eager, err_F=err_F, err_E=err_E,
                        stages_ms=stages)
        for t in (plan, tplan):
            t.close()

    # Real-space sum beside the path (FP32, cutoff REAL_SPACE_RC): timed on its
    # own, reported next to the k-space line
    real_space = None
    if not args.no_real_space and 3 * REAL_SPACE_RC <= L:
        from paper_1712_04718_amd import RealSpacePlan
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
        from paper_1712_04718_amd import SEPlan, ewald_total
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
        from paper_1712_04718_amd import _lib as rs_lib, tolerance as rs_tol
        unit = {n: 0.0 for n, _ in rs_lib.SeCostModel._fields_}
        unit["real_cell"] = 1.0
        nc = round(rs_tol.predict(unit, "f32", N, L, REAL_SPACE_RC, 48, 4)[0] ** (1.0 / 3.0))
        w = 5 if nc > int(L // REAL_SPACE_RC) else 3
        tested = N * float(w) ** 3 * (L / nc) ** 3 * N / L ** 3
        in_range = N * 4.0 / 3.0 * math.pi * REAL_SPACE_RC ** 3 * N / L ** 3
        flops = tested * RS_FLOPS_TEST + in_range * RS_FLOPS_PAIR
        real_space = {"rc": REAL_SPACE_RC, "ms_per_eval": ms_rs, "reps": reps,
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
        log(f"real space rc={REAL_SPACE_RC}: {ms_rs * 1e3:.1f} us/eval")

    # CPU baseline: the oracle as it stands, FP64, repeated full evaluations
    # of the same workload for about ten seconds
    cpu = None
    if not args.no_cpu:
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

    f32 = out["f32"]
    ms = f32["ms_eager"]
    value = N / (ms * 1e-3)
    stages = f32["stages_ms"]
    dom = max(stages, key=stages.get)
    kind, amount = kernel_work(dom, N, M, P, 4, window)
    dur_s = stages[dom] * 1e-3
    if kind == "bytes":
        roof = {"bound": "hbm", "achieved": amount / dur_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": amount / dur_s / 1e12,
                "peak": VALU_PEAK_TFLOPS["f32"], "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    traffic, traffic_src = stored_traffic(dom, args.workload, P, window, "f32")
    roof["traffic"] = traffic
    roof["kernel"] = dom
    roof["kernel_us"] = stages[dom] * 1e3
    roof["algorithmic"] = {"kind": kind, "per_launch": amount}
    roof["traffic_source"] = traffic_src

    hbm_frac = {}
    for st in stages:
        k, b = kernel_work(st, N, M, P, 4, window)
        if k == "bytes":
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
        "stages_region_ms_per_step": f32["ms_timed_eager"],
        "grid_pass_hbm_frac": hbm_frac,
        "roofline": roof,
        "cpu_baseline": cpu,
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
                       "stages_us": {k: round(v * 1e3, 2) for k, v in f64["stages_ms"].items()}}
        res["fp32_over_fp64"] = f64["ms_eager"] / ms
    print(json.dumps(res), flush=True)


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
    ap.add_argument("--no-real-space", action="store_true")
    ap.add_argument("--no-total", action="store_true",
                    help="skip the total Ewald sum timing (its overlapped form runs k-space "
                         "kernels beside the pair kernel, which a kernel trace would mix in)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "FETCH_LOG",
                                                       "WRITE_LOG"),
                    help="summarize two rocprofv3 --pmc runs of this script into profiles/ "
                         "(host only)")
    args = ap.parse_args()
    if args.traffic_from:
        summarize_counters(*args.traffic_from)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
