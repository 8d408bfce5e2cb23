"""Fit the runtime model of se_cost_model to this GPU.

The model is the library's (se_cost_model, se_cost_predict): the form of
the paper's section 7 plus the terms of a GPU launch sequence,
    t_real   = real_fixed + real_atom N + real_pair N nbar + real_cell ncells
               + real_test N ntest q
    t_kspace = k_fixed + k_atom N + k_window N P^3 + k_block nt^3 (T+P-1)^3
               + k_grid M^3 + k_fft (M^3/2) ln(M^3/2).
Each term's value for a configuration is read back from se_cost_predict with
a model that has that coefficient 1 and the others 0, so the fit and the
library price the same quantities.
Times are the mean of ``reps`` calls of se_rs_eval and se_kspace (SE window)
between HIP events, inputs resident on the device, uniform random charges at
0.1 per unit volume (water's number density in A^-3).  Each model is fitted
by non-negative least squares on relative residuals.

    python -m paper_1712_04718_amd.calibrate [--dtype f32|f64] [--out file.json]

prints one JSON object: the constants, each measured point and the largest
relative deviation of the fit;

    python -m paper_1712_04718_amd.calibrate --markdown calib_f32.json calib_f64.json

(host only) writes the two fits as the markdown summary of profiles/.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
import torch
from scipy.optimize import nnls

from . import RealSpacePlan, SEPlan, _lib, tolerance

DENSITY = 0.1
K_POINTS = [(N, M, P) for N in (20_000, 100_000, 400_000) for M in (48, 96, 144, 192, 256)
            for P in (4, 8, 12, 16)]
R_POINTS = [(N, rc) for N in (20_000, 100_000, 400_000) for rc in (4.0, 6.0, 8.0, 10.0, 12.0)]


def _system(N, dtype, seed=0):
    L = (N / DENSITY) ** (1.0 / 3.0)
    g = torch.Generator().manual_seed(seed)
    x = torch.rand(N, 3, generator=g, dtype=torch.float64) * L
    q = torch.where(torch.arange(N) % 2 == 0, 1.0, -1.0).to(torch.float64)
    return L, x.to("cuda", dtype), q.to("cuda", dtype)


def _time(fn, reps):
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e-3


REAL_TERMS = ("real_fixed", "real_atom", "real_pair", "real_cell", "real_test")
K_TERMS = ("k_fixed", "k_atom", "k_window", "k_block", "k_grid", "k_fft")


def _features(dtype, N, L, rc, M, P, terms, which):
    row = []
    for name in terms:
        unit = {n: 0.0 for n, _ in _lib.SeCostModel._fields_}
        unit[name] = 1.0
        row.append(tolerance.predict(unit, dtype, N, L, rc, M, P)[which])
    return row


def measure(dtype, reps):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    kpts, rpts = [], []
    for N, M, P in K_POINTS:
        L, x, q = _system(N, tdt)
        xi = math.sqrt(0.5 * 0.95 ** 2 * math.pi * M * M / (P * L * L))  # eta = 0.5
        try:
            plan = SEPlan(M, P, L, xi, dtype=tdt, n_max=N)
        except RuntimeError as e:  # a support the LDS of this precision cannot hold
            print(f"[calibrate] skip k-space N={N} M={M} P={P}: {e}", file=sys.stderr, flush=True)
            continue
        t = _time(lambda: plan.kspace(x, q), reps)
        plan.close()
        kpts.append({"N": N, "L": L, "M": M, "P": P, "t": t})
        print(f"[calibrate] k-space N={N} M={M} P={P}: {t * 1e6:.1f} us", file=sys.stderr,
              flush=True)
    for N, rc in R_POINTS:
        L, x, q = _system(N, tdt)
        plan = RealSpacePlan(L, 0.3, rc, dtype=tdt, n_max=N)
        t = _time(lambda: plan.eval(x, q), reps)
        plan.close()
        rpts.append({"N": N, "L": L, "rc": rc, "t": t})
        print(f"[calibrate] real space N={N} rc={rc}: {t * 1e6:.1f} us", file=sys.stderr,
              flush=True)
    return kpts, rpts


def fit(dtype, kpts, rpts):
    def solve(A, t):
        w = 1.0 / t
        c, _ = nnls(A * w[:, None], np.ones_like(t))
        rel = A @ c / t - 1.0
        return c, float(np.abs(rel).max())

    A = np.array([_features(dtype, p["N"], p["L"], 1.0, p["M"], p["P"], K_TERMS, 1)
                  for p in kpts])
    ck, ek = solve(A, np.array([p["t"] for p in kpts]))
    B = np.array([_features(dtype, p["N"], p["L"], p["rc"], 48, 4, REAL_TERMS, 0)
                  for p in rpts])
    cr, er = solve(B, np.array([p["t"] for p in rpts]))
    model = dict(zip(REAL_TERMS, map(float, cr)))
    model.update(zip(K_TERMS, map(float, ck)))
    return model, ek, er


def markdown(paths):
    """The fits of calibration runs (JSON files of --out) as markdown."""
    md = ["# Runtime model of the parameter selection, fitted on one MI355X", "",
          "Command (run from the repository root on the GPU box, once per precision):", "",
          "    python -m paper_1712_04718_amd.calibrate --dtype f32 --out <out-dir>/calib_f32.json",
          "    python -m paper_1712_04718_amd.calibrate --dtype f64 --out <out-dir>/calib_f64.json",
          "    python -m paper_1712_04718_amd.calibrate --markdown <out-dir>/calib_f32.json "
          "<out-dir>/calib_f64.json", "",
          "Each point: mean of 10 calls between HIP events after 3 warm-ups, uniform",
          "random +-1 charges at 0.1 per A^3.  k space: `se_kspace`, SE window,",
          "eta = 0.5.  Real space: `se_rs_eval`, xi = 0.3.  The fits are the constants",
          "`se_cost_model_mi355x` returns (non-negative least squares on relative",
          "residuals; terms as in `include/sekspace.h`).", ""]
    for path in paths:
        with open(path) as f:
            rec = json.loads(f.readline())
        md += ["", f"## {rec['dtype'].upper()}", "", "| term | seconds per unit |", "|---|---|"]
        md += [f"| {k} | {v:.4e} |" for k, v in rec["model"].items()]
        dev = rec["max_rel_dev"]
        md += ["", f"Largest relative deviation of the fit: k space {dev['kspace']:.2f}, "
               f"real space {dev['real']:.2f}.", "", "Real-space points (us):", "",
               "| N | rc | measured |", "|---|---|---|"]
        md += [f"| {p['N']} | {p['rc']:g} | {p['t'] * 1e6:.1f} |" for p in rec["real_points"]]
        md += ["", "k-space points (us):", "", "| N | M | P | measured |", "|---|---|---|---|"]
        md += [f"| {p['N']} | {p['M']} | {p['P']} | {p['t'] * 1e6:.1f} |"
               for p in rec["kspace_points"]]
    return "\n".join(md) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--dtype", choices=("f32", "f64"), default="f32")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=None)
    ap.add_argument("--markdown", nargs="+", metavar="JSON",
                    help="print the fits of earlier runs as markdown (host only)")
    a = ap.parse_args(argv)
    if a.markdown:
        print(markdown(a.markdown), end="")
        return
    kpts, rpts = measure(a.dtype, a.reps)
    model, ek, er = fit(a.dtype, kpts, rpts)
    rec = {"dtype": a.dtype, "gpu": torch.cuda.get_device_name(0), "model": model,
           "max_rel_dev": {"kspace": ek, "real": er}, "kspace_points": kpts,
           "real_points": rpts}
    line = json.dumps(rec)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
