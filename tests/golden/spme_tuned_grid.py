"""Tuned parameters of the 10^6-ion workload at a relative rms k-space force
error <= 1e-4: the smallest SPME grid size M (2^a 3^b 5^c, even) for B-spline
orders p = 4 and 6, and the smallest even SE support P at M = 192.

Reference: the SE k-space force at P = 12, M = 192 (window error ~e^{-pi P
c^2 / 2} = 4e-8, section 5; Fourier truncation of the M = 192 cube ~2e-7,
eq. 2.2), on 2000 sampled ions.  Errors follow the relative rms definition
used throughout (sum |F - F*|^2 / sum |F*|^2)^(1/2).

Calls only the oracle.  Writes spme_tuned_grid.json beside this file:
    python tests/golden/spme_tuned_grid.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import se_oracle as O  # noqa: E402
from workloads import make_system  # noqa: E402

TARGET = 1e-4


def good_sizes(lo, hi):
    out = []
    for m in range(lo, hi + 1, 2):
        r = m
        for f in (2, 3, 5):
            while r % f == 0:
                r //= f
        if r == 1:
            out.append(m)
    return out


def main():
    x, q, spec = make_system("ions_1M")
    L, xi = spec.L, spec.xi
    idx = np.random.default_rng(7).choice(len(q), size=2000, replace=False)
    t0 = time.time()
    eta = O.se_eta(L, xi, 192, 12)
    G = O.se_spread(x, q, L, 192, 12, xi, eta)
    _, Phi = O.scale_and_energy(G, O.se_influence(L, xi, 192, eta), L)
    _, Fref = O.se_gather(x[idx], q[idx], L, 192, 12, xi, eta, Phi, want_phi=False)
    print(f"reference SE P=12 M=192: {time.time() - t0:.1f} s", flush=True)

    def se_err(M, P):
        e = O.se_eta(L, xi, M, P)
        G = O.se_spread(x, q, L, M, P, xi, e)
        _, Phi = O.scale_and_energy(G, O.se_influence(L, xi, M, e), L)
        _, F = O.se_gather(x[idx], q[idx], L, M, P, xi, e, Phi, want_phi=False)
        return O.rel_rms(F, Fref)

    def spme_err(M, p):
        Q = O.spme_spread(x, q, L, M, p)
        _, Phi = O.scale_and_energy(Q, O.spme_influence(L, xi, M, p), L)
        _, F = O.spme_gather(x[idx], q[idx], L, M, p, Phi, want_phi=False)
        return O.rel_rms(F, Fref)

    res = {"workload": "ions_1M", "reference": "SE P=12 M=192 (FP64 oracle), 2000 sampled ions",
           "target_rel_rms_force": TARGET, "se": {}, "spme": {}}
    trail = []
    for P in (8, 10):
        err = se_err(192, P)
        trail.append([P, err])
        print(f"SE M=192 P={P}: {err:.3e}", flush=True)
        if err <= TARGET:
            break
    res["se"] = {"M": 192, "P": trail[-1][0], "rel_rms_force": trail[-1][1], "trail": trail}
    for p in (4, 6):
        trail = []
        for M in good_sizes(192, 512):
            err = spme_err(M, p)
            trail.append([M, err])
            print(f"SPME p={p} M={M}: {err:.3e}", flush=True)
            if err <= TARGET:
                break
        res["spme"][f"p{p}"] = {"M": trail[-1][0], "rel_rms_force": trail[-1][1], "trail": trail}
    with open(os.path.join(HERE, "spme_tuned_grid.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
