"""Method error of the SE k-space force on the 100,200-atom water workload
(L = 100 A, xi = 0.3 A^-1, M = 96) for supports P = 6, 8, 10, 12, against
the SE force at P = 24 on the same grid (window error e^{-pi P c^2/2} =
1.7e-15, section 5; Fourier truncation of the M = 96 cube e^{-(pi 48 /
(0.3 100))^2} = 1e-11, eq. 2.2), on 3000 sampled atoms: the accuracy the
FP32 headline at P = 8 is quoted at.  Errors are relative rms,
(sum |F - F*|^2 / sum |F*|^2)^(1/2), as used throughout.

Calls only the oracle.  Writes water_L100_method_error.json beside this file:
    python tests/golden/water_L100_method_error.py
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

M = 96


def force_at(x, q, L, xi, P, idx):
    eta = O.se_eta(L, xi, M, P)
    G = O.se_spread(x, q, L, M, P, xi, eta)
    _, Phi = O.scale_and_energy(G, O.se_influence(L, xi, M, eta), L)
    _, F = O.se_gather(x[idx], q[idx], L, M, P, xi, eta, Phi, want_phi=False)
    return F


def main():
    x, q, spec = make_system("water_L100")
    L, xi = spec.L, spec.xi
    idx = np.random.default_rng(9).choice(len(q), size=3000, replace=False)
    t0 = time.time()
    Fref = force_at(x, q, L, xi, 24, idx)
    print(f"reference P=24: {time.time() - t0:.1f} s", flush=True)
    out = {"workload": "water_L100", "M": M, "reference": "SE P=24, M=96 (FP64 oracle)",
           "samples": len(idx), "rel_rms_force": {}}
    for P in (6, 8, 10, 12):
        e = O.rel_rms(force_at(x, q, L, xi, P, idx), Fref)
        out["rel_rms_force"][str(P)] = e
        print(f"P={P}: {e:.3e}", flush=True)
    with open(os.path.join(HERE, "water_L100_method_error.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
