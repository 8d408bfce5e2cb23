"""Coefficients of the FP32 erfc used by the real-space pair kernel.

erfc(x) = e^{-x^2} t sum_{i=0}^{7} a_i t^i,  t = 1 / (1 + p x),  x >= 0,

the form of Abramowitz and Stegun 7.1.26 (p = 0.3275911 as there) with three
more terms, fitted here for relative (not absolute) accuracy on [0, 8] by
iteratively reweighted least squares on the scaled complementary error
function erfcx(x) = e^{x^2} erfc(x) (scipy).  Prints the coefficients as a C
initialiser and the largest relative error of the fit; realspace.hip holds the
printed values.  Run:  python paper_1712_04718_amd/csrc/erfc_fit.py
"""
import numpy as np
from scipy.special import erfcx

P = 0.3275911
DEG = 7


def fit():
    x = np.linspace(0.0, 8.0, 40001)
    t = 1.0 / (1.0 + P * x)
    y = erfcx(x) / t
    V = np.vander(t, DEG + 1, increasing=True)
    w = np.ones_like(x)
    for _ in range(60):
        c = np.linalg.lstsq(V * (w / y)[:, None], w, rcond=None)[0]
        rel = V @ c / y - 1.0
        w *= 1.0 + 5.0 * np.abs(rel) / np.abs(rel).max()
        w /= w.mean()
    return c, float(np.abs(rel).max())


if __name__ == "__main__":
    c, err = fit()
    print("// max relative error of the fit on [0, 8]: %.2e" % err)
    print("{" + ", ".join("%.9ef" % v for v in c) + "}")
