"""Coefficients of the erfc used by the real-space pair kernel.

erfc(x) = e^{-x^2} t sum_{i=0}^{D} a_i t^i,  t = 1 / (1 + p x),  x >= 0,

the form of Abramowitz and Stegun 7.1.26 (p = 0.3275911 as there) with more
terms, fitted for relative (not absolute) accuracy by iteratively reweighted
least squares on the scaled complementary error function
erfcx(x) = e^{x^2} erfc(x):
  FP32: D = 7 on [0, 8] against scipy's erfcx;
  FP64: D = 16 on [0, 6.5] against mpmath's erfc at 40 digits, in the
        Chebyshev basis of t (the monomial Vandermonde matrix is too ill
        conditioned at this degree) and then expanded to monomials.  Past
        x = 6.5 (erfc < 1e-19) the polynomial stays between 0.18 and 0.27,
        so the absolute error there is below 1e-19.
Prints the coefficients as C initialisers and the largest relative error of
each fit; realspace.hip holds the printed values.  Run:
  python paper_1712_04718_amd/csrc/erfc_fit.py
"""
import numpy as np
from numpy.polynomial import chebyshev as cheb
from scipy.special import erfcx

P = 0.3275911


def fit32(deg=7, xmax=8.0):
    x = np.linspace(0.0, xmax, 40001)
    t = 1.0 / (1.0 + P * x)
    y = erfcx(x) / t
    V = np.vander(t, deg + 1, increasing=True)
    w = np.ones_like(x)
    for _ in range(60):
        c = np.linalg.lstsq(V * (w / y)[:, None], w, rcond=None)[0]
        rel = V @ c / y - 1.0
        w *= 1.0 + 5.0 * np.abs(rel) / np.abs(rel).max()
        w /= w.mean()
    return c, float(np.abs(rel).max())


def fit64(deg=16, xmax=6.5):
    import mpmath as mp
    mp.mp.dps = 40
    x = np.linspace(0.0, xmax, 8001)
    # erfcx(x) / t in 40-digit arithmetic, rounded once
    y = np.array([float(mp.erfc(mp.mpf(v)) * mp.e ** (mp.mpf(v) ** 2) * (1 + P * mp.mpf(v)))
                  for v in x])
    t = 1.0 / (1.0 + P * x)
    tmin = 1.0 / (1.0 + P * xmax)
    a, b = 2.0 / (1.0 - tmin), -(1.0 + tmin) / (1.0 - tmin)  # t -> [-1, 1]
    u = a * t + b
    w = np.ones_like(x)
    best = (np.inf, None)
    for _ in range(80):
        c = cheb.chebfit(u, y, deg, w=w / y)
        rel = cheb.chebval(u, c) / y - 1.0
        if np.abs(rel).max() < best[0]:
            best = (float(np.abs(rel).max()), c)
        w *= 1.0 + 5.0 * np.abs(rel) / np.abs(rel).max()
        w /= w.mean()
    mono = np.polynomial.Polynomial(cheb.cheb2poly(best[1]))(np.polynomial.Polynomial([b, a])).coef
    h = np.zeros_like(t)
    for cc in mono[::-1]:  # Horner in FP64, as the kernel evaluates it
        h = h * t + cc
    return mono, float(np.abs(h / y - 1.0).max())


if __name__ == "__main__":
    c, err = fit32()
    print("// FP32: max relative error of the fit on [0, 8]: %.2e" % err)
    print("{" + ", ".join("%.9ef" % v for v in c) + "}")
    c, err = fit64()
    print("// FP64: max relative error of the fit on [0, 6.5] (Horner in FP64): %.2e" % err)
    print("{" + ", ".join("%.17e" % v for v in c) + "}")
