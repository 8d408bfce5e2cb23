"""The erfc of the real-space pair kernel, checked on the host: the
coefficients written in csrc/realspace.hip, evaluated in the kernel's form
e^{-x^2} t sum a_i t^i (t = 1/(1 + p x), Horner from the highest term, FP64
arithmetic), against scipy's erfc: relative error at most 6e-8 (FP32 set) and
1e-14 (FP64 set) where the fits hold, and a bounded absolute error beyond."""
import os
import re

import numpy as np
import pytest
from scipy.special import erfc

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1712_04718_amd", "csrc",
                   "realspace.hip")


def _coeffs(kind):
    s = open(SRC).read()
    body = s[s.index(f"__device__ inline {kind} erfc_from_exp"):]
    body = body[:body.index("return")]
    lead = re.search(rf"{kind} s = ([-+0-9.e]+)f?;", body).group(1)
    rest = re.findall(r"s = fmaf?\(s, t, ([-+0-9.e]+)f?\);", body)
    return [float(lead)] + [float(v) for v in rest]  # highest power first


def _eval(c, x):
    t = 1.0 / (1.0 + 0.3275911 * x)
    s = np.zeros_like(x)
    for a in c:
        s = s * t + a
    return np.exp(-x * x) * t * s


@pytest.mark.parametrize("kind,n,xmax,rtol", [("float", 8, 8.0, 6e-8), ("double", 17, 6.5, 1e-14)])
def test_kernel_erfc_coefficients(kind, n, xmax, rtol):
    c = _coeffs(kind)
    assert len(c) == n
    x = np.linspace(0.0, xmax, 20001)
    rel = np.abs(_eval(c, x) / erfc(x) - 1.0)
    assert rel.max() <= rtol, (kind, rel.max(), x[rel.argmax()])
    # past the fitted range erfc < 1e-19 (FP64 set) and the kernel's value
    # stays as small
    far = np.linspace(xmax, 30.0, 2001)
    assert np.all(_eval(c, far) >= 0.0)
    assert np.abs(_eval(c, far) - erfc(far)).max() <= 2.0 * erfc(xmax)
