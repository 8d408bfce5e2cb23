"""Parameters from an error tolerance: binding of the host-only estimate
functions of libsekspace.so (Kolafa-Perram truncation estimates and their
inversions, section 2.1; SE approximation error, section 5; runtime model
of section 7).  No torch and no device needed.

    ch = choose_params("force", eps=1e-3, N=N, Q=(q**2).sum(), L=L,
                       rc_range=(4.0, 12.0), model=cost_model_mi355x("f32"))
    SEPlan(ch["M"], ch["P"], L, ch["xi"], ...); RealSpacePlan(L, ch["xi"], ch["rc"], ...)
"""
from __future__ import annotations

import ctypes

from . import _lib

_KIND = _lib.EST_KINDS
_DT = {"f32": _lib.SE_FP32, "f64": _lib.SE_FP64}


def _call(name, *args, out_type=ctypes.c_double):
    out = out_type(0)
    _lib.check(getattr(_lib.load(), name)(*args, ctypes.byref(out)))
    return out.value


def real_error(kind, Q, L, xi, rc):
    """Real-space truncation estimate (eq. 2.1)."""
    return _call("se_est_real_error", _KIND[kind], Q, L, xi, rc)


def fourier_error(kind, Q, L, xi, kinf):
    """Fourier truncation estimate (eq. 2.2)."""
    return _call("se_est_fourier_error", _KIND[kind], Q, L, xi, kinf)


def xi_for(kind, eps, Q, L, rc):
    """xi meeting eps in real space at cutoff rc (eq. 2.3)."""
    return _call("se_est_xi", _KIND[kind], eps, Q, L, rc)


def kinf_for(kind, eps, Q, L, xi):
    """Fourier cut meeting eps at xi (eq. 2.4)."""
    return _call("se_est_kinf", _KIND[kind], eps, Q, L, xi)


def se_error(kind, Q, L, xi, P, c=0.95):
    """SE approximation-error estimate (sections 5.1-5.3)."""
    return _call("se_est_se_error", _KIND[kind], Q, L, xi, int(P), c)


def se_support_for(kind, eps, Q, L, xi, c=0.95):
    """Smallest even P meeting eps (section 5.3)."""
    return _call("se_est_se_support", _KIND[kind], eps, Q, L, xi, c, out_type=ctypes.c_int)


def cost_model_mi355x(dtype="f32") -> dict:
    """The library's fitted MI355X runtime model (seconds)."""
    m = _lib.SeCostModel()
    _lib.check(_lib.load().se_cost_model_mi355x(_DT[dtype], ctypes.byref(m)))
    return {name: getattr(m, name) for name, _ in _lib.SeCostModel._fields_}


def paper_cpu_model() -> dict:
    """Section 7's constants for the paper's CPU runs, in the same form."""
    m = {name: 0.0 for name, _ in _lib.SeCostModel._fields_}
    m.update(real_pair=2.4e-8, k_fft=4.5e-9, k_window=5e-9, k_grid=2e-9)
    return m


def predict(model, dtype, N, L, rc, M, P):
    """(t_real, t_kspace) of the runtime model for one configuration."""
    mdl = _lib.SeCostModel(**model)
    tr, tk = ctypes.c_double(0), ctypes.c_double(0)
    _lib.check(_lib.load().se_cost_predict(ctypes.byref(mdl), _DT[dtype], int(N), float(L),
                                           float(rc), int(M), int(P), ctypes.byref(tr),
                                           ctypes.byref(tk)))
    return tr.value, tk.value


def choose_params(kind, eps, N, Q, L, rc_range, n_rc=256, model=None, c=0.95,
                  dtype="f32") -> dict:
    """Cheapest (rc, xi, M, P) meeting eps with each error source held to eps
    on its own (see se_choose_params)."""
    mdl = _lib.SeCostModel(**(model if model is not None else cost_model_mi355x(dtype)))
    ch = _lib.SeChoice()
    lo, hi = rc_range
    _lib.check(_lib.load().se_choose_params(_KIND[kind], eps, int(N), Q, L, lo, hi, int(n_rc), c,
                                            _DT[dtype], ctypes.byref(mdl), ctypes.byref(ch)))
    return {name: getattr(ch, name) for name, _ in _lib.SeChoice._fields_}
