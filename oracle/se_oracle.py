"""Plain FP64 CPU oracle for the Spectral Ewald (SE) and SPME k-space sums.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the GPU library (it never loads it) and the GPU library never loads
this.

The particle loops (spread, gather, direct Ewald sums) are plain C in
``oracle/se_oracle.c``, compiled with gcc into ``oracle/liboracle.so``; the
3D FFT is ``numpy.fft`` used as a library primitive.  Each function cites
the passage of the paper (arXiv:1712.04718) it follows.

Conventions: Coulomb constant 1, box [0, L)^3, h = L/M, grids indexed
G[jz, jy, jx] with grid point j at x_j = j h, wave vectors k = 2 pi n / L.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "se_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
             "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        lib.or_se_spread.argtypes = [i, _dp, _dp, d, i, i, d, d, _dp]
        lib.or_se_gather.argtypes = [i, _dp, _dp, d, i, i, d, d, _dp,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.or_spme_spread.argtypes = [i, _dp, _dp, d, i, i, _dp]
        lib.or_spme_gather.argtypes = [i, _dp, _dp, d, i, i, _dp,
                                       ctypes.c_void_p, ctypes.c_void_p]
        lib.or_bspline.argtypes = [i, d]
        lib.or_bspline.restype = d
        lib.or_bspline_deriv.argtypes = [i, d]
        lib.or_bspline_deriv.restype = d
        lib.or_ewald_kspace.argtypes = [i, _dp, _dp, d, d, d, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        lib.or_ewald_real.argtypes = [i, _dp, _dp, d, d, d, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------

def se_eta(L: float, xi: float, M: int, P: int, c: float = 0.95) -> float:
    """Gaussian shape parameter, section 4 and eq. (5.2):
    w = P h / 2, m = c sqrt(pi P), eta = (2 w xi / m)^2 = P L^2 xi^2 / (c^2 pi M^2)."""
    h = L / M
    w = P * h / 2.0
    m = c * math.sqrt(math.pi * P)
    return (2.0 * w * xi / m) ** 2


def wave_numbers_sq(L: float, M: int) -> np.ndarray:
    """|k|^2 on the full M^3 DFT grid, k_d = 2 pi n_d / L with n_d the signed
    frequency (n for n < M/2, n - M otherwise; the Nyquist row n = M/2 gets
    |n| = M/2 either way).  Indexed [nz, ny, nx] like the grids."""
    n = np.fft.fftfreq(M, d=1.0 / M)  # 0..M/2-1, -M/2..-1
    k = 2.0 * math.pi * n / L
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    return k2


def se_influence(L: float, xi: float, M: int, eta: float) -> np.ndarray:
    """SE scaling factor of eq. (4.6): exp(-(1 - eta) k^2 / 4 xi^2) / k^2,
    with the k = 0 mode set to zero (section 1: zero mean potential)."""
    k2 = wave_numbers_sq(L, M)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.exp(-(1.0 - eta) * k2 / (4.0 * xi * xi)) / k2
    w[0, 0, 0] = 0.0
    return w


def bspline(p: int, u: float) -> float:
    """Cardinal B-spline M_p(u) of section 6.1 (recursive definition)."""
    return _load().or_bspline(int(p), float(u))


def spme_bmod2(p: int, M: int) -> np.ndarray:
    """|b(n)|^2 along one axis for the SPME influence function (eq. 6.2).

    The printed b_j is garbled (missing i in the numerator phase, M_p taken
    at multiples of h, b_2 written twice).  Reading used: Essmann et al.'s
    definition in grid units,
        |b(n)|^2 = 1 / |sum_{l=0}^{p-2} M_p(l+1) e^{2 pi i n l / M}|^2 ;
    the numerator phase has modulus one.  Where the denominator vanishes
    (odd p at the Nyquist mode n = M/2) the mode gets B = 0."""
    vals = np.array([bspline(p, l + 1.0) for l in range(p - 1)])
    n = np.arange(M)
    phase = np.exp(2j * math.pi * np.outer(n, np.arange(p - 1)) / M)
    den = np.abs(phase @ vals) ** 2
    out = np.zeros(M)
    good = den > 1e-10
    out[good] = 1.0 / den[good]
    return out


def spme_influence(L: float, xi: float, M: int, p: int) -> np.ndarray:
    """SPME scaling of eq. (6.2): B(k) exp(-k^2 / 4 xi^2) / k^2, k = 0 dropped."""
    k2 = wave_numbers_sq(L, M)
    b = spme_bmod2(p, M)
    B = b[:, None, None] * b[None, :, None] * b[None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        w = B * np.exp(-k2 / (4.0 * xi * xi)) / k2
    w[0, 0, 0] = 0.0
    return w


# --------------------------------------------------------------------------
# Steps of Algorithm 1 (section 3), SE and SPME windows (Table 2)
# --------------------------------------------------------------------------

def se_spread(x, q, L, M, P, xi, eta) -> np.ndarray:
    """Step 2, SE: grid G = h^3 H(x_j) of eq. (4.5), truncated to P^3 points."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    G = np.empty((M, M, M))
    _load().or_se_spread(len(q), x, q, float(L), int(M), int(P), float(xi), float(eta), G)
    return G


def spme_spread(x, q, L, M, p) -> np.ndarray:
    """Step 2, SPME: grid Q of eq. (6.1)."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    Q = np.empty((M, M, M))
    _load().or_spme_spread(len(q), x, q, float(L), int(M), int(p), Q)
    return Q


def scale_and_energy(G: np.ndarray, w: np.ndarray, L: float):
    """Steps 3-5: forward DFT (e^{-i k.x}), multiply by the influence factor w,
    inverse DFT.  Returns (E, Phi) with
        E   = (2 pi / L^3) sum_k w_k |G^_k|^2          (eq. 1.6 via Parseval)
        Phi = (4 pi / L^3) sum_k w_k G^_k e^{+i k.x_j}  (real)
    so that gathering Phi with the window gives phi (eqs. 4.9, 6.3)."""
    M = G.shape[0]
    V = L ** 3
    Gh = np.fft.fftn(G)
    E = 2.0 * math.pi / V * float(np.sum(w * (Gh.real ** 2 + Gh.imag ** 2)))
    Phi = (4.0 * math.pi / V) * np.real(np.fft.ifftn(w * Gh)) * (M ** 3)
    return E, np.ascontiguousarray(Phi)


def se_gather(x, q, L, M, P, xi, eta, Phi, want_phi=True, want_F=True):
    """Step 6, SE: eq. (4.9) for phi and the analytic-derivative force."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    N = len(q)
    phi = np.empty(N) if want_phi else None
    F = np.empty((N, 3)) if want_F else None
    _load().or_se_gather(N, x, q, float(L), int(M), int(P), float(xi), float(eta),
                         _f64(Phi), _ptr(phi), _ptr(F))
    return phi, F


def spme_gather(x, q, L, M, p, Phi, want_phi=True, want_F=True):
    """Step 6, SPME: eq. (6.3) for phi and the analytic-derivative force."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    N = len(q)
    phi = np.empty(N) if want_phi else None
    F = np.empty((N, 3)) if want_F else None
    _load().or_spme_gather(N, x, q, float(L), int(M), int(p), _f64(Phi),
                           _ptr(phi), _ptr(F))
    return phi, F


def se_kspace(x, q, L, xi, M, P, c=0.95, return_grids=False):
    """SE k-space sum (Algorithm 1 with the SE column of Table 2).

    Returns (E, phi[N], F[N,3]) of the Fourier-space (long-range) parts of
    eqs. (1.5)-(1.7) as approximated by the SE method; with
    ``return_grids`` also the spread grid G and the scaled grid Phi."""
    eta = se_eta(L, xi, M, P, c)
    G = se_spread(x, q, L, M, P, xi, eta)
    E, Phi = scale_and_energy(G, se_influence(L, xi, M, eta), L)
    phi, F = se_gather(x, q, L, M, P, xi, eta, Phi)
    if return_grids:
        return E, phi, F, G, Phi
    return E, phi, F


def spme_kspace(x, q, L, xi, M, p, return_grids=False):
    """SPME k-space sum (Algorithm 1 with the SPME column of Table 2)."""
    Q = spme_spread(x, q, L, M, p)
    E, Phi = scale_and_energy(Q, spme_influence(L, xi, M, p), L)
    phi, F = spme_gather(x, q, L, M, p, Phi)
    if return_grids:
        return E, phi, F, Q, Phi
    return E, phi, F


def field_grids(G: np.ndarray, w: np.ndarray, L: float):
    """Section 3.1, the ik differentiation: the three components of the field
    -grad Phi on the grid,
        E_d = (4 pi / L^3) sum_k (-i k_d) w_k G^_k e^{+i k.x_j},
    with k_d = 0 on the Nyquist row of axis d (the derivative of that mode is
    not defined on the grid).  Returned as (E_x, E_y, E_z), indexed like G."""
    M = G.shape[0]
    V = L ** 3
    Gh = np.fft.fftn(G)
    n = np.fft.fftfreq(M, d=1.0 / M)
    if M % 2 == 0:
        n[M // 2] = 0.0
    k = 2.0 * math.pi * n / L
    shapes = ((1, 1, M), (1, M, 1), (M, 1, 1))  # x, y, z along the [z, y, x] axes
    return tuple(np.ascontiguousarray(
        (4.0 * math.pi / V) * np.real(np.fft.ifftn(-1j * k.reshape(sh) * w * Gh)) * M ** 3)
        for sh in shapes)


def se_kspace_ik(x, q, L, xi, M, P, c=0.95):
    """SE k-space sum with ik-differentiated forces (section 3.1): E and phi
    as in se_kspace, F_m = q_m (E_x, E_y, E_z) gathered at x_m with the window
    (eq. 4.9 applied to each field grid)."""
    eta = se_eta(L, xi, M, P, c)
    G = se_spread(x, q, L, M, P, xi, eta)
    w = se_influence(L, xi, M, eta)
    E, Phi = scale_and_energy(G, w, L)
    phi, _ = se_gather(x, q, L, M, P, xi, eta, Phi, want_F=False)
    comps = [se_gather(x, q, L, M, P, xi, eta, Ed, want_F=False)[0] for Ed in field_grids(G, w, L)]
    return E, phi, np.asarray(q)[:, None] * np.stack(comps, axis=1)


def spme_kspace_ik(x, q, L, xi, M, p):
    """SPME k-space sum with ik-differentiated forces (section 3.1)."""
    Q = spme_spread(x, q, L, M, p)
    w = spme_influence(L, xi, M, p)
    E, Phi = scale_and_energy(Q, w, L)
    phi, _ = spme_gather(x, q, L, M, p, Phi, want_F=False)
    comps = [spme_gather(x, q, L, M, p, Ed, want_F=False)[0] for Ed in field_grids(Q, w, L)]
    return E, phi, np.asarray(q)[:, None] * np.stack(comps, axis=1)


# --------------------------------------------------------------------------
# Exact Ewald sums (section 1) for pinning
# --------------------------------------------------------------------------

def ewald_kspace_direct(x, q, L, xi, tol=1e-20):
    """Direct k-space sum of eqs. (1.5)-(1.7) over every k != 0 whose Gaussian
    factor exp(-k^2/4xi^2) exceeds ``tol`` (a sphere in k)."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    N = len(q)
    kcut = 2.0 * xi * math.sqrt(-math.log(tol))
    E = np.zeros(1)
    phi = np.empty(N)
    F = np.empty((N, 3))
    _load().or_ewald_kspace(N, x, q, float(L), float(xi), float(kcut),
                            _ptr(E), _ptr(phi), _ptr(F))
    return float(E[0]), phi, F


def ewald_real(x, q, L, xi, rc):
    """Real-space sum of eqs. (1.5)-(1.7) truncated at r <= rc (all images)."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    N = len(q)
    E = np.zeros(1)
    phi = np.empty(N)
    F = np.empty((N, 3))
    _load().or_ewald_real(N, x, q, float(L), float(xi), float(rc),
                          _ptr(E), _ptr(phi), _ptr(F))
    return float(E[0]), phi, F


def ewald_real_targets(x, q, L, xi, rc, idx):
    """phi[len(idx)], F[len(idx), 3] of ewald_real for the particles idx
    only (all N particles are sources)."""
    x = _f64(x, (-1, 3))
    q = _f64(q)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    phi = np.empty(len(idx))
    F = np.empty((len(idx), 3))
    lib = _load()
    lib.or_ewald_real_targets.argtypes = [
        ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.c_int, np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS"), _dp, _dp]
    lib.or_ewald_real_targets(len(q), x, q, float(L), float(xi), float(rc), len(idx), idx,
                              phi, F)
    return phi, F


def ewald_self(q, xi):
    """Self terms of eqs. (1.5)-(1.6): phi = -2 xi q / sqrt(pi),
    E = -(xi / sqrt(pi)) sum q^2."""
    q = _f64(q)
    return (-xi / math.sqrt(math.pi) * float(np.sum(q * q)),
            -2.0 * xi / math.sqrt(math.pi) * q)


def ewald_total(x, q, L, xi, rc, tol=1e-20):
    """Total Ewald sum (real + Fourier + self), eqs. (1.5)-(1.7)."""
    Er, pr, Fr = ewald_real(x, q, L, xi, rc)
    Ek, pk, Fk = ewald_kspace_direct(x, q, L, xi, tol)
    Es, ps = ewald_self(q, xi)
    return Er + Ek + Es, pr + pk + ps, Fr + Fk


# --------------------------------------------------------------------------
# Error measures (section 2.1 rms error; relative form as used in section 8)
# --------------------------------------------------------------------------

def rms(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((a - ref) ** 2) / ref.shape[0]))


def rel_rms(a, ref):
    """sqrt(sum |a - ref|^2 / sum |ref|^2) over all particles/components."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((a - ref) ** 2) / np.sum(ref ** 2)))
