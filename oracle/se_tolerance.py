"""Plain FP64 oracle for choosing Ewald and SE parameters from a tolerance.

TEST INFRASTRUCTURE.  Only ``tests/`` may import this module.  It shares no
code with the GPU library and never loads it.

What it computes, each function citing the passage it follows
(arXiv:1712.04718):

* the Kolafa-Perram rms truncation estimates of the real-space sum
  (section 2.1, eq. 2.1 a-c) and of the Fourier sum cut at |n| <= k_inf
  (eq. 2.2 a-c), with Q = sum q^2;
* their inversions for xi given rc (eq. 2.3 a-c) and for k_inf given xi
  (eq. 2.4 a-c); the Lambert W function is scipy's principal branch, used
  as a library primitive;
* the SE approximation-error estimates A e^{-pi P c^2 / 2} with
  A_phi = sqrt(Q xi L)/L, A_E = Q sqrt(xi L)/L, A_F = 4 pi Q sqrt(xi^3/L)
  (section 5.1-5.3) and the smallest even P meeting a tolerance;
* the runtime model of section 7 (t_real = c_real nbar N;
  t_fourier = c_fft (M^3/2) log(M^3/2) + c_sg N P^3 + c_solve M^3) and the
  choice of (xi, rc, M, P) that minimises it over a list of cutoffs, each
  source of error held to the tolerance on its own.

Estimates are absolute, in the units of the quantity with the Coulomb
constant 1: per-particle rms for the potential; for the force the root of
the summed squared errors over the particles (the printed force forms carry
Q where a per-particle rms would carry q_n sqrt(Q)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import lambertw

KINDS = ("potential", "energy", "force")


def _W(z: float) -> float:
    """Principal branch of Lambert W (the inverse of w -> w e^w), real z >= 0."""
    return float(lambertw(z, 0).real)


# ------------------------------------------------------------ eq. 2.1, 2.2

def real_error(kind: str, Q: float, L: float, xi: float, rc: float) -> float:
    """Real-space truncation estimate, section 2.1 eq. 2.1 (a) potential,
    (b) energy, (c) force."""
    g = math.exp(-(rc * xi) ** 2)
    if kind == "potential":
        return math.sqrt(Q * rc / (2 * L ** 3)) * (xi * rc) ** -2 * g
    if kind == "energy":
        return Q * math.sqrt(rc / (2 * L ** 3)) * (xi * rc) ** -2 * g
    if kind == "force":
        return 2 * Q * math.sqrt(1 / (rc * L ** 3)) * g
    raise ValueError(kind)


def fourier_error(kind: str, Q: float, L: float, xi: float, kinf: float) -> float:
    """Fourier-space truncation estimate for the sum over |k| <= 2 pi k_inf / L,
    section 2.1 eq. 2.2 (a)-(c)."""
    g = math.exp(-(math.pi * kinf / (xi * L)) ** 2)
    if kind == "potential":
        return xi * math.pi ** -2 * kinf ** -1.5 * math.sqrt(Q) * g
    if kind == "energy":
        return xi * math.pi ** -2 * kinf ** -1.5 * Q * g
    if kind == "force":
        return xi / (L * math.pi) * math.sqrt(8 / kinf) * Q * g
    raise ValueError(kind)


# ------------------------------------------------------------ eq. 2.3, 2.4

def xi_for(kind: str, eps: float, Q: float, L: float, rc: float) -> float:
    """Ewald parameter at which the real-space estimate equals eps,
    section 2.1 eq. 2.3 (a)-(c)."""
    if kind == "potential":
        return math.sqrt(_W(math.sqrt(Q * rc / (2 * L ** 3)) / eps)) / rc
    if kind == "energy":
        return math.sqrt(_W(Q * math.sqrt(rc / (2 * L ** 3)) / eps)) / rc
    if kind == "force":
        return math.sqrt(math.log(2 * Q / eps * math.sqrt(1 / (rc * L ** 3)))) / rc
    raise ValueError(kind)


def kinf_for(kind: str, eps: float, Q: float, L: float, xi: float) -> float:
    """Fourier cut k_inf at which the Fourier estimate equals eps,
    section 2.1 eq. 2.4 (a)-(c)."""
    if kind == "potential":
        z = 4 / (3 * L ** 2) * (Q / (math.pi * xi * eps ** 2)) ** (2 / 3)
        return math.sqrt(3) * L * xi / (2 * math.pi) * math.sqrt(_W(z))
    if kind == "energy":
        z = 4 / (3 * L ** 2) * (Q ** 2 / (math.pi * xi * eps ** 2)) ** (2 / 3)
        return math.sqrt(3) * L * xi / (2 * math.pi) * math.sqrt(_W(z))
    if kind == "force":
        z = 2 ** 8 * xi ** 2 * Q ** 4 / (eps ** 4 * L ** 6 * math.pi ** 2)
        return L * xi / (2 * math.pi) * math.sqrt(_W(z))
    raise ValueError(kind)


# ------------------------------------------------------------ section 5

def se_amplitude(kind: str, Q: float, L: float, xi: float) -> float:
    """Prefactor A of the SE approximation error A e^{-pi P c^2/2}:
    A_phi (section 5.1), A_E (section 5.2), A_F (section 5.3)."""
    if kind == "potential":
        return math.sqrt(Q * xi * L) / L
    if kind == "energy":
        return Q * math.sqrt(xi * L) / L
    if kind == "force":
        return 4 * math.pi * Q * math.sqrt(xi ** 3 / L)
    raise ValueError(kind)


def se_approx_error(kind: str, Q: float, L: float, xi: float, P: int, c: float = 0.95) -> float:
    """SE approximation-error estimate at support P, sections 5.1-5.3."""
    return se_amplitude(kind, Q, L, xi) * math.exp(-math.pi * P * c * c / 2)


def se_support_for(kind: str, eps: float, Q: float, L: float, xi: float,
                   c: float = 0.95) -> int:
    """Smallest even P (P >= 2) whose estimate is <= eps: P is rounded up to
    an even number as section 5.3 prescribes.  Searched by counting up."""
    P = 2
    while se_approx_error(kind, Q, L, xi, P, c) > eps:
        P += 2
    return P


def se_support_for_relative(eps_rel: float, c: float = 0.95) -> int:
    """Smallest even P with e^{-pi P c^2/2} <= eps_rel (the relative form of
    the remark closing section 5.3)."""
    P = 2
    while math.exp(-math.pi * P * c * c / 2) > eps_rel:
        P += 2
    return P


# ------------------------------------------------------------ section 7

PAPER_CPU_MODEL = {
    # constants of section 7 as printed in the text of sections 7.1 and 7.2
    "c_real": 2.4e-8, "c_fft": 4.5e-9, "c_sg": 5e-9, "c_solve": 2e-9,
}


def neighbours(N: int, L: float, rc: float) -> float:
    """Mean number of neighbours within rc of a uniform system, section 7.1."""
    return 4.0 / 3.0 * math.pi * rc ** 3 / L ** 3 * N


def runtime_estimate(model: dict, N: int, L: float, rc: float, M: int, P: int):
    """(t_real, t_fourier) of the section 7 model."""
    t_real = model["c_real"] * neighbours(N, L, rc) * N
    M3 = float(M) ** 3
    t_fourier = (model["c_fft"] * M3 / 2 * math.log(M3 / 2) + model["c_sg"] * N * P ** 3
                 + model["c_solve"] * M3)
    return t_real, t_fourier


def choose(kind: str, eps: float, N: int, Q: float, L: float, rcs, grid_sizes, model: dict,
           P_min: int = 4, P_max: int = 16, c: float = 0.95, eta_max: float = 1.0,
           P_fixed: int | None = None):
    """For each cutoff rc in ``rcs``: xi from eq. 2.3, k_inf from eq. 2.4,
    M the smallest of ``grid_sizes`` with M >= 2 k_inf (section 5.3 takes
    M = 2 k_inf) and eta = P L^2 xi^2/(c^2 pi M^2) below 1 (section 4) and
    at most eta_max, P from section 5 (raised to P_min, cutoff skipped above
    P_max), or ``P_fixed`` at every cutoff (section 7's experiment takes P
    from its relative error target, independent of xi);
    keep the cutoff with the least t_real + t_fourier (section 7).  Returns a
    dict, or None when no cutoff is feasible (M or P out of range)."""
    best = None
    for rc in rcs:
        xi = xi_for(kind, eps, Q, L, rc)
        kinf = kinf_for(kind, eps, Q, L, xi)
        if P_fixed is not None:
            P = int(P_fixed)
        else:
            P = se_support_for(kind, eps, Q, L, xi, c)
            if P > P_max:
                continue
            P = max(P, P_min)
        M = None
        for m in sorted(grid_sizes):
            eta = P * L ** 2 * xi ** 2 / (c * c * math.pi * m * m)
            if m >= 2 * kinf and eta < 1 and eta <= eta_max:
                M = m
                break
        if M is None:
            continue
        tr, tf = runtime_estimate(model, N, L, rc, M, P)
        if best is None or tr + tf < best["t_real"] + best["t_fourier"]:
            best = {"rc": rc, "xi": xi, "kinf": kinf, "M": M, "P": P,
                    "t_real": tr, "t_fourier": tf}
    return best
