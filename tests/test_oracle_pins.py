"""Pins of the FP64 oracle against values fixed by the paper and by mathematics.

Nothing here compares the oracle with itself re-typed: the checks are
textbook lattice constants, exact Ewald sums evaluated a different way
(direct k-space sums, real-space erfc sums), invariances, identities of the
discrete scheme, finite differences, an explicit DFT, and the paper's error
law.  Each test names the passage it follows.
"""
import json
import math
import os

import numpy as np
import pytest

from workloads import ions, nacl_lattice

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


def _rand_neutral(N, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((N, 3)) * L
    q = rng.standard_normal(N)
    q -= q.mean()
    return x, q


# ---------------------------------------------------------------- exact sums

@pytest.mark.parametrize("xi", [1.6, 2.2])
def test_nacl_madelung_direct_ewald(oracle, xi):
    """Eqs. (1.5)-(1.7) summed exactly reproduce the rock-salt Madelung
    constant: E = -N alpha / 2, phi_m = -q_m alpha, F = 0 (nn distance 1)."""
    alpha = GOLD["nacl_madelung"]["value"]
    x, q, L = nacl_lattice(2)
    E, phi, F = oracle.ewald_total(x, q, L, xi, rc=4.0)
    N = len(q)
    assert abs(E / (-N * alpha / 2) - 1) < 1e-12
    assert np.max(np.abs(phi + q * alpha)) < 1e-11
    assert np.max(np.abs(F)) < 1e-11


def test_cscl_madelung_direct_ewald(oracle):
    """Second lattice: CsCl, nn distance sqrt(3)/2 for a unit cubic cell."""
    alpha = GOLD["cscl_madelung"]["value"]
    n = 3
    corners = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = np.concatenate([corners, corners + 0.5]).astype(float)
    q = np.concatenate([np.ones(len(corners)), -np.ones(len(corners))])
    L = float(n)
    d = math.sqrt(3) / 2
    E, phi, F = oracle.ewald_total(x, q, L, 3.0, rc=2.5)
    assert abs(E / (-len(q) / 2 * alpha / d) - 1) < 1e-12
    assert np.max(np.abs(F)) < 1e-11


def test_single_charge_wigner(oracle):
    """One charge with the k = 0 mode dropped (section 1) is a charge in a
    neutralising background; adding that background's Ewald term
    -pi Q^2 / (2 V xi^2) gives the simple-cubic lattice sum E = q^2 zeta / 2L,
    for any xi (section 1: the sums are exact and xi-independent)."""
    zeta = GOLD["sc_wigner"]["value"]
    L = 5.0
    for xi in (0.8, 1.3):
        E, _, _ = oracle.ewald_total(np.array([[1.0, 2.0, 3.0]]), np.array([1.0]), L, xi, rc=7.0)
        Ebg = -math.pi / (2 * L ** 3 * xi ** 2)
        assert abs((E + Ebg) / (zeta / (2 * L)) - 1) < 1e-12


def test_total_energy_xi_independent(oracle):
    """Section 1: the Ewald sums are exact and invariant to xi."""
    x, q = _rand_neutral(30, 6.0, 3)
    ref = None
    for xi in (0.9, 1.3, 1.8):
        E, phi, F = oracle.ewald_total(x, q, 6.0, xi, rc=3.0 * 6.0 / 2 * 1.5 / xi * 1.3)
        if ref is None:
            ref = (E, phi, F)
        else:
            assert abs(E - ref[0]) < 1e-10 * abs(ref[0])
            assert np.max(np.abs(phi - ref[1])) < 1e-9 * np.max(np.abs(ref[1]))
            assert np.max(np.abs(F - ref[2])) < 1e-9 * np.max(np.abs(ref[2]))


def test_direct_kspace_force_is_energy_gradient(oracle):
    """Eq. (1.7) read as F = -dE/dx of eq. (1.6): central differences."""
    x, q = _rand_neutral(6, 4.0, 5)
    _, _, F = oracle.ewald_kspace_direct(x, q, 4.0, 1.2)
    dx = 1e-5
    for m in range(3):
        for d in range(3):
            xp = x.copy(); xp[m, d] += dx
            xm = x.copy(); xm[m, d] -= dx
            Ep, _, _ = oracle.ewald_kspace_direct(xp, q, 4.0, 1.2)
            Em, _, _ = oracle.ewald_kspace_direct(xm, q, 4.0, 1.2)
            assert abs(-(Ep - Em) / (2 * dx) - F[m, d]) < 1e-7 * max(1.0, abs(F[m, d]))


# ------------------------------------------------------------ SE vs exact

def test_se_matches_direct_ewald_at_P24(oracle):
    """Section 5: with P = 24 (scaled error ~1e-15) and a grid large enough
    that Fourier truncation is negligible, SE equals the exact k-space sum."""
    x, q = ions(20, 10.0, 11)
    xi, L, M = 1.5, 10.0, 64
    Ek, pk, Fk = oracle.ewald_kspace_direct(x, q, L, xi)
    E, phi, F = oracle.se_kspace(x, q, L, xi, M, 24)
    assert abs(E - Ek) < 1e-12 * abs(Ek)
    assert oracle.rel_rms(phi, pk) < 1e-12
    assert oracle.rel_rms(F, Fk) < 1e-11


def test_se_total_reproduces_madelung(oracle):
    """SE k-space (P = 24) + real space + self term reproduces the NaCl
    Madelung constant: pins the SE oracle to a textbook value directly."""
    alpha = GOLD["nacl_madelung"]["value"]
    x, q, L = nacl_lattice(2)
    xi = 2.0
    Er, pr, Fr = oracle.ewald_real(x, q, L, xi, rc=3.5)
    Es, ps = oracle.ewald_self(q, xi)
    Ek, pk, Fk = oracle.se_kspace(x, q, L, xi, 32, 24)
    N = len(q)
    assert abs((Er + Es + Ek) / (-N * alpha / 2) - 1) < 1e-12
    assert np.max(np.abs(pr + ps + pk + q * alpha)) < 1e-11
    assert np.max(np.abs(Fr + Fk)) < 1e-11


def test_se_error_follows_paper_law(oracle):
    """Eqs. (5.3), (5.6): the approximation error decays like
    exp(-pi P c^2 / 2) with prefactors A_P = sqrt(Q xi L)/L for phi and
    A_F = 4 pi Q sqrt(xi^3 / L) for F.  The scaled rms errors must sit at or
    below the bound and not far below it (a wrong eta would break either)."""
    c = 0.95
    for (N, L, xiL, seed) in [(200, 5.0, 15.0, 21), (300, 10.0, 20.0, 22), (400, 1.0, 5.0, 23)]:
        xi = xiL / L
        x, q = ions(N, L, seed)
        Q = float(np.sum(q * q))
        M = int(2 * math.ceil(4 * xi * L / 2))  # M = 2 k_inf ~ 4 xi L (section 5.3)
        _, pk, Fk = oracle.ewald_kspace_direct(x, q, L, xi)
        for P in (6, 8, 10, 12):
            _, phi, F = oracle.se_kspace(x, q, L, xi, M, P)
            bound = math.exp(-math.pi * P * c * c / 2)
            sp = oracle.rms(phi, pk) / (math.sqrt(Q * xi * L) / L) / bound
            sf = math.sqrt(np.sum((F - Fk) ** 2) / N) / (4 * math.pi * Q * math.sqrt(xi ** 3 / L)) / bound
            assert 0.05 < sp < 1.0, (N, L, P, sp)
            assert 1e-3 < sf < 1.0, (N, L, P, sf)


def test_paper_accuracy_ladder():
    """Section 5 remark: exp(-pi P c^2/2) with c = 0.95 is below 1e-6, 1e-12
    at P = 10, 20 and about 1e-15 at P = 24."""
    g = GOLD["paper_accuracy_ladder"]
    c = g["c"]
    for P, lim in zip(g["P"], g["scaled_error_below"]):
        v = math.exp(-math.pi * P * c * c / 2)
        assert v < 2 * lim


def test_se_grid_holds_the_charge(oracle):
    """Eq. (4.5): the spread Gaussians are normalised, so the trapezoidal sum
    of the grid returns the charge up to the truncation level erfc(m/sqrt 2)
    (Theorem 1), for any net charge."""
    rng = np.random.default_rng(4)
    x = rng.random((50, 3)) * 8.0
    q = rng.random(50) + 0.5
    for P, tol in ((8, None), (24, 1e-13)):
        eta = oracle.se_eta(8.0, 1.0, 32, P)
        G = oracle.se_spread(x, q, 8.0, 32, P, 1.0, eta)
        m = 0.95 * math.sqrt(math.pi * P)
        lim = tol if tol else 10 * math.erfc(m / math.sqrt(2))
        assert abs(G.sum() / q.sum() - 1) < lim


# ------------------------------------------------- identities of the scheme

def _se_energy(oracle, x, q, L, xi, M, P):
    return oracle.se_kspace(x, q, L, xi, M, P)[0]


def _safe_atoms(x, h, P, dx, count):
    """Atoms whose +/- dx move keeps every axis inside one stencil (the
    truncated window switches stencil where x/h crosses an integer for even
    P, and E jumps there)."""
    u = x / h
    frac = u - np.floor(u)
    ok = np.all((frac > dx / h * 2) & (frac < 1 - dx / h * 2), axis=1)
    return np.nonzero(ok)[0][:count]


@pytest.mark.parametrize("P", [6, 8])
def test_se_force_is_minus_energy_gradient(oracle, P):
    """Section 3.1 and eq. (4.12): the analytic force is -dE/dx of the
    discrete SE energy (pins the sign and factor of eq. 4.12)."""
    L, xi, M = 8.0, 1.0, 24
    x, q = _rand_neutral(40, L, 7)
    _, _, F = oracle.se_kspace(x, q, L, xi, M, P)
    dx = 1e-5
    for m in _safe_atoms(x, L / M, P, dx, 5):
        for d in range(3):
            xp = x.copy(); xp[m, d] += dx
            xm = x.copy(); xm[m, d] -= dx
            g = -(_se_energy(oracle, xp, q, L, xi, M, P) - _se_energy(oracle, xm, q, L, xi, M, P)) / (2 * dx)
            assert abs(g - F[m, d]) < 1e-6 * max(1.0, np.abs(F).max())


def test_se_potential_is_charge_gradient(oracle):
    """E is quadratic in q (eq. 1.2), so dE/dq_m = phi_m exactly; central
    differences in q carry rounding only."""
    L, xi, M, P = 8.0, 1.0, 24, 8
    x, q = _rand_neutral(30, L, 8)
    _, phi, _ = oracle.se_kspace(x, q, L, xi, M, P)
    dq = 1e-3
    for m in range(5):
        qp = q.copy(); qp[m] += dq
        qm = q.copy(); qm[m] -= dq
        g = (_se_energy(oracle, x, qp, L, xi, M, P) - _se_energy(oracle, x, qm, L, xi, M, P)) / (2 * dq)
        assert abs(g - phi[m]) < 1e-9 * np.abs(phi).max()


@pytest.mark.parametrize("window", ["se", "spme"])
def test_parseval_energy(oracle, window):
    """E = 1/2 sum_m q_m phi_m (eq. 1.2) equals the Fourier-side energy
    (2 pi / V) sum w |G^|^2 exactly (discrete Parseval)."""
    L, xi, M = 9.0, 1.1, 30
    x, q = _rand_neutral(60, L, 9)
    if window == "se":
        E, phi, _ = oracle.se_kspace(x, q, L, xi, M, 8)
    else:
        E, phi, _ = oracle.spme_kspace(x, q, L, xi, M, 6)
    assert abs(0.5 * np.dot(q, phi) - E) < 1e-13 * abs(E)


def test_explicit_dft_agrees(oracle):
    """Steps 3-5 with an explicit DFT matrix (no FFT library) on a tiny grid:
    the same E and Phi as the FFT-based driver."""
    L, xi, M, P = 4.0, 1.0, 6, 4
    x, q = _rand_neutral(7, L, 10)
    eta = oracle.se_eta(L, xi, M, P)
    G = oracle.se_spread(x, q, L, M, P, xi, eta)
    w = oracle.se_influence(L, xi, M, eta)
    E, Phi = oracle.scale_and_energy(G, w, L)
    j = np.arange(M)
    Wm = np.exp(-2j * np.pi * np.outer(j, j) / M)      # forward, e^{-i k x}
    Gh = np.einsum("az,by,cx,zyx->abc", Wm, Wm, Wm, G)
    V = L ** 3
    E2 = 2 * np.pi / V * np.sum(w * np.abs(Gh) ** 2)
    Phi2 = 4 * np.pi / V * np.einsum("az,by,cx,abc->zyx", Wm.conj(), Wm.conj(), Wm.conj(), w * Gh).real
    assert abs(E - E2) < 1e-13 * abs(E2)
    assert np.max(np.abs(Phi - Phi2)) < 1e-13 * np.max(np.abs(Phi2))


def test_translation_by_grid_vector(oracle):
    """Shifting every particle by a grid vector shifts the grids by whole
    cells and leaves E, phi and F unchanged up to rounding."""
    L, xi, M, P = 8.0, 1.0, 32, 8
    x, q = _rand_neutral(40, L, 12)
    h = L / M
    E0, p0, F0 = oracle.se_kspace(x, q, L, xi, M, P)
    E1, p1, F1 = oracle.se_kspace(np.mod(x + h * np.array([3, -5, 7]), L), q, L, xi, M, P)
    assert abs(E1 - E0) < 1e-12 * abs(E0)
    assert np.max(np.abs(p1 - p0)) < 1e-11 * np.max(np.abs(p0))
    assert np.max(np.abs(F1 - F0)) < 1e-11 * np.max(np.abs(F0))


def test_arbitrary_translation_within_method_error(oracle):
    """A shift by a non-grid vector changes results only at the level of the
    approximation error (section 5)."""
    L, xi, M, P = 8.0, 1.0, 32, 12
    x, q = _rand_neutral(40, L, 13)
    _, p0, F0 = oracle.se_kspace(x, q, L, xi, M, P)
    _, p1, F1 = oracle.se_kspace(np.mod(x + np.array([0.123, 0.456, 0.789]), L), q, L, xi, M, P)
    assert oracle.rel_rms(p1, p0) < 1e-6
    assert oracle.rel_rms(F1, F0) < 1e-5


def test_scale_invariance(oracle):
    """(L, x, xi) -> (sL, sx, xi/s) at fixed (M, P) leaves eta unchanged and
    scales E, phi by 1/s and F by 1/s^2 (Coulomb 1/r)."""
    L, xi, M, P, s = 8.0, 1.0, 24, 8, 2.5
    x, q = _rand_neutral(30, L, 14)
    E0, p0, F0 = oracle.se_kspace(x, q, L, xi, M, P)
    E1, p1, F1 = oracle.se_kspace(s * x, q, s * L, xi / s, M, P)
    assert abs(E1 * s - E0) < 1e-12 * abs(E0)
    assert np.max(np.abs(p1 * s - p0)) < 1e-11 * np.max(np.abs(p0))
    assert np.max(np.abs(F1 * s * s - F0)) < 1e-11 * np.max(np.abs(F0))


def test_charge_symmetries(oracle):
    """q -> -q: E, F unchanged, phi flips; q -> lambda q: E -> lambda^2 E;
    permuting particles permutes outputs."""
    L, xi, M, P = 8.0, 1.0, 24, 8
    x, q = _rand_neutral(30, L, 15)
    E0, p0, F0 = oracle.se_kspace(x, q, L, xi, M, P)
    E1, p1, F1 = oracle.se_kspace(x, -q, L, xi, M, P)
    assert abs(E1 - E0) < 1e-13 * abs(E0)
    assert np.allclose(p1, -p0, rtol=0, atol=1e-13 * np.abs(p0).max())
    assert np.allclose(F1, F0, rtol=0, atol=1e-13 * np.abs(F0).max())
    E2, _, _ = oracle.se_kspace(x, 3.0 * q, L, xi, M, P)
    assert abs(E2 - 9.0 * E0) < 1e-12 * abs(E2)
    perm = np.random.default_rng(1).permutation(len(q))
    E3, p3, F3 = oracle.se_kspace(x[perm], q[perm], L, xi, M, P)
    assert abs(E3 - E0) < 1e-12 * abs(E0)
    assert np.allclose(p3, p0[perm], rtol=0, atol=1e-12 * np.abs(p0).max())
    assert np.allclose(F3, F0[perm], rtol=0, atol=1e-12 * np.abs(F0).max())


def test_net_force_nonzero_but_small(oracle):
    """Section 5.5: SE conserves energy, not momentum; the net force on an
    opposite-charge pair is not zero but of the order of the rms error."""
    L, xi, M = 10.0, 1.0, 32
    x = np.array([[1.3, 2.2, 3.1], [4.4, 5.7, 6.05]])
    q = np.array([1.0, -1.0])
    _, _, Fk = oracle.ewald_kspace_direct(x, q, L, xi)
    _, _, F = oracle.se_kspace(x, q, L, xi, M, 6)
    net = np.abs(F.sum(0)).max()
    err = np.abs(F - Fk).max()
    assert net > 0
    assert net < 10 * err + 1e-15


# ------------------------------------------------------------------- SPME

def test_bspline_values(oracle):
    """Section 6.1 recursion gives the standard cardinal B-spline values."""
    g = GOLD["bspline_values"]
    assert abs(oracle.bspline(3, 1.0) - g["M3_at_1"]) < 1e-15
    assert abs(oracle.bspline(3, 2.0) - g["M3_at_2"]) < 1e-15
    for k in (1, 2, 3):
        assert abs(oracle.bspline(4, float(k)) - g[f"M4_at_{k}"]) < 1e-15
    # partition of unity at arbitrary u
    for p in (3, 4, 5, 6, 8):
        for u in (0.1, 0.37, 0.9):
            assert abs(sum(oracle.bspline(p, u + j) for j in range(p)) - 1.0) < 1e-14


def test_spme_nyquist_denominator():
    """sum_{l=0}^{p-2} M_p(l+1) (-1)^l vanishes for odd p and equals -1/3,
    2/15 for p = 4, 6; the oracle sets B = 0 where it vanishes."""
    from oracle import se_oracle as o
    expect = {3: 0.0, 4: -1.0 / 3.0, 5: 0.0, 6: 2.0 / 15.0, 7: 0.0}
    for p, v in expect.items():
        s = sum(o.bspline(p, l + 1.0) * (-1) ** l for l in range(p - 1))
        assert abs(s - v) < 1e-14
    b = o.spme_bmod2(5, 16)
    assert b[8] == 0.0
    b = o.spme_bmod2(4, 16)
    assert abs(b[8] - 9.0) < 1e-12


def test_spme_grid_holds_the_charge_exactly(oracle):
    """B-splines form a partition of unity, so sum(Q) = sum(q) (eq. 6.1)."""
    rng = np.random.default_rng(16)
    x = rng.random((40, 3)) * 7.0
    q = rng.random(40)
    for p in (3, 4, 6):
        Q = oracle.spme_spread(x, q, 7.0, 20, p)
        assert abs(Q.sum() - q.sum()) < 1e-13 * q.sum()


def test_spme_converges_as_h_to_the_p(oracle):
    """Section 6.2: SPME's approximation error is O(h^p); doubling M cuts the
    force error by roughly 2^p."""
    L, xi = 10.0, 1.0
    x, q = ions(40, L, 17)
    _, _, Fk = oracle.ewald_kspace_direct(x, q, L, xi)
    for p in (4, 6):
        e1 = oracle.rel_rms(oracle.spme_kspace(x, q, L, xi, 32, p)[2], Fk)
        e2 = oracle.rel_rms(oracle.spme_kspace(x, q, L, xi, 64, p)[2], Fk)
        rate = math.log2(e1 / e2)
        assert p - 1.5 < rate < p + 2.5, (p, e1, e2, rate)


def test_spme_force_is_minus_energy_gradient(oracle):
    """SPME forces by analytic differentiation (section 6.1) are -dE/dx."""
    L, xi, M, p = 8.0, 1.0, 24, 6
    x, q = _rand_neutral(30, L, 18)
    _, _, F = oracle.spme_kspace(x, q, L, xi, M, p)
    dx = 1e-5
    for m in range(4):
        for d in range(3):
            xp = x.copy(); xp[m, d] += dx
            xm = x.copy(); xm[m, d] -= dx
            g = -(oracle.spme_kspace(xp, q, L, xi, M, p)[0] - oracle.spme_kspace(xm, q, L, xi, M, p)[0]) / (2 * dx)
            assert abs(g - F[m, d]) < 1e-6 * max(1.0, np.abs(F).max())


def test_real_space_targets_match_full_sum(oracle):
    """The target-subset real-space sum equals the full one on the targets."""
    rng = np.random.default_rng(21)
    x = rng.random((300, 3)) * 8.0
    q = rng.standard_normal(300)
    E, phi, F = oracle.ewald_real(x, q, 8.0, 1.1, 2.5)
    idx = np.array([0, 7, 150, 299, 42])
    phit, Ft = oracle.ewald_real_targets(x, q, 8.0, 1.1, 2.5, idx)
    np.testing.assert_allclose(phit, phi[idx], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Ft, F[idx], rtol=1e-13, atol=1e-14)


def test_potential_and_field_at_points_match_direct_sum(oracle):
    """Evaluation at points that are not sources (a unit test charge gathering
    the grid, eq. 4.9 and the force of eq. 4.12 per unit charge): at P = 24
    the SE values equal the exact k-space potential and field at those points,
    computed by the direct sum with zero charges placed there (section 1)."""
    x, q = _rand_neutral(60, 5.0, 11)
    rng = np.random.default_rng(12)
    xt = rng.random((25, 3)) * 7.0 - 1.0  # some points outside [0, L)
    L, xi, M, P = 5.0, 2.0, 40, 24
    _, _, _, _, Phi = oracle.se_kspace(x, q, L, xi, M, P, return_grids=True)
    eta = oracle.se_eta(L, xi, M, P)
    phi_t, field_t = oracle.se_gather(xt, np.ones(len(xt)), L, M, P, xi, eta, Phi)
    xa = np.concatenate([x, xt])
    qa = np.concatenate([q, np.zeros(len(xt))])
    _, phi_d, _ = oracle.ewald_kspace_direct(xa, qa, L, xi)
    # field = force on a unit charge: differentiate the direct potential
    h = 1e-5
    fd = np.empty((len(xt), 3))
    for d in range(3):
        xp, xm = xa.copy(), xa.copy()
        xp[len(x):, d] += h
        xm[len(x):, d] -= h
        pp = oracle.ewald_kspace_direct(xp, qa, L, xi)[1][len(x):]
        pm = oracle.ewald_kspace_direct(xm, qa, L, xi)[1][len(x):]
        fd[:, d] = -(pp - pm) / (2 * h)
    assert np.max(np.abs(phi_t - phi_d[len(x):])) < 1e-11 * np.max(np.abs(phi_d))
    assert np.max(np.abs(field_t - fd)) < 1e-7 * np.max(np.abs(fd))


def test_ik_forces_reach_the_exact_force(oracle):
    """Section 3.1: ik differentiation is the most accurate force.  At P = 24
    on a grid fine enough for the Fourier truncation to vanish, the ik forces
    equal the exact k-space forces (direct sum) to near machine precision (a
    k_d applied along the wrong axis fails this) and agree with the
    analytic-derivative forces of the same method.  At P = 8 both are
    approximations; the ik forces are the more accurate (1e-5 against 2.5e-4
    here), and the two differ by about the larger error."""
    x, q = _rand_neutral(80, 5.0, 17)
    L, xi = 5.0, 2.0
    _, _, Fd = oracle.ewald_kspace_direct(x, q, L, xi)
    E, phi, Fik = oracle.se_kspace_ik(x, q, L, xi, 48, 24)
    Ea, phia, Fa = oracle.se_kspace(x, q, L, xi, 48, 24)
    assert oracle.rel_rms(Fik, Fd) < 1e-11
    assert E == Ea and np.array_equal(phi, phia)
    assert oracle.rel_rms(Fik, Fa) < 1e-11
    # at a loose support both are approximations: ik and analytic forces
    # differ at the level of the method error
    _, _, Fik8 = oracle.se_kspace_ik(x, q, L, xi, 32, 8)
    _, _, Fa8 = oracle.se_kspace(x, q, L, xi, 32, 8)
    e_ik, e_a = oracle.rel_rms(Fik8, Fd), oracle.rel_rms(Fa8, Fd)
    assert 1e-8 < e_ik < 1e-3 and 1e-8 < e_a < 1e-3
    assert oracle.rel_rms(Fik8, Fa8) < 3 * max(e_ik, e_a)


def test_ik_forces_spme(oracle):
    """The same ik differentiation behind the SPME window: the force error
    against the exact force falls with the grid like the analytic one."""
    x, q = _rand_neutral(80, 5.0, 18)
    L, xi = 5.0, 2.0
    _, _, Fd = oracle.ewald_kspace_direct(x, q, L, xi)
    errs = [oracle.rel_rms(oracle.spme_kspace_ik(x, q, L, xi, M, 6)[2], Fd) for M in (24, 48)]
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-4
