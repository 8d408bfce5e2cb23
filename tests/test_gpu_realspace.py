"""Real-space (erfc) part of the Ewald sums on the GPU vs the FP64 oracle,
and the total Ewald sum (k space + real space + self) on crystals.

Bar: relative rms error of E, phi and F <= 1e-5 in FP32 and <= 1e-9 in FP64
against the oracle's real-space sum with the same cutoff."""
import math

import numpy as np
import pytest
import torch

from gpu_util import DEV, TOL, array_errors, as_oracle_inputs, cached_system, to_dev
from oracle import se_oracle as O
from paper_1712_04718_amd import RealSpacePlan, SEPlan, _lib, ewald_total
from workloads import nacl_lattice

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]


def _rs(x, q, L, xi, rc, dtype):
    xt, qt = to_dev(x, q, dtype)
    plan = RealSpacePlan(L, xi, rc, dtype=dtype, n_max=max(1, len(q)))
    E, phi, F = plan.eval(xt, qt)
    torch.cuda.synchronize()
    out = (E.item(), phi.double().cpu().numpy(), F.double().cpu().numpy())
    plan.close()
    return out, xt, qt


def _errors(gpu, ref):
    """|E - E*| / |E*|, then the rms and largest-element errors of phi and F
    (gpu_util.array_errors), all to be held below the tolerance."""
    (E, phi, F), (Eo, phio, Fo) = gpu, ref
    return (abs(E - Eo) / abs(Eo),) + array_errors(phi, phio) + array_errors(F, Fo)


def _parity(x, q, L, xi, rc, dtype):
    print(f"[realspace] N={len(q)} L={L} xi={xi} rc={rc} {dtype}", flush=True)
    out, xt, qt = _rs(x, q, L, xi, rc, dtype)
    xo, qo = as_oracle_inputs(xt, qt)
    e = _errors(out, O.ewald_real(xo, qo, L, xi, rc))
    assert max(e) < TOL[dtype], e


@pytest.mark.parametrize("dtype", DTYPES)
def test_ions_1k(dtype):
    """1000 ions in L = 10, xi = 1.5, rc = 2.4 (4 cells per side searched 3
    wide: 2 particles per cell of the finer list are too few for it)."""
    x, q, spec = cached_system("ions_1k")
    _parity(x, q, spec.L, spec.xi, 2.4, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_water_L40(dtype):
    """6411-atom water, xi = 0.3, rc = 9 (8 cells per side of edge 5 >= rc/2,
    searched 5 wide; molecules split across cells)."""
    x, q, spec = cached_system("water_L40")
    _parity(x, q, spec.L, spec.xi, 9.0, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("crowd", [700, 2000])
def test_minimum_cells_and_crowded_cell(crowd, dtype):
    """rc = L/3, the fewest cells each list allows, with `crowd` particles in
    one cell (more than a work-group takes at once) and 200 spread out:
    900 particles use three cells per side searched 3 wide (every cell is
    everyone's neighbour), 2200 (10 per cell of the finer list) six cells
    per side searched 5 wide."""
    rng = np.random.default_rng(3)
    L = 12.0
    x = np.concatenate([rng.random((crowd, 3)) * 1.5 + 2.0, rng.random((200, 3)) * L])
    q = rng.standard_normal(crowd + 200)
    _parity(x, q, L, 0.8, L / 3, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_empty_and_single(dtype):
    """N = 0 gives E = 0; a lone charge has no partner within rc <= L/3."""
    plan = RealSpacePlan(10.0, 1.0, 3.0, dtype=dtype, n_max=4)
    x = torch.zeros(0, 3, dtype=dtype, device=DEV)
    q = torch.zeros(0, dtype=dtype, device=DEV)
    E, _, _ = plan.eval(x, q)
    assert E.item() == 0.0
    x1, q1 = to_dev(np.array([[1.0, 2.0, 3.0]]), np.array([2.0]), dtype)
    E, phi, F = plan.eval(x1, q1)
    torch.cuda.synchronize()
    assert E.item() == 0.0 and phi.item() == 0.0 and float(F.abs().max()) == 0.0
    plan.close()


def test_full_water_L100_sampled():
    """100k-atom water, rc = 10, FP32, 2000 sampled atoms against the oracle."""
    x, q, spec = cached_system("water_L100")
    print(f"[realspace] water_L100 N={len(q)} rc=10", flush=True)
    xt, qt = to_dev(x, q, torch.float32)
    plan = RealSpacePlan(spec.L, spec.xi, 10.0, dtype=torch.float32, n_max=len(q))
    E, phi, F = plan.eval(xt, qt)
    torch.cuda.synchronize()
    xo, qo = as_oracle_inputs(xt, qt)
    idx = np.random.default_rng(8).choice(len(q), size=2000, replace=False)
    phio, Fo = O.ewald_real_targets(xo, qo, spec.L, spec.xi, 10.0, idx)
    e = array_errors(phi.double().cpu().numpy()[idx], phio) + \
        array_errors(F.double().cpu().numpy()[idx], Fo)
    print(f"[realspace] water_L100: phi {e[0]:.2e} F {e[2]:.2e} (max/10: {e[1]:.2e}, "
          f"{e[3]:.2e})", flush=True)
    assert max(e) < TOL[torch.float32], e
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_sparse_cells_sampled(dtype):
    """20,000 random ions in L = 60 with rc = 5: 1728 cells of edge 5 hold
    about 12 each, the half-edge cells fewer than 2, so the 27-cell list is
    taken, and with more cells than four work-groups per CU the FP32 pair
    kernel runs its 512-particle stage with the 12-entry queue; 2000 sampled
    atoms against the oracle's direct sum."""
    L, xi, rc, N = 60.0, 0.5, 5.0, 20000
    rng = np.random.default_rng(77)
    x = rng.random((N, 3)) * L
    q = np.where(np.arange(N) < N // 2, 1.0, -1.0)
    print(f"[realspace] sparse cells N={N} L={L} rc={rc} {dtype}", flush=True)
    xt, qt = to_dev(x, q, dtype)
    plan = RealSpacePlan(L, xi, rc, dtype=dtype, n_max=N)
    E, phi, F = plan.eval(xt, qt)
    torch.cuda.synchronize()
    xo, qo = as_oracle_inputs(xt, qt)
    idx = np.random.default_rng(9).choice(N, size=2000, replace=False)
    phio, Fo = O.ewald_real_targets(xo, qo, L, xi, rc, idx)
    e = array_errors(phi.double().cpu().numpy()[idx], phio) + \
        array_errors(F.double().cpu().numpy()[idx], Fo)
    print(f"[realspace] sparse cells {dtype}: {e}", flush=True)
    assert max(e) < TOL[dtype], e
    plan.close()


def test_total_ewald_nacl_madelung():
    """Total Ewald sum of a rock-salt crystal on the GPU (SE k space with the
    self terms, P = 16, FP64, plus the real space) against the oracle's exact
    total at the same xi and rc, and against the Madelung constant."""
    x, q, L = nacl_lattice(3)          # 216 ions, nearest-neighbour distance 1
    xi, rc = 2.4, L / 3                 # erfc(xi rc) ~ 1e-10
    xt, qt = to_dev(x, q, torch.float64)
    kplan = SEPlan(48, 16, L, xi, dtype=torch.float64, n_max=len(q), add_self=True)
    rplan = RealSpacePlan(L, xi, rc, dtype=torch.float64, n_max=len(q))
    E, phi, F = ewald_total(xt, qt, kplan, rplan)
    torch.cuda.synchronize()
    Eo, phio, Fo = O.ewald_total(x, q, L, xi, rc)
    assert abs(E.item() - Eo) / abs(Eo) < 1e-8, (E.item(), Eo)
    alpha = 1.7475645946331822
    assert abs(E.item() / len(q) * 2 + alpha) < 1e-7
    np.testing.assert_allclose(phi.cpu().numpy(), -q * alpha, rtol=0, atol=1e-7)
    assert float(F.abs().max()) < 1e-7
    for p in (kplan, rplan):
        p.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_total_overlapped_matches_sequential(dtype):
    """ewald_total with the real-space sum on a second stream gives the sums
    of the two parts taken in sequence, call after call, with the inputs
    freed right after each call and eager work on the caller's stream in
    between (the FP32 pair sums depend on the order of particles in a cell,
    which comes from atomics, so FP32 agrees to rounding; FP64 to 1e-12)."""
    print(f"[realspace] ewald_total overlapped vs sequential {dtype}", flush=True)
    N, L, xi, rc = 20000, 30.0, 0.5, 6.0
    rng = np.random.default_rng(61)
    x = rng.random((N, 3)) * L
    q = rng.standard_normal(N)
    q -= q.mean()
    xt, qt = to_dev(x, q, dtype)
    kplan = SEPlan(48, 8, L, xi, dtype=dtype, n_max=N, add_self=True)
    rplan = RealSpacePlan(L, xi, rc, dtype=dtype, n_max=N)
    Es, phis, Fs = ewald_total(xt, qt, kplan, rplan, overlap=False)
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    for rep in range(3):
        xc, qc = xt.clone(), qt.clone()
        Eo, phio, Fo = ewald_total(xc, qc, kplan, rplan, overlap=True)
        del xc, qc
        junk = torch.randn(N, 3, dtype=dtype, device=DEV) * 1e6  # reuses freed memory
        torch.cuda.synchronize()
        assert abs(Eo.item() - Es.item()) <= tol * abs(Es.item())
        for got, want in ((phio, phis), (Fo, Fs)):
            d = (got.double() - want.double()).norm() / want.double().norm()
            assert d.item() <= tol, (rep, d.item())
        del junk
    for p in (kplan, rplan):
        p.close()
