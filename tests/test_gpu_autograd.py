"""Differentiation: SEEnergy's adjoint against the forward gather, central
finite differences of the FP64 GPU energy, and the oracle's analytic forces
(water box L = 60 A, 21,642 atoms, xi = 0.3, M = 64, P = 8)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, array_errors, as_oracle_inputs, cached_system, to_dev
from oracle import se_oracle as O
from paper_1712_04718_amd import SEEnergy, SEPlan

pytestmark = pytest.mark.gpu


def test_adjoint_equals_gather():
    """grad_x = -gE F and grad_q = gE phi, reusing the stored grid."""
    rng = np.random.default_rng(3)
    x = rng.random((600, 3)) * 10.0
    q = rng.standard_normal(600)
    for dtype in (torch.float32, torch.float64):
        xt, qt = to_dev(x, q, dtype)
        plan = SEPlan(32, 8, 10.0, 1.2, dtype=dtype, n_max=600)
        xg = xt.clone().requires_grad_(True)
        qg = qt.clone().requires_grad_(True)
        Eg = SEEnergy.apply(xg, qg, plan)
        phi, F = plan.gather()          # same forward pass as the backward below
        Eg.backward()
        torch.cuda.synchronize()
        assert torch.equal(xg.grad, -F)
        assert torch.equal(qg.grad, phi)
        # scaled upstream gradient
        xg.grad = None
        qg.grad = None
        Eg = SEEnergy.apply(xg, qg, plan)
        phi, F = plan.gather()
        (2.5 * Eg).backward()
        tol = 1e-6 if dtype == torch.float32 else 1e-14
        assert torch.allclose(xg.grad, -2.5 * F, rtol=tol, atol=tol * F.abs().max().item())
        assert torch.allclose(qg.grad, 2.5 * phi, rtol=tol, atol=tol * phi.abs().max().item())


def test_stale_plan_backward_raises():
    plan = SEPlan(16, 6, 5.0, 1.0, dtype=torch.float64, n_max=8)
    x = torch.rand(8, 3, dtype=torch.float64, device=DEV, requires_grad=True)
    q = torch.randn(8, dtype=torch.float64, device=DEV, requires_grad=True)
    E = SEEnergy.apply(x, q, plan)
    plan.forward(x.detach(), q.detach())
    with pytest.raises(RuntimeError):
        E.backward()


def _safe_atoms(x, h, dx, count, seed):
    """Seeded choice of atoms whose +/- dx move crosses no stencil switch
    (x/h crossing an integer) on any axis."""
    u = x / h
    frac = u - np.floor(u)
    ok = np.all((frac > 2 * dx / h) & (frac < 1 - 2 * dx / h), axis=1)
    cand = np.nonzero(ok)[0]
    return np.random.default_rng(seed).choice(cand, size=count, replace=False)


def test_gradient_vs_finite_differences_water_L60():
    x, q, spec = cached_system("water_L60")
    L, xi, M, P = spec.L, spec.xi, spec.M, 8
    h = L / M
    dx = 1e-4
    atoms = _safe_atoms(x, h, dx, 32, seed=7)
    print(f"[fd] N={len(q)} atoms={atoms[:4]}...", flush=True)

    # analytic gradients in both precisions through autograd
    grads = {}
    for dtype in (torch.float32, torch.float64):
        xt, qt = to_dev(x, q, dtype)
        plan = SEPlan(M, P, L, xi, dtype=dtype, n_max=len(q))
        xg = xt.clone().requires_grad_(True)
        qg = qt.clone().requires_grad_(True)
        E = SEEnergy.apply(xg, qg, plan)
        E.backward()
        torch.cuda.synchronize()
        grads[dtype] = (xg.grad.double().cpu().numpy(), qg.grad.double().cpu().numpy())

    # central differences of the FP64 GPU energy (x is exactly representable)
    x64, q64 = to_dev(x, q, torch.float64)
    plan = SEPlan(M, P, L, xi, dtype=torch.float64, n_max=len(q))
    fd = np.zeros((len(atoms), 3))
    for a, m in enumerate(atoms):
        for d in range(3):
            xp = x64.clone()
            xp[m, d] += dx
            Ep = plan.forward(xp, q64).item()
            xm = x64.clone()
            xm[m, d] -= dx
            Em = plan.forward(xm, q64).item()
            fd[a, d] = (Ep - Em) / (2 * dx)
    for dtype, lim_rms, lim_max in ((torch.float32, 1e-5, 1e-4), (torch.float64, 1e-6, 1e-5)):
        g = grads[dtype][0][atoms]
        rel = np.sqrt(np.sum((g - fd) ** 2) / np.sum(fd ** 2))
        mx = np.max(np.abs(g - fd)) / np.sqrt(np.mean(fd ** 2))
        print(f"[fd] {dtype}: rms-rel {rel:.2e} max-rel {mx:.2e}", flush=True)
        assert rel < lim_rms and mx < lim_max, (rel, mx)

    # dE/dq: E is quadratic in q, so central differences are exact up to rounding
    fdq = []
    for m in atoms[:8]:
        qp = q64.clone(); qp[m] += 1e-3
        qm = q64.clone(); qm[m] -= 1e-3
        fdq.append((plan.forward(x64, qp).item() - plan.forward(x64, qm).item()) / 2e-3)
    fdq = np.array(fdq)
    gq = grads[torch.float64][1][atoms[:8]]
    assert np.max(np.abs(gq - fdq)) < 1e-8 * np.max(np.abs(gq))

    # against the oracle's analytic forces on the same atoms
    xo, qo = as_oracle_inputs(x64, q64)
    eta = O.se_eta(L, xi, M, P)
    G = O.se_spread(xo, qo, L, M, P, xi, eta)
    _, Phi = O.scale_and_energy(G, O.se_influence(L, xi, M, eta), L)
    _, Fo = O.se_gather(xo[atoms], qo[atoms], L, M, P, xi, eta, Phi)
    for dtype, lim in ((torch.float32, 1e-5), (torch.float64, 1e-9)):
        assert max(array_errors(-grads[dtype][0][atoms], Fo)) < lim
