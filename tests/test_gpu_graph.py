"""Evaluations captured in a HIP graph: every replay, with new positions and
charges copied into the captured inputs and eager work between the replays,
equals an eager evaluation of the same inputs: the k-space path bit for bit
in both precisions (its spread accumulates in fixed point, order-free), the
real-space sum to rounding (the order of particles in a cell comes from
atomics)."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import DEV
from paper_1712_04718_amd import RealSpacePlan, SEPlan, _lib

pytestmark = pytest.mark.gpu


def _inputs(rng, N, L):
    x = rng.random((N, 3)) * L
    q = rng.standard_normal(N)
    return x, q - q.mean()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("window,M,P", [("gaussian", 48, 8), ("bspline", 40, 6)])
def test_kspace_graph_replays(window, M, P, dtype):
    print(f"[graph] {window} M={M} P={P} {dtype}", flush=True)
    N, L, xi = 3000, 16.0, 1.0
    rng = np.random.default_rng(51)
    lib = _lib.load()
    plan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=N, add_self=True)
    eager = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=N, add_self=True)
    xs = torch.zeros(N, 3, dtype=dtype, device=DEV)
    qs = torch.zeros(N, dtype=dtype, device=DEV)
    E = torch.zeros((), dtype=torch.float64, device=DEV)
    phi = torch.zeros(N, dtype=dtype, device=DEV)
    F = torch.zeros(N, 3, dtype=dtype, device=DEV)
    gE = torch.ones((), dtype=torch.float64, device=DEV)
    gx = torch.zeros(N, 3, dtype=dtype, device=DEV)
    gq = torch.zeros(N, dtype=dtype, device=DEV)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731

    def step():
        s = torch.cuda.current_stream().cuda_stream
        _lib.check(lib.se_plan_set_stream(plan._plan, ctypes.c_void_p(s)))
        _lib.check(lib.se_kspace(plan._plan, N, ptr(xs), ptr(qs), ptr(E), ptr(phi), ptr(F)))
        _lib.check(lib.se_backward(plan._plan, ptr(gE), ptr(gx), ptr(gq)))

    x0, q0 = _inputs(rng, N, L)
    xs.copy_(torch.tensor(x0, dtype=dtype))
    qs.copy_(torch.tensor(q0, dtype=dtype))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    rt = 0.0
    for rep in range(4):
        x, q = _inputs(rng, N, L)
        xs.copy_(torch.tensor(x, dtype=dtype))
        qs.copy_(torch.tensor(q, dtype=dtype))
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays, on another plan
        xe, qe = xs.clone(), qs.clone()
        Ee, phie, Fe = eager.kspace(xe, qe)
        gxe, gqe = eager.backward(torch.ones((), dtype=torch.float64, device=DEV))
        torch.cuda.synchronize()
        np.testing.assert_allclose(E.item(), Ee.item(), rtol=rt, atol=0)
        for got, want in ((phi, phie), (F, Fe), (gx, gxe), (gq, gqe)):
            np.testing.assert_allclose(got.cpu().numpy(), want.cpu().numpy(), rtol=0,
                                       atol=rt * float(want.abs().max()))
    for p in (plan, eager):
        p.close()


def test_realspace_graph_replays():
    print("[graph] real space fp32", flush=True)
    N, L, xi, rc = 4000, 20.0, 0.6, 5.0
    rng = np.random.default_rng(52)
    lib = _lib.load()
    plan = RealSpacePlan(L, xi, rc, dtype=torch.float32, n_max=N)
    eager = RealSpacePlan(L, xi, rc, dtype=torch.float32, n_max=N)
    xs = torch.zeros(N, 3, dtype=torch.float32, device=DEV)
    qs = torch.zeros(N, dtype=torch.float32, device=DEV)
    E = torch.zeros((), dtype=torch.float64, device=DEV)
    phi = torch.zeros(N, dtype=torch.float32, device=DEV)
    F = torch.zeros(N, 3, dtype=torch.float32, device=DEV)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731

    def step():
        s = torch.cuda.current_stream().cuda_stream
        _lib.check(lib.se_rs_plan_set_stream(plan._plan, ctypes.c_void_p(s)))
        _lib.check(lib.se_rs_eval(plan._plan, N, ptr(xs), ptr(qs), ptr(E), ptr(phi), ptr(F)))

    x0, q0 = _inputs(rng, N, L)
    xs.copy_(torch.tensor(x0, dtype=torch.float32))
    qs.copy_(torch.tensor(q0, dtype=torch.float32))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        x, q = _inputs(rng, N, L)
        xs.copy_(torch.tensor(x, dtype=torch.float32))
        qs.copy_(torch.tensor(q, dtype=torch.float32))
        g.replay()
        torch.cuda.synchronize()
        Ee, phie, Fe = eager.eval(xs.clone(), qs.clone())
        torch.cuda.synchronize()
        # the order of particles inside a cell comes from atomics, so the FP32
        # sums agree to rounding
        assert abs(E.item() - Ee.item()) <= 1e-5 * abs(Ee.item())
        for got, want in ((phi, phie), (F, Fe)):
            d = (got.double() - want.double()).norm() / want.double().norm()
            assert d < 1e-5, d.item()
    for p in (plan, eager):
        p.close()


def test_autograd_step_graph_replays():
    """SEEnergy forward + backward captured in a HIP graph (the adjoint reads
    dL/dE from device memory): every replay with new inputs gives the
    gradients an eager autograd step gives (FP32, bit for bit)."""
    from paper_1712_04718_amd import SEEnergy
    print("[graph] autograd fp32", flush=True)
    N, L, xi = 3000, 16.0, 1.0
    rng = np.random.default_rng(53)
    plan = SEPlan(48, 8, L, xi, dtype=torch.float32, n_max=N)
    eager = SEPlan(48, 8, L, xi, dtype=torch.float32, n_max=N)
    x0, q0 = _inputs(rng, N, L)
    xg = torch.tensor(x0, dtype=torch.float32, device=DEV).requires_grad_(True)
    qg = torch.tensor(q0, dtype=torch.float32, device=DEV).requires_grad_(True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            xg.grad = None
            qg.grad = None
            SEEnergy.apply(xg, qg, plan).backward()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    xg.grad = None
    qg.grad = None
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        SEEnergy.apply(xg, qg, plan).backward()
    for rep in range(3):
        x, q = _inputs(rng, N, L)
        with torch.no_grad():
            xg.copy_(torch.tensor(x, dtype=torch.float32))
            qg.copy_(torch.tensor(q, dtype=torch.float32))
        g.replay()
        torch.cuda.synchronize()
        xe = xg.detach().clone().requires_grad_(True)
        qe = qg.detach().clone().requires_grad_(True)
        SEEnergy.apply(xe, qe, eager).backward()
        torch.cuda.synchronize()
        assert torch.equal(xg.grad, xe.grad) and torch.equal(qg.grad, qe.grad)
    for p in (plan, eager):
        p.close()
