"""A plan on a caller-owned workspace (SE_FLAG_CALLER_WORKSPACE with
se_plan_set_workspace, here memory of PyTorch's caching allocator) gives the
results of a plan that owns its workspace, bit for bit: the same kernels and
tables, and the spread accumulates in fixed point."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, to_dev
from paper_1712_04718_amd import SeError, SEPlan, _lib

pytestmark = pytest.mark.gpu


def _run(plan, xt, qt):
    E, phi, F = plan.kspace(xt, qt)
    gx, gq = plan.backward(torch.tensor(0.75, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    return E, phi, F, gx, gq


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("window,M,P", [("gaussian", 30, 8), ("gaussian", 32, 12),
                                        ("bspline", 32, 5)])
def test_caller_workspace_matches_owned(window, M, P, dtype):
    L, xi = 10.0, 1.2
    rng = np.random.default_rng(61)
    x = rng.random((900, 3)) * 12.0 - 1.0
    q = rng.standard_normal(900)
    print(f"[workspace] {window} M={M} P={P} {dtype}", flush=True)
    xt, qt = to_dev(x, q, dtype)
    owned = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=900)
    ws = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=900, workspace=True)
    assert ws.workspace is not None and ws.workspace.dtype == torch.uint8
    ref = _run(owned, xt, qt)
    got = _run(ws, xt, qt)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    # a second, smaller input on the same workspace
    ref2 = _run(owned, xt[:333], qt[:333])
    got2 = _run(ws, xt[:333], qt[:333])
    for a, b in zip(ref2, got2):
        assert torch.equal(a, b)
    owned.close()
    ws.close()


def test_caller_workspace_reattach_and_errors():
    """A supplied tensor is used as given; re-attaching another one drops the
    stored grid (gather is refused until the next forward) and then gives
    the same results; too small a tensor is refused."""
    M, P, L, xi, N = 32, 8, 10.0, 1.2, 500
    rng = np.random.default_rng(62)
    xt, qt = to_dev(rng.random((N, 3)) * L, rng.standard_normal(N), torch.float32)
    prm = _lib.make_params(M, P, L, xi, flags=_lib.SE_FLAG_CALLER_WORKSPACE)
    st, need = _lib.workspace_size(prm, N)
    assert st == 0
    buf = torch.empty(need + 4096, dtype=torch.uint8, device=DEV)
    plan = SEPlan(M, P, L, xi, n_max=N, workspace=buf)
    assert plan.workspace.data_ptr() == buf.data_ptr()
    E1, phi1, F1 = plan.kspace(xt, qt)
    buf2 = torch.empty(need, dtype=torch.uint8, device=DEV)
    _lib.check(plan.lib.se_plan_set_workspace(plan._plan, ctypes_ptr(buf2), need))
    with pytest.raises(SeError):
        _lib.check(plan.lib.se_gather(plan._plan, None, None))
    E2, phi2, F2 = plan.kspace(xt, qt)
    torch.cuda.synchronize()
    assert torch.equal(E1, E2) and torch.equal(phi1, phi2) and torch.equal(F1, F2)
    with pytest.raises(SeError):
        SEPlan(M, P, L, xi, n_max=N, workspace=buf2[: need - 256])
    plan.close()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())
