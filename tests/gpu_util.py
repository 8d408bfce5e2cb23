"""Helpers shared by the GPU tests: run the GPU path and the oracle on the
same (exactly representable) inputs and measure their disagreement."""
import numpy as np
import torch

from oracle import se_oracle as O
from paper_1712_04718_amd import SEPlan

DEV = torch.device("cuda:0")
TOL = {torch.float32: 1e-5, torch.float64: 1e-9}


def to_dev(x, q, dtype):
    xt = torch.tensor(np.asarray(x), dtype=dtype, device=DEV)
    qt = torch.tensor(np.asarray(q), dtype=dtype, device=DEV)
    return xt, qt


def as_oracle_inputs(xt, qt):
    """The device inputs, promoted exactly to float64 for the oracle."""
    return xt.double().cpu().numpy(), qt.double().cpu().numpy()


def oracle_kspace(window, x, q, L, xi, M, P):
    if window == "gaussian":
        return O.se_kspace(x, q, L, xi, M, P)
    return O.spme_kspace(x, q, L, xi, M, P)


def gpu_kspace(x, q, L, xi, M, P, dtype, window="gaussian", add_self=False):
    xt, qt = to_dev(x, q, dtype)
    plan = SEPlan(M, P, L, xi, window=window, dtype=dtype, n_max=max(1, len(q)),
                  add_self=add_self)
    E, phi, F = plan.kspace(xt, qt)
    torch.cuda.synchronize()
    out = (E.item(), phi.double().cpu().numpy(), F.double().cpu().numpy())
    return out, plan, xt, qt


# Every parity check holds both norms: the relative rms error of an array to
# the tolerance, and its largest element error (relative to the rms of the
# reference values) to MAX_FACTOR times the tolerance, so that a defect
# confined to a few particles (a wrong stencil at a tile seam, one bad tile)
# cannot hide in the rms.
MAX_FACTOR = 10.0


def max_rel(a, ref):
    """max |a - ref| over all elements / rms(ref)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = np.sqrt(np.mean(ref ** 2))
    return float(np.max(np.abs(a - ref)) / rms) if a.size else 0.0


def array_errors(a, ref):
    """(relative rms error, largest element error / MAX_FACTOR): both must
    stay below the tolerance."""
    return O.rel_rms(a, ref), max_rel(a, ref) / MAX_FACTOR


def errors(gpu, ref):
    """Errors of (E, phi, F) against the oracle's, each to be held below the
    tolerance: |E - E*| / |E*|, then array_errors of phi and of F."""
    (E, phi, F), (Eo, phio, Fo) = gpu, ref
    return ((abs(E - Eo) / abs(Eo) if Eo != 0 else abs(E),)
            + array_errors(phi, phio) + array_errors(F, Fo))


_SYSTEMS = {}


def cached_system(name):
    """(x, q, spec) of a named workload, generated once per test session."""
    from workloads import make_system
    if name not in _SYSTEMS:
        _SYSTEMS[name] = make_system(name)
    return _SYSTEMS[name]
