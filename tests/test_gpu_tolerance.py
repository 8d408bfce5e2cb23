"""Parameters chosen from a tolerance deliver it: the total Ewald force of
1000 random ions computed on the GPU (FP64) with the (rc, xi, M, P) that
se_choose_params picks, against the oracle's exact Ewald sum.

The force estimates of section 2.1 (eqs. 2.1c, 2.2c) and section 5.3 are for
the root of the summed squared errors over all particles, sqrt(sum_n
|dF_n|^2).  With each of the three sources held to eps (and eta <= 0.5, the
regime the approximation estimate holds in) the total stays within 2 eps:
the real-space term, which the estimate predicts closely, dominates it."""
import math

import numpy as np
import pytest
import torch

from gpu_util import DEV
from oracle import se_oracle as O
from paper_1712_04718_amd import RealSpacePlan, SEPlan, ewald_total, tolerance

pytestmark = pytest.mark.gpu

N, L = 1000, 10.0


@pytest.fixture(scope="module")
def system():
    rng = np.random.default_rng(5)
    x = rng.random((N, 3)) * L
    q = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    _, _, F = O.ewald_total(x, q, L, 1.0, 9.0)  # xi-independent; truncation below 1e-30
    return x, q, F


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3, 1e-4])
def test_chosen_parameters_meet_force_tolerance(system, eps):
    x, q, Fref = system
    ch = tolerance.choose_params("force", eps, N, float(np.sum(q * q)), L, (1.0, L / 3),
                                 n_rc=64, dtype="f64")
    print(f"[tolerance] eps={eps}: rc={ch['rc']:.3f} xi={ch['xi']:.3f} M={ch['M']} P={ch['P']}",
          flush=True)
    xt = torch.tensor(x, dtype=torch.float64, device=DEV)
    qt = torch.tensor(q, dtype=torch.float64, device=DEV)
    kplan = SEPlan(ch["M"], ch["P"], L, ch["xi"], dtype=torch.float64, n_max=N, add_self=True)
    rplan = RealSpacePlan(L, ch["xi"], ch["rc"], dtype=torch.float64, n_max=N)
    _, _, F = ewald_total(xt, qt, kplan, rplan)
    torch.cuda.synchronize()
    err = math.sqrt(float(np.sum((F.cpu().numpy() - Fref) ** 2)))
    print(f"[tolerance] eps={eps}: error {err:.3e} ({err / eps:.2f} eps)", flush=True)
    assert err <= 2 * eps
    for p in (kplan, rplan):
        p.close()
