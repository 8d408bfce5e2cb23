"""Per-kernel timing plans (SE_FLAG_TIMING): every launch is counted, the
ring of event pairs wraps without losing launches, and timing changes no
result."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, to_dev
from paper_1712_04718_amd import SEPlan, _lib

pytestmark = pytest.mark.gpu


FIVE_PASSES = {"fft_x", "fft_y", "ifft_y", "ifft_x"}
PLANE_PASSES = {"fft_xy", "ifft_yx"}


# M = 40 and M = 192: the plane fits in LDS (twice, or once with in-place
# stages), so x and y run as one pass each way; M = 216 in FP32 does not
# fit and runs the five separate passes
@pytest.mark.parametrize("M,fft_stages", [(40, PLANE_PASSES), (192, PLANE_PASSES),
                                          (216, FIVE_PASSES)])
def test_stage_means_cover_every_launch_and_reset(M, fft_stages):
    print(f"[timing] N=3000 L=20 M={M} P=8 fp32, 40 steps", flush=True)
    rng = np.random.default_rng(11)
    x = rng.random((3000, 3)) * 20.0
    q = rng.standard_normal(3000)
    q -= q.mean()
    xt, qt = to_dev(x, q, torch.float32)
    ref = SEPlan(M, 8, 20.0, 0.6, dtype=torch.float32, n_max=3000)
    tim = SEPlan(M, 8, 20.0, 0.6, dtype=torch.float32, n_max=3000, timing=True)
    E0, phi0, F0 = ref.kspace(xt, qt)
    for _ in range(40):  # more launches than the ring of event pairs holds
        E1, phi1, F1 = tim.kspace(xt, qt)
    times = tim.stage_times()
    # up to 8192 tiles the scan runs inside the scatter kernel
    assert set(times) == (set(_lib.STAGES) - FIVE_PASSES - PLANE_PASSES - {"bin_scan"}) | fft_stages
    assert all(v > 0 for v in times.values()), times
    # nothing launched since the read: every stage reports "not launched"
    assert tim.stage_times() == {}
    # the FP32 spread is order-independent, so timing changes no bit
    torch.cuda.synchronize()
    assert E0.item() == E1.item()
    assert torch.equal(phi0, phi1) and torch.equal(F0, F1)
    for p in (ref, tim):
        p.close()


def test_stage_times_needs_timing_plan():
    plan = SEPlan(16, 4, 10.0, 0.5, dtype=torch.float32, n_max=10)
    with pytest.raises(_lib.SeError, match="SE_ERR_STATE"):
        plan.stage_times()
    plan.close()
