"""MI355X-native Spectral Ewald (SE) and SPME k-space evaluation, with the
real-space part of the Ewald sums beside it.

The computation lives in libsekspace.so (HIP kernels for gfx950, C ABI in
include/sekspace.h); this package only binds it to PyTorch tensors.
"""
from ._lib import EXPORTS, LIB_PATH, SeError  # noqa: F401
from . import tolerance  # noqa: F401  (host-only parameter selection)


def __getattr__(name):
    # torch is imported lazily so that the C-ABI helpers work without it
    if name in ("SEPlan", "SEEnergy", "se_kspace", "RealSpacePlan", "ewald_total"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
