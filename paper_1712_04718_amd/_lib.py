"""ctypes view of libsekspace.so (declared in include/sekspace.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsekspace.so")

SE_OK = 0
SE_WINDOW_GAUSSIAN = 0
SE_WINDOW_BSPLINE = 1
SE_FP32 = 0
SE_FP64 = 1
SE_FLAG_ADD_SELF = 1
SE_FLAG_TIMING = 2
SE_FLAG_IK_FORCE = 4
SE_FLAG_CALLER_WORKSPACE = 8
STAGES = ("bin_count", "bin_scan", "bin_scatter", "spread", "fold", "fft_x", "fft_y",
          "fft_z_scale", "ifft_y", "ifft_x", "gather", "fft_xy", "ifft_yx")

STATUS_NAMES = {
    0: "SE_OK", 1: "SE_ERR_ARG", 2: "SE_ERR_GRID", 3: "SE_ERR_ETA",
    4: "SE_ERR_UNSUPPORTED", 5: "SE_ERR_WORKSPACE", 6: "SE_ERR_HIP", 7: "SE_ERR_STATE",
}

# Every entry point the header declares.
EXPORTS = (
    "se_status_string", "se_last_error", "se_params_check", "se_plan_workspace_size",
    "se_plan_create", "se_plan_set_workspace", "se_plan_set_stream", "se_plan_eta",
    "se_plan_destroy",
    "se_forward", "se_gather", "se_kspace", "se_kspace_noalloc", "se_backward",
    "se_plan_stage_times",
    "se_plan_reserve_targets", "se_eval_targets",
    "se_rs_plan_create", "se_rs_plan_set_stream", "se_rs_eval", "se_rs_plan_destroy",
    "se_est_real_error", "se_est_fourier_error", "se_est_xi", "se_est_kinf",
    "se_est_se_error", "se_est_se_support", "se_cost_model_mi355x", "se_cost_predict",
    "se_choose_params",
)

EST_KINDS = {"potential": 0, "energy": 1, "force": 2}


class SeParams(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int),
        ("P", ctypes.c_int),
        ("L", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("c", ctypes.c_double),
        ("window", ctypes.c_int),
        ("dtype", ctypes.c_int),
        ("flags", ctypes.c_uint),
    ]


class SeCostModel(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "real_fixed", "real_atom", "real_pair", "real_cell", "real_test",
        "k_fixed", "k_atom", "k_window", "k_block", "k_grid", "k_fft")]


class SeChoice(ctypes.Structure):
    _fields_ = [
        ("rc", ctypes.c_double), ("xi", ctypes.c_double), ("kinf", ctypes.c_double),
        ("M", ctypes.c_int), ("P", ctypes.c_int), ("eta", ctypes.c_double),
        ("t_real", ctypes.c_double), ("t_kspace", ctypes.c_double),
        ("est_real", ctypes.c_double), ("est_fourier", ctypes.c_double),
        ("est_approx", ctypes.c_double),
    ]


class SeError(RuntimeError):
    """A non-zero se_status, with the library's message."""

    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1712_04718_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pp = ctypes.POINTER(SeParams)
    lib.se_status_string.restype = ctypes.c_char_p
    lib.se_status_string.argtypes = [i]
    lib.se_last_error.restype = ctypes.c_char_p
    lib.se_last_error.argtypes = []
    lib.se_params_check.restype = i
    lib.se_params_check.argtypes = [pp, ctypes.POINTER(d)]
    lib.se_plan_workspace_size.restype = i
    lib.se_plan_workspace_size.argtypes = [pp, i, ctypes.POINTER(ctypes.c_size_t)]
    lib.se_plan_create.restype = i
    lib.se_plan_create.argtypes = [pp, i, vp, ctypes.POINTER(vp)]
    lib.se_plan_set_workspace.restype = i
    lib.se_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    lib.se_plan_set_stream.restype = i
    lib.se_plan_set_stream.argtypes = [vp, vp]
    lib.se_plan_eta.restype = i
    lib.se_plan_eta.argtypes = [vp, ctypes.POINTER(d)]
    lib.se_plan_destroy.restype = i
    lib.se_plan_destroy.argtypes = [vp]
    lib.se_forward.restype = i
    lib.se_forward.argtypes = [vp, i, vp, vp, vp]
    lib.se_gather.restype = i
    lib.se_gather.argtypes = [vp, vp, vp]
    lib.se_kspace.restype = i
    lib.se_kspace.argtypes = [vp, i, vp, vp, vp, vp, vp]
    lib.se_kspace_noalloc.restype = i
    lib.se_kspace_noalloc.argtypes = [pp, i, vp, vp, vp, vp, vp, vp]
    lib.se_backward.restype = i
    lib.se_backward.argtypes = [vp, vp, vp, vp]
    lib.se_plan_reserve_targets.restype = i
    lib.se_plan_reserve_targets.argtypes = [vp, i]
    lib.se_eval_targets.restype = i
    lib.se_eval_targets.argtypes = [vp, i, vp, vp, vp]
    lib.se_plan_stage_times.restype = i
    lib.se_plan_stage_times.argtypes = [vp, ctypes.POINTER(d), i]
    lib.se_rs_plan_create.restype = i
    lib.se_rs_plan_create.argtypes = [d, d, d, i, i, vp, ctypes.POINTER(vp)]
    lib.se_rs_plan_set_stream.restype = i
    lib.se_rs_plan_set_stream.argtypes = [vp, vp]
    lib.se_rs_eval.restype = i
    lib.se_rs_eval.argtypes = [vp, i, vp, vp, vp, vp, vp]
    lib.se_rs_plan_destroy.restype = i
    lib.se_rs_plan_destroy.argtypes = [vp]
    pd = ctypes.POINTER(d)
    for name in ("se_est_real_error", "se_est_fourier_error", "se_est_xi", "se_est_kinf"):
        getattr(lib, name).restype = i
        getattr(lib, name).argtypes = [i, d, d, d, d, pd]
    lib.se_est_se_error.restype = i
    lib.se_est_se_error.argtypes = [i, d, d, d, i, d, pd]
    lib.se_est_se_support.restype = i
    lib.se_est_se_support.argtypes = [i, d, d, d, d, d, ctypes.POINTER(i)]
    lib.se_cost_model_mi355x.restype = i
    lib.se_cost_model_mi355x.argtypes = [i, ctypes.POINTER(SeCostModel)]
    lib.se_cost_predict.restype = i
    lib.se_cost_predict.argtypes = [ctypes.POINTER(SeCostModel), i, i, d, d, i, i, pd, pd]
    lib.se_choose_params.restype = i
    lib.se_choose_params.argtypes = [i, d, i, d, d, d, d, i, d, i, ctypes.POINTER(SeCostModel),
                                     ctypes.POINTER(SeChoice)]
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != SE_OK:
        msg = load().se_last_error().decode(errors="replace")
        raise SeError(status, msg)


def make_params(M, P, L, xi, c=0.95, window=SE_WINDOW_GAUSSIAN, dtype=SE_FP32, flags=0) -> SeParams:
    return SeParams(int(M), int(P), float(L), float(xi), float(c), int(window), int(dtype),
                    int(flags))


def params_check(prm: SeParams):
    """(status, eta) from the host-only parameter check."""
    eta = ctypes.c_double(0.0)
    st = load().se_params_check(ctypes.byref(prm), ctypes.byref(eta))
    return st, eta.value


def workspace_size(prm: SeParams, n_max: int):
    b = ctypes.c_size_t(0)
    st = load().se_plan_workspace_size(ctypes.byref(prm), int(n_max), ctypes.byref(b))
    return st, b.value
