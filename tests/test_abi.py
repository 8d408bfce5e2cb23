"""The C-ABI library: it loads, exports every symbol the header declares, and
its host-side argument checks behave as documented.  No GPU calls."""
import math
import os
import re

import pytest

from paper_1712_04718_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "sekspace.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(se_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib.load()
    for code, name in _lib.STATUS_NAMES.items():
        assert lib.se_status_string(code).decode().startswith(name)


def _check(**kw):
    base = dict(M=96, P=8, L=100.0, xi=0.3, c=0.95, window=0, dtype=0, flags=0)
    base.update(kw)
    prm = _lib.make_params(**base)
    return _lib.params_check(prm)


def test_eta_matches_paper_formula():
    """eta = P L^2 xi^2 / (c^2 pi M^2) (section 4, eq. 5.2)."""
    for (M, P, L, xi) in [(96, 8, 100.0, 0.3), (32, 8, 10.0, 1.5), (192, 8, 220.0, 0.35),
                          (40, 10, 40.0, 0.3)]:
        st, eta = _check(M=M, P=P, L=L, xi=xi)
        assert st == _lib.SE_OK
        assert abs(eta - P * L * L * xi * xi / (0.95 ** 2 * math.pi * M * M)) < 1e-15


@pytest.mark.parametrize("kw,status", [
    (dict(L=0.0), 1), (dict(L=-1.0), 1), (dict(xi=0.0), 1), (dict(L=float("nan")), 1),
    (dict(window=7), 1), (dict(dtype=3), 1), (dict(flags=32), 1),
    (dict(M=33), 2), (dict(M=14), 2), (dict(M=6), 2), (dict(M=1024), 2), (dict(M=10, P=12), 2),
    (dict(P=7), 4), (dict(P=18), 4), (dict(P=2), 4), (dict(P=26, dtype=1), 4),
    (dict(P=19, dtype=1), 4), (dict(P=18, dtype=1, xi=0.2, flags=4), 4), (dict(flags=16), 1),
    (dict(window=1, P=2), 4), (dict(window=1, P=9), 4),
    (dict(xi=3.0), 3),
])
def test_invalid_parameters_rejected(kw, status):
    st, _ = _check(**kw)
    assert st == status
    assert _lib.load().se_last_error().decode() != ""


def test_valid_parameter_sets():
    for kw in [dict(), dict(dtype=1), dict(window=1, P=4), dict(window=1, P=3),
               dict(window=1, P=7), dict(M=40, L=40.0, P=6), dict(M=30, L=10.0, xi=1.0, P=8),
               dict(dtype=1, P=18, xi=0.2), dict(dtype=1, P=24, xi=0.2), dict(flags=4),
               dict(window=1, P=5, flags=4)]:
        st, _ = _check(**kw)
        assert st == _lib.SE_OK, kw


def test_workspace_size():
    prm = _lib.make_params(96, 8, 100.0, 0.3)
    st, b = _lib.workspace_size(prm, 100200)
    assert st == 0
    M, K = 96, 49
    assert b >= M ** 3 * 4 + M * M * K * 8 + 100200 * 16
    st, b64 = _lib.workspace_size(_lib.make_params(96, 8, 100.0, 0.3, dtype=1), 100200)
    assert st == 0 and b64 > b
    st, _ = _lib.workspace_size(prm, 0)
    assert st == 1  # SE_ERR_ARG


@pytest.mark.parametrize("L,xi,rc,dtype,n_max", [
    (10.0, 1.0, 4.0, _lib.SE_FP32, 10),      # rc > L/3: more than one image within rc
    (10.0, 1.0, 0.0, _lib.SE_FP32, 10),      # rc = 0
    (-1.0, 1.0, 0.2, _lib.SE_FP32, 10),      # L <= 0
    (10.0, 0.0, 2.0, _lib.SE_FP32, 10),      # xi = 0
    (10.0, 1.0, 2.0, 7, 10),                 # unknown dtype
    (10.0, 1.0, 2.0, _lib.SE_FP64, 0),       # n_max < 1
])
def test_realspace_plan_rejects_bad_arguments(L, xi, rc, dtype, n_max):
    """The real-space plan checks its arguments on the host before touching
    the device (so this runs without a GPU)."""
    import ctypes
    lib = _lib.load()
    out = ctypes.c_void_p(None)
    st = lib.se_rs_plan_create(L, xi, rc, dtype, n_max, None, ctypes.byref(out))
    assert _lib.STATUS_NAMES.get(st) == "SE_ERR_ARG", st
    assert out.value is None
    assert lib.se_last_error().decode()


def test_target_entry_points_reject_bad_arguments():
    lib = _lib.load()
    assert _lib.STATUS_NAMES[lib.se_plan_reserve_targets(None, 10)] == "SE_ERR_ARG"
    assert _lib.STATUS_NAMES[lib.se_eval_targets(None, 1, None, None, None)] == "SE_ERR_ARG"


def test_caller_workspace_host_checks():
    """A plan created with SE_FLAG_CALLER_WORKSPACE allocates nothing and
    makes no HIP call until a workspace is attached, so its checks run here:
    a buffer smaller than se_plan_workspace_size or not 256-byte aligned is
    SE_ERR_WORKSPACE, a NULL one SE_ERR_ARG, and forward/gather before any
    workspace SE_ERR_STATE (all before any HIP call)."""
    import ctypes
    lib = _lib.load()
    prm = _lib.make_params(32, 8, 10.0, 1.5, flags=_lib.SE_FLAG_CALLER_WORKSPACE)
    st, need = _lib.workspace_size(prm, 1000)
    assert st == 0 and need > 0
    plan = ctypes.c_void_p(None)
    assert lib.se_plan_create(ctypes.byref(prm), 1000, None, ctypes.byref(plan)) == 0
    try:
        name = lambda st: _lib.STATUS_NAMES[st]  # noqa: E731
        fake = ctypes.c_void_p(1 << 40)  # never dereferenced: every check fails first
        assert name(lib.se_plan_set_workspace(plan, fake, need - 1)) == "SE_ERR_WORKSPACE"
        assert "smaller" in lib.se_last_error().decode()
        assert name(lib.se_plan_set_workspace(plan, ctypes.c_void_p((1 << 40) + 64), need)) \
            == "SE_ERR_WORKSPACE"
        assert "256" in lib.se_last_error().decode()
        assert name(lib.se_plan_set_workspace(plan, None, need)) == "SE_ERR_ARG"
        assert name(lib.se_plan_set_workspace(None, fake, need)) == "SE_ERR_ARG"
        E = ctypes.c_void_p(1 << 40)
        assert name(lib.se_forward(plan, 0, None, None, E)) == "SE_ERR_STATE"
        assert name(lib.se_gather(plan, None, None)) == "SE_ERR_STATE"
    finally:
        assert lib.se_plan_destroy(plan) == 0
