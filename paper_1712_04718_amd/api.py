"""PyTorch-facing binding of the Spectral Ewald k-space library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsekspace.so.  PyTorch supplies device memory and the stream.

    plan = SEPlan(M=96, P=8, L=100.0, xi=0.3, dtype=torch.float32, n_max=N)
    E, phi, F = plan.kspace(x, q)           # x [N,3], q [N] on the GPU
    E = SEEnergy.apply(x, q, plan)          # differentiable in x and q
"""
from __future__ import annotations

import contextlib
import ctypes

import torch

from . import _lib

_DTYPES = {torch.float32: _lib.SE_FP32, torch.float64: _lib.SE_FP64}
_WINDOWS = {"gaussian": _lib.SE_WINDOW_GAUSSIAN, "se": _lib.SE_WINDOW_GAUSSIAN,
            "bspline": _lib.SE_WINDOW_BSPLINE, "spme": _lib.SE_WINDOW_BSPLINE}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _on(device):
    """Context making ``device`` current; a no-op when it already is (the
    common case, and the switch costs microseconds per call)."""
    if torch.cuda.current_device() == device.index:
        return contextlib.nullcontext()
    return torch.cuda.device(device)


class SEPlan:
    """A k-space plan (grid size M, support P or B-spline order p, box L,
    Ewald parameter xi, window, precision) for up to ``n_max`` particles on
    one GPU.  The plan keeps the scaled grid of its last forward pass for
    ``gather`` and ``backward``."""

    def __init__(self, M, P, L, xi, window="gaussian", dtype=torch.float32, c=0.95,
                 n_max=1 << 20, add_self=False, device=None, timing=False, ik_force=False,
                 workspace=None):
        """``workspace``: None (the library allocates the plan's device
        memory), True (a uint8 tensor from PyTorch's caching allocator of
        the size the library asks for), or such a tensor supplied by the
        caller (contiguous, on the plan's device, large enough, 256-byte
        aligned); the plan keeps a reference to it."""
        if not torch.cuda.is_available():
            raise RuntimeError("SEPlan needs a GPU (no HIP device visible)")
        if dtype not in _DTYPES:
            raise TypeError(f"dtype must be float32 or float64, got {dtype}")
        if window not in _WINDOWS:
            raise ValueError(f"window must be one of {sorted(_WINDOWS)}")
        self.lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.M, self.P, self.L, self.xi = int(M), int(P), float(L), float(xi)
        self.window = window
        self.dtype = dtype
        self.n_max = int(n_max)
        flags = ((_lib.SE_FLAG_ADD_SELF if add_self else 0) | (_lib.SE_FLAG_TIMING if timing else 0)
                 | (_lib.SE_FLAG_IK_FORCE if ik_force else 0)
                 | (_lib.SE_FLAG_CALLER_WORKSPACE if workspace is not None else 0))
        self.params = _lib.make_params(M, P, L, xi, c, _WINDOWS[window], _DTYPES[dtype], flags)
        self._plan = ctypes.c_void_p(None)
        self.workspace = None
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _lib.check(self.lib.se_plan_create(ctypes.byref(self.params), self.n_max,
                                               ctypes.c_void_p(stream), ctypes.byref(self._plan)))
            if workspace is not None:
                st, nbytes = _lib.workspace_size(self.params, self.n_max)
                _lib.check(st)
                if workspace is True:
                    workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                if (not isinstance(workspace, torch.Tensor) or workspace.device != self.device
                        or not workspace.is_contiguous()):
                    raise ValueError(f"workspace must be a contiguous tensor on {self.device}")
                _lib.check(self.lib.se_plan_set_workspace(
                    self._plan, _ptr(workspace), workspace.numel() * workspace.element_size()))
                self.workspace = workspace
        eta = ctypes.c_double(0.0)
        _lib.check(self.lib.se_plan_eta(self._plan, ctypes.byref(eta)))
        self.eta = eta.value
        self.generation = 0     # bumped by every forward pass
        self._N = None

    # ------------------------------------------------------------ helpers
    def _bind_stream(self):
        # every call enqueues on torch's current stream of the plan's device
        # (set each time: the plan may also be driven through the C ABI)
        s = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(self.lib.se_plan_set_stream(self._plan, ctypes.c_void_p(s)))

    def _check_inputs(self, x, q):
        if x.device != self.device or q.device != self.device:
            raise ValueError(f"x and q must be on {self.device}")
        if x.dtype != self.dtype or q.dtype != self.dtype:
            raise TypeError(f"x and q must be {self.dtype}")
        if x.dim() != 2 or x.shape[1] != 3 or q.dim() != 1 or q.shape[0] != x.shape[0]:
            raise ValueError("expected x [N,3] and q [N]")
        if x.shape[0] > self.n_max:
            raise ValueError(f"N={x.shape[0]} exceeds n_max={self.n_max}")
        return x.contiguous(), q.contiguous()

    # ---------------------------------------------------------------- API
    def forward(self, x, q):
        """Steps 1-5: returns E (0-d float64 tensor on the device)."""
        x, q = self._check_inputs(x, q)
        E = torch.empty((), dtype=torch.float64, device=self.device)
        with _on(self.device):
            self._bind_stream()
            _lib.check(self.lib.se_forward(self._plan, int(x.shape[0]), _ptr(x), _ptr(q), _ptr(E)))
        self._keep = (x, q)  # inputs stay alive until the enqueued work has used them
        self._N = int(x.shape[0])
        self.generation += 1
        return E

    def gather(self, want_phi=True, want_F=True):
        """Step 6 for the last forward: (phi [N], F [N,3])."""
        if self._N is None:
            raise RuntimeError("gather before forward")
        phi = torch.empty(self._N, dtype=self.dtype, device=self.device) if want_phi else None
        F = torch.empty(self._N, 3, dtype=self.dtype, device=self.device) if want_F else None
        with _on(self.device):
            self._bind_stream()
            _lib.check(self.lib.se_gather(self._plan, _ptr(phi), _ptr(F)))
        return phi, F

    def kspace(self, x, q):
        """(E, phi, F) of the k-space sum."""
        E = self.forward(x, q)
        phi, F = self.gather()
        return E, phi, F

    def backward(self, gE, want_x=True, want_q=True):
        """Adjoint of the last forward: (gE * dE/dx, gE * dE/dq)."""
        if self._N is None:
            raise RuntimeError("backward before forward")
        gE = gE.to(device=self.device, dtype=torch.float64).reshape(()).contiguous()
        gx = torch.empty(self._N, 3, dtype=self.dtype, device=self.device) if want_x else None
        gq = torch.empty(self._N, dtype=self.dtype, device=self.device) if want_q else None
        with _on(self.device):
            self._bind_stream()
            _lib.check(self.lib.se_backward(self._plan, _ptr(gE), _ptr(gx), _ptr(gq)))
        self._keep_g = gE
        return gx, gq

    def eval_targets(self, xt, want_phi=True, want_field=True):
        """(phi [nt], field [nt,3]) of the charges of the last forward pass at
        the points xt [nt,3] (unit test charges, no self term)."""
        if self._N is None:
            raise RuntimeError("eval_targets before forward")
        if xt.device != self.device or xt.dtype != self.dtype or xt.dim() != 2 or xt.shape[1] != 3:
            raise ValueError(f"xt must be [nt,3] {self.dtype} on {self.device}")
        xt = xt.contiguous()
        nt = int(xt.shape[0])
        if nt > getattr(self, "_tcap", 0):
            _lib.check(self.lib.se_plan_reserve_targets(self._plan, max(nt, 1)))
            self._tcap = max(nt, 1)
        phi = torch.empty(nt, dtype=self.dtype, device=self.device) if want_phi else None
        field = torch.empty(nt, 3, dtype=self.dtype, device=self.device) if want_field else None
        with _on(self.device):
            self._bind_stream()
            _lib.check(self.lib.se_eval_targets(self._plan, nt, _ptr(xt), _ptr(phi), _ptr(field)))
        self._keep_t = xt
        return phi, field

    def stage_times(self):
        """{stage: mean milliseconds per launch} over the launches since the
        previous call (plans created with ``timing=True``); waits for them."""
        n = len(_lib.STAGES)
        buf = (ctypes.c_double * n)()
        _lib.check(self.lib.se_plan_stage_times(self._plan, buf, n))
        return {name: buf[i] for i, name in enumerate(_lib.STAGES) if buf[i] >= 0}

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            _lib.check(self.lib.se_plan_destroy(self._plan))
            self._plan = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RealSpacePlan:
    """The real-space (erfc) part of the Ewald sums for up to ``n_max``
    particles in a cube of side L, truncated at rc <= L/3 (cell list on the
    GPU).  ``eval(x, q)`` returns (E, phi, F); the total Ewald sum is this
    plus the k-space part of an SEPlan created with ``add_self=True``."""

    def __init__(self, L, xi, rc, dtype=torch.float32, n_max=1 << 20, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("RealSpacePlan needs a GPU (no HIP device visible)")
        if dtype not in _DTYPES:
            raise TypeError(f"dtype must be float32 or float64, got {dtype}")
        self.lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.L, self.xi, self.rc, self.dtype, self.n_max = float(L), float(xi), float(rc), dtype, int(n_max)
        self._plan = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _lib.check(self.lib.se_rs_plan_create(self.L, self.xi, self.rc, _DTYPES[dtype],
                                                  self.n_max, ctypes.c_void_p(stream),
                                                  ctypes.byref(self._plan)))

    def eval(self, x, q, want_phi=True, want_F=True):
        if x.device != self.device or q.device != self.device:
            raise ValueError(f"x and q must be on {self.device}")
        if x.dtype != self.dtype or q.dtype != self.dtype:
            raise TypeError(f"x and q must be {self.dtype}")
        if x.dim() != 2 or x.shape[1] != 3 or q.dim() != 1 or q.shape[0] != x.shape[0]:
            raise ValueError("expected x [N,3] and q [N]")
        x, q = x.contiguous(), q.contiguous()
        N = int(x.shape[0])
        E = torch.empty((), dtype=torch.float64, device=self.device)
        phi = torch.empty(N, dtype=self.dtype, device=self.device) if want_phi else None
        F = torch.empty(N, 3, dtype=self.dtype, device=self.device) if want_F else None
        with _on(self.device):
            s = torch.cuda.current_stream(self.device).cuda_stream
            _lib.check(self.lib.se_rs_plan_set_stream(self._plan, ctypes.c_void_p(s)))
            _lib.check(self.lib.se_rs_eval(self._plan, N, _ptr(x), _ptr(q), _ptr(E), _ptr(phi),
                                           _ptr(F)))
        self._keep = (x, q)
        return E, phi, F

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            _lib.check(self.lib.se_rs_plan_destroy(self._plan))
            self._plan = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_SIDE_STREAMS = {}


def _side_stream(device):
    """A second stream (default priority) on ``device`` for work that may
    overlap the caller's current stream."""
    s = _SIDE_STREAMS.get(device)
    if s is None:
        s = _SIDE_STREAMS[device] = torch.cuda.Stream(device=device)
    return s


def ewald_total(x, q, kplan: SEPlan, rplan: RealSpacePlan, overlap=True):
    """(E, phi, F) of the total Ewald sum: real space + k space + self terms
    (the k-space plan must have been created with ``add_self=True``).

    With ``overlap`` the real-space sum runs on a second stream of the device
    while the k-space evaluation runs on the caller's stream (the two only
    read x and q and have separate workspaces): the k-space kernels leave
    CUs idle that the pair kernel can use.  The caller's stream waits for
    both before the sums, so the result is ordered on it as usual."""
    if not overlap or kplan.device != rplan.device:
        Ek, phik, Fk = kplan.kspace(x, q)
        Er, phir, Fr = rplan.eval(x, q)
        return Ek + Er, phik + phir, Fk + Fr
    dev = kplan.device
    main = torch.cuda.current_stream(dev)
    side = _side_stream(dev)
    side.wait_stream(main)  # x and q are ready on the side stream
    with torch.cuda.stream(side):
        Er, phir, Fr = rplan.eval(x, q)
    Ek, phik, Fk = kplan.kspace(x, q)
    main.wait_stream(side)
    # memory used across the two streams is not reused before both are done
    x.record_stream(side)
    q.record_stream(side)
    for t in (Er, phir, Fr):
        t.record_stream(main)
    return Ek + Er, phik + phir, Fk + Fr


def se_kspace(x, q, plan: SEPlan):
    """(E, phi[N], F[N,3]) of the k-space sum on ``plan``."""
    return plan.kspace(x, q)


class SEEnergy(torch.autograd.Function):
    """E(x, q) of the k-space sum, differentiable in x and q.

    The backward pass is the adjoint gather on the grid stored by the forward
    pass (no re-spreading): dE/dx = -F and dE/dq = phi.  The plan holds one
    forward pass at a time; the backward must run before the next forward on
    the same plan.  Double backward is not supported."""

    @staticmethod
    def forward(ctx, x, q, plan):
        E = plan.forward(x.detach(), q.detach())
        ctx.plan = plan
        ctx.generation = plan.generation
        return E

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gE):
        plan = ctx.plan
        if plan.generation != ctx.generation:
            raise RuntimeError("SEEnergy.backward: the plan ran another forward pass since")
        gx, gq = plan.backward(gE, want_x=ctx.needs_input_grad[0], want_q=ctx.needs_input_grad[1])
        return gx, gq, None
