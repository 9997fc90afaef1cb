"""ctypes binding of the differentiable edge rollout (kpx_diff_* of
include/kpx.h) and a torch.autograd.Function over it: argument marshalling
only; the rollout, loss, adjoint and polish steps run in the library's HIP
kernel.

Layouts are structure-of-arrays over the E edges, as the kernel reads them:
x0 (12, E) float32, u (16, E) float32 (row 4 j + c = control c of segment j),
n (E,) int32 step counts in 4..40.  Losses are (E,), gradients (16, E).
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from .kpx import KPXError, OK, _f, lib

_vp = C.c_void_p


class DiffProblemC(C.Structure):
    _fields_ = [("dyn_params", C.c_float * 8), ("dt", C.c_float),
                ("boxes", C.POINTER(C.c_float)), ("n_boxes", C.c_int32),
                ("goal", C.c_float * 3), ("w_ctrl", C.c_float), ("w_obst", C.c_float),
                ("k_obst", C.c_float), ("d_safe", C.c_float), ("w_goal", C.c_float),
                ("u_lo", C.c_float * 4), ("u_hi", C.c_float * 4),
                ("x_lo", C.c_float * 12), ("x_hi", C.c_float * 12),
                ("ws_lo", C.c_float * 3), ("ws_hi", C.c_float * 3), ("w_len", C.c_float)]


_bound = False


def _lib():
    global _bound
    L = lib()
    if not _bound:
        i32, i64 = C.c_int32, C.c_int64
        L.kpx_diff_create.argtypes = [C.POINTER(DiffProblemC), _vp, C.POINTER(_vp)]
        L.kpx_diff_loss_grad.argtypes = [_vp, _vp, _vp, _vp, i64, _vp, _vp]
        L.kpx_diff_polish.argtypes = [_vp, _vp, _vp, _vp, i64, i32, C.c_float, _vp, _vp]
        L.kpx_diff_destroy.argtypes = [_vp]
        L.kpx_diff_last_error.argtypes = [_vp]
        L.kpx_diff_last_error.restype = C.c_char_p
        for name in ("kpx_diff_create", "kpx_diff_loss_grad", "kpx_diff_polish", "kpx_diff_destroy"):
            getattr(L, name).restype = C.c_int
        _bound = True
    return L


def diff_problem_struct(problem, dt, goal=None, w_ctrl=0.1, w_obst=1.0, k_obst=50.0, d_safe=0.02,
                        w_goal=1.0, w_len=0.0):
    """kpx_diff_problem from a workloads.Problem (QUAD12); returns (struct,
    kept-alive boxes).  The goal defaults to the problem's goal centre."""
    boxes = np.ascontiguousarray(problem.boxes, dtype=np.float32).reshape(-1, 6)
    s = DiffProblemC()
    s.dyn_params = _f(problem.dyn_params, 8)
    s.dt = dt
    s.boxes = boxes.ctypes.data_as(C.POINTER(C.c_float)) if boxes.size else None
    s.n_boxes = boxes.shape[0]
    s.goal = _f(problem.goal_center if goal is None else goal, 3)
    s.w_ctrl, s.w_obst, s.k_obst, s.d_safe, s.w_goal = w_ctrl, w_obst, k_obst, d_safe, w_goal
    s.w_len = w_len
    s.u_lo = _f(problem.u_lo, 4)
    s.u_hi = _f(problem.u_hi, 4)
    s.x_lo = _f(problem.x_lo, 12)
    s.x_hi = _f(problem.x_hi, 12)
    s.ws_lo = _f(problem.ws_lo, 3)
    s.ws_hi = _f(problem.ws_hi, 3)
    return s, boxes


def create_status(problem, dt, **weights) -> int:
    """Status of kpx_diff_create for arguments that fail host-side validation
    (no GPU call is made on those paths); used by the argument tests."""
    s, keep = diff_problem_struct(problem, dt, **weights)
    h = _vp()
    rc = _lib().kpx_diff_create(C.byref(s), None, C.byref(h))
    if rc == OK:
        _lib().kpx_diff_destroy(h)
    return rc


class Rollout:
    """A scene and loss (a kpx_diff object) on the current GPU, ordered on one
    stream (torch's current stream by default)."""

    def __init__(self, problem, dt, device: str = "cuda", stream=None, **weights):
        import torch

        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        s, self._boxes = diff_problem_struct(problem, dt, **weights)
        h = _vp()
        rc = _lib().kpx_diff_create(C.byref(s), _vp(self.stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise KPXError(rc, "kpx_diff_create")
        self.h = h

    def _check(self, rc: int):
        if rc < 0:
            raise KPXError(rc, _lib().kpx_diff_last_error(self.h).decode())

    def _args(self, x0, u, n):
        import torch

        E = int(n.numel())
        for t, rows, dt in ((x0, 12, torch.float32), (u, 16, torch.float32)):
            if t.dtype != dt or t.device != self.device or tuple(t.shape) != (rows, E) or not t.is_contiguous():
                raise ValueError(f"expected a contiguous ({rows}, {E}) {dt} tensor on {self.device}")
        if n.dtype != torch.int32 or n.device != self.device or not n.is_contiguous():
            raise ValueError("n must be a contiguous int32 tensor on the device")
        return E

    def loss_grad(self, x0, u, n, want_grad: bool = True):
        """(loss (E,), grad (16, E) or None), enqueued on the stream."""
        import torch

        E = self._args(x0, u, n)
        loss = torch.empty(E, dtype=torch.float32, device=self.device)
        grad = torch.empty((16, E), dtype=torch.float32, device=self.device) if want_grad else None
        self.loss_grad_into(x0, u, n, loss, grad)
        return loss, grad

    def loss_grad_into(self, x0, u, n, loss, grad=None):
        """As loss_grad, into caller tensors (no allocation)."""
        import torch

        E = self._args(x0, u, n)
        if loss.dtype != torch.float32 or loss.device != self.device or loss.numel() != E or not loss.is_contiguous():
            raise ValueError(f"loss must be a contiguous float32 tensor of {E} entries on {self.device}")
        if grad is not None and (grad.dtype != torch.float32 or grad.device != self.device
                                 or tuple(grad.shape) != (16, E) or not grad.is_contiguous()):
            raise ValueError(f"grad must be a contiguous (16, {E}) float32 tensor on {self.device}")
        self._check(_lib().kpx_diff_loss_grad(self.h, x0.data_ptr(), u.data_ptr(), n.data_ptr(), E,
                                              loss.data_ptr(),
                                              None if grad is None else grad.data_ptr()))

    def polish(self, x0, u, n, steps: int = 3, lr: float = 1e-3, loss=None, validity: bool = False):
        """Projected gradient steps on u in place; returns the final losses, and
        with validity=True also the first invalid step of every edge (int32)."""
        import torch

        E = self._args(x0, u, n)
        if loss is None:
            loss = torch.empty(E, dtype=torch.float32, device=self.device)
        elif loss.dtype != torch.float32 or loss.device != self.device or loss.numel() != E or not loss.is_contiguous():
            raise ValueError(f"loss must be a contiguous float32 tensor of {E} entries on {self.device}")
        bad = torch.empty(E, dtype=torch.int32, device=self.device) if validity else None
        self._check(_lib().kpx_diff_polish(self.h, x0.data_ptr(), u.data_ptr(), n.data_ptr(), E,
                                           int(steps), float(lr), loss.data_ptr(),
                                           None if bad is None else bad.data_ptr()))
        return (loss, bad) if validity else loss

    def close(self):
        if getattr(self, "h", None):
            _lib().kpx_diff_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_function():
    import torch

    class EdgeLoss(torch.autograd.Function):
        """Per-edge loss of the rollout as a differentiable function of the
        controls u (16, E): forward evaluates the loss only; backward runs the
        kernel again with the adjoint and scales the gradient by the incoming
        gradient of each edge's loss."""

        @staticmethod
        def forward(ctx, u, rollout, x0, n):
            with torch.no_grad():
                loss, _ = rollout.loss_grad(x0, u.contiguous(), n, want_grad=False)
            ctx.rollout = rollout
            ctx.save_for_backward(u, x0, n)
            return loss

        @staticmethod
        def backward(ctx, g):
            u, x0, n = ctx.saved_tensors
            _, grad = ctx.rollout.loss_grad(x0, u.contiguous(), n, want_grad=True)
            return grad * g.unsqueeze(0), None, None, None

    return EdgeLoss


_EdgeLoss = None


def edge_loss(u, rollout: Rollout, x0, n):
    """Differentiable per-edge losses (E,) of controls u (16, E)."""
    global _EdgeLoss
    if _EdgeLoss is None:
        _EdgeLoss = _make_function()
    return _EdgeLoss.apply(u, rollout, x0, n)
