"""The relaxed MaxSAT loss as a differentiable PyTorch function.

Section 4 of the paper models the loss as a network whose only trainable
parameter is the relaxed assignment x and solves by backpropagation.  Here the
forward pass (scores, unsat mask, loss) and the backward pass (transposed sum,
tanh derivative) are the library's hand-written kernels behind
``torch.autograd.Function``; autograd only routes the incoming gradient.

``checkpoint=True`` keeps nothing between forward and backward and recomputes
the clause scores inside backward; the gradient is bitwise the same.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import LOSS_UNSAT, Cnf, _check, _device_points, _stream_ptr, lib


def adjoint_bytes(cnf: Cnf, restarts: int) -> int:
    out = C.c_int64()
    _check(lib().hms_adjoint_bytes(cnf.handle, int(restarts), C.byref(out)))
    return out.value


class _MaxSatLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, cnf, loss_mode, checkpoint):
        X = _device_points(x.detach().contiguous(), cnf, "x")
        R = X.shape[1]
        loss = torch.empty(R, dtype=torch.float64, device=X.device)
        unsat = torch.empty(R, dtype=torch.int64, device=X.device)
        adj = None
        if not checkpoint:
            adj = torch.empty(adjoint_bytes(cnf, R), dtype=torch.uint8, device=X.device)
        stream = _stream_ptr(None)
        _check(lib().hms_forward(cnf.handle, C.c_void_p(X.data_ptr()), R, int(loss_mode),
                                 C.c_void_p(loss.data_ptr()), C.c_void_p(unsat.data_ptr()),
                                 C.c_void_p(adj.data_ptr()) if adj is not None else None, stream))
        ctx.cnf = cnf
        ctx.loss_mode = int(loss_mode)
        ctx.shape = x.shape
        ctx.save_for_backward(X, adj if adj is not None else torch.empty(0, device=X.device))
        ctx.checkpoint = checkpoint
        ctx.mark_non_differentiable(unsat)
        return loss, unsat

    @staticmethod
    def backward(ctx, grad_loss, grad_unsat):
        X, adj = ctx.saved_tensors
        R = X.shape[1]
        gl = grad_loss.detach().to(torch.float32).contiguous()
        grad = torch.empty_like(X)
        _check(lib().hms_backward(ctx.cnf.handle, C.c_void_p(X.data_ptr()), R, ctx.loss_mode,
                                  None if ctx.checkpoint else C.c_void_p(adj.data_ptr()),
                                  C.c_void_p(gl.data_ptr()), C.c_void_p(grad.data_ptr()),
                                  _stream_ptr(None)))
        return grad.view(ctx.shape), None, None, None


def maxsat_loss(cnf: Cnf, x: torch.Tensor, loss_mode: int = LOSS_UNSAT, checkpoint: bool = False):
    """Loss per restart (float64 [R]) and unsat count per restart (int64 [R]) at
    x (cuda float32 [n] or [n][R]); differentiable in x."""
    return _MaxSatLoss.apply(x, cnf, loss_mode, checkpoint)
