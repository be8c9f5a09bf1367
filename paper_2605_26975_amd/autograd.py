"""torch.autograd.Function wrappers of the HIP kernels.

``objective(U, graph, p, eps)`` returns F_p(U) of Eq. (1) (Section 2 of the paper) as a 0-dim
FP64 tensor and is differentiable to any order in U:

* its backward is the hand-written gradient kernel (``pspec_grad``, the EucGrad callback);
* the gradient itself is a Function whose backward (vector-Jacobian product) and forward-mode
  ``jvp`` are the fused Hessian-vector product kernel (``pspec_hvp``, the EucHessianEta callback of
  Algorithm 1).  The Hessian of Eq. (1) is symmetric, so H v serves both directions.

So ``torch.autograd.grad`` twice (reverse-over-reverse) and ``torch.autograd.forward_ad`` on the
gradient (forward-over-reverse) both land on the same HVP kernel.  The kernels take raw device
pointers, so the functorch transforms (``torch.func``), whose wrapped tensors have no storage, are
not supported.  ``eps`` caps |x|^(p-2) near x = 0 in the
Hessian (psi(x) = max(|x|, eps)^(p-2)); the objective and gradient do not depend on it.
"""
from __future__ import annotations

import torch

from . import pspec


class _Grad(torch.autograd.Function):
    """G = dF_p/dU (EucGrad); backward and jvp are Hessian-vector products (EucHessianEta)."""

    @staticmethod
    def forward(U, graph, p, eps):
        G, _ = pspec.grad(graph, U.contiguous(), p)
        return G

    @staticmethod
    def setup_context(ctx, inputs, output):
        U, graph, p, eps = inputs
        ctx.save_for_backward(U)
        ctx.save_for_forward(U)
        ctx.graph, ctx.p, ctx.eps = graph, p, eps

    @staticmethod
    def backward(ctx, gG):
        (U,) = ctx.saved_tensors
        HV = _Hvp.apply(U, gG, ctx.graph, ctx.p, ctx.eps)
        return HV, None, None, None

    @staticmethod
    def jvp(ctx, tU, _graph, _p, _eps):
        (U,) = ctx.saved_tensors
        HV, _, _ = pspec.hvp(ctx.graph, U.contiguous(), tU.contiguous(), ctx.p, ctx.eps)
        return HV


class _Hvp(torch.autograd.Function):
    """H(U) V.  Third derivatives are not provided (double backward through it raises)."""

    @staticmethod
    def forward(U, V, graph, p, eps):
        HV, _, _ = pspec.hvp(graph, U.contiguous(), V.contiguous().to(U.dtype), p, eps)
        return HV

    @staticmethod
    def setup_context(ctx, inputs, output):
        pass

    @staticmethod
    def backward(ctx, gHV):
        raise RuntimeError("third derivatives of F_p are not implemented")


class _Objective(torch.autograd.Function):
    """F_p(U) (Eq. (1)); backward is the gradient Function above."""

    @staticmethod
    def forward(U, graph, p, eps):
        F, _ = pspec.objective(graph, U.contiguous(), p)
        return F

    @staticmethod
    def setup_context(ctx, inputs, output):
        U, graph, p, eps = inputs
        ctx.save_for_backward(U)
        ctx.save_for_forward(U)
        ctx.graph, ctx.p, ctx.eps = graph, p, eps

    @staticmethod
    def backward(ctx, gF):
        (U,) = ctx.saved_tensors
        G = _Grad.apply(U, ctx.graph, ctx.p, ctx.eps)
        return gF.to(G.dtype) * G, None, None, None

    @staticmethod
    def jvp(ctx, tU, _graph, _p, _eps):
        (U,) = ctx.saved_tensors
        G, _ = pspec.grad(ctx.graph, U.contiguous(), ctx.p)
        return pspec.dot(G, tU.contiguous().to(G.dtype))


def objective(U: torch.Tensor, graph: pspec.Graph, p: float, eps: float = 1e-8) -> torch.Tensor:
    """F_p(U), differentiable in U (reverse and forward mode)."""
    return _Objective.apply(U, graph, p, eps)


def gradient(U: torch.Tensor, graph: pspec.Graph, p: float, eps: float = 1e-8) -> torch.Tensor:
    """dF_p/dU, differentiable in U (its derivative is the Hessian-vector product kernel)."""
    return _Grad.apply(U, graph, p, eps)


# Public names of the two Functions: PSpecF.apply(U, graph, p, eps) is F_p(U) as a 0-dim FP64 tensor,
# PSpecGrad.apply(U, graph, p, eps) its gradient (backward and jvp: Hessian-vector products).
PSpecF = _Objective
PSpecGrad = _Grad
