"""Differentiable X-ray transform: torch.autograd.Function wrappers of the C-ABI calls.

The transform is linear, so the vector-Jacobian product of the forward projection A is
the adjoint A^T and that of the adjoint is A (Introduction: the adjoint is the transpose
of the projection matrix).  Both directions run in the library's HIP kernels; torch only
provides the tensors and the current stream.
"""
from __future__ import annotations

import torch

from .xrt import Plan


class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, img: torch.Tensor, plan: Plan, adjoint_mode: str):
        ctx.plan = plan
        ctx.adjoint_mode = adjoint_mode
        return plan.forward(img.contiguous())

    @staticmethod
    def backward(ctx, grad: torch.Tensor):
        # through _Adjoint, so that higher derivatives stay differentiable
        return _Adjoint.apply(grad, ctx.plan, ctx.adjoint_mode), None, None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sino: torch.Tensor, plan: Plan, adjoint_mode: str):
        ctx.plan = plan
        ctx.adjoint_mode = adjoint_mode
        return plan.adjoint(sino.contiguous(), mode=adjoint_mode)

    @staticmethod
    def backward(ctx, grad: torch.Tensor):
        return _Forward.apply(grad, ctx.plan, ctx.adjoint_mode), None, None


def project(img: torch.Tensor, plan: Plan, adjoint_mode: str = "auto") -> torch.Tensor:
    """A f, differentiable in f (batch dimensions in front of the image shape)."""
    return _Forward.apply(img, plan, adjoint_mode)


def backproject(sino: torch.Tensor, plan: Plan, adjoint_mode: str = "auto") -> torch.Tensor:
    """A^T g, differentiable in g."""
    return _Adjoint.apply(sino, plan, adjoint_mode)


class XrayTransform(torch.nn.Module):
    """nn.Module form of `project` for a fixed plan."""

    def __init__(self, plan: Plan, adjoint_mode: str = "auto"):
        super().__init__()
        self.plan = plan
        self.adjoint_mode = adjoint_mode

    def forward(self, img: torch.Tensor) -> torch.Tensor:
        return project(img, self.plan, self.adjoint_mode)
