"""Differentiable camera operator.

A is linear, so the vector-Jacobian product of y = A x is A^T g: the
backward pass is the library's adjoint kernel (ltm_backproject) and the
backward of A^T is ltm_project.  No torch compute op is involved.
"""
from __future__ import annotations

import torch

from . import ltm as _ltm


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.project(x.detach().contiguous().reshape(-1))

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.backproject(g.contiguous().reshape(-1)), None


class _Backproject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, plan):
        ctx.plan = plan
        return plan.backproject(y.detach().contiguous().reshape(-1))

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.project(g.contiguous().reshape(-1)), None


def project(x: torch.Tensor, plan: "_ltm.Plan") -> torch.Tensor:
    """y = A x with autograd support (x: N float32 on the GPU)."""
    return _Project.apply(x, plan)


def backproject(y: torch.Tensor, plan: "_ltm.Plan") -> torch.Tensor:
    """x = A^T y with autograd support (y: M float32 on the GPU)."""
    return _Backproject.apply(y, plan)
