"""Differentiable multifrontal solve.

u = MFSolve.apply(K, b, plan) solves A(K) u = b with A = sum_e P_e^T K_e P_e on the GPU.  The
backward pass reuses the factors of the forward pass: lambda = A^{-T} g is one transposed
multifrontal solve (U^T then L^T sweeps), and the gradients are
    dL/db = lambda,    dL/dK_e[a, b] = -sum_r lambda[conn_e[a], r] u[conn_e[b], r].
Gradients with respect to per-element coefficients follow from torch's autograd through
whatever builds K (e.g. K = k[:, None, None] * S + M).
"""
from __future__ import annotations

import torch

from .solver import Plan


class MFSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, K: torch.Tensor, b: torch.Tensor, plan: Plan, precision: str = "fp64",
                refine_tol: float = 0.0):
        Kc = K.detach().contiguous()
        plan.factor(Kc, precision)
        bc = b.detach().contiguous()
        if refine_tol > 0:
            u, _, _ = plan.refine(Kc, bc, tol=refine_tol)
        else:
            u = plan.solve(bc)
        ctx.plan = plan
        ctx.version = plan.factor_version
        ctx.precision = precision
        ctx.save_for_backward(u, Kc)
        return u

    @staticmethod
    def backward(ctx, gu: torch.Tensor):
        plan: Plan = ctx.plan
        u, Kc = ctx.saved_tensors
        if plan.factor_version != ctx.version:
            raise RuntimeError("the plan was refactored after this forward pass; its stored "
                               "factors no longer belong to this graph")
        lam = plan.solve(gu.contiguous(), transpose=True)
        gK = plan.elem_grad(lam, u) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gK, gb, None, None, None


def mf_solve(K: torch.Tensor, b: torch.Tensor, plan: Plan, precision: str = "fp64",
             refine_tol: float = 0.0) -> torch.Tensor:
    return MFSolve.apply(K, b, plan, precision, refine_tol)
