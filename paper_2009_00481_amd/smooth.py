"""The smoothed bound as a differentiable function of the costs (App. "Smoothing").

``smoothed_bound(cost, solver, alpha, iters)`` runs the smoothed method on the GPU for ``iters``
iterations from lambda = c / |J_i| and returns LB_alpha; its backward pass is the library's
hand-written adjoint (reverse accumulation over per-iteration multiplier checkpoints, each
iteration recomputed from its checkpoint). Both directions run in ``libbddmp.so``; this module
only marshals tensors.
"""
from __future__ import annotations

import torch

from . import binding as B


class SmoothedBound(torch.autograd.Function):
    """LB_alpha(c) after a fixed number of smoothed iterations; d LB / d c by the adjoint kernels."""

    @staticmethod
    def forward(ctx, cost, solver, alpha: float, iters: int):
        assert cost.is_cuda and cost.dim() == 1 and cost.numel() == solver.plan.n
        c64 = cost.detach().to(torch.float64).contiguous()
        B.bddmp_solver_set_costs(solver.h, c64)
        nb = B.bddmp_smooth_workspace_bytes(solver.plan.h, iters)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=cost.device)
        B.bddmp_solver_smooth_run(solver.h, alpha, iters, ws, nb)
        lb = solver.lb_history(1)[-1]
        ctx.solver, ctx.alpha, ctx.iters, ctx.ws, ctx.nb = solver, float(alpha), int(iters), ws, nb
        ctx.c64, ctx.dtype = c64, cost.dtype
        return torch.tensor(lb, dtype=torch.float64, device=cost.device)

    @staticmethod
    def backward(ctx, g):
        s = ctx.solver
        grad = torch.empty(max(s.plan.n, 1), dtype=torch.float32, device=ctx.ws.device)
        # the checkpoints belong to these costs; another forward on the solver would replace them
        B.bddmp_solver_set_costs(s.h, ctx.c64)
        B.bddmp_solver_smooth_grad(s.h, ctx.alpha, ctx.iters, ctx.ws, ctx.nb, float(g.item()), grad)
        return grad[: s.plan.n].to(ctx.dtype), None, None, None


def smoothed_bound(cost, solver, alpha: float, iters: int):
    return SmoothedBound.apply(cost, solver, alpha, iters)
