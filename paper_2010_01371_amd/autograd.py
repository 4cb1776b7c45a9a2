"""torch.autograd.Function for the polyenergetic forward model.

forward:  ybar = S exp(-(Q (x) A) x), saving only the line integrals l = A x
          (no ray x energy tensor);
backward: dx = A^T [ sum_E Q_Ek (-t_E) sum_c S_cE gbar_c ], recomputing
          t_E = exp(-sum_k Q_Ek l_k) per ray (mbmd_forward_vjp).
"""

from __future__ import annotations

import torch


class PolyForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, problem):
        ybar, l = problem.forward(x.detach().contiguous(), keep_l=True)
        ctx.save_for_backward(l)
        ctx.problem = problem
        return ybar

    @staticmethod
    def backward(ctx, gbar):
        (l,) = ctx.saved_tensors
        dx = ctx.problem.forward_vjp(l, gbar.contiguous().to(torch.float32))
        return dx, None


def poly_forward(x, problem):
    return PolyForward.apply(x, problem)
