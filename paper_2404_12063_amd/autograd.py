"""torch.autograd wrapper of the fused loss: the forward call computes the loss and, in the same
launch sequence, its gradient; backward only scales the stored gradient.

torch supplies memory, streams and the optimiser loop; every FLOP of the loss and its gradient
runs in the HIP library (include/vpinn.h).
"""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import vpinn as V


class VpinnLoss(torch.autograd.Function):
    """L(theta, eps) of Algorithm 3 plus the Dirichlet and sensor terms.

    forward(params, eps, problem, cfg) -> (L, components) where components = [L, L_v, L_b, L_s]
    (not differentiable).  d/dparams and d/deps come from vpinn_loss_and_grad.
    """

    @staticmethod
    def forward(ctx, params: torch.Tensor, eps: Optional[torch.Tensor], problem, cfg) -> Tuple[torch.Tensor, torch.Tensor]:
        p = params.detach().contiguous()
        e = None if eps is None else eps.detach().reshape(1).contiguous()
        loss = torch.empty(4, dtype=torch.float32, device=p.device)
        grad = torch.empty_like(p)
        geps = None if e is None else torch.empty(1, dtype=torch.float32, device=p.device)
        need_grad = ctx.needs_input_grad[0] or (eps is not None and ctx.needs_input_grad[1])
        V.vpinn_loss_and_grad(problem, cfg, p, eps=e, loss=loss, grad=grad if need_grad else None,
                              grad_eps=geps if need_grad else None)
        ctx.has_eps = eps is not None
        ctx.save_for_backward(grad, geps if geps is not None else grad.new_zeros(1))
        comps = loss.detach().clone()
        ctx.mark_non_differentiable(comps)
        return loss[0].clone(), comps

    @staticmethod
    def backward(ctx, gL, _gcomps):
        grad, geps = ctx.saved_tensors
        g_params = gL * grad
        g_eps = (gL * geps).reshape(1) if ctx.has_eps else None
        return g_params, g_eps, None, None


def vpinn_loss(params: torch.Tensor, problem, cfg, eps: Optional[torch.Tensor] = None):
    """Differentiable total loss (0-dim tensor) and its components [L, L_v, L_b, L_s]."""
    return VpinnLoss.apply(params, eps, problem, cfg)
