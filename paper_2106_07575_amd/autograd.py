"""torch.autograd wrappers of the HIP operator (Eq. fwd_model, Eq. gradient).

FarField: (obj, probe) -> G(obj, probe) = F(probe * obj[pos_k]).  G is linear
in obj and in probe separately, so torch's vector-Jacobian product for each
is the adjoint of that partial map applied to the incoming gradient:
grad_obj = sum_k place_k(conj(p) * F^H g_k), grad_probe = sum_k conj(obj[pos_k])
* F^H g_k -- both from the hand-written adjoint kernel (ptyg_adjoint).

MLLoss: (obj, probe) -> Phi (deviance form of Eq. ML, FP64) or F (Eq. ML),
computed with the fused GRAD kernel, which also yields the Wirtinger
derivatives dF/d conj(obj), dF/d conj(probe) (Eq. gradient).  torch's
gradient of a real loss with respect to a complex leaf is 2 dL/d conj(z)
(e.g. grad |z|^2 = 2 z), so backward returns 2 * grad_out * (grad_obj,
grad_probe).
"""
from __future__ import annotations

import torch

from . import ptyg


class FarField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, obj, probe, pos):
        far = ptyg.forward(obj.detach(), probe.detach(), pos)
        ctx.save_for_backward(obj.detach(), probe.detach(), pos)
        return far

    @staticmethod
    def backward(ctx, grad_far):
        obj, probe, pos = ctx.saved_tensors
        want_obj, want_probe = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_obj or want_probe):
            return None, None, None
        go, gp = ptyg.adjoint(grad_far.contiguous(), probe, pos, obj.shape, obj=obj, want_probe=want_probe)
        return (go if want_obj else None), (gp if want_probe else None), None


class MLLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, obj, probe, pos, data, which: str = "deviance", eps: float = 1e-32):
        want_probe = probe.requires_grad
        objective, g, gp = ptyg.grad(obj.detach(), probe.detach(), pos, data, want_probe=want_probe, eps=eps)
        ctx.save_for_backward(g, gp if gp is not None else torch.empty(0, device=obj.device))
        ctx.has_probe = gp is not None
        return objective[0] if which == "deviance" else objective[1]

    @staticmethod
    def backward(ctx, grad_out):
        g, gp = ctx.saved_tensors
        s = (2.0 * grad_out).to(torch.float32)
        go = s * g if ctx.needs_input_grad[0] else None
        gpo = s * gp if (ctx.needs_input_grad[1] and ctx.has_probe) else None
        return go, gpo, None, None, None, None


def far_field(obj: torch.Tensor, probe: torch.Tensor, pos: torch.Tensor) -> torch.Tensor:
    """Differentiable G(obj, probe): complex64 [k, n, n]."""
    return FarField.apply(obj, probe, ptyg.positions(pos))


def ml_loss(obj: torch.Tensor, probe: torch.Tensor, pos: torch.Tensor, data: torch.Tensor,
            which: str = "deviance", eps: float = 1e-32) -> torch.Tensor:
    """Differentiable Poisson objective (float64 scalar): deviance Phi or Eq. ML's F."""
    if which not in ("deviance", "eq_ml"):
        raise ValueError("which must be 'deviance' or 'eq_ml'")
    return MLLoss.apply(obj, probe, ptyg.positions(pos), data, which, eps)
