"""Amplitude loss L(psi, w) = sum_i sum_q (|F(w T_i psi)|_q - a_iq)^2 (the
least-squares form of Eq. (data0)) with the hand-written adjoint as its
backward.  Gradients follow torch's complex convention dL/dRe + i dL/dIm."""
from __future__ import annotations

import torch


class AmplitudeLoss(torch.autograd.Function):
    """``AmplitudeLoss.apply(psi, w, plan)`` -> scalar float32 loss.

    The forward pass runs the library's gradient kernels once and keeps the
    gradients; backward scales them by the incoming gradient."""

    @staticmethod
    def forward(ctx, psi, w, plan):
        loss, gpsi, gw = plan.grad(psi.detach(), w.detach(), want_psi=psi.requires_grad,
                                   want_w=w.requires_grad)
        ctx.save_for_backward(*(t for t in (gpsi, gw) if t is not None))
        ctx.have = (gpsi is not None, gw is not None)
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        saved = list(ctx.saved_tensors)
        gpsi = saved.pop(0) * grad_out if ctx.have[0] else None
        gw = saved.pop(0) * grad_out if ctx.have[1] else None
        return gpsi, gw, None
