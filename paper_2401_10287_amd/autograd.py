"""torch.autograd glue: log|psi| as a differentiable function of the flat
parameter vector, with the backward pass in the HIP library.

    lp = log_psi(cfg, theta, x)              # [B] FP64, forward on the GPU
    loss = (coeff.detach() * lp).sum()
    loss.backward()                          # theta.grad = sum_p coeff_p d log|psi_p| / d theta

With coeff_p = 2 (E_p - mean E) / B this is the training gradient of Eq. 6
of the paper (vmc_loss below).  Argument marshalling only.
"""
from __future__ import annotations

import torch

from . import fnvmc


class LogPsi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, x, cfg, ws):
        lp, _ = fnvmc.fn_log_psi(cfg, theta.detach(), x, ws=ws)
        ctx.save_for_backward(theta, x)
        ctx.cfg = cfg
        ctx.ws = ws
        return lp

    @staticmethod
    def backward(ctx, g):
        theta, x = ctx.saved_tensors
        grad = fnvmc.fn_log_psi_vjp(ctx.cfg, theta.detach(), x, g.detach().to(torch.float64).contiguous(), ws=ctx.ws)
        return grad, None, None, None


def log_psi(cfg: "fnvmc.Config", theta: torch.Tensor, x: torch.Tensor, ws: "fnvmc.Workspace | None" = None):
    return LogPsi.apply(theta, x, cfg, ws)


def vmc_loss(cfg: "fnvmc.Config", theta: torch.Tensor, x: torch.Tensor, e_loc: torch.Tensor,
             ws: "fnvmc.Workspace | None" = None):
    """Surrogate whose gradient is Eq. 6: 2 E_p[(E_p - E_p(E_p)) d log|psi| / d theta].
    The weights 2 (E_p - mean) / B come from the library (fn_energy_stats)."""
    _, coeff = fnvmc.fn_energy_stats(e_loc.detach().contiguous())
    return (coeff * log_psi(cfg, theta, x, ws)).sum()
