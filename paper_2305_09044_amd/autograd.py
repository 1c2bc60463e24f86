"""Differentiation form: the Welsch/correntropy loss of the observed residual as a
torch.autograd.Function whose forward and backward are libtrd calls.

L = sum over observed entries of sigma^2 (1 - exp(-e^2 / 2 sigma^2)), e = x - Tr(prod Z_k),
the correntropy objective of eq. (4) written as a loss (sigma = +inf: sum e^2 / 2).
Backward: dL/dZ_k = -fold(d_k) for every core, d_k of eq. (9) with the weights of
eq. (7) at the same cores (half-quadratic identity); subchain tables are rebuilt per
core inside the library rather than stored for all k.
"""
from __future__ import annotations

import torch


class CorrentropyLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, problem, sigma, *cores):
        ctx.problem = problem
        ctx.sigma = float(sigma)
        ctx.save_for_backward(*cores)
        return problem.loss_fwd(list(cores), ctx.sigma)[0]

    @staticmethod
    def backward(ctx, grad_out):
        cores = [c.contiguous() for c in ctx.saved_tensors]
        scale = float(grad_out)  # one device->host read per backward call
        grads = ctx.problem.loss_bwd(cores, ctx.sigma, grad_scale=scale)
        return (None, None, *grads)


def correntropy_loss(problem, cores, sigma):
    """Loss of the bound problem at the given cores (flat core-layout device tensors)."""
    return CorrentropyLoss.apply(problem, sigma, *cores)
