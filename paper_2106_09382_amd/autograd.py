"""Differentiable CONCORD estimate: Omega-hat(S, lam) as a torch function.

The forward pass is one CONCORD-PCD solve (concord_fit); the backward pass is
the implicit gradient through the stationarity conditions on the active set
(concord_backward), solved by the same coloured sweeps.  Both run in the
library's HIP kernels; this module only wires them into autograd.
"""
from __future__ import annotations

import torch

from . import _lib


class ConcordFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, lam, tol, maxit, btol, bmaxit):
        om, info = _lib.fit(S.contiguous(), float(lam), tol, maxit)
        ctx.save_for_backward(S, om)
        ctx.btol, ctx.bmaxit = btol, bmaxit
        ctx.fit_info = info
        return om

    @staticmethod
    def backward(ctx, grad):
        S, om = ctx.saved_tensors
        gS, gl, _ = _lib.backward(S.contiguous(), om, grad.contiguous(), ctx.btol, ctx.bmaxit)
        glam = torch.tensor(gl, dtype=S.dtype, device=S.device)
        return gS, glam, None, None, None, None


def concord(S: torch.Tensor, lam, tol: float = 1e-8, maxit: int = 1000,
            backward_tol: float = 1e-10, backward_maxit: int = 5000) -> torch.Tensor:
    """Omega-hat(S, lam), differentiable in S and lam (lam: float or 0-d tensor).

    S is the p x p (symmetric) sample covariance on the device; the returned
    gradient with respect to S is the symmetric one.  The estimate is a
    piecewise-smooth function of (S, lam): the gradient is that of the smooth
    piece on the current active set (entries with omega_ij != 0).
    """
    if not torch.is_tensor(lam):
        lam = torch.tensor(float(lam), dtype=S.dtype, device=S.device)
    return ConcordFunction.apply(S, lam, tol, maxit, backward_tol, backward_maxit)
