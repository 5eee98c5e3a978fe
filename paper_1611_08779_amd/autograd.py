"""Differentiable unfolded OCD: a ``torch.autograd.Function`` around
``ocd_detect`` (forward, keeping the per-sweep history of z) and
``ocd_detect_backward`` (the hand-written adjoint kernel).

Learnable quantities: the per-sweep regularisers ``lam`` ([K], the HYBRID
mode's lambda_k), the box half-width ``beta`` (a one-element tensor) and the
receive vectors ``y``.  H is not differentiated.  Both passes run in the HIP
kernels; torch only allocates and orders the work on its current stream.
"""

from __future__ import annotations

import torch

from . import (backward as _ocd_backward, detect as _ocd_detect, problem as _problem)

__all__ = ["OCDFunction", "ocd_llr"]


class OCDFunction(torch.autograd.Function):
    """llr = OCD(y; lam, beta, H) with the approximate max-log soft output."""

    @staticmethod
    def forward(ctx, y, lam, beta, H, K, Q, mode, N0, Es, storage):
        # The box half-width travels in the problem descriptor as a host scalar.
        beta_val = float(beta.detach().reshape(-1)[0].item()) if beta is not None else 0.0
        lam_c = lam.detach().contiguous().float() if lam is not None else None
        y_c = y.detach().contiguous()
        _, llr, z_hist = _ocd_detect(H, y_c, K, Q, mode, N0, Es, beta_val, lam=lam_c,
                                     storage=storage, want_z=False, want_llr=True, want_hist=True)
        ctx.save_for_backward(y_c, H, z_hist, lam_c)
        ctx.cfg = (K, Q, mode, N0, Es, beta_val, storage, lam is not None, beta is not None)
        return llr

    @staticmethod
    def backward(ctx, grad_llr):
        y, H, z_hist, lam = ctx.saved_tensors
        K, Q, mode, N0, Es, beta_val, storage, has_lam, has_beta = ctx.cfg
        dlam, dbeta, dy = _ocd_backward(H, y, z_hist, grad_llr.contiguous().float(), K, Q, mode,
                                        N0, Es, beta_val, lam=lam, storage=storage,
                                        want_dy=ctx.needs_input_grad[0])
        gy = dy if ctx.needs_input_grad[0] else None
        glam = dlam if has_lam and ctx.needs_input_grad[1] else None
        gbeta = dbeta if has_beta and ctx.needs_input_grad[2] else None
        return gy, glam, gbeta, None, None, None, None, None, None, None


def ocd_llr(y, H, K, Q, mode="hybrid", N0=1.0, Es=1.0, lam=None, beta=None, storage="f32"):
    """Differentiable LLRs [W, S, U, Q] of OCD detection (see OCDFunction)."""
    return OCDFunction.apply(y, lam, beta, H, K, Q, mode, N0, Es, storage)


def problem_of(y, H, K, Q, mode, N0, Es, beta=0.0, storage="f32"):
    W, U, B = H.shape[:3]
    return _problem(B, U, W, y.shape[1], Q, K, mode, storage, N0, Es, beta)
