"""Differentiable unfolded OCD: a ``torch.autograd.Function`` around
``ocd_detect`` (forward, keeping the per-sweep history of z) and
``ocd_detect_backward`` (the hand-written adjoint kernel), and a second one for
the training loss itself, the mean binary cross-entropy of the LLRs against the
transmitted bits, whose forward is one launch of the training step
``ocd_detect_train_bce`` (the loss and its gradients together).

Learnable quantities: the per-sweep regularisers ``lam`` ([K], the HYBRID
mode's lambda_k), the box half-width ``beta`` (a one-element tensor) and the
receive vectors ``y``.  H is not differentiated.  Both passes run in the HIP
kernels; torch only allocates and orders the work on its current stream.
"""

from __future__ import annotations

import torch

from . import (backward as _ocd_backward, detect as _ocd_detect, problem as _problem,
               train_step as _train_step)

__all__ = ["OCDFunction", "ocd_llr", "OCDBCEFunction", "ocd_bce_loss"]


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


class OCDBCEFunction(torch.autograd.Function):
    """loss = mean over the W S U Q bits of softplus(L) - bit L, L = OCD(y; lam, beta, H):
    one launch of the training step (ocd_detect_train_bce) computes the loss and its
    gradients together; the backward only scales them by the upstream gradient."""

    @staticmethod
    def forward(ctx, y, lam, beta, H, bits, K, Q, mode, N0, Es, storage):
        beta_val = float(beta.detach().reshape(-1)[0].item()) if beta is not None else 0.0
        lam_c = lam.detach().contiguous().float() if lam is not None else None
        y_c = y.detach().contiguous()
        bits_u8 = bits.detach().to(torch.uint8).contiguous()
        loss, dlam, dbeta, dy, _, _ = _train_step(H, y_c, bits_u8, K, Q, mode, N0, Es, beta_val,
                                                  lam=lam_c, storage=storage,
                                                  want_dy=ctx.needs_input_grad[0])
        ctx.save_for_backward(dlam, dbeta, dy)
        ctx.cfg = (lam is not None, beta is not None)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_loss):
        dlam, dbeta, dy = ctx.saved_tensors
        has_lam, has_beta = ctx.cfg
        gy = dy * grad_loss if ctx.needs_input_grad[0] else None
        glam = dlam * grad_loss if has_lam and ctx.needs_input_grad[1] else None
        gbeta = dbeta * grad_loss if has_beta and ctx.needs_input_grad[2] else None
        return gy, glam, gbeta, None, None, None, None, None, None, None, None


def ocd_bce_loss(y, H, bits, K, Q, mode="hybrid", N0=1.0, Es=1.0, lam=None, beta=None,
                 storage="f32"):
    """Differentiable mean binary cross-entropy of OCD's LLRs against bits [W, S, U, Q]
    (0/1, any dtype), P(bit = 1) = sigmoid(L) (see OCDBCEFunction)."""
    return OCDBCEFunction.apply(y, lam, beta, H, bits, K, Q, mode, N0, Es, storage)


def problem_of(y, H, K, Q, mode, N0, Es, beta=0.0, storage="f32"):
    W, U, B = H.shape[:3]
    return _problem(B, U, W, y.shape[1], Q, K, mode, storage, N0, Es, beta)
